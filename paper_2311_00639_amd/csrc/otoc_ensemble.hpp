// Disorder average of the normalised OTOC over a run of realisations (host driver).
#pragma once

#include "internal.hpp"

namespace syk {

// Realisation r: Hamiltonian seed d.seed + r, Haar vectors from o.state_seed + r.  Path:
// the batched persistent launch when allowed (complex64, 18 <= N <= 32, m <= 60) and not
// excluded by d.path, else the single-request path one realisation at a time.  F_rows
// (n_real x nt, may be null) receives each realisation's normalised curve; F_mean and
// F_sem (may be null) their mean and standard error.  Synchronises s.
void otoc_ensemble(const syk_ensemble_desc &d, const double *t, int nt, const syk_otoc_opts &o, double *F_mean,
                   double *F_sem, double *F_rows, syk_ensemble_stats &st, hipStream_t s);

// Whether the batched path serves this request (path == -1 chooses it when it does).
bool ensemble_batch_eligible(const syk_ensemble_desc &d, const syk_otoc_opts &o);

}  // namespace syk
