// OTOC driver (host side).
#pragma once

#include <atomic>
#include <complex>
#include <vector>

#include "internal.hpp"

namespace syk {

size_t otoc_workspace_bytes(uint64_t n, int m, size_t elem_bytes);

// The two correlators of the random-state estimator: the regularised OTOC of Eq. (2)
// (W = chi_i, V = chi_j) and the Green function of the supplement (chi_i twice).
enum class Correlator { Otoc, Green };

template <typename T>
void apply_gamma(int N, int n, int src, int rot, const T *x, T *y, uint64_t amps, hipStream_t s);

// F[k] = mean over vectors of F_v(ts[k]) (complex); ws: otoc_workspace_bytes(2^L, m, sizeof(T)).
// cancel (may be null): checked after every t point; a non-zero value ends the run with
// SYK_ECANCELLED.
template <typename T>
void otoc_run(Hamiltonian &h, int i, int j, double beta, const std::vector<double> &ts, const syk_otoc_opts &o,
              std::vector<std::complex<double>> &F, syk_otoc_stats &st, char *ws, hipStream_t s,
              const std::atomic<int> *cancel = nullptr, Correlator kind = Correlator::Otoc);

// Argument checks of one request (throws SYK_EINVAL); j is ignored for the Green function.
void check_otoc_args(int N, int i, int j, double beta, const double *t, int nt, const syk_otoc_opts &o,
                     Correlator kind = Correlator::Otoc);

// The whole OTOC request: t = 0 prepended when missing, the chain in the dtype of `o`,
// F_raw / F_norm / F_imag (host, nt doubles, any may be null) and stats.  `ws` grows to
// otoc_workspace_bytes as needed.
void otoc_compute(Hamiltonian &H, int i, int j, double beta, const double *t, int nt, const syk_otoc_opts &o,
                  DeviceBuffer &ws, hipStream_t s, double *F_raw, double *F_norm, double *F_imag,
                  syk_otoc_stats &st, const std::atomic<int> *cancel = nullptr,
                  Correlator kind = Correlator::Otoc);

}  // namespace syk
