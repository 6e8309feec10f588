// Disorder average of the normalised OTOC of Eq. (2), the quantity whose crossing of F0
// defines t*(N) (main text before Eq. (4)): each realisation is normalised by its own
// F(0), then the curves are averaged with their standard error.
#include "otoc_ensemble.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "batch.hpp"
#include "otoc.hpp"

namespace syk {

bool ensemble_batch_eligible(const syk_ensemble_desc &d, const syk_otoc_opts &o) {
    const int L = d.N / 2 - 1;
    return o.dtype == SYK_C64 && L >= 8 && L <= 15 && o.krylov.m <= kMaxKrylov && o.profile == 0;
}

void otoc_ensemble(const syk_ensemble_desc &d, const double *t, int nt, const syk_otoc_opts &o, double *F_mean,
                   double *F_sem, double *F_rows, syk_ensemble_stats &st, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int R = d.n_real;
    std::vector<double> rows(static_cast<size_t>(R) * nt);
    const bool batch = d.path == 0 || (d.path == -1 && ensemble_batch_eligible(d, o));
    st = syk_ensemble_stats{};
    if (batch) {
        std::vector<syk_batch_item> items(R);
        for (int r = 0; r < R; ++r)
            items[r] = syk_batch_item{d.N, d.k, d.seed + static_cast<uint64_t>(r), d.i, d.j,
                                      o.state_seed + static_cast<uint64_t>(r), d.ensemble};
        syk_batch_opts bo{o.nvec, d.beta, o.krylov.m, o.krylov.tol, -1, o.krylov.max_substeps};
        syk_batch_stats bs{};
        otoc_batch(items.data(), R, t, nt, bo, nullptr, rows.data(), nullptr, bs, s);
        st.path = 0;
        st.matvecs = bs.matvecs;
    } else {
        DeviceBuffer ws;
        syk_otoc_opts oo = o;
        for (int r = 0; r < R; ++r) {
            Hamiltonian h;
            build_hamiltonian(h, d.N, d.k, d.seed + static_cast<uint64_t>(r), d.ensemble);
            oo.state_seed = o.state_seed + static_cast<uint64_t>(r);
            syk_otoc_stats os{};
            otoc_compute(h, d.i, d.j, d.beta, t, nt, oo, ws, s, nullptr, rows.data() + static_cast<size_t>(r) * nt,
                         nullptr, os);
            st.matvecs += os.matvecs;
        }
        st.path = 1;
    }
    for (int n = 0; n < nt; ++n) {
        double m = 0.0;
        for (int r = 0; r < R; ++r) m += rows[static_cast<size_t>(r) * nt + n];
        m /= R;
        double v = 0.0;
        for (int r = 0; r < R; ++r) {
            const double e = rows[static_cast<size_t>(r) * nt + n] - m;
            v += e * e;
        }
        if (F_mean) F_mean[n] = m;
        if (F_sem) F_sem[n] = R > 1 ? std::sqrt(v / (R - 1) / R) : 0.0;
    }
    if (F_rows) std::copy(rows.begin(), rows.end(), F_rows);
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace syk
