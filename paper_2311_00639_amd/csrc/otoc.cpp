// Regularised OTOC of Eq. (2) and the Green function of the supplement, by the
// random-state estimator of the supplement.  The OTOC is computed as
// the sum of the U-block and D-block chains ("+ swap UD"):
//
//   F_v(t) = <psi| e^{(it-b/8)H} W e^{-(it+b/4)H} V e^{(it-b/4)H} W e^{-(it+b/4)H} V e^{-bH/8} |psi>
//
// with W = chi_i, V = chi_j.  Every Majorana maps one parity block to the other, so reading
// the chain from the right, for the block A of psi and the other block B:
//   r0 = e^{-b H_A/8} psi_A,                       l  = r0
//   r2 = e^{-b H_B/4} V_BA r0                      (t-independent)
//   for increasing t:  r2 <- e^{-i dt H_B} r2,  l <- e^{-i dt H_A} l      (incremental)
//   r4 = e^{(it - b/4) H_A} W_AB r2,  r6 = e^{(-it - b/4) H_B} V_BA r4
//   F_A(t) = <l, W_AB r6> / 4          (1/4 = (1/sqrt 2)^4 from chi = gamma / sqrt 2)
// since <psi_A| e^{(it-b/8)H_A} = (e^{(-it-b/8)H_A} psi_A)^dagger = (e^{-itH_A} r0)^dagger.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "krylov.hpp"
#include "otoc.hpp"

namespace syk {

namespace {
auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
}

size_t otoc_workspace_bytes(uint64_t n, int m, size_t elem_bytes) {
    return 4 * up(static_cast<size_t>(n) * 2 * elem_bytes) + krylov_workspace_bytes(n, m, elem_bytes);
}

// y = gamma_n block mapping `src` to the other block, vectors in layout rotation `rot`
template <typename T>
void apply_gamma(int N, int n, int src, int rot, const T *x, T *y, uint64_t amps, hipStream_t s) {
    if (n == N - 1) {
        // gamma_{N-1}^{UD} = -i (from D), gamma_{N-1}^{DU} = +i (from U)
        launch_majorana<T>(0u, 0u, 0, 0.0, src == 0 ? 1.0 : -1.0, x, y, amps, s);
    } else {
        const int L = N / 2 - 1;
        uint32_t bx, bz;
        int bw;
        block_majorana(N, n, bx, bz, bw);
        launch_majorana<T>(rotr_bits(bx, rot, L), rotr_bits(bz, rot, L), bw, 1.0, 0.0, x, y, amps, s);
    }
}

template <typename T>
void otoc_run(Hamiltonian &h, int i, int j, double beta, const std::vector<double> &ts, const syk_otoc_opts &o,
              std::vector<std::complex<double>> &F, syk_otoc_stats &st, char *ws, hipStream_t s,
              const std::atomic<int> *cancel, Correlator kind) {
    const uint64_t n = 1ULL << h.L;
    const size_t vb = up(static_cast<size_t>(n) * 2 * sizeof(T));
    T *l = reinterpret_cast<T *>(ws);
    T *r2 = reinterpret_cast<T *>(ws + vb);
    T *r4 = reinterpret_cast<T *>(ws + 2 * vb);
    T *tmp = reinterpret_cast<T *>(ws + 3 * vb);
    char *kws = ws + 4 * vb;
    // every vector of the chain lives in the planner's layout rotation; overlaps are
    // invariant under the permutation
    if (use_tiled<T>(h.L) && o.autotune) autotune<T>(h, l, tmp, s, false);     // l, tmp: scratch here
    const int rot = !use_tiled<T>(h.L) ? 0 : (o.layout >= 0 ? o.layout : h.internal_rotation<T>(h.variant<T>()));
    KrylovRun<T> kr[2] = {KrylovRun<T>(h, 0, rot, n, o.krylov.m, kws, s),
                          KrylovRun<T>(h, 1, rot, n, o.krylov.m, kws, s)};
    ApplyTimer timer;
    if (o.profile) {
        kr[0].set_timer(&timer);
        kr[1].set_timer(&timer);
    }
    const int nt = static_cast<int>(ts.size());
    F.assign(nt, 0.0);
    std::vector<double> hd(2);
    using cd = std::complex<double>;
    auto prop = [&](int blk, cd z, T *v) {
        syk_krylov_stats ks{};
        kr[blk].run(z, v, v, o.krylov, ks);
        st.matvecs += ks.matvecs;
        st.substeps += ks.substeps;
        st.max_err_est = std::max(st.max_err_est, ks.err_est);
    };
    // <a, b> over the block, reduced in double on the device, read back (synchronises)
    auto overlap = [&](const T *a, const T *b) {
        launch_dot_partials<T>(a, b, n, kr[0].partials(), kr[0].n_part(), s);
        launch_reduce_partials(kr[0].partials(), kr[0].n_part(), 2, kr[0].scratch(), s);
        SYK_HIP(hipMemcpyAsync(hd.data(), kr[0].scratch(), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        SYK_HIP(hipStreamSynchronize(s));
        if (!std::isfinite(hd[0]) || !std::isfinite(hd[1])) fail(SYK_ENUMERIC, "non-finite overlap");
        return cd(hd[0], hd[1]);
    };
    int done = 0;
    const int total = o.nvec * 2 * nt;
    auto point_done = [&]() {
        ++done;
        if (o.progress) o.progress(o.progress_ctx, done, total);
        if (cancel && cancel->load()) fail(SYK_ECANCELLED, "request cancelled");
    };
    for (int v = 0; v < o.nvec; ++v) {
        for (int A = 0; A < 2; ++A) {
            const int B = 1 - A;
            // psi: the A part into l, the B part into tmp (discarded), normalised over both
            T *pu = (A == 0) ? l : tmp;
            T *pd = (A == 0) ? tmp : l;
            launch_haar_raw<T>(o.state_seed, v, h.L, rot, pu, pd, kr[0].partials(), kr[0].n_part(), s);
            launch_reduce_partials(kr[0].partials(), kr[0].n_part(), 1, kr[0].scratch(), s);
            launch_scale_pair<T>(pu, pd, n, kr[0].scratch(), s);
            if (kind == Correlator::Green) {
                // G_A(t) = <psi_A| e^{(it-b/2)H_A} chi^{AB} e^{-itH_B} chi^{BA} e^{-bH_A/2} |psi_A>:
                // l = e^{-itH_A} r0 and r2 = e^{-itH_B} chi^{BA} r0, both incremental in t
                prop(A, cd(-beta / 2.0, 0.0), l);                 // l = r0
                apply_gamma<T>(h.N, i, A, rot, l, r2, n, s);                 // gamma^{BA} r0
                double tprev = 0.0;
                for (int k = 0; k < nt; ++k) {
                    const double dt = ts[k] - tprev;
                    if (dt > 0.0) {
                        prop(B, cd(0.0, -dt), r2);
                        prop(A, cd(0.0, -dt), l);
                    }
                    tprev = ts[k];
                    apply_gamma<T>(h.N, i, B, rot, r2, tmp, n, s);            // gamma^{AB} r2
                    F[k] += 0.5 * overlap(l, tmp);             // (1/sqrt 2)^2 from chi = gamma / sqrt 2
                    point_done();
                }
                continue;
            }
            prop(A, cd(-beta / 8.0, 0.0), l);                     // l = r0
            apply_gamma<T>(h.N, j, A, rot, l, r2, n, s);                // V_BA r0
            prop(B, cd(-beta / 4.0, 0.0), r2);                     // r2
            double tprev = 0.0;
            for (int k = 0; k < nt; ++k) {
                const double t = ts[k];
                const double dt = t - tprev;
                if (dt > 0.0) {
                    prop(B, cd(0.0, -dt), r2);
                    prop(A, cd(0.0, -dt), l);
                }
                tprev = t;
                apply_gamma<T>(h.N, i, B, rot, r2, r4, n, s);           // W_AB r2
                prop(A, cd(-beta / 4.0, t), r4);                   // r4
                apply_gamma<T>(h.N, j, A, rot, r4, tmp, n, s);          // V_BA r4
                prop(B, cd(-beta / 4.0, -t), tmp);                 // r6
                apply_gamma<T>(h.N, i, B, rot, tmp, r4, n, s);          // W_AB r6
                F[k] += 0.25 * overlap(l, r4);
                point_done();
            }
        }
    }
    for (auto &f : F) f /= static_cast<double>(o.nvec);
    SYK_HIP(hipStreamSynchronize(s));
    timer.flush();
    st.apply_ms += timer.ms;
    st.apply_launches += timer.launches;
}

template void otoc_run<float>(Hamiltonian &, int, int, double, const std::vector<double> &, const syk_otoc_opts &,
                              std::vector<std::complex<double>> &, syk_otoc_stats &, char *, hipStream_t,
                              const std::atomic<int> *, Correlator);
template void otoc_run<double>(Hamiltonian &, int, int, double, const std::vector<double> &, const syk_otoc_opts &,
                               std::vector<std::complex<double>> &, syk_otoc_stats &, char *, hipStream_t,
                               const std::atomic<int> *, Correlator);

void check_otoc_args(int N, int i, int j, double beta, const double *t, int nt, const syk_otoc_opts &o,
                     Correlator kind) {
    auto require = [](bool c, const char *msg) {
        if (!c) fail(SYK_EINVAL, msg);
    };
    require(t != nullptr, "NULL argument");
    if (kind == Correlator::Green)
        require(i >= 0 && i < N, "Majorana index must lie in [0, N)");
    else
        require(i >= 0 && i < N && j >= 0 && j < N && i != j, "Majorana indices must be distinct and in [0, N)");
    require(nt >= 1, "nt must be >= 1");
    require(std::isfinite(beta) && beta >= 0.0, "beta must be finite and >= 0");
    require(o.nvec >= 1, "nvec must be >= 1");
    require(o.autotune == 0 || o.autotune == 1, "autotune must be 0 or 1");
    require(o.precision_check == 0 || o.precision_check == 1, "precision_check must be 0 or 1");
    require(o.dtype == SYK_C64 || o.dtype == SYK_C128, "invalid dtype");
    require(o.layout >= -1 && o.layout < std::max(N / 2 - 1, 1), "layout must be -1 or a rotation in [0, L)");
    check_krylov_opts(o.krylov);
    for (int k = 0; k < nt; ++k) {
        require(std::isfinite(t[k]) && t[k] >= 0.0, "t must be finite and >= 0");
        if (k) require(t[k] >= t[k - 1], "t must be non-decreasing");
    }
}

void otoc_compute(Hamiltonian &H, int i, int j, double beta, const double *t, int nt, const syk_otoc_opts &o,
                  DeviceBuffer &ws, hipStream_t s, double *F_raw, double *F_norm, double *F_imag,
                  syk_otoc_stats &st, const std::atomic<int> *cancel, Correlator kind) {
    std::vector<double> ts(t, t + nt);
    const bool prepend = ts[0] != 0.0;
    if (prepend) ts.insert(ts.begin(), 0.0);
    const uint64_t n = 1ULL << H.L;
    std::vector<std::complex<double>> F;
    st.mp_err = -1.0;
    st.mp_seconds = 0.0;
    if (o.dtype == SYK_C64) {
        ws.ensure(otoc_workspace_bytes(n, o.krylov.m, sizeof(float)));
        otoc_run<float>(H, i, j, beta, ts, o, F, st, ws.ptr(), s, cancel, kind);
    } else {
        ws.ensure(otoc_workspace_bytes(n, o.krylov.m, sizeof(double)));
        otoc_run<double>(H, i, j, beta, ts, o, F, st, ws.ptr(), s, cancel, kind);
    }
    if (o.precision_check && o.dtype == SYK_C64) {
        // the same vectors and chain with complex128 states at t = 0 and the last t
        const auto c0 = std::chrono::steady_clock::now();
        std::vector<double> tc{0.0};
        if (ts.back() > 0.0) tc.push_back(ts.back());
        syk_otoc_opts o2 = o;
        o2.dtype = SYK_C128;
        syk_krylov_default_opts(SYK_C128, &o2.krylov);
        o2.krylov.m = o.krylov.m;
        o2.krylov.reorth = o.krylov.reorth;
        o2.krylov.max_substeps = o.krylov.max_substeps;
        o2.profile = 0;
        o2.progress = nullptr;
        o2.precision_check = 0;
        std::vector<std::complex<double>> F2;
        syk_otoc_stats st2{};
        ws.ensure(otoc_workspace_bytes(n, o.krylov.m, sizeof(double)));
        otoc_run<double>(H, i, j, beta, tc, o2, F2, st2, ws.ptr(), s, cancel, kind);
        const double r0 = F2[0].real();
        double err = std::abs(F[0].real() - r0) / std::abs(r0);
        if (tc.size() > 1)
            err = std::max(err, std::abs(F.back().real() / F[0].real() - F2[1].real() / r0));
        st.mp_err = err;
        st.mp_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - c0).count();
    }
    const double f0 = F[0].real();
    const int off = prepend ? 1 : 0;
    for (int k = 0; k < nt; ++k) {
        const std::complex<double> f = F[k + off];
        if (F_raw) F_raw[k] = f.real();
        if (F_imag) F_imag[k] = f.imag();
        if (F_norm) F_norm[k] = f.real() / f0;
    }
}
template void apply_gamma<float>(int, int, int, int, const float *, float *, uint64_t, hipStream_t);
template void apply_gamma<double>(int, int, int, int, const double *, double *, uint64_t, hipStream_t);

}  // namespace syk
