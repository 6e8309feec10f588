// extern "C" entry points of libsyk: argument checks, error translation, dispatch.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "analysis.hpp"
#include "apply_plan.hpp"
#include "batch.hpp"
#include "engine.hpp"
#include "krylov.hpp"
#include "op.hpp"
#include "otoc.hpp"
#include "otoc_ensemble.hpp"

struct syk_ham {
    syk::Hamiltonian h;
};

struct syk_engine {
    std::unique_ptr<syk::Engine> e;
};

struct syk_op {
    syk::Operator op;
};

namespace {

thread_local std::string g_last_error;

template <typename F>
syk_status guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return SYK_OK;
    } catch (const syk::Error &e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return SYK_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return SYK_EDEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return SYK_EDEVICE;
    }
}

void require(bool c, const char *msg) {
    if (!c) syk::fail(SYK_EINVAL, msg);
}

void check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) syk::fail(SYK_EDEVICE, "no HIP device available");
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

uint64_t block_amps(int N) { return 1ULL << (N / 2 - 1); }

void check_N(int N) { require(N % 2 == 0 && N >= 6 && N <= 64, "N must be even with 6 <= N <= 64"); }

}  // namespace

extern "C" {

syk_status syk_create_hamiltonian_ensemble(int N, int q, double k, uint64_t seed, syk_ensemble ensemble,
                                           syk_ham **out) {
    return guarded([&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        check_N(N);
        if (q != 4) syk::fail(SYK_EUNSUPPORTED, "only q = 4 is defined (Eq. (1))");
        require(std::isfinite(k) && k > 0.0, "k must be positive");
        require(ensemble == SYK_ENSEMBLE_EXACT_K || ensemble == SYK_ENSEMBLE_BERNOULLI, "unknown ensemble");
        auto *h = new syk_ham();
        try {
            syk::build_hamiltonian(h->h, N, k, seed, ensemble);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

syk_status syk_create_hamiltonian(int N, int q, double k, uint64_t seed, syk_ham **out) {
    return syk_create_hamiltonian_ensemble(N, q, k, seed, SYK_ENSEMBLE_EXACT_K, out);
}

syk_status syk_op_create(int L, size_t n, const uint64_t *x, const uint64_t *z, const double *c_re,
                         const double *c_im, syk_op **out) {
    return guarded([&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        require(L >= 1 && L <= 31, "L must lie in [1, 31]");
        require(n == 0 || (x && z && (c_re || c_im)), "NULL term array");
        const uint64_t mask = (1ULL << L) - 1ULL;
        auto *o = new syk_op();
        o->op.L = L;
        for (size_t a = 0; a < n; ++a) {
            if ((x[a] & ~mask) || (z[a] & ~mask)) {
                delete o;
                syk::fail(SYK_EINVAL, "Pauli string acts beyond qubit L-1");
            }
            const std::complex<double> c(c_re ? c_re[a] : 0.0, c_im ? c_im[a] : 0.0);
            if (!std::isfinite(c.real()) || !std::isfinite(c.imag())) {
                delete o;
                syk::fail(SYK_EINVAL, "non-finite coefficient");
            }
            o->op.terms.push_back(syk::OpTerm{x[a], z[a], c});
        }
        o->op.canonicalise(0.0);
        *out = o;
    });
}

syk_status syk_op_destroy(syk_op *o) {
    return guarded([&] { delete o; });
}

syk_status syk_op_product(const syk_op *a, const syk_op *b, syk_op **out) {
    return guarded([&] {
        require(a && b && out, "NULL argument");
        *out = nullptr;
        auto *o = new syk_op();
        try {
            o->op = syk::op_product(a->op, b->op);
        } catch (...) {
            delete o;
            throw;
        }
        *out = o;
    });
}

syk_status syk_op_sum(const syk_op *a, const syk_op *b, double alpha_re, double alpha_im, double beta_re,
                      double beta_im, syk_op **out) {
    return guarded([&] {
        require(a && b && out, "NULL argument");
        *out = nullptr;
        auto *o = new syk_op();
        try {
            o->op = syk::op_sum(a->op, b->op, {alpha_re, alpha_im}, {beta_re, beta_im});
        } catch (...) {
            delete o;
            throw;
        }
        *out = o;
    });
}

syk_status syk_op_adjoint(const syk_op *a, syk_op **out) {
    return guarded([&] {
        require(a && out, "NULL argument");
        *out = nullptr;
        auto *o = new syk_op();
        o->op = syk::op_adjoint(a->op);
        *out = o;
    });
}

syk_status syk_op_get_terms(const syk_op *a, size_t cap, size_t *n, uint64_t *x, uint64_t *z, double *c_re,
                            double *c_im) {
    return guarded([&] {
        require(a && n, "NULL argument");
        *n = a->op.terms.size();
        if (!x && !z && !c_re && !c_im) return;
        require(cap >= a->op.terms.size(), "cap is smaller than the number of terms");
        for (size_t i = 0; i < a->op.terms.size(); ++i) {
            const auto &t = a->op.terms[i];
            if (x) x[i] = t.x;
            if (z) z[i] = t.z;
            if (c_re) c_re[i] = t.c.real();
            if (c_im) c_im[i] = t.c.imag();
        }
    });
}

syk_status syk_op_is_hermitian(const syk_op *a, int *out) {
    return guarded([&] {
        require(a && out, "NULL argument");
        *out = syk::op_is_hermitian(a->op, 1e-13) ? 1 : 0;
    });
}

syk_status syk_op_to_hamiltonian(const syk_op *a, syk_ham **out) {
    return guarded([&] {
        require(a && out, "NULL argument");
        *out = nullptr;
        require(a->op.L >= 2, "apply needs L >= 2 qubits");
        auto *h = new syk_ham();
        try {
            syk::build_operator_hamiltonian(h->h, a->op);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

syk_status syk_destroy_hamiltonian(syk_ham *h) {
    return guarded([&] { delete h; });
}

syk_status syk_ham_get_info(const syk_ham *h, syk_ham_info *out) {
    return guarded([&] {
        require(h && out, "NULL argument");
        const auto &H = h->h;
        out->N = H.N;
        out->L = H.L;
        out->K = H.K;
        out->k = H.k;
        out->p = H.p;
        out->sigma = H.sigma;
        out->sum_J2 = H.sum_J2;
        out->seed = H.seed;
        out->block_dim = 1ULL << H.L;
    });
}

syk_status syk_get_terms(const syk_ham *h, size_t cap, int32_t *ijkl, double *J, uint64_t *xmask, uint64_t *zmask,
                         int8_t *phase_U, int8_t *phase_D) {
    return guarded([&] {
        require(h != nullptr, "NULL handle");
        const auto &H = h->h;
        require(cap >= static_cast<size_t>(H.K), "cap is smaller than the number of terms");
        const size_t K = static_cast<size_t>(H.K);
        if (ijkl) std::memcpy(ijkl, H.ijkl.data(), 4 * K * sizeof(int32_t));
        if (J) std::memcpy(J, H.J.data(), K * sizeof(double));
        if (xmask) std::memcpy(xmask, H.xmask.data(), K * sizeof(uint64_t));
        if (zmask) std::memcpy(zmask, H.zmask.data(), K * sizeof(uint64_t));
        if (phase_U) std::memcpy(phase_U, H.phase[0].data(), K);
        if (phase_D) std::memcpy(phase_D, H.phase[1].data(), K);
    });
}

syk_status syk_apply_H(const syk_ham *h, syk_block blk, syk_dtype dt, const void *x, void *y, uint64_t n_amps,
                       int nvec, uint64_t ld, void *stream) {
    return guarded([&] {
        require(h && x && y, "NULL argument");
        require(blk == SYK_BLOCK_U || blk == SYK_BLOCK_D || blk == SYK_FULL, "invalid block");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        const uint64_t nb = block_amps(h->h.N);
        require(n_amps == (blk == SYK_FULL ? 2 * nb : nb), "n_amps must equal 2^(N/2-1) (2^(N/2) for SYK_FULL)");
        require(nvec >= 1 && nvec <= 65535, "nvec must lie in [1, 65535]");
        require(ld >= n_amps, "ld must be >= n_amps");
        if (blk == SYK_FULL && h->h.ensemble < 0)
            syk::fail(SYK_EUNSUPPORTED, "an operator handle has no parity sectors");
        check_device();
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        // the full space is the U block followed by the D block
        const int b0 = blk == SYK_FULL ? SYK_BLOCK_U : blk, b1 = blk == SYK_FULL ? SYK_BLOCK_D : -1;
        if (dt == SYK_C64) {
            const float *xf = static_cast<const float *>(x);
            float *yf = static_cast<float *>(y);
            syk::apply_block<float>(H, b0, 0, xf, yf, nvec, ld, as_stream(stream));
            if (b1 >= 0) syk::apply_block<float>(H, b1, 0, xf + 2 * nb, yf + 2 * nb, nvec, ld, as_stream(stream));
        } else {
            const double *xd = static_cast<const double *>(x);
            double *yd = static_cast<double *>(y);
            syk::apply_block<double>(H, b0, 0, xd, yd, nvec, ld, as_stream(stream));
            if (b1 >= 0) syk::apply_block<double>(H, b1, 0, xd + 2 * nb, yd + 2 * nb, nvec, ld, as_stream(stream));
        }
    });
}

syk_status syk_haar_state(int N, uint64_t state_seed, int v, syk_dtype dt, void *psi_U, void *psi_D, void *stream) {
    return guarded([&] {
        check_N(N);
        require(psi_U && psi_D && psi_U != psi_D, "psi_U, psi_D must be distinct non-NULL buffers");
        require(v >= 0, "v must be >= 0");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        check_device();
        const uint64_t n = block_amps(N);
        const int np = syk::reduction_blocks(n);
        auto &ws = syk::thread_workspace(1);
        ws.ensure(static_cast<size_t>(np + 1) * sizeof(double));
        double *part = reinterpret_cast<double *>(ws.ptr());
        double *sum = part + np;
        hipStream_t s = as_stream(stream);
        if (dt == SYK_C64) {
            syk::launch_haar_raw<float>(state_seed, v, N / 2 - 1, 0, static_cast<float *>(psi_U),
                                        static_cast<float *>(psi_D), part, np, s);
            syk::launch_reduce_partials(part, np, 1, sum, s);
            syk::launch_scale_pair<float>(static_cast<float *>(psi_U), static_cast<float *>(psi_D), n, sum, s);
        } else {
            syk::launch_haar_raw<double>(state_seed, v, N / 2 - 1, 0, static_cast<double *>(psi_U),
                                         static_cast<double *>(psi_D), part, np, s);
            syk::launch_reduce_partials(part, np, 1, sum, s);
            syk::launch_scale_pair<double>(static_cast<double *>(psi_U), static_cast<double *>(psi_D), n, sum, s);
        }
        // the workspace is reused by later calls on this thread: keep it alive until done
        SYK_HIP(hipStreamSynchronize(s));
    });
}

syk_status syk_haar_state_noalloc(int N, uint64_t state_seed, int v, syk_dtype dt, void *psi_U, void *psi_D,
                                  void *stream) {
    return guarded([&] {
        check_N(N);
        require(psi_U && psi_D && psi_U != psi_D, "psi_U, psi_D must be distinct non-NULL buffers");
        require(v >= 0, "v must be >= 0");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        check_device();
        const uint64_t n = block_amps(N);
        const int np = syk::reduction_blocks(n);
        // the partials and their total live in the fixed scratch; every partial is written
        // by haar_raw before reduce_partials reads it, so nothing needs clearing
        double *part = syk::fixed_scratch(static_cast<size_t>(np) + 1);
        double *sum = part + np;
        hipStream_t s = as_stream(stream);
        if (dt == SYK_C64) {
            syk::launch_haar_raw<float>(state_seed, v, N / 2 - 1, 0, static_cast<float *>(psi_U),
                                        static_cast<float *>(psi_D), part, np, s);
            syk::launch_reduce_partials(part, np, 1, sum, s);
            syk::launch_scale_pair<float>(static_cast<float *>(psi_U), static_cast<float *>(psi_D), n, sum, s);
        } else {
            syk::launch_haar_raw<double>(state_seed, v, N / 2 - 1, 0, static_cast<double *>(psi_U),
                                         static_cast<double *>(psi_D), part, np, s);
            syk::launch_reduce_partials(part, np, 1, sum, s);
            syk::launch_scale_pair<double>(static_cast<double *>(psi_U), static_cast<double *>(psi_D), n, sum, s);
        }
    });
}

syk_status syk_apply_majorana(int N, int n, syk_block src, syk_dtype dt, const void *x, void *y, uint64_t n_amps,
                              double scale_re, double scale_im, void *stream) {
    return guarded([&] {
        check_N(N);
        require(n >= 0 && n < N, "Majorana index out of range");
        require(src == SYK_BLOCK_U || src == SYK_BLOCK_D, "invalid block");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        require(x && y, "NULL argument");
        require(n_amps == block_amps(N), "n_amps must equal 2^(N/2-1)");
        uint32_t bx = 0, bz = 0;
        int bw = 0;
        if (n < N - 1) syk::block_majorana(N, n, bx, bz, bw);
        require(x != y || bx == 0, "in-place Majorana insertion needs a string without flips");
        check_device();
        std::complex<double> sc(scale_re, scale_im);
        if (n == N - 1) sc *= std::complex<double>(0.0, src == SYK_BLOCK_U ? 1.0 : -1.0);
        hipStream_t s = as_stream(stream);
        if (dt == SYK_C64)
            syk::launch_majorana<float>(bx, bz, bw, sc.real(), sc.imag(), static_cast<const float *>(x),
                                        static_cast<float *>(y), n_amps, s);
        else
            syk::launch_majorana<double>(bx, bz, bw, sc.real(), sc.imag(), static_cast<const double *>(x),
                                         static_cast<double *>(y), n_amps, s);
    });
}

void syk_krylov_default_opts(syk_dtype dt, syk_krylov_opts *o) {
    if (!o) return;
    o->m = 30;
    o->tol = (dt == SYK_C64) ? 1e-7 : 1e-12;
    o->reorth = 0;
    o->max_substeps = 0;
}

syk_status syk_krylov_expm(const syk_ham *h, syk_block blk, syk_dtype dt, double z_re, double z_im, const void *v,
                           void *out, uint64_t n_amps, const syk_krylov_opts *o, syk_krylov_stats *stats,
                           void *stream) {
    return guarded([&] {
        if (h && !h->h.hermitian) syk::fail(SYK_EUNSUPPORTED, "Lanczos propagation needs a Hermitian operator");
        require(h && v && out && o, "NULL argument");
        require(reinterpret_cast<uintptr_t>(v) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0,
                "v and out must be 16-byte aligned");
        require(blk == SYK_BLOCK_U || blk == SYK_BLOCK_D || blk == SYK_FULL, "invalid block");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        const uint64_t nb = block_amps(h->h.N);
        require(n_amps == (blk == SYK_FULL ? 2 * nb : nb), "n_amps must equal 2^(N/2-1) (2^(N/2) for SYK_FULL)");
        require(std::isfinite(z_re) && std::isfinite(z_im), "z must be finite");
        if (blk == SYK_FULL && h->h.ensemble < 0)
            syk::fail(SYK_EUNSUPPORTED, "an operator handle has no parity sectors");
        syk::check_krylov_opts(*o);
        check_device();
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        syk_krylov_stats st{};
        auto &ws = syk::thread_workspace(0);
        hipStream_t s = as_stream(stream);
        const std::complex<double> z(z_re, z_im);
        // one block, or both halves of the full space (U first), each its own Lanczos run
        const int nblk = blk == SYK_FULL ? 2 : 1;
        for (int q = 0; q < nblk; ++q) {
            const int b = blk == SYK_FULL ? q : blk;
            const uint64_t off = static_cast<uint64_t>(q) * 2 * nb;   // in scalars
            syk_krylov_stats sq{};
            if (dt == SYK_C64) {
                ws.ensure(syk::krylov_workspace_bytes(nb, o->m, sizeof(float)));
                syk::KrylovRun<float> kr(H, b, 0, nb, o->m, ws.ptr(), s);
                kr.run(z, static_cast<const float *>(v) + off, static_cast<float *>(out) + off, *o, sq);
            } else {
                ws.ensure(syk::krylov_workspace_bytes(nb, o->m, sizeof(double)));
                syk::KrylovRun<double> kr(H, b, 0, nb, o->m, ws.ptr(), s);
                kr.run(z, static_cast<const double *>(v) + off, static_cast<double *>(out) + off, *o, sq);
            }
            st.substeps += sq.substeps;
            st.matvecs += sq.matvecs;
            st.breakdown |= sq.breakdown;
            st.err_est += sq.err_est;
            st.reorths += sq.reorths;
        }
        SYK_HIP(hipStreamSynchronize(s));
        if (stats) *stats = st;
    });
}

syk_status syk_otoc(const syk_ham *h, int i, int j, double beta, const double *t, int nt, const syk_otoc_opts *o,
                    double *F_raw, double *F_norm, double *F_imag, syk_otoc_stats *stats, void *stream) {
    return guarded([&] {
        require(h && t && o, "NULL argument");
        if (h->h.ensemble < 0) syk::fail(SYK_EUNSUPPORTED, "the OTOC needs an SYK Hamiltonian (Majorana blocks)");
        syk::check_otoc_args(h->h.N, i, j, beta, t, nt, *o);
        check_device();
        auto t0 = std::chrono::steady_clock::now();
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        syk_otoc_stats st{};
        syk::otoc_compute(H, i, j, beta, t, nt, *o, syk::thread_workspace(0), as_stream(stream), F_raw, F_norm,
                          F_imag, st);
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = st;
    });
}

syk_status syk_green(const syk_ham *h, int n, double beta, const double *t, int nt, const syk_otoc_opts *o,
                     double *G_raw, double *G_norm, double *G_imag, syk_otoc_stats *stats, void *stream) {
    return guarded([&] {
        require(h && t && o, "NULL argument");
        if (h->h.ensemble < 0) syk::fail(SYK_EUNSUPPORTED, "the Green function needs an SYK Hamiltonian (Majorana blocks)");
        syk::check_otoc_args(h->h.N, n, -1, beta, t, nt, *o, syk::Correlator::Green);
        check_device();
        auto t0 = std::chrono::steady_clock::now();
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        syk_otoc_stats st{};
        syk::otoc_compute(H, n, -1, beta, t, nt, *o, syk::thread_workspace(0), as_stream(stream), G_raw, G_norm,
                          G_imag, st, nullptr, syk::Correlator::Green);
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = st;
    });
}

syk_status syk_otoc_batch(const syk_batch_item *items, int n_items, const double *t, int nt,
                          const syk_batch_opts *o, double *F_raw, double *F_norm, double *F_imag,
                          syk_batch_stats *stats, void *stream) {
    return guarded([&] {
        require(items && t && o, "NULL argument");
        require(n_items >= 1, "n_items must be >= 1");
        require(o->nvec >= 1, "nvec must be >= 1");
        require(std::isfinite(o->beta) && o->beta >= 0.0, "beta must be finite and >= 0");
        require(o->m >= 2 && o->m <= syk::kMaxKrylov, "m must lie in [2, 60]");
        require(o->tol > 0.0 && std::isfinite(o->tol), "tol must be positive");
        require(o->variant >= -1 && o->variant < static_cast<int>(syk::batch_variants().size()),
                "variant must be -1 or a launch shape index");
        require(o->max_substeps >= 0, "max_substeps must be >= 0");
        require(nt >= 1, "nt must be >= 1");
        for (int k = 0; k < nt; ++k) {
            require(std::isfinite(t[k]) && t[k] >= 0.0, "t must be finite and >= 0");
            if (k) require(t[k] >= t[k - 1], "t must be non-decreasing");
        }
        for (int r = 0; r < n_items; ++r) {
            const syk_batch_item &it = items[r];
            check_N(it.N);
            require(it.N / 2 - 1 >= 8 && it.N / 2 - 1 <= 15, "batched items need 18 <= N <= 32");
            require(std::isfinite(it.k) && it.k > 0.0, "k must be positive");
            require(it.ensemble == SYK_ENSEMBLE_EXACT_K || it.ensemble == SYK_ENSEMBLE_BERNOULLI,
                    "unknown ensemble");
            const double C4 = it.N * (it.N - 1.0) * (it.N - 2.0) * (it.N - 3.0) / 24.0;
            if (it.ensemble == SYK_ENSEMBLE_EXACT_K) {
                const double K = std::floor(it.k * it.N + 0.5);
                require(K >= 1.0 && K <= C4, "K = round(k N) must lie in [1, C(N,4)]");
            } else {
                require(it.k * it.N <= C4, "Bernoulli ensemble needs p = k N / C(N,4) <= 1");
            }
            require(it.i >= 0 && it.i < it.N && it.j >= 0 && it.j < it.N && it.i != it.j,
                    "Majorana indices must be distinct and in [0, N)");
        }
        check_device();
        syk_batch_stats st{};
        syk::otoc_batch(items, n_items, t, nt, *o, F_raw, F_norm, F_imag, st, as_stream(stream));
        if (stats) *stats = st;
    });
}

syk_status syk_otoc_ensemble(const syk_ensemble_desc *d, const double *t, int nt, const syk_otoc_opts *o,
                             double *F_mean, double *F_sem, double *F_rows, syk_ensemble_stats *stats,
                             void *stream) {
    return guarded([&] {
        require(d && t && o, "NULL argument");
        check_N(d->N);
        require(std::isfinite(d->k) && d->k > 0.0, "k must be positive");
        require(d->ensemble == SYK_ENSEMBLE_EXACT_K || d->ensemble == SYK_ENSEMBLE_BERNOULLI, "unknown ensemble");
        require(d->n_real >= 1, "n_real must be >= 1");
        require(d->path >= -1 && d->path <= 1, "path must be -1, 0 or 1");
        syk::check_otoc_args(d->N, d->i, d->j, d->beta, t, nt, *o);
        if (d->path == 0 && !syk::ensemble_batch_eligible(*d, *o))
            syk::fail(SYK_EUNSUPPORTED, "the batched path needs complex64, 18 <= N <= 32, m <= 60 and no profiling");
        check_device();
        syk_ensemble_stats st{};
        syk::otoc_ensemble(*d, t, nt, *o, F_mean, F_sem, F_rows, st, as_stream(stream));
        if (stats) *stats = st;
    });
}

syk_status syk_crossing_time(const double *t, const double *F, const double *F_err, int nt, double F0,
                             double *tstar, double *tstar_err) {
    return guarded([&] {
        require(t && F && tstar, "NULL argument");
        require(nt >= 2, "nt must be >= 2");
        require(std::isfinite(F0), "F0 must be finite");
        for (int k = 0; k < nt; ++k) {
            require(std::isfinite(t[k]) && std::isfinite(F[k]), "t and F must be finite");
            if (F_err) require(std::isfinite(F_err[k]) && F_err[k] >= 0.0, "F_err must be finite and >= 0");
            if (k) require(t[k] >= t[k - 1], "t must be non-decreasing");
        }
        syk::crossing_time(t, F, F_err, nt, F0, *tstar, tstar_err);
    });
}

syk_status syk_lyapunov_fit(const double *N, const double *tstar, const double *tstar_err, int n,
                            const syk_fit_opts *o, syk_fit_result *out, double *pts_N, double *pts_y,
                            double *pts_err, int cap) {
    return guarded([&] {
        require(N && tstar && o && out, "NULL argument");
        require(n >= 1, "n must be >= 1");
        require(o->method == SYK_FIT_SLOPE || o->method == SYK_FIT_GLOBAL, "unknown fit method");
        require(o->terms >= 0 && o->terms <= 3, "terms must be a mask of bits 0 and 1");
        for (int a = 0; a < n; ++a) {
            require(std::isfinite(N[a]) && N[a] > 1.0, "N must be finite and > 1");
            require(std::isfinite(tstar[a]), "t* must be finite");
            if (tstar_err) require(std::isfinite(tstar_err[a]) && tstar_err[a] > 0.0, "t* errors must be positive");
        }
        const double nan = std::numeric_limits<double>::quiet_NaN();
        // points (x = N or N_mid, value, sigma)
        std::vector<double> px, py, pe;
        if (o->method == SYK_FIT_SLOPE) {
            require(o->dN >= 1, "dN must be >= 1");
            for (const auto &sp : syk::slope_points(N, tstar, tstar_err, n, o->dN)) {
                px.push_back(sp.N_mid);
                py.push_back(sp.y);
                pe.push_back(sp.err);
            }
        } else {
            for (int a = 0; a < n; ++a) {
                px.push_back(N[a]);
                py.push_back(tstar[a]);
                pe.push_back(tstar_err ? tstar_err[a] : nan);
            }
        }
        const int np = static_cast<int>(px.size());
        require(np >= 1, "no pair (N, N + dN) in the data");
        const bool t1 = o->terms & 1, t2 = o->terms & 2;
        // columns: SLOPE 1, 1/N, 1/N^2; GLOBAL 1, log N, log N/N, log N/N^2
        std::vector<double> A;
        int k = 0;
        for (int a = 0; a < np; ++a) {
            const double x = px[a];
            std::vector<double> row;
            if (o->method == SYK_FIT_SLOPE) {
                row.push_back(1.0);
                if (t1) row.push_back(1.0 / x);
                if (t2) row.push_back(1.0 / (x * x));
            } else {
                const double lg = std::log(x);
                row.push_back(1.0);
                row.push_back(lg);
                if (t1) row.push_back(lg / x);
                if (t2) row.push_back(lg / (x * x));
            }
            k = static_cast<int>(row.size());
            A.insert(A.end(), row.begin(), row.end());
        }
        std::vector<double> w(np, 1.0);
        if (tstar_err)
            for (int a = 0; a < np; ++a) {
                require(std::isfinite(pe[a]) && pe[a] > 0.0, "fit point error must be positive");
                w[a] = 1.0 / (pe[a] * pe[a]);
            }
        const syk::LsqSolution sol = syk::least_squares(A, py, w, np, k);
        std::vector<double> cov = sol.cov;
        const int dof = np - k;
        if (!tstar_err)
            for (double &c : cov) c = dof > 0 ? c * sol.rss / dof : nan;
        syk_fit_result r{};
        r.chi2 = sol.rss;
        r.n_points = np;
        r.dof = dof;
        if (o->method == SYK_FIT_SLOPE) {
            r.lambda = sol.p[0];
            r.lambda_err = std::sqrt(cov[0]);
            int c = 1;
            if (t1) { r.coef[0] = sol.p[c]; r.coef_err[0] = std::sqrt(cov[c * k + c]); ++c; }
            if (t2) { r.coef[1] = sol.p[c]; r.coef_err[1] = std::sqrt(cov[c * k + c]); }
        } else {
            // q = (gamma_0, a, b, c): lambda = 1/a, gamma_1 = b/a, gamma_2 = c/a; J dq -> dparams
            const double a = sol.p[1];
            std::vector<double> J(static_cast<size_t>(k) * k, 0.0);
            J[0] = 1.0;
            J[1 * k + 1] = -1.0 / (a * a);
            for (int c = 2; c < k; ++c) {
                J[c * k + 1] = -sol.p[c] / (a * a);
                J[c * k + c] = 1.0 / a;
            }
            auto var = [&](int row) {
                double s = 0.0;
                for (int x = 0; x < k; ++x)
                    for (int y = 0; y < k; ++y) s += J[row * k + x] * cov[x * k + y] * J[row * k + y];
                return std::sqrt(s);
            };
            r.lambda = 1.0 / a;
            r.lambda_err = var(1);
            r.coef[0] = sol.p[0];
            r.coef_err[0] = var(0);
            int c = 2;
            if (t1) { r.coef[1] = sol.p[c] / a; r.coef_err[1] = var(c); ++c; }
            if (t2) { r.coef[2] = sol.p[c] / a; r.coef_err[2] = var(c); }
        }
        if (pts_N || pts_y || pts_err) {
            require(cap >= np, "cap is below the number of fitted points");
            for (int a = 0; a < np; ++a) {
                if (pts_N) pts_N[a] = px[a];
                if (pts_y) pts_y[a] = py[a];
                if (pts_err) pts_err[a] = pe[a];
            }
        }
        *out = r;
    });
}

syk_status syk_engine_create(const syk_engine_opts *o, syk_engine **out) {
    return guarded([&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        check_device();
        syk_engine_opts d{};
        if (o) {
            require(o->max_active >= 0 && o->max_active <= 64, "max_active must lie in [0, 64]");
            d = *o;
        } else {
            d.max_bypass = -1;
        }
        auto *e = new syk_engine();
        try {
            e->e.reset(new syk::Engine(d));
        } catch (...) {
            delete e;
            throw;
        }
        *out = e;
    });
}

syk_status syk_engine_submit(syk_engine *e, const syk_request *r, uint64_t *id) {
    return guarded([&] {
        require(e && r && id, "NULL argument");
        *id = e->e->submit(*r);
    });
}

syk_status syk_engine_poll(syk_engine *e, int wait_ms, syk_result_info *info, double *F_raw, double *F_norm,
                           double *F_imag, int cap) {
    syk_status st = SYK_OK;
    const syk_status g = guarded([&] {
        require(e && info, "NULL argument");
        st = e->e->poll(wait_ms, *info, F_raw, F_norm, F_imag, cap);
        if (st == SYK_EINVAL) syk::fail(SYK_EINVAL, "cap is smaller than the request's nt");
    });
    return g != SYK_OK ? g : st;
}

syk_status syk_engine_cancel(syk_engine *e, uint64_t id) {
    return guarded([&] {
        require(e != nullptr, "NULL argument");
        e->e->cancel(id);
    });
}

syk_status syk_engine_get_stats(syk_engine *e, syk_engine_stats *st) {
    return guarded([&] {
        require(e && st, "NULL argument");
        e->e->stats(*st);
    });
}

syk_status syk_engine_destroy(syk_engine *e) {
    return guarded([&] { delete e; });
}

syk_status syk_workspace_bytes(int N, int m, syk_dtype dt, int nvec, uint64_t *bytes) {
    return guarded([&] {
        check_N(N);
        require(m >= 2 && m <= 128, "m must lie in [2, 128]");
        require(nvec >= 1, "nvec must be >= 1");
        require(bytes != nullptr, "bytes is NULL");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        const size_t e = (dt == SYK_C64) ? sizeof(float) : sizeof(double);
        *bytes = syk::otoc_workspace_bytes(block_amps(N), m, e);
    });
}

syk_status syk_tridiag_expm(int n, const double *alpha, const double *beta, double z_re, double z_im, double *c_re,
                            double *c_im) {
    return guarded([&] {
        require(n >= 1 && n <= 1024, "n must lie in [1, 1024]");
        require(alpha && c_re && c_im && (n == 1 || beta), "NULL argument");
        syk::TriExp te(n, alpha, beta);
        if (!te.ok()) syk::fail(SYK_ENUMERIC, "tridiagonal eigensolver failed");
        std::vector<std::complex<double>> c(n);
        te.apply(std::complex<double>(z_re, z_im), c.data());
        for (int i = 0; i < n; ++i) {
            c_re[i] = c[i].real();
            c_im[i] = c[i].imag();
        }
    });
}

syk_status syk_plan_blocks(const syk_ham *h, syk_block blk, syk_dtype dt, int layout, uint32_t *out, size_t cap,
                           size_t *n_words) {
    return guarded([&] {
        require(h && n_words, "NULL argument");
        require(blk == SYK_BLOCK_U || blk == SYK_BLOCK_D, "invalid block");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        require(layout >= -1 && layout < std::max(H.L, 1), "layout must be -1 or a rotation in [0, L)");
        const bool c64 = dt == SYK_C64;
        if (!(c64 ? syk::use_tiled<float>(H.L) : syk::use_tiled<double>(H.L)))
            syk::fail(SYK_EUNSUPPORTED, "the block is not served by the tiled kernel");
        const int var = c64 ? H.variant<float>() : H.variant<double>();
        const syk::TiledVariant tv = c64 ? syk::tiled_variants<float>()[var] : syk::tiled_variants<double>()[var];
        if (tv.sr != 2) syk::fail(SYK_EUNSUPPORTED, "the variant in use has no control blocks");
        const int rot = layout >= 0 ? layout : (c64 ? H.internal_rotation<float>(var) : H.internal_rotation<double>(var));
        const syk::HostPlan hp = syk::build_host_plan(H.block_terms[blk], H.L, tv.bt, tv.rb, tv.nbuf, tv.pf, rot,
                                                      c64 ? 8u : 16u, syk::resident_bits(tv), tv.sr, tv.w);
        *n_words = hp.meta.size();
        if (out) {
            require(cap >= hp.meta.size(), "cap is smaller than the control blocks");
            std::copy(hp.meta.begin(), hp.meta.end(), out);
        }
    });
}

syk_status syk_plan_describe(const syk_ham *h, syk_block blk, syk_dtype dt, int layout, syk_plan_desc *out) {
    return guarded([&] {
        require(h && out, "NULL argument");
        require(blk == SYK_BLOCK_U || blk == SYK_BLOCK_D, "invalid block");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        require(layout >= -1 && layout < std::max(H.L, 1), "layout must be -1 or a rotation in [0, L)");
        *out = syk_plan_desc{};
        const bool c64 = dt == SYK_C64;
        out->tiled = c64 ? syk::use_tiled<float>(H.L) : syk::use_tiled<double>(H.L);
        if (!out->tiled) {
            out->n_groups = syk::gather_groups(H.block_terms[blk]);
            return;
        }
        const int var = c64 ? H.variant<float>() : H.variant<double>();
        const syk::TiledVariant tv = c64 ? syk::tiled_variants<float>()[var] : syk::tiled_variants<double>()[var];
        const int bt = tv.bt, rb = tv.rb;
        out->tile_bits = bt;
        out->variant = var;
        const int rot = layout >= 0 ? layout : (c64 ? H.internal_rotation<float>(var) : H.internal_rotation<double>(var));
        const syk::HostPlan hp = syk::build_host_plan(H.block_terms[blk], H.L, bt, rb, tv.nbuf, tv.pf, rot, c64 ? 8u : 16u,
                                                      syk::resident_bits(tv), tv.sr, tv.w);
        // consistency: the workgroups' tiles cover the block once, and every (tile, term)
        // pair is applied exactly once over the partner schedule
        std::vector<char> seen(hp.n_tiles, 0);
        for (uint32_t t0 : hp.tile_map)
            for (uint32_t h : hp.hvec) {
                const uint32_t t = t0 ^ h;
                if (t >= hp.n_tiles || seen[t]) syk::fail(SYK_EDEVICE, "tile map is not a bijection");
                seen[t] = 1;
            }
        const size_t tpw = hp.hvec.size();
        for (size_t i = 0; i < tpw; ++i) {
            std::vector<int> hits(H.K, 0);
            for (int st = 0; st < hp.n_pi; ++st) {
                const uint32_t *r = &hp.ranges[(st * tpw + i) * 3];
                for (uint32_t a = r[0]; a < r[2]; ++a) ++hits[a];
            }
            for (int a = 0; a < H.K; ++a)
                if (hits[a] != 1) syk::fail(SYK_EDEVICE, "partner schedule does not apply every term once");
        }
        out->rot = rot;
        out->n_groups = hp.D;
        out->tiles_per_wg = static_cast<int>(tpw);
        out->n_partners = hp.n_partners;
        out->classes_xcd = hp.classes_xcd;
        out->classes_gpu = hp.classes_gpu;
        out->res_bits = hp.res_bits;
        out->n_tiles = hp.n_tiles;
    });
}

syk_status syk_autotune(const syk_ham *h, syk_dtype dt, int *variant, float *ms, int cap, void *stream) {
    return guarded([&] {
        require(h != nullptr, "NULL handle");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        check_device();
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        const uint64_t n = 1ULL << H.L;
        const size_t es = (dt == SYK_C64) ? 2 * sizeof(float) : 2 * sizeof(double);
        auto &ws = syk::thread_workspace(0);
        ws.ensure(2 * n * es);
        hipStream_t s = as_stream(stream);
        std::vector<float> times;
        int v = (dt == SYK_C64)
                    ? syk::autotune<float>(H, reinterpret_cast<float *>(ws.ptr()),
                                           reinterpret_cast<float *>(ws.ptr() + n * es), s, true, &times)
                    : syk::autotune<double>(H, reinterpret_cast<double *>(ws.ptr()),
                                            reinterpret_cast<double *>(ws.ptr() + n * es), s, true, &times);
        SYK_HIP(hipStreamSynchronize(s));
        if (variant) *variant = v;
        if (ms)
            for (int k = 0; k < cap; ++k) ms[k] = k < static_cast<int>(times.size()) ? times[k] : -1.0f;
    });
}

syk_status syk_select_variant(const syk_ham *h, syk_dtype dt, int variant) {
    return guarded([&] {
        require(h != nullptr, "NULL handle");
        require(dt == SYK_C64 || dt == SYK_C128, "invalid dtype");
        const int nv = (dt == SYK_C64) ? static_cast<int>(syk::tiled_variants<float>().size())
                                       : static_cast<int>(syk::tiled_variants<double>().size());
        require(variant >= 0 && variant < nv, "variant out of range (see syk_autotune's ms array)");
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;     // host-only use: plans of device 0
        auto &H = const_cast<syk::Hamiltonian &>(h->h);
        std::lock_guard<std::mutex> g(H.dev_mu);
        H.tuned[{dt == SYK_C128 ? 1 : 0, dev}] = variant;
    });
}

syk_status syk_release_workspace(void) {
    return guarded([&] {
        check_device();
        syk::thread_workspace(0).release();
        syk::thread_workspace(1).release();
    });
}

const char *syk_status_string(syk_status s) {
    switch (s) {
        case SYK_OK: return "SYK_OK";
        case SYK_EINVAL: return "SYK_EINVAL";
        case SYK_EUNSUPPORTED: return "SYK_EUNSUPPORTED";
        case SYK_ENOMEM: return "SYK_ENOMEM";
        case SYK_EDEVICE: return "SYK_EDEVICE";
        case SYK_ENOTCONV: return "SYK_ENOTCONV";
        case SYK_ENUMERIC: return "SYK_ENUMERIC";
        case SYK_ECANCELLED: return "SYK_ECANCELLED";
        case SYK_EAGAIN: return "SYK_EAGAIN";
    }
    return "SYK_UNKNOWN";
}

const char *syk_last_error(void) { return g_last_error.c_str(); }

const char *syk_kernel_revision(void) { return "tiled-block-14"; }

}  // extern "C"
