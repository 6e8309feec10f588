// Lanczos propagator out = e^{z H_blk} v (the restarted Krylov time evolution of
// supplement Sec. I.A), with a-posteriori step control.
//
// One sub-step: Lanczos on the normalised start vector builds V_k and the real symmetric
// tridiagonal T_k (alpha_j = Re <v_j, H v_j - beta_{j-1} v_{j-1}>, beta_j = ||w_j||, both
// reduced in double on the device).  The small exponential c(tau) = e^{tau z T_k} e_1 comes
// from the eigendecomposition of T_k (implicit QL, double).  The estimate
// err(tau) = beta_k |c_{k-1}(tau)| bounds the error of ||v|| V_k c(tau) relative to ||v||
// (Saad 1992).  A sub-step of fraction tau of z is accepted when err(tau) <= tol * tau,
// so accepted errors sum to at most tol.  beta_k ~ 0 means V_k spans an invariant
// subspace and the result is exact.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "krylov.hpp"

namespace syk {

// ------------------------------------------------------------------ tridiagonal eigensolver
// Implicit QL iteration with shifts for a real symmetric tridiagonal matrix (Bowdler,
// Martin, Reinsch & Wilkinson, Numer. Math. 11 (1968)): d <- eigenvalues, Z <- orthonormal
// eigenvectors (column k of Z, row-major n x n).  e[i] couples d[i] and d[i+1].
bool tridiag_eig(int n, std::vector<double> &d, std::vector<double> e, std::vector<double> &Z) {
    Z.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Z[static_cast<size_t>(i) * n + i] = 1.0;
    e.resize(n, 0.0);
    e[n - 1] = 0.0;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 200) return false;
            // shift: eigenvalue of the leading 2x2 block closest to d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {          // underflow: split here and restart the sweep
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int k = 0; k < n; ++k) {
                    double *row = &Z[static_cast<size_t>(k) * n];
                    const double zf = row[i + 1];
                    row[i + 1] = s * row[i] + c * zf;
                    row[i] = c * row[i] - s * zf;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

TriExp::TriExp(int n, const double *alpha, const double *beta_off) : n_(n) {
    lam_.assign(alpha, alpha + n);
    std::vector<double> e(std::max(n, 1), 0.0);
    for (int i = 0; i + 1 < n; ++i) e[i] = beta_off[i];
    ok_ = tridiag_eig(n, lam_, e, Z_);
    for (double v : lam_)
        if (!std::isfinite(v)) ok_ = false;
}

// c = Z diag(e^{z lam}) Z^T e_1
void TriExp::apply(std::complex<double> z, std::complex<double> *c) const {
    std::vector<std::complex<double>> w(n_);
    for (int k = 0; k < n_; ++k) w[k] = std::exp(z * lam_[k]) * Z_[k];          // Z[0][k] = Z_[k]
    for (int i = 0; i < n_; ++i) {
        std::complex<double> acc = 0.0;
        const double *row = &Z_[static_cast<size_t>(i) * n_];
        for (int k = 0; k < n_; ++k) acc += row[k] * w[k];
        c[i] = acc;
    }
}

std::complex<double> TriExp::last(std::complex<double> z) const {
    std::complex<double> acc = 0.0;
    const double *row = &Z_[static_cast<size_t>(n_ - 1) * n_];
    for (int k = 0; k < n_; ++k) acc += row[k] * std::exp(z * lam_[k]) * Z_[k];
    return acc;
}

// ------------------------------------------------------------------ apply_H timing
ApplyTimer::~ApplyTimer() {
    for (auto e : pool_) ignore_status(hipEventDestroy(e));
}

void ApplyTimer::begin(hipStream_t s) {
    while (pool_.size() < used_ + 2) {
        hipEvent_t e;
        SYK_HIP(hipEventCreate(&e));
        pool_.push_back(e);
    }
    SYK_HIP(hipEventRecord(pool_[used_], s));
}

void ApplyTimer::end(hipStream_t s) {
    SYK_HIP(hipEventRecord(pool_[used_ + 1], s));
    used_ += 2;
}

void ApplyTimer::flush() {
    for (size_t k = 0; k + 1 < used_; k += 2) {
        float t = 0.0f;
        SYK_HIP(hipEventElapsedTime(&t, pool_[k], pool_[k + 1]));
        ms += t;
        launches += 1;
    }
    used_ = 0;
}

// ------------------------------------------------------------------ Lanczos driver
static int log2_of(uint64_t n) { return 63 - __builtin_clzll(n); }

void check_krylov_opts(const syk_krylov_opts &o) {
    auto require = [](bool c, const char *msg) {
        if (!c) fail(SYK_EINVAL, msg);
    };
    require(o.m >= 2 && o.m <= 128, "Krylov m must lie in [2, 128]");
    require(o.tol > 0.0 && std::isfinite(o.tol), "Krylov tol must be positive");
    require(o.reorth >= 0 && o.reorth <= 3, "reorth must be 0, 1, 2 or 3");
    require(o.max_substeps >= 0, "max_substeps must be >= 0");
}

// bytes from one Krylov basis vector to the next: the vector rounded up to 256 bytes plus
// 4 KiB, so that vectors read side by side (the recombination reads up to m of them at the
// same index) do not all start at the same low address bits (measured on a 60-vector
// recombination of 2^27 complex64 amplitudes: 11.7 ms against 12.9 ms with a stride of
// exactly 1 GiB)
static size_t basis_stride_bytes(uint64_t n, size_t elem_bytes) {
    return ((static_cast<size_t>(n) * 2 * elem_bytes + 255) & ~static_cast<size_t>(255)) + 4096;
}

size_t krylov_workspace_bytes(uint64_t n, int m, size_t elem_bytes) {
    const size_t vec = basis_stride_bytes(n, elem_bytes);
    const size_t part = static_cast<size_t>(reduction_blocks(n)) * 2 * (m + 2) * sizeof(double);
    const size_t scal = static_cast<size_t>(8 * (m + 4)) * sizeof(double);
    const size_t fused = static_cast<size_t>(lanczos_partials_max(log2_of(n))) * 4 * sizeof(double);
    auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    return static_cast<size_t>(m + 1) * up(vec) + up(part) + up(scal) + up(fused);
}

template <typename T>
KrylovRun<T>::KrylovRun(Hamiltonian &h, int blk, int rot, uint64_t n, int m, char *ws, hipStream_t s)
    : h_(h), blk_(blk), rot_(rot), n_(n), m_(m), s_(s) {
    auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    vec_stride_ = basis_stride_bytes(n, sizeof(T)) / (2 * sizeof(T));
    basis_ = reinterpret_cast<T *>(ws);
    char *p = ws + static_cast<size_t>(m + 1) * vec_stride_ * 2 * sizeof(T);
    n_part_ = reduction_blocks(n);
    partials_ = reinterpret_cast<double *>(p);
    p += up(static_cast<size_t>(n_part_) * 2 * (m + 2) * sizeof(double));
    alpha_ = reinterpret_cast<double *>(p);   // 2 (m+1)
    beta2_ = alpha_ + 2 * (m + 2);            // m+2
    coef_ = beta2_ + (m + 2);                 // 2 (m+2)
    scratch_ = coef_ + 2 * (m + 2);           // 2 (m+2)
    p += up(static_cast<size_t>(8 * (m + 4)) * sizeof(double));
    fused_ = reinterpret_cast<double *>(p);   // 4 per tile
}

template <typename T>
double KrylovRun<T>::norm(const T *v) {
    launch_norm2_partials<T>(v, n_, partials_, n_part_, s_);
    launch_reduce_partials(partials_, n_part_, 1, scratch_, s_);
    double h = 0.0;
    SYK_HIP(hipMemcpyAsync(&h, scratch_, sizeof(double), hipMemcpyDeviceToHost, s_));
    SYK_HIP(hipStreamSynchronize(s_));
    if (timer_) timer_->flush();
    if (!std::isfinite(h)) fail(SYK_ENUMERIC, "non-finite norm in Krylov propagation");
    return std::sqrt(h);
}

// one Lanczos iteration j: fills slot j+1, alpha[j], beta2[j+1]
template <typename T>
bool KrylovRun<T>::iterate(int j, int reorth) {
    T *vj = vec(j);
    T *w = vec(j + 1);
    if (reorth == 0 && use_tiled<T>(h_.L)) {
        // fused step: the apply epilogue forms w = H v_j - beta v_{j-1} and the sums for
        // alpha_j and beta_j; one more pass normalises
        // basis slots hold u_i unnormalised (||u_i|| = beta_{i-1}); the scales enter the
        // apply epilogue, the residual pass and the recombination coefficients
        LanczosFuse<T> lf;
        lf.vprev = j > 0 ? vec(j - 1) : nullptr;
        lf.vcur = vj;
        lf.beta2 = beta2_;
        lf.j = j;
        lf.partials = fused_;
        if (timer_) timer_->begin(s_);
        const int np = apply_block_lanczos<T>(h_, blk_, rot_, vj, w, lf, s_);
        if (timer_) timer_->end(s_);
        launch_lanczos_scalars(fused_, np, alpha_ + 2 * j, nullptr, s_);
        // alpha_j is formed: the epilogue's partials buffer takes the residual's partials
        // (the stage buffer needs 512 doubles; tiled blocks have at least 2^18 amplitudes)
        if (static_cast<size_t>(n_part_) * 2 * (m_ + 2) < 512) fail(SYK_EDEVICE, "partials buffer too small");
        launch_lanczos_residual<T>(w, vj, alpha_ + 2 * j, beta2_, j, n_, fused_,
                                   lanczos_partials_max(log2_of(n_)) * 4, partials_, beta2_ + j + 1, s_);
        unnormalised_ = true;
        return false;
    }
    if (timer_) timer_->begin(s_);
    apply_block<T>(h_, blk_, rot_, vj, w, 1, n_, s_);
    if (timer_) timer_->end(s_);
    launch_lanczos_orth1<T>(w, j > 0 ? vec(j - 1) : nullptr, vj, beta2_ + j, n_, partials_, n_part_, s_);
    launch_reduce_partials(partials_, n_part_, 2, alpha_ + 2 * j, s_);
    launch_lanczos_orth2<T>(w, vj, alpha_ + 2 * j, n_, partials_, n_part_, s_);
    // reorth 1: one more pass against v_{j-1}, v_j; reorth 2: two full classical
    // Gram-Schmidt passes against v_0 .. v_j; reorth 3: the same two passes on the steps
    // where the estimated loss of orthogonality calls for them
    bool full = reorth == 2;
    if (reorth == 3) {
        launch_reduce_partials(partials_, n_part_, 1, beta2_ + j + 1, s_);
        full = partial_estimate(j);
    }
    if (reorth == 1 || full) {
        const int first = (reorth == 1) ? std::max(0, j - 1) : 0;
        const int nb = j + 1 - first;
        for (int pass = 0; pass < (full ? 2 : 1); ++pass) {
            launch_multi_dot_partials<T>(vec(first), vec_stride_, nb, w, n_, partials_, n_part_, s_);
            launch_reduce_partials(partials_, n_part_, 2 * nb, scratch_, s_);
            launch_subtract_proj<T>(w, vec(first), vec_stride_, nb, scratch_, n_, s_);
        }
        launch_norm2_partials<T>(w, n_, partials_, n_part_, s_);
    }
    launch_reduce_partials(partials_, n_part_, 1, beta2_ + j + 1, s_);
    launch_lanczos_normalize<T>(w, beta2_ + j + 1, n_, s_);
    return full;
}

// Partial reorthogonalisation (H. D. Simon, Math. Comp. 42 (1984) 115-142).  With
// normalised Lanczos vectors and beta_j v_{j+1} = H v_j - alpha_j v_j - beta_{j-1} v_{j-1},
// omega_{j,k} = <v_j, v_k> obeys
//   beta_j omega_{j+1,k} = beta_k omega_{j,k+1} + (alpha_k - alpha_j) omega_{j,k}
//                          + beta_{k-1} omega_{j,k-1} - beta_{j-1} omega_{j-1,k}
// up to rounding, which is modelled by adding 2 eps ||T|| with the sign of the sum
// (omega_{j,j} = 1, omega_{j+1,j} = eps).  When max_k |omega_{j+1,k}| exceeds sqrt(eps),
// v_{j+1} is reorthogonalised against every earlier vector, and so is v_{j+2} (the loss
// of v_{j+1} also reaches the next vector through the recurrence); the estimates of a
// reorthogonalised vector are reset to eps.  eps is the unit roundoff of the vectors.
template <typename T>
bool KrylovRun<T>::partial_estimate(int j) {
    const double eps = sizeof(T) == 4 ? 5.9604644775390625e-8 : 1.1102230246251565e-16;
    ha_.resize(static_cast<size_t>(m_) + 1);
    hb_.resize(static_cast<size_t>(m_) + 2);
    double ab[2];
    std::vector<double> b2(static_cast<size_t>(j) + 2);
    SYK_HIP(hipMemcpyAsync(ab, alpha_ + 2 * j, 2 * sizeof(double), hipMemcpyDeviceToHost, s_));
    SYK_HIP(hipMemcpyAsync(b2.data(), beta2_, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s_));
    SYK_HIP(hipStreamSynchronize(s_));
    ha_[j] = ab[0];
    for (int k = 0; k <= j; ++k) hb_[k] = std::sqrt(b2[k + 1]);   // beta_k = ||w_k||
    if (!std::isfinite(ha_[j]) || !std::isfinite(hb_[j])) fail(SYK_ENUMERIC, "non-finite Lanczos scalars");
    if (j == 0) {
        omega_[0].assign(static_cast<size_t>(m_) + 2, 0.0);
        omega_[1].assign(static_cast<size_t>(m_) + 2, 0.0);
        omega_[1][0] = 1.0;                  // row 0: <v_0, v_0>
        anorm_ = 0.0;
        force_next_ = false;
    }
    anorm_ = std::max({anorm_, std::fabs(ha_[j]), hb_[j]});
    const double bj = hb_[j];
    std::vector<double> next(static_cast<size_t>(m_) + 2, 0.0);
    double worst = 0.0;
    if (bj > 0.0) {
        const std::vector<double> &cur = omega_[1], &prev = omega_[0];
        for (int k = 0; k < j; ++k) {
            double t = hb_[k] * cur[k + 1] + (ha_[k] - ha_[j]) * cur[k];
            if (k > 0) t += hb_[k - 1] * cur[k - 1];
            if (j > 0) t -= hb_[j - 1] * prev[k];
            t += std::copysign(2.0 * eps * anorm_, t);
            next[k] = t / bj;
            worst = std::max(worst, std::fabs(next[k]));
        }
    }
    next[j] = eps;
    next[j + 1] = 1.0;
    const bool due = force_next_ || worst > std::sqrt(eps);
    force_next_ = due && !force_next_;
    if (due)
        for (int k = 0; k <= j; ++k) next[k] = eps;
    omega_[0].swap(omega_[1]);
    omega_[1].swap(next);
    return due;
}

template <typename T>
void KrylovRun<T>::run(std::complex<double> z, const T *v, T *out, const syk_krylov_opts &o, syk_krylov_stats &st) {
    double nrm = norm(v);
    if (nrm == 0.0 || z == std::complex<double>(0.0, 0.0)) {
        if (out != v) launch_scale_copy<T>(v, out, n_, 1.0, s_);
        return;
    }
    const bool every = n_ >= (1ULL << 20);        // large vectors: a host check per iteration is cheap
    double remaining = 1.0;
    const T *cur = v;
    std::vector<double> ha(2 * (m_ + 2)), hb(m_ + 2);
    std::vector<std::complex<double>> c(m_ + 1);
    std::vector<double> coef(2 * (m_ + 1));
    while (remaining > 0.0) {
        if (o.max_substeps > 0 && st.substeps >= o.max_substeps)
            fail(SYK_ENOTCONV, "Krylov propagation exceeded max_substeps");
        launch_scale_copy<T>(cur, vec(0), n_, 1.0 / nrm, s_);
        SYK_HIP(hipMemsetAsync(beta2_, 0, sizeof(double), s_));
        unnormalised_ = false;
        int k = 0;                 // Lanczos vectors built
        double tau = 0.0;
        bool done = false;
        int next_check = every ? 1 : 4;
        for (int j = 0; j < m_ && !done; ++j) {
            if (iterate(j, o.reorth)) st.reorths += 1;
            k = j + 1;
            st.matvecs += 1;
            if (k < next_check && k < m_) continue;
            next_check = every ? k + 1 : k + std::max(2, k / 4);
            SYK_HIP(hipMemcpyAsync(ha.data(), alpha_, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s_));
            SYK_HIP(hipMemcpyAsync(hb.data(), beta2_, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, s_));
            SYK_HIP(hipStreamSynchronize(s_));
            if (timer_) timer_->flush();
            std::vector<double> al(k), bo(std::max(k - 1, 1));
            double tnorm = 0.0;
            for (int i = 0; i < k; ++i) {
                al[i] = ha[2 * i];
                if (!std::isfinite(al[i])) fail(SYK_ENUMERIC, "non-finite Lanczos alpha");
                tnorm = std::max(tnorm, std::fabs(al[i]));
            }
            for (int i = 0; i + 1 < k; ++i) {
                bo[i] = std::sqrt(hb[i + 1]);
                tnorm = std::max(tnorm, bo[i]);
            }
            const double bk = std::sqrt(hb[k]);
            if (!std::isfinite(bk)) fail(SYK_ENUMERIC, "non-finite Lanczos beta");
            TriExp te(k, al.data(), bo.data());
            if (!te.ok()) fail(SYK_ENUMERIC, "tridiagonal eigensolver failed");
            const bool breakdown = bk <= 1e-14 * std::max(tnorm, 1e-300);
            auto err = [&](double f) { return breakdown ? 0.0 : bk * std::abs(te.last(f * z)); };
            if (err(remaining) <= o.tol * remaining) {
                tau = remaining;
                done = true;
                if (breakdown) st.breakdown = 1;
            } else if (k == m_) {
                // largest fraction f <= remaining with err(f) <= tol f (bisection in log f)
                double lo = 0.0, hi = remaining;
                for (int it = 0; it < 200; ++it) {
                    const double mid = (lo == 0.0) ? hi * 0.5 : std::sqrt(lo * hi);
                    if (err(mid) <= o.tol * mid)
                        lo = mid;
                    else
                        hi = mid;
                    if (lo > 0.0 && hi / lo < 1.0 + 1e-3) break;
                    if (lo == 0.0 && hi < 1e-14 * remaining) break;
                }
                if (lo <= 1e-12 * remaining) fail(SYK_ENOTCONV, "Krylov step size underflow (tolerance too strict)");
                tau = lo;
                done = true;
            }
            if (done) {
                te.apply(tau * z, c.data());
                st.err_est += err(tau);
                for (int i = 0; i < k; ++i) {
                    // fused path: slot i >= 1 holds u_i = ||u_i|| v_i
                    const double ni = std::sqrt(hb[i]);
                    const double sc = (unnormalised_ && i >= 1) ? (ni > 1e-300 ? nrm / ni : 0.0) : nrm;
                    coef[2 * i] = sc * c[i].real();
                    coef[2 * i + 1] = sc * c[i].imag();
                }
            }
        }
        // the combination writes `out`; the start vector already lives in the basis
        SYK_HIP(hipMemcpyAsync(coef_, coef.data(), 2 * k * sizeof(double), hipMemcpyHostToDevice, s_));
        launch_combine<T>(basis_, vec_stride_, k, coef_, out, n_, s_);
        st.substeps += 1;
        remaining -= tau;
        if (remaining <= 1e-15) break;
        cur = out;
        nrm = norm(out);
        if (nrm == 0.0) break;
    }
}

template class KrylovRun<float>;
template class KrylovRun<double>;

}  // namespace syk
