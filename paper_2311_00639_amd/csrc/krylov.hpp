// Lanczos propagator and the small tridiagonal exponential (host side).
#pragma once

#include <complex>
#include <vector>

#include "internal.hpp"

namespace syk {

bool tridiag_eig(int n, std::vector<double> &d, std::vector<double> e, std::vector<double> &Z);

// e^{z T} e_1 for a real symmetric tridiagonal T, through T = Z diag(lam) Z^T
class TriExp {
  public:
    TriExp(int n, const double *alpha, const double *beta_off);
    bool ok() const { return ok_; }
    void apply(std::complex<double> z, std::complex<double> *c) const;   // all n components
    std::complex<double> last(std::complex<double> z) const;             // component n-1

  private:
    int n_;
    bool ok_ = false;
    std::vector<double> lam_, Z_;
};

// Argument checks of Krylov options (throws SYK_EINVAL).
void check_krylov_opts(const syk_krylov_opts &o);

size_t krylov_workspace_bytes(uint64_t n, int m, size_t elem_bytes);

// Optional timing of apply_H launches with HIP events recorded on the launch stream.
// Pairs are read back (flush) only after the stream has been synchronised.
class ApplyTimer {
  public:
    ~ApplyTimer();
    void begin(hipStream_t s);
    void end(hipStream_t s);
    void flush();              // the stream must be synchronised
    double ms = 0.0;
    long long launches = 0;

  private:
    std::vector<hipEvent_t> pool_;
    size_t used_ = 0;
};

template <typename T>
class KrylovRun {
  public:
    // ws: device workspace of at least krylov_workspace_bytes(n, m, sizeof(T)) bytes
    // rot: layout rotation of the vectors (0 = standard index order)
    KrylovRun(Hamiltonian &h, int blk, int rot, uint64_t n, int m, char *ws, hipStream_t s);
    // out = e^{z H} v (out may equal v); accumulates into st
    void run(std::complex<double> z, const T *v, T *out, const syk_krylov_opts &o, syk_krylov_stats &st);
    double norm(const T *v);
    void set_timer(ApplyTimer *t) { timer_ = t; }
    double *partials() { return partials_; }
    double *scratch() { return scratch_; }
    int n_part() const { return n_part_; }

  private:
    T *vec(int j) { return basis_ + static_cast<size_t>(j) * vec_stride_ * 2; }
    // one Lanczos step; returns true if w was fully reorthogonalised
    bool iterate(int j, int reorth);
    // reorth = 3: update the estimates of |<v_{j+1}, v_k>| from alpha, beta; true if a
    // full reorthogonalisation is due
    bool partial_estimate(int j);

    Hamiltonian &h_;
    int blk_, rot_;
    uint64_t n_;
    int m_;
    hipStream_t s_;
    size_t vec_stride_ = 0;    // complex elements between basis vectors
    T *basis_ = nullptr;
    double *partials_ = nullptr, *alpha_ = nullptr, *beta2_ = nullptr, *coef_ = nullptr, *scratch_ = nullptr;
    double *fused_ = nullptr;
    bool unnormalised_ = false;   // fused path: basis slots >= 1 hold u_i = beta_{i-1} v_i
    // partial reorthogonalisation state: omega_[0] row j - 1, omega_[1] row j of the
    // estimated <v_j, v_k>; host copies of alpha and beta; whether the next step must be
    // reorthogonalised too
    std::vector<double> omega_[2], ha_, hb_;
    double anorm_ = 0.0;
    bool force_next_ = false;
    int n_part_ = 0;
    ApplyTimer *timer_ = nullptr;
};

}  // namespace syk
