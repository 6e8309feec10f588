// Internal declarations of libsyk shared by the host sources and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstddef>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/syk.h"

namespace syk {

// ------------------------------------------------------------------ errors
struct Error {
    syk_status status;
    std::string msg;
};
[[noreturn]] void fail(syk_status s, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define SYK_HIP(call) ::syk::hip_check((call), #call)

// ------------------------------------------------------------------ terms
// One term of Eq. (1) on one parity block, reduced for the kernels:
//   (J/4) i^p X^x Z^z acting as  y[m] += c * i^{imag} * (-1)^{popc(m & z)} * x[m ^ x]
// where the sign (-1)^{popc(x & z)} of reading the Z bits from the source index m ^ x has
// been folded into c together with the real sign of i^p; imag = p odd.
struct BlockTerm {
    uint32_t x, z;
    double c;
    bool imag;
};

struct DeviceTables {            // per device, per block: real terms first, then imaginary
    uint32_t *x = nullptr;       // K entries
    uint32_t *z = nullptr;
    float *c32 = nullptr;
    double *c64 = nullptr;
    int n_real = 0;
    int K = 0;
};

// ------------------------------------------------------------------ host-side model
uint64_t splitmix_mix(uint64_t z);

struct Hamiltonian {
    int N = 0, L = 0, K = 0;
    double k = 0, p = 0, sigma = 0, sum_J2 = 0;
    uint64_t seed = 0;
    std::vector<int32_t> ijkl;         // 4K, sorted subsets
    std::vector<double> J;             // K
    std::vector<uint64_t> xmask, zmask;
    std::vector<int8_t> phase[2];      // U, D
    std::vector<BlockTerm> block_terms[2];   // kernel order: real first, then imaginary
    int n_real[2] = {0, 0};

    std::mutex dev_mu;
    std::vector<DeviceTables> dev[2];  // indexed by device ordinal
    const DeviceTables &tables(int blk);
    ~Hamiltonian();
};

void build_hamiltonian(Hamiltonian &h, int N, double k, uint64_t seed);

// canonical Pauli string i^w X^x Z^z of block Majorana A_n (0 <= n <= N-2) on L qubits
void block_majorana(int N, int n, uint32_t &x, uint32_t &z, int &w);

// ------------------------------------------------------------------ device workspace
class DeviceBuffer {
  public:
    DeviceBuffer() = default;
    ~DeviceBuffer();
    DeviceBuffer(const DeviceBuffer &) = delete;
    DeviceBuffer &operator=(const DeviceBuffer &) = delete;
    void ensure(size_t bytes);
    void release();
    char *ptr() const { return p_; }
    size_t size() const { return n_; }

  private:
    char *p_ = nullptr;
    size_t n_ = 0;
};

// per-(device, thread) cached workspace used by the convenience entry points
DeviceBuffer &thread_workspace(int slot);

// ------------------------------------------------------------------ kernels (HIP side)
// All launchers enqueue on `s` and never synchronise.
template <typename T>
void launch_apply_h(const DeviceTables &tb, const T *x, T *y, uint32_t n_amps, int nvec, uint64_t ld,
                    hipStream_t s);
template <typename T>
void launch_haar_raw(uint64_t state_seed, int v, int L, T *psi_U, T *psi_D, double *partials, int n_part,
                     hipStream_t s);
template <typename T>
void launch_scale_pair(T *a, T *b, uint64_t n, const double *inv_norm_dev, hipStream_t s);
template <typename T>
void launch_majorana(uint32_t x, uint32_t z, int w, double sre, double sim, const T *src, T *dst, uint64_t n,
                     hipStream_t s);
// partial reductions: out[b] for b < n_part, each (re, im) or (sum) in double
template <typename T>
void launch_dot_partials(const T *a, const T *b, uint64_t n, double *partials, int n_part, hipStream_t s);
template <typename T>
void launch_norm2_partials(const T *a, uint64_t n, double *partials, int n_part, hipStream_t s);
// reduce `n_part` partials of width `width` into dst[0..width) (single workgroup, fixed order)
void launch_reduce_partials(const double *partials, int n_part, int width, double *dst, hipStream_t s);

// Lanczos building blocks (scalars live on the device, see krylov.cpp)
template <typename T>
void launch_lanczos_orth1(T *w, const T *vprev, const T *vcur, const double *beta_prev, uint64_t n,
                          double *partials, int n_part, hipStream_t s);
template <typename T>
void launch_lanczos_orth2(T *w, const T *vcur, const double *alpha, uint64_t n, double *partials, int n_part,
                          hipStream_t s);
template <typename T>
void launch_lanczos_normalize(T *w, const double *beta, uint64_t n, hipStream_t s);
template <typename T>
void launch_scale_copy(const T *src, T *dst, uint64_t n, double scale, hipStream_t s);
template <typename T>
void launch_combine(const T *basis, uint64_t stride, int nb, const double *coef_dev, T *out, uint64_t n,
                    hipStream_t s);
// subtract projections: w -= sum_k c_k v_k with c_k = <v_k, w> taken from coef_dev (complex)
template <typename T>
void launch_subtract_proj(T *w, const T *basis, uint64_t stride, int nb, const double *coef_dev, uint64_t n,
                          hipStream_t s);
template <typename T>
void launch_multi_dot_partials(const T *basis, uint64_t stride, int nb, const T *w, uint64_t n, double *partials,
                               int n_part, hipStream_t s);

int reduction_blocks(uint64_t n);   // number of partials the reduction launchers produce

}  // namespace syk
