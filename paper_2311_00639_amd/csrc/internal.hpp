// Internal declarations of libsyk shared by the host sources and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstddef>
#include <map>
#include <mutex>
#include <tuple>
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
// Cleanup paths (destructors, unwinding after an error): a failure to release a resource
// cannot be reported from there, so its status is dropped on purpose.
inline void ignore_status(hipError_t) {}

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

// A region of device memory handed out front to back in 256-byte aligned pieces; nothing
// in it is freed piece by piece (its owner returns the region as a whole).
struct DeviceSlab {
    char *base = nullptr;
    size_t size = 0, used = 0;
    // next piece of `bytes`; ENOMEM naming `what` when the region is exhausted
    void *take(size_t bytes, const char *what);
};

struct DeviceTables {            // per device, per block: the gather kernel's term tables
    bool in_slab = false;        // carved from a DeviceSlab: not freed by the library
    int n_real = 0;              // real-phase terms of the block
    int K = 0;
    // terms grouped by x mask: group g has mask gx[g], real-phase terms [gs[g], gm[g]) and
    // i-phase terms [gm[g], gs[g + 1]) of gz / gc32 / gc64
    uint32_t *gx = nullptr, *gs = nullptr, *gm = nullptr, *gz = nullptr;
    float *gc32 = nullptr;
    double *gc64 = nullptr;
    int G = 0;
};

// distinct x masks of a block's terms: the groups the gather kernel loads once each
int gather_groups(const std::vector<BlockTerm> &terms);

// Compiled variant of the tiled apply_H kernel: tiles of 2^bt amplitudes, 2^rb per
// thread, nbuf LDS partner buffers (nbuf - 1 copies in flight; 1 = copy, then compute),
// pf extra partner entries at the end of the group list, occ workgroups resident per CU
// (the planner's XCD-resident subspace has dimension 5 + log2(occ)); sr = 1: each term's
// register permutation and register signs select a compiled code path (4-dword term
// records), sr = 0: they are read from the term record (4 + 2 * 2^rb dwords), sr = 2: each
// partner step's records sit in a 64-dword control block that a wave holds in one VGPR
// and reads with readlane (no scalar memory loads in the term loop; two buffers); each
// workgroup keeps 2^w output tiles in registers and streams the union of their partner
// tiles once.
struct TiledVariant {
    int bt, rb, nbuf, pf, occ, sr, w;   // w: each workgroup holds 2^w output tiles
};
inline int resident_bits(const TiledVariant &v) { return 5 + (v.occ >= 4 ? 2 : v.occ >= 2 ? 1 : 0); }
template <typename T>
const std::vector<TiledVariant> &tiled_variants();
// variant used before (or without) autotuning, for blocks of 2^L amplitudes
template <typename T>
int default_variant(int L);
// smallest block (in qubits) served by the tiled kernel
constexpr int kTiledMinL = 18;

// bit rotations within L bits: layout rotation s stores qubit (b + s) mod L at index bit b
uint32_t rotr_bits(uint32_t v, int s, int L);
uint32_t rotl_bits(uint32_t v, int s, int L);

struct ApplyPlan {
    bool in_slab = false;            // device arrays carved from a DeviceSlab: not freed by the library
    int bt = 0, rb = 0, rot = 0, variant = 0, w = 0;
    uint32_t n_tiles = 0;            // output tiles
    uint32_t n_wg = 0;               // workgroups (n_tiles >> w)
    uint32_t hvec[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // tiles of a workgroup: t0 ^ hvec[i], i < 2^w
    uint32_t *tile_map = nullptr;    // n_wg: blockIdx -> t0
    int n_pi = 0;
    uint32_t *pi = nullptr;          // n_pi + pf partner offsets (partner tile t0 ^ pi)
    uint32_t *ranges = nullptr;      // n_pi * 2^w * 3 term ranges (first, mid, end)
    uint32_t *meta = nullptr;        // K + 1 term records (see apply_tiled.hip)
    float *c32 = nullptr;
    double *c64 = nullptr;
};

// Optional epilogue of the tiled apply_H for Lanczos step j of the fused path, where the
// basis is stored unnormalised: slot i >= 1 holds u_i with ||u_i|| = sqrt(beta2[i]) (so
// v_i = u_i / sqrt(beta2[i])), slot 0 holds v_0.  With x = u_j (vcur) the epilogue forms
//   y = H v_j - beta_{j-1} v_{j-1} = s_j H u_j - (beta_{j-1} s_{j-1}) u_{j-1}
// (s_i = 1 / ||u_i||, s_0 = 1, beta_{j-1} = ||u_j||; vprev = u_{j-1}, null for j = 0) and
// per-workgroup partial sums (re <v_j,y>, im <v_j,y>, ||y||^2, ||v_j||^2) at
// partials[4 * blockIdx.x].
template <typename T>
struct LanczosFuse {
    const T *vprev = nullptr;
    const T *vcur = nullptr;
    const double *beta2 = nullptr;     // device, indexed by basis slot
    int j = 0;
    double *partials = nullptr;
};

// ------------------------------------------------------------------ host-side model
uint64_t splitmix_mix(uint64_t z);

struct Hamiltonian {
    int N = 0, L = 0, K = 0;
    double k = 0, p = 0, sigma = 0, sum_J2 = 0;
    uint64_t seed = 0;
    int ensemble = 0;                  // -1: a general operator (syk_op_to_hamiltonian)
    bool hermitian = true;
    std::vector<int32_t> ijkl;         // 4K, sorted subsets
    std::vector<double> J;             // K
    std::vector<uint64_t> xmask, zmask;
    std::vector<int8_t> phase[2];      // U, D
    std::vector<BlockTerm> block_terms[2];   // kernel order: real first, then imaginary
    int n_real[2] = {0, 0};

    // where device tables and plans come from: hipMalloc (null) or a slab that outlives the
    // handle (the request engine carves each request's tables from its arena)
    DeviceSlab *slab = nullptr;
    std::mutex dev_mu;
    std::vector<DeviceTables> dev[2];  // indexed by device ordinal
    // plans keyed by (block, double?, device, rotation, variant)
    std::map<std::tuple<int, int, int, int, int>, ApplyPlan> plans;
    std::map<std::pair<int, int>, int> rotation;               // (double?, variant) -> planned rotation
    std::map<std::pair<int, int>, int> tuned;                   // (double?, device) -> variant
    const DeviceTables &tables(int blk);
    template <typename T>
    const ApplyPlan &plan(int blk, int rot, int variant);
    template <typename T>
    int internal_rotation(int variant);   // layout used inside Krylov/OTOC runs (0 if not tiled)
    template <typename T>
    int variant();                        // tuned variant on the current device, else the default
    ~Hamiltonian();
};

void build_hamiltonian(Hamiltonian &h, int N, double k, uint64_t seed, int ensemble = SYK_ENSEMBLE_EXACT_K);

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
    // use caller-owned device memory of `bytes` instead of allocating: ensure() then never
    // allocates (ENOMEM beyond `bytes`) and release() only forgets the pointer
    void adopt(void *p, size_t bytes);
    char *ptr() const { return p_; }
    size_t size() const { return n_; }

  private:
    char *p_ = nullptr;
    size_t n_ = 0;
    bool owned_ = true;
};

// per-(device, thread) cached workspace used by the convenience entry points
DeviceBuffer &thread_workspace(int slot);

// y = H_blk x on the device: tiled kernel for large blocks, gather kernel otherwise
template <typename T>
inline bool use_tiled(int L) {
    return L >= kTiledMinL;
}
template <typename T>
void apply_block(Hamiltonian &h, int blk, int rot, const T *x, T *y, int nvec, uint64_t ld, hipStream_t s);
// y = H_blk x with the fused Lanczos epilogue (tiled blocks only); returns the number of
// partials written (one per tile)
template <typename T>
int apply_block_lanczos(Hamiltonian &h, int blk, int rot, const T *x, T *y, const LanczosFuse<T> &lf,
                        hipStream_t s);
// upper bound on the partials apply_block_lanczos writes for a block of 2^L amplitudes
inline uint64_t lanczos_partials_max(int L) { return 1ULL << (L > 10 ? L - 10 : 0); }
// time the tiled-kernel variants and keep the fastest; returns it (-1: block not tiled)
template <typename T>
int autotune(Hamiltonian &h, T *x, T *y, hipStream_t s, bool force, std::vector<float> *times = nullptr);

// ------------------------------------------------------------------ kernels (HIP side)
// All launchers enqueue on `s` and never synchronise.
template <typename T>
void launch_apply_h(const DeviceTables &tb, const T *x, T *y, uint32_t n_amps, int nvec, uint64_t ld,
                    hipStream_t s);
// psi in layout rotation `rot`: index p holds standard amplitude rotl(p, rot)
template <typename T>
void launch_haar_raw(uint64_t state_seed, int v, int L, int rot, T *psi_U, T *psi_D, double *partials, int n_part,
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
// sums[0..4) = (re <v,w>, im <v,w>, ||w||^2, ||v||^2) -> alpha = (re, im) at alpha_out[0..2),
// beta^2 = ||w - alpha_re v||^2 at beta2_out (expanded in the sums)
void launch_lanczos_scalars(const double *partials, int n_part, double *alpha_out, double *beta2_out,
                            hipStream_t s);
// fused path: w <- w - alpha_j s_j u_j (v = u_j, s_j from beta2[j], j >= 1; 1 for j = 0) and
// ||w||^2 at beta2_out, summed in a fixed order over per-workgroup partials (one workgroup
// per 256 amplitudes, at most partials_cap of them) and a 512-double stage buffer
template <typename T>
void launch_lanczos_residual(T *w, const T *v, const double *alpha, const double *beta2, int j, uint64_t n,
                             double *partials, uint64_t partials_cap, double *stage, double *beta2_out,
                             hipStream_t s);
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
// this device's copy of the library's fixed device scratch (at least n_doubles doubles;
// EINVAL beyond its size); looked up once per device, never allocated
double *fixed_scratch(size_t n_doubles);
size_t fixed_scratch_doubles();

}  // namespace syk
