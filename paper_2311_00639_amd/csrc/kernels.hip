// HIP kernels of libsyk for gfx950: matrix-free apply_H (supplement Algorithm 1), Haar
// states, Majorana insertions, and the vector kernels of the Lanczos propagator.
//
// Complex vectors are interleaved (re, im) of float or double, addressed as float2 /
// double2.  Every reduction accumulates in double and writes one partial per workgroup;
// partials are combined in a fixed order by reduce_partials, so results are repeatable.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "internal.hpp"

namespace syk {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T> using V2 = typename Vec2<T>::type;

constexpr int kBlock = 256;

static inline int grid_for(uint64_t n, int per_thread = 1) {
    uint64_t g = (n + static_cast<uint64_t>(kBlock) * per_thread - 1) / (static_cast<uint64_t>(kBlock) * per_thread);
    if (g < 1) g = 1;
    if (g > 65535ULL * 16) g = 65535ULL * 16;
    return static_cast<int>(g);
}

int reduction_blocks(uint64_t n) {
    uint64_t g = n / (kBlock * 8);
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return static_cast<int>(g);
}

// block-wide sum of W doubles per thread into out[0..W) (thread 0 writes)
template <int W>
__device__ inline void block_sum(double (&v)[W], double *out) {
    __shared__ double sh[W][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        double s = v[k];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += sh[k][w];
            out[k] = s;
        }
    }
}

// ------------------------------------------------------------------ apply_H
// Blocks below the tiled size.  Terms are grouped by x mask (one term per mask for sparse
// Hamiltonians, about 19 for dense SYK): per output amplitude and group, the diagonal
// D_x(m) = sum_t c_t (-1)^popc(m & z_t) (the parity of x & z folded into c_t) is summed
// over the group's real-phase terms (Re) and i-phase terms (Im), then multiplied once by
// the partner x[m ^ x] gathered straight from memory.  One gather per mask.  Small
// blocks have too few amplitudes to fill the GPU, so a workgroup of kBlock threads holds
// A = kBlock / S amplitudes and S slices of the group list (slice s takes groups s, s + S,
// ...); the slices' sums are added in slice order in LDS, so the result does not depend on
// scheduling.
template <typename T, int S>
__global__ void __launch_bounds__(kBlock) apply_h_grouped(const uint32_t *__restrict__ gx,
                                                          const uint32_t *__restrict__ gs,
                                                          const uint32_t *__restrict__ gm,
                                                          const uint32_t *__restrict__ gz,
                                                          const T *__restrict__ gc, int G,
                                                          const V2<T> *__restrict__ x, V2<T> *__restrict__ y,
                                                          uint32_t n_amps, uint64_t ld) {
    constexpr int A = kBlock / S;
    __shared__ V2<T> part[S > 1 ? S : 1][A];
    const uint64_t vo = static_cast<uint64_t>(blockIdx.y) * ld;
    x += vo;
    y += vo;
    const int slice = static_cast<int>(threadIdx.x) / A, a = static_cast<int>(threadIdx.x) % A;
    for (uint32_t base = blockIdx.x * A; base < n_amps; base += gridDim.x * A) {
        const uint32_t m = base + a;
        T ar = 0, ai = 0;
        if (m < n_amps) {
            for (int g = slice; g < G; g += S) {
                const V2<T> v = x[m ^ gx[g]];
                const uint32_t t0 = gs[g], t1 = gm[g], t2 = gs[g + 1];
                T dre = 0, dim = 0;
                for (uint32_t t = t0; t < t1; ++t) dre += (__popc(m & gz[t]) & 1) ? -gc[t] : gc[t];
                for (uint32_t t = t1; t < t2; ++t) dim += (__popc(m & gz[t]) & 1) ? -gc[t] : gc[t];
                ar += dre * v.x - dim * v.y;
                ai += dre * v.y + dim * v.x;
            }
        }
        if constexpr (S == 1) {
            if (m < n_amps) y[m] = V2<T>{ar, ai};
        } else {
            part[slice][a] = V2<T>{ar, ai};
            __syncthreads();
            if (slice == 0 && m < n_amps) {
                V2<T> acc = part[0][a];
#pragma unroll
                for (int k = 1; k < S; ++k) {
                    acc.x += part[k][a].x;
                    acc.y += part[k][a].y;
                }
                y[m] = acc;
            }
            __syncthreads();
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_zero(V2<T> *__restrict__ y, uint32_t n_amps, uint64_t ld) {
    y += static_cast<uint64_t>(blockIdx.y) * ld;
    for (uint32_t m = blockIdx.x * kBlock + threadIdx.x; m < n_amps; m += gridDim.x * kBlock) y[m] = V2<T>{T(0), T(0)};
}

template <typename T> static const T *gcoef_ptr(const DeviceTables &tb);
template <> const float *gcoef_ptr<float>(const DeviceTables &tb) { return tb.gc32; }
template <> const double *gcoef_ptr<double>(const DeviceTables &tb) { return tb.gc64; }

template <typename T>
void launch_apply_h(const DeviceTables &tb, const T *x, T *y, uint32_t n_amps, int nvec, uint64_t ld,
                    hipStream_t s) {
    if (tb.G > 0) {
        // slices of the group list per amplitude: enough workgroups (about 1024) for small blocks
        int S = 1;
        while (S < 16 && static_cast<uint64_t>(n_amps) * S < 1024ull * kBlock) S *= 2;
        const dim3 gg(static_cast<unsigned>((n_amps + kBlock / S - 1) / (kBlock / S)), nvec);
        auto go = [&](auto sc) {
            constexpr int SS = decltype(sc)::value;
            hipLaunchKernelGGL((apply_h_grouped<T, SS>), gg, dim3(kBlock), 0, s, tb.gx, tb.gs, tb.gm, tb.gz,
                               gcoef_ptr<T>(tb), tb.G, reinterpret_cast<const V2<T> *>(x), reinterpret_cast<V2<T> *>(y),
                               n_amps, ld);
        };
        switch (S) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 4: go(std::integral_constant<int, 4>{}); break;
            case 8: go(std::integral_constant<int, 8>{}); break;
            default: go(std::integral_constant<int, 16>{}); break;
        }
    } else {
        hipLaunchKernelGGL(fill_zero<T>, dim3(grid_for(n_amps), nvec), dim3(kBlock), 0, s, reinterpret_cast<V2<T> *>(y),
                           n_amps, ld);                        // no terms: H = 0
    }
    SYK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Haar states
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ inline double2 haar_amp(uint64_t base, uint64_t n) {
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    const uint64_t w1 = mix64(base + (2 * n + 1) * G);
    const uint64_t w2 = mix64(base + (2 * n + 2) * G);
    const double u1 = static_cast<double>((w1 >> 11) + 1) * 0x1p-53;
    const double u2 = static_cast<double>(w2 >> 11) * 0x1p-53;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    return double2{r * cs, r * sn};
}

// index b of the stored (layout-rotated) block holds standard block index m = rotl(b, rot)
template <typename T>
__global__ void __launch_bounds__(kBlock) haar_raw(uint64_t base, int L, int rot, V2<T> *__restrict__ pu,
                                                   V2<T> *__restrict__ pd, double *__restrict__ partials) {
    const uint64_t h = 1ULL << L;
    const uint64_t mask = h - 1;
    double acc[1] = {0.0};
    for (uint64_t b = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; b < h;
         b += static_cast<uint64_t>(gridDim.x) * kBlock) {
        const uint64_t m = rot ? (((b << rot) | (b >> (L - rot))) & mask) : b;
        const double2 a = haar_amp(base, m);
        const double2 d = haar_amp(base, h + m);
        acc[0] += a.x * a.x + a.y * a.y + d.x * d.x + d.y * d.y;
        pu[b] = V2<T>{static_cast<T>(a.x), static_cast<T>(a.y)};
        pd[b] = V2<T>{static_cast<T>(d.x), static_cast<T>(d.y)};
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

template <typename T>
void launch_haar_raw(uint64_t state_seed, int v, int L, int rot, T *psi_U, T *psi_D, double *partials, int n_part,
                     hipStream_t s) {
    const uint64_t base = splitmix_mix(state_seed + static_cast<uint64_t>(v + 1) * 0x9E3779B97F4A7C15ULL);
    hipLaunchKernelGGL(haar_raw<T>, dim3(n_part), dim3(kBlock), 0, s, base, L, rot % (L > 0 ? L : 1),
                       reinterpret_cast<V2<T> *>(psi_U),
                       reinterpret_cast<V2<T> *>(psi_D), partials);
    SYK_HIP(hipGetLastError());
}

// a, b *= 1/sqrt(norm2[0]) -- the normalisation of a full-space state split in two blocks.
// For double the raw amplitudes are rescaled as stored; for float the stored rounded raw
// values are rescaled (a relative change of at most one float ulp from normalising first).
template <typename T>
__global__ void __launch_bounds__(kBlock) scale_pair(V2<T> *__restrict__ a, V2<T> *__restrict__ b, uint64_t n,
                                                     const double *__restrict__ norm2) {
    const double inv = 1.0 / sqrt(norm2[0]);
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        V2<T> u = a[i], w = b[i];
        a[i] = V2<T>{static_cast<T>(u.x * inv), static_cast<T>(u.y * inv)};
        b[i] = V2<T>{static_cast<T>(w.x * inv), static_cast<T>(w.y * inv)};
    }
}

template <typename T>
void launch_scale_pair(T *a, T *b, uint64_t n, const double *norm2_dev, hipStream_t s) {
    hipLaunchKernelGGL(scale_pair<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, reinterpret_cast<V2<T> *>(a),
                       reinterpret_cast<V2<T> *>(b), n, norm2_dev);
    SYK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ fixed scratch
// Device memory of the allocation-free Haar entry point: the per-workgroup partial sums of
// the norm and their total.  Each device holds its own copy of this array (at its own
// address) from module load until the process ends; every call on a device reuses it, so
// calls that overlap on one device race.  Host code must use the address returned by
// hipGetSymbolAddress on that device, never the array's name.
constexpr size_t kScratchDoubles = 4096;
static __device__ __align__(256) double scratch[kScratchDoubles];

double *fixed_scratch(size_t n_doubles) {
    if (n_doubles > kScratchDoubles)
        fail(SYK_EINVAL, "request needs " + std::to_string(n_doubles) + " doubles of fixed scratch, more than the " +
                             std::to_string(kScratchDoubles) + " available");
    int dev = 0;
    SYK_HIP(hipGetDevice(&dev));
    static std::mutex mu;
    static std::map<int, double *> ptrs;     // device ordinal -> that device's copy of the array
    std::lock_guard<std::mutex> g(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    void *p = nullptr;
    SYK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) fail(SYK_EDEVICE, "hipGetSymbolAddress returned no address for the fixed scratch");
    ptrs[dev] = static_cast<double *>(p);
    return static_cast<double *>(p);
}

size_t fixed_scratch_doubles() { return kScratchDoubles; }

// ------------------------------------------------------------------ Majorana insertion
// dst[m] = s * (-1)^{popc((m ^ x) & z)} * src[m ^ x],  s complex (phase i^w folded in).
template <typename T>
__global__ void __launch_bounds__(kBlock) majorana_kernel(uint32_t x, uint32_t z, double sre, double sim,
                                                          const V2<T> *__restrict__ src, V2<T> *__restrict__ dst,
                                                          uint64_t n) {
    for (uint64_t m = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; m < n;
         m += static_cast<uint64_t>(gridDim.x) * kBlock) {
        const uint32_t k = static_cast<uint32_t>(m) ^ x;
        const V2<T> v = src[k];
        const double sg = (__popc(k & z) & 1) ? -1.0 : 1.0;
        const double vr = sg * static_cast<double>(v.x), vi = sg * static_cast<double>(v.y);
        dst[m] = V2<T>{static_cast<T>(sre * vr - sim * vi), static_cast<T>(sre * vi + sim * vr)};
    }
}

template <typename T>
void launch_majorana(uint32_t x, uint32_t z, int w, double sre, double sim, const T *src, T *dst, uint64_t n,
                     hipStream_t s) {
    // fold i^w into the scale
    for (int k = 0; k < (w & 3); ++k) {
        const double r = -sim, i = sre;
        sre = r;
        sim = i;
    }
    hipLaunchKernelGGL(majorana_kernel<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, x, z, sre, sim,
                       reinterpret_cast<const V2<T> *>(src), reinterpret_cast<V2<T> *>(dst), n);
    SYK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ reductions
template <typename T>
__global__ void __launch_bounds__(kBlock) dot_partials(const V2<T> *__restrict__ a, const V2<T> *__restrict__ b,
                                                       uint64_t n, double *__restrict__ partials) {
    double acc[2] = {0.0, 0.0};
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        const V2<T> u = a[i], v = b[i];
        acc[0] += static_cast<double>(u.x) * v.x + static_cast<double>(u.y) * v.y;
        acc[1] += static_cast<double>(u.x) * v.y - static_cast<double>(u.y) * v.x;
    }
    block_sum<2>(acc, partials + 2 * blockIdx.x);
}

template <typename T>
void launch_dot_partials(const T *a, const T *b, uint64_t n, double *partials, int n_part, hipStream_t s) {
    hipLaunchKernelGGL(dot_partials<T>, dim3(n_part), dim3(kBlock), 0, s, reinterpret_cast<const V2<T> *>(a),
                       reinterpret_cast<const V2<T> *>(b), n, partials);
    SYK_HIP(hipGetLastError());
}

template <typename T>
__global__ void __launch_bounds__(kBlock) norm2_partials(const V2<T> *__restrict__ a, uint64_t n,
                                                         double *__restrict__ partials) {
    double acc[1] = {0.0};
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        const V2<T> u = a[i];
        acc[0] += static_cast<double>(u.x) * u.x + static_cast<double>(u.y) * u.y;
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

template <typename T>
void launch_norm2_partials(const T *a, uint64_t n, double *partials, int n_part, hipStream_t s) {
    hipLaunchKernelGGL(norm2_partials<T>, dim3(n_part), dim3(kBlock), 0, s, reinterpret_cast<const V2<T> *>(a), n,
                       partials);
    SYK_HIP(hipGetLastError());
}

// dst[k] = sum_p partials[p * width + k], fixed order; width <= 2 * 130
__global__ void __launch_bounds__(kBlock) reduce_partials_kernel(const double *__restrict__ partials, int n_part,
                                                                 int width, double *__restrict__ dst) {
    for (int k = 0; k < width; ++k) {
        double acc[1] = {0.0};
        for (int p = threadIdx.x; p < n_part; p += kBlock) acc[0] += partials[static_cast<size_t>(p) * width + k];
        block_sum<1>(acc, dst + k);
        __syncthreads();
    }
}

void launch_reduce_partials(const double *partials, int n_part, int width, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kBlock), 0, s, partials, n_part, width, dst);
    SYK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Lanczos vector kernels
// w -= beta_prev * vprev (vprev may be null, beta_prev = sqrt(beta2_prev[0])); partial <vcur, w>
template <typename T>
__global__ void __launch_bounds__(kBlock) lanczos_orth1(V2<T> *__restrict__ w, const V2<T> *__restrict__ vprev,
                                                        const V2<T> *__restrict__ vcur,
                                                        const double *__restrict__ beta2_prev, uint64_t n,
                                                        double *__restrict__ partials) {
    const T bp = vprev ? static_cast<T>(sqrt(beta2_prev[0])) : T(0);
    double acc[2] = {0.0, 0.0};
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        V2<T> u = w[i];
        if (vprev) {
            const V2<T> p = vprev[i];
            u.x -= bp * p.x;
            u.y -= bp * p.y;
            w[i] = u;
        }
        const V2<T> c = vcur[i];
        acc[0] += static_cast<double>(c.x) * u.x + static_cast<double>(c.y) * u.y;
        acc[1] += static_cast<double>(c.x) * u.y - static_cast<double>(c.y) * u.x;
    }
    block_sum<2>(acc, partials + 2 * blockIdx.x);
}

template <typename T>
void launch_lanczos_orth1(T *w, const T *vprev, const T *vcur, const double *beta_prev, uint64_t n,
                          double *partials, int n_part, hipStream_t s) {
    hipLaunchKernelGGL(lanczos_orth1<T>, dim3(n_part), dim3(kBlock), 0, s, reinterpret_cast<V2<T> *>(w),
                       reinterpret_cast<const V2<T> *>(vprev), reinterpret_cast<const V2<T> *>(vcur), beta_prev,
                       n, partials);
    SYK_HIP(hipGetLastError());
}

// w -= alpha_re * vcur; partial ||w||^2
template <typename T>
__global__ void __launch_bounds__(kBlock) lanczos_orth2(V2<T> *__restrict__ w, const V2<T> *__restrict__ vcur,
                                                        const double *__restrict__ alpha, uint64_t n,
                                                        double *__restrict__ partials) {
    const T al = static_cast<T>(alpha[0]);
    double acc[1] = {0.0};
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        V2<T> u = w[i];
        const V2<T> c = vcur[i];
        u.x -= al * c.x;
        u.y -= al * c.y;
        w[i] = u;
        acc[0] += static_cast<double>(u.x) * u.x + static_cast<double>(u.y) * u.y;
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

template <typename T>
void launch_lanczos_orth2(T *w, const T *vcur, const double *alpha, uint64_t n, double *partials, int n_part,
                          hipStream_t s) {
    hipLaunchKernelGGL(lanczos_orth2<T>, dim3(n_part), dim3(kBlock), 0, s, reinterpret_cast<V2<T> *>(w),
                       reinterpret_cast<const V2<T> *>(vcur), alpha, n, partials);
    SYK_HIP(hipGetLastError());
}

// w *= 1/beta where beta = sqrt(norm2[0]); w = 0 if beta underflows (invariant subspace)
template <typename T>
__global__ void __launch_bounds__(kBlock) lanczos_normalize(V2<T> *__restrict__ w, const double *__restrict__ norm2,
                                                            uint64_t n) {
    const double b = sqrt(norm2[0]);
    const T inv = (b > 1e-300) ? static_cast<T>(1.0 / b) : T(0);
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        V2<T> u = w[i];
        u.x *= inv;
        u.y *= inv;
        w[i] = u;
    }
}

template <typename T>
void launch_lanczos_normalize(T *w, const double *norm2, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(lanczos_normalize<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, reinterpret_cast<V2<T> *>(w),
                       norm2, n);
    SYK_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(kBlock) lanczos_scalars_kernel(const double *__restrict__ partials, int n_part,
                                                                 double *__restrict__ alpha_out,
                                                                 double *__restrict__ beta2_out) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < n_part; p += kBlock)
        for (int k = 0; k < 4; ++k) acc[k] += partials[static_cast<size_t>(p) * 4 + k];
    __shared__ double tot[4];
    block_sum<4>(acc, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        alpha_out[0] = tot[0];
        alpha_out[1] = tot[1];
        // beta is not formed from these sums (||y||^2 - alpha^2 cancels when the Krylov
        // space is nearly invariant); the residual pass computes it from the vector
        if (beta2_out) beta2_out[0] = 0.0;
    }
}

void launch_lanczos_scalars(const double *partials, int n_part, double *alpha_out, double *beta2_out,
                            hipStream_t s) {
    hipLaunchKernelGGL(lanczos_scalars_kernel, dim3(1), dim3(kBlock), 0, s, partials, n_part, alpha_out, beta2_out);
    SYK_HIP(hipGetLastError());
}

// 16 bytes of complex amplitudes per lane (two complex64 or one complex128): the
// recombination below moves whole 16-byte units so each wave reads or writes 1 KiB per
// instruction (the residual pass takes one amplitude per thread instead).
template <typename T> struct Wide;
template <> struct Wide<float> { using type = float4; static constexpr int amps = 2; };
template <> struct Wide<double> { using type = double2; static constexpr int amps = 1; };

// fused Lanczos: w <- w - (alpha_j / ||u_j||) u_j, with one partial of ||w||^2 per
// workgroup.  One amplitude per thread and as many workgroups as that takes: at 2^27
// complex64 amplitudes this streams at 6.2 TB/s, against 5.3 TB/s for 2048 workgroups
// walking contiguous slices and 5.6-5.9 TB/s for two or four amplitudes per thread.
template <typename T>
__global__ void __launch_bounds__(kBlock) lanczos_residual(V2<T> *__restrict__ w, const V2<T> *__restrict__ v,
                                                           const double *__restrict__ alpha,
                                                           const double *__restrict__ beta2, int j, uint64_t n,
                                                           double *__restrict__ partials) {
    const double nj = j >= 1 ? sqrt(beta2[j]) : 1.0;
    const double sj = nj > 1e-300 ? 1.0 / nj : 0.0;
    const T a = static_cast<T>(alpha[0] * sj);
    double acc[1] = {0.0};
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        V2<T> u = w[i];
        const V2<T> c = v[i];
        u.x -= a * c.x;
        u.y -= a * c.y;
        w[i] = u;
        acc[0] += static_cast<double>(u.x) * u.x + static_cast<double>(u.y) * u.y;
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

// first stage of a two-stage sum: workgroup b adds the partials of its contiguous chunk
// in index order (the sum does not depend on timing)
__global__ void __launch_bounds__(kBlock) sum_chunks_kernel(const double *__restrict__ partials, int n_part,
                                                            double *__restrict__ out) {
    const int per = (n_part + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
    const int b0 = static_cast<int>(blockIdx.x) * per;
    const int b1 = b0 + per < n_part ? b0 + per : n_part;
    double acc[1] = {0.0};
    for (int p = b0 + static_cast<int>(threadIdx.x); p < b1; p += kBlock) acc[0] += partials[p];
    block_sum<1>(acc, out + blockIdx.x);
}

template <typename T>
void launch_lanczos_residual(T *w, const T *v, const double *alpha, const double *beta2, int j, uint64_t n,
                             double *partials, uint64_t partials_cap, double *stage, double *beta2_out,
                             hipStream_t s) {
    constexpr int kStage = 512;              // first-stage workgroups (stage holds this many doubles)
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g > partials_cap) g = partials_cap;  // then each thread takes several amplitudes
    if (g < 1 || g > (1u << 30)) fail(SYK_EDEVICE, "lanczos_residual: bad partials capacity");
    hipLaunchKernelGGL(lanczos_residual<T>, dim3(static_cast<unsigned>(g)), dim3(kBlock), 0, s,
                       reinterpret_cast<V2<T> *>(w), reinterpret_cast<const V2<T> *>(v), alpha, beta2, j, n,
                       partials);
    SYK_HIP(hipGetLastError());
    const int st = g < static_cast<uint64_t>(kStage) ? static_cast<int>(g) : kStage;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(st), dim3(kBlock), 0, s, partials, static_cast<int>(g), stage);
    SYK_HIP(hipGetLastError());
    launch_reduce_partials(stage, st, 1, beta2_out, s);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) scale_copy(const V2<T> *__restrict__ src, V2<T> *__restrict__ dst,
                                                     uint64_t n, double scale) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        const V2<T> u = src[i];
        dst[i] = V2<T>{static_cast<T>(u.x * scale), static_cast<T>(u.y * scale)};
    }
}

template <typename T>
void launch_scale_copy(const T *src, T *dst, uint64_t n, double scale, hipStream_t s) {
    hipLaunchKernelGGL(scale_copy<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, reinterpret_cast<const V2<T> *>(src),
                       reinterpret_cast<V2<T> *>(dst), n, scale);
    SYK_HIP(hipGetLastError());
}

// the recombination: kUnroll basis vectors in flight per thread
constexpr int kUnroll = 4;

// out[i] = sum_k coef[k] basis[k][i], coef complex double (re, im interleaved); summed in
// double over 16-byte units of each basis vector, kUnroll vectors in flight per step
__device__ inline void cmac(double (&acc)[4], double cr, double ci, float4 b) {
    acc[0] += cr * b.x - ci * b.y;
    acc[1] += cr * b.y + ci * b.x;
    acc[2] += cr * b.z - ci * b.w;
    acc[3] += cr * b.w + ci * b.z;
}
__device__ inline void cmac(double (&acc)[4], double cr, double ci, double2 b) {
    acc[0] += cr * b.x - ci * b.y;
    acc[1] += cr * b.y + ci * b.x;
}
__device__ inline void store_unit(float4 *p, const double (&acc)[4]) {
    *p = float4{static_cast<float>(acc[0]), static_cast<float>(acc[1]), static_cast<float>(acc[2]),
                static_cast<float>(acc[3])};
}
__device__ inline void store_unit(double2 *p, const double (&acc)[4]) { *p = double2{acc[0], acc[1]}; }

template <typename T>
__global__ void __launch_bounds__(kBlock) combine_kernel(const V2<T> *__restrict__ basis, uint64_t stride, int nb,
                                                         const double *__restrict__ coef, V2<T> *__restrict__ out,
                                                         uint64_t n) {
    using W = typename Wide<T>::type;
    const W *bw = reinterpret_cast<const W *>(basis);
    W *ow = reinterpret_cast<W *>(out);
    const uint64_t nw = n / Wide<T>::amps, sw = stride / Wide<T>::amps;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < nw;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int k = 0;
        for (; k + kUnroll <= nb; k += kUnroll) {
            W b[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) b[u] = bw[(k + u) * sw + i];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) cmac(acc, coef[2 * (k + u)], coef[2 * (k + u) + 1], b[u]);
        }
        for (; k < nb; ++k) cmac(acc, coef[2 * k], coef[2 * k + 1], bw[k * sw + i]);
        store_unit(ow + i, acc);
    }
}

template <typename T>
void launch_combine(const T *basis, uint64_t stride, int nb, const double *coef_dev, T *out, uint64_t n,
                    hipStream_t s) {
    if (n % Wide<T>::amps != 0 || stride % Wide<T>::amps != 0 || reinterpret_cast<uintptr_t>(basis) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(out) % 16 != 0)
        fail(SYK_EDEVICE, "combine needs 16-byte aligned vectors of whole 16-byte units");
    hipLaunchKernelGGL(combine_kernel<T>, dim3(grid_for(n / Wide<T>::amps)), dim3(kBlock), 0, s,
                       reinterpret_cast<const V2<T> *>(basis), stride, nb, coef_dev,
                       reinterpret_cast<V2<T> *>(out), n);
    SYK_HIP(hipGetLastError());
}

// partials[p][k] = sum_i conj(v_k[i]) w[i] for k < nb (complex, width 2 nb)
template <typename T>
__global__ void __launch_bounds__(kBlock) multi_dot_kernel(const V2<T> *__restrict__ basis, uint64_t stride, int nb,
                                                           const V2<T> *__restrict__ w, uint64_t n,
                                                           double *__restrict__ partials) {
    for (int k = 0; k < nb; ++k) {
        double acc[2] = {0.0, 0.0};
        const V2<T> *v = basis + k * stride;
        for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
             i += static_cast<uint64_t>(gridDim.x) * kBlock) {
            const V2<T> a = v[i], b = w[i];
            acc[0] += static_cast<double>(a.x) * b.x + static_cast<double>(a.y) * b.y;
            acc[1] += static_cast<double>(a.x) * b.y - static_cast<double>(a.y) * b.x;
        }
        block_sum<2>(acc, partials + (static_cast<size_t>(blockIdx.x) * nb + k) * 2);
        __syncthreads();
    }
}

template <typename T>
void launch_multi_dot_partials(const T *basis, uint64_t stride, int nb, const T *w, uint64_t n, double *partials,
                               int n_part, hipStream_t s) {
    hipLaunchKernelGGL(multi_dot_kernel<T>, dim3(n_part), dim3(kBlock), 0, s, reinterpret_cast<const V2<T> *>(basis),
                       stride, nb, reinterpret_cast<const V2<T> *>(w), n, partials);
    SYK_HIP(hipGetLastError());
}

// w -= sum_k c_k v_k (c complex double); partial ||w||^2 of the result
template <typename T>
__global__ void __launch_bounds__(kBlock) subtract_proj_kernel(V2<T> *__restrict__ w, const V2<T> *__restrict__ basis,
                                                               uint64_t stride, int nb,
                                                               const double *__restrict__ coef, uint64_t n) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kBlock) {
        V2<T> u = w[i];
        double ar = u.x, ai = u.y;
        for (int k = 0; k < nb; ++k) {
            const V2<T> v = basis[k * stride + i];
            const double cr = coef[2 * k], ci = coef[2 * k + 1];
            ar -= cr * v.x - ci * v.y;
            ai -= cr * v.y + ci * v.x;
        }
        w[i] = V2<T>{static_cast<T>(ar), static_cast<T>(ai)};
    }
}

template <typename T>
void launch_subtract_proj(T *w, const T *basis, uint64_t stride, int nb, const double *coef_dev, uint64_t n,
                          hipStream_t s) {
    hipLaunchKernelGGL(subtract_proj_kernel<T>, dim3(grid_for(n, 2)), dim3(kBlock), 0, s, reinterpret_cast<V2<T> *>(w),
                       reinterpret_cast<const V2<T> *>(basis), stride, nb, coef_dev, n);
    SYK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ instantiations
#define SYK_INST(T)                                                                                                \
    template void launch_apply_h<T>(const DeviceTables &, const T *, T *, uint32_t, int, uint64_t, hipStream_t);   \
    template void launch_haar_raw<T>(uint64_t, int, int, int, T *, T *, double *, int, hipStream_t);                    \
    template void launch_scale_pair<T>(T *, T *, uint64_t, const double *, hipStream_t);                           \
    template void launch_majorana<T>(uint32_t, uint32_t, int, double, double, const T *, T *, uint64_t,            \
                                     hipStream_t);                                                                 \
    template void launch_dot_partials<T>(const T *, const T *, uint64_t, double *, int, hipStream_t);              \
    template void launch_norm2_partials<T>(const T *, uint64_t, double *, int, hipStream_t);                       \
    template void launch_lanczos_orth1<T>(T *, const T *, const T *, const double *, uint64_t, double *, int,      \
                                          hipStream_t);                                                            \
    template void launch_lanczos_orth2<T>(T *, const T *, const double *, uint64_t, double *, int, hipStream_t);   \
    template void launch_lanczos_normalize<T>(T *, const double *, uint64_t, hipStream_t);                         \
    template void launch_lanczos_residual<T>(T *, const T *, const double *, const double *, int, uint64_t,          \
                                             double *, uint64_t, double *, double *, hipStream_t);              \
    template void launch_scale_copy<T>(const T *, T *, uint64_t, double, hipStream_t);                             \
    template void launch_combine<T>(const T *, uint64_t, int, const double *, T *, uint64_t, hipStream_t);         \
    template void launch_subtract_proj<T>(T *, const T *, uint64_t, int, const double *, uint64_t, hipStream_t);   \
    template void launch_multi_dot_partials<T>(const T *, uint64_t, int, const T *, uint64_t, double *, int,       \
                                               hipStream_t);
SYK_INST(float)
SYK_INST(double)

}  // namespace syk
