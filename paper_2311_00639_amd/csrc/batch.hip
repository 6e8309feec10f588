// Batched OTOC: many small-N realisations and random vectors in one persistent launch.
//
// A job is one (realisation, Haar vector) pair: both parity-block chains of the OTOC of
// Eq. (2) over the whole t grid (the random-state estimator of the supplement).  The grid
// holds one workgroup per resident slot; each workgroup takes jobs from a device counter
// until none is left and runs a whole job by itself, with no host round trip: Haar state,
// Majorana insertions, overlaps and every Lanczos propagator (matrix-free apply_H with the
// vector staged in LDS, Lanczos recurrence with double reductions, small exponential,
// step control, recombination).  Vectors are complex64 in the standard layout; every
// reduction and the tridiagonal exponential are double.
//
// Small exponential.  c = e^{w T} e_1 for the k x k Lanczos tridiagonal T (k <= 64) is
// evaluated by one wavefront, lane i holding component i: T = a + b Y with [a - b, a + b]
// the Gershgorin interval, e^{w b y} expanded in Chebyshev polynomials on [-1, 1] with
// coefficients from 64 Chebyshev nodes (a discrete cosine transform), and the series summed
// with the three-term recurrence of T_n(Y) e_1.  Accurate to rounding while |w b| <= 25;
// a larger argument counts as not converged, so the step control shortens the sub-step.
// The host path (krylov.cpp) uses an eigendecomposition instead; both compute the same
// matrix function.
#include <hip/hip_runtime.h>

#include "batch.hpp"

namespace syk {

namespace {

// Explicit address spaces.  The job code runs in out-of-line functions, where pointers that
// are not typed by address space turn into generic (flat) accesses: slower for LDS, and each
// one waits on both memory counters.
typedef __attribute__((address_space(1))) float2 gf2;          // device memory
typedef __attribute__((address_space(3))) float2 lf2;          // LDS
typedef __attribute__((address_space(1))) const BatchTerm gterm;
typedef __attribute__((address_space(3))) const BatchTerm lterm;

// loads and stores through typed pointers use clang's builtin vector types (the HIP vector
// classes cannot be copied from address-space-qualified objects)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 ld(const gf2 *p) {
    const f32x2 u = *(__attribute__((address_space(1))) const f32x2 *)p;
    return float2{u.x, u.y};
}
__device__ __forceinline__ void st(gf2 *p, float2 v) { *(__attribute__((address_space(1))) f32x2 *)p = f32x2{v.x, v.y}; }
__device__ __forceinline__ float2 ld(const lf2 *p) {
    const f32x2 u = *(__attribute__((address_space(3))) const f32x2 *)p;
    return float2{u.x, u.y};
}
__device__ __forceinline__ void st(lf2 *p, float2 v) { *(__attribute__((address_space(3))) f32x2 *)p = f32x2{v.x, v.y}; }
__device__ __forceinline__ BatchTerm ld(gterm *p) {
    return __builtin_bit_cast(BatchTerm, *(__attribute__((address_space(1))) const u32x4 *)p);
}
__device__ __forceinline__ BatchTerm ld(lterm *p) {
    return __builtin_bit_cast(BatchTerm, *(__attribute__((address_space(3))) const u32x4 *)p);
}

constexpr int kCheb = 64;               // Chebyshev nodes and series length
constexpr double kMaxArg = 25.0;        // largest |w| b evaluated

__device__ __forceinline__ uint64_t bmix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// amplitude n (full-space index) of the Haar state with base = mix(seed + (v + 1) G)
__device__ __forceinline__ double2 bhaar(uint64_t base, uint64_t n) {
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    const uint64_t w1 = bmix(base + (2 * n + 1) * G);
    const uint64_t w2 = bmix(base + (2 * n + 2) * G);
    const double u1 = static_cast<double>((w1 >> 11) + 1) * 0x1p-53;
    const double u2 = static_cast<double>(w2 >> 11) * 0x1p-53;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    return double2{r * cs, r * sn};
}

__device__ __forceinline__ float fsign(float c, uint32_t bit) { return __int_as_float(__float_as_int(c) ^ (bit << 31)); }

// LDS written by some lanes of a wavefront, then read by others of the same wavefront
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

template <int NT>
struct Shared {
    double red[4][NT / 64];
    double al[kMaxKrylov + 2];
    double bt[kMaxKrylov + 2];
    float sc[kMaxKrylov + 2];          // basis vector i is stored as beta_{i-1} v_i: v_i = sc[i] * stored
    double cre[kMaxKrylov + 2], cim[kMaxKrylov + 2];
    double fre[kCheb], fim[kCheb];
    double cosb[4 * kCheb];            // cos(pi j / (2 kCheb)), j < 4 kCheb
    double ctl_d[4];
    int ctl_i[4];
};

template <int NT>
using LShared = __attribute__((address_space(3))) Shared<NT>;

// whole-workgroup context of one job
template <int NT, int CHB>
struct Ctx {
    const BatchParams &p;
    LShared<NT> &sh;
    lf2 *buf;                          // LDS staging, 2^CHB amplitudes
    const BatchJob &job;
    gf2 *basis;                        // (m + 1) vectors
    gf2 *vec[4];                       // l, r2, r4, tmp
    uint32_t tid;
    lterm *lterms[2];                  // the job's terms staged in LDS (null: read from memory)
    long long matvecs = 0;
    int substeps = 0;
    int status = 0;
};

// sum of two doubles over the workgroup, same value and order in every thread
template <int NT>
__device__ __forceinline__ void bsum2(double &a, double &b, LShared<NT> &sh, uint32_t tid) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((tid & 63) == 0) {
        sh.red[0][tid >> 6] = a;
        sh.red[1][tid >> 6] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        a += sh.red[0][w];
        b += sh.red[1][w];
    }
    __syncthreads();
}

// sum of one double over the workgroup, same value and order in every thread
template <int NT>
__device__ __forceinline__ double bsum1(double a, LShared<NT> &sh, uint32_t tid) {
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((tid & 63) == 0) sh.red[0][tid >> 6] = a;
    __syncthreads();
    a = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) a += sh.red[0][w];
    __syncthreads();
    return a;
}

// ------------------------------------------------------------------ vector kernels
// Thread tid owns amplitudes r * NT + tid, r < R = 2^L / NT.

// One term on a thread's RC registers.  xr and zr are wave-uniform: the partner register
// offset (r ^ xr) << LNT and the register sign are scalar values, so each register costs
// one vector add for its LDS address and one vector XOR for its sign besides the FMAs.
template <int NT, int RC, bool IM>
__device__ __forceinline__ void term_regs(float2 (&acc)[RC], const lf2 *buf_lane, float cl, uint32_t xr,
                                          uint32_t zr) {
    constexpr int LNT = __builtin_ctz(NT);
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const float2 q = ld(buf_lane + ((static_cast<uint32_t>(r) ^ xr) << LNT));
        uint32_t sg = (__popc(static_cast<uint32_t>(r) & zr) & 1u) << 31;
        asm("" : "+s"(sg));              // keep the register sign a scalar operand
        const float cr = r == 0 ? cl : __int_as_float(__float_as_int(cl) ^ static_cast<int>(sg));
        if (IM) {
            acc[r].x -= cr * q.y;
            acc[r].y += cr * q.x;
        } else {
            acc[r].x += cr * q.x;
            acc[r].y += cr * q.y;
        }
    }
}

// y = H_blk v (v, y: global, standard layout); returns this thread's share of Re <v, y>.
// The block is cut into NCH chunks of CH amplitudes; output chunk o is accumulated in
// registers (RC per thread) while every chunk ch of v is staged in LDS in turn, and the
// terms whose partner offset x >> log2(CH) equals o ^ ch are applied from it.
template <int NT, int CHB, int L>
__device__ double apply_h(Ctx<NT, CHB> &c, int blk, const gf2 *v, gf2 *y, float vs) {
    constexpr int n = 1 << L;
    constexpr int LCH = L < CHB ? L : CHB;
    constexpr int CH = 1 << LCH;
    constexpr int NCH = n / CH;
    constexpr int RC = CH / NT;
    constexpr int LNT = __builtin_ctz(NT);
    static_assert(NCH >= 1 && NCH <= 4 && RC >= 1 && RC <= 16, "chunking");
    const uint32_t tid = c.tid;
    gterm *terms = (gterm *)(c.p.terms + c.job.term_off[blk]);
    lterm *lterms = c.lterms[blk];
    const int K = c.job.K;
    double dre = 0.0;
    // one term with wave-uniform fields (scalar registers)
    auto term = [&](auto im, float2 (&acc)[RC], uint32_t tx, uint32_t tz, float tc, int o) __attribute__((always_inline)) {
        const uint32_t xl = tx & (CH - 1);
        const uint32_t lane = tid ^ (xl & (NT - 1));
        const uint32_t xr = xl >> LNT;
        const uint32_t zr = (tz >> LNT) & (RC - 1);
        // sign of output m = (o RC + r) NT + tid: thread bits, chunk bits, register bits
        const uint32_t par = (__popc(tid & tz & (NT - 1)) + __popc((tz >> LCH) & static_cast<uint32_t>(o))) & 1u;
        const float cl = fsign(tc, par);
        term_regs<NT, RC, decltype(im)::value>(acc, c.buf + lane, cl, xr, zr);
    };
    // the terms of [lo, hi) with the given phase, from LDS or from memory; the two phases
    // run as separate loops so that each loop body is one straight FMA sequence
    const bool staged = __builtin_amdgcn_readfirstlane(lterms != nullptr ? 1 : 0) != 0;   // uniform
    auto phase = [&](auto im, float2 (&acc)[RC], int lo, int hi, int o) __attribute__((always_inline)) {
        auto one = [&](const BatchTerm &tm) __attribute__((always_inline)) {
            if ((__builtin_amdgcn_readfirstlane(tm.imag) != 0) != decltype(im)::value) return;
            term(im, acc, __builtin_amdgcn_readfirstlane(tm.x), __builtin_amdgcn_readfirstlane(tm.z),
                 __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(tm.c))), o);
        };
        if (staged)
            for (int t = lo; t < hi; ++t) one(ld(lterms + t));
        else
            for (int t = lo; t < hi; ++t) one(ld(terms + t));
    };
    for (int o = 0; o < NCH; ++o) {
        float2 acc[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[r] = float2{0.0f, 0.0f};
        for (int ch = 0; ch < NCH; ++ch) {
            __syncthreads();                              // earlier readers of buf are done
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                const float2 q = ld(v + (ch * CH + r * NT + tid));
                st(c.buf + (r * NT + tid), float2{vs * q.x, vs * q.y});
            }
            __syncthreads();
            // the terms with partner chunk offset x >> LCH == o ^ ch (terms sorted by x)
            const uint32_t want = static_cast<uint32_t>(o ^ ch);
            int lo = 0, hi = K;
            if constexpr (L >= 12) {
                constexpr int SH = LCH - 12;
                lo = c.job.gstart[blk][want << SH];
                hi = c.job.gstart[blk][(want + 1) << SH];
            }
            phase(std::false_type{}, acc, lo, hi, o);
            phase(std::true_type{}, acc, lo, hi, o);
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int i = o * CH + r * NT + static_cast<int>(tid);
            const float2 q = ld(v + i);
            dre += static_cast<double>(vs * q.x) * acc[r].x + static_cast<double>(vs * q.y) * acc[r].y;
            st(y + i, acc[r]);
        }
    }
    return dre;
}

template <int NT, int CHB, int L>
__device__ double norm2(Ctx<NT, CHB> &c, const gf2 *v) {
    constexpr int R = (1 << L) / NT;
    double a = 0.0;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
        const float2 q = ld(v + (r * NT + c.tid));
        a += static_cast<double>(q.x) * q.x + static_cast<double>(q.y) * q.y;
    }
    return bsum1<NT>(a, c.sh, c.tid);
}

// <u, v> = sum conj(u) v
template <int NT, int CHB, int L>
__device__ double2 dot(Ctx<NT, CHB> &c, const gf2 *u, const gf2 *v) {
    constexpr int R = (1 << L) / NT;
    double a = 0.0, b = 0.0;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
        const float2 p = ld(u + (r * NT + c.tid)), q = ld(v + (r * NT + c.tid));
        a += static_cast<double>(p.x) * q.x + static_cast<double>(p.y) * q.y;
        b += static_cast<double>(p.x) * q.y - static_cast<double>(p.y) * q.x;
    }
    bsum2<NT>(a, b, c.sh, c.tid);
    return double2{a, b};
}

template <int NT, int CHB, int L>
__device__ void scale_copy(Ctx<NT, CHB> &c, const gf2 *src, gf2 *dst, double s) {
    constexpr int R = (1 << L) / NT;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
        const float2 q = ld(src + (r * NT + c.tid));
        st(dst + (r * NT + c.tid), float2{static_cast<float>(s * q.x), static_cast<float>(s * q.y)});
    }
    __syncthreads();
}

// dst = chi block map of Majorana n from block `src_blk` (times sqrt 2: the Pauli string)
template <int NT, int CHB, int L>
__device__ void gamma(Ctx<NT, CHB> &c, bool top, uint32_t x, uint32_t z, int w, int src_blk, const gf2 *src,
                      gf2 *dst) {
    constexpr int R = (1 << L) / NT;
    // scale i^w, or +-i for n = N - 1 (U -> D: +i, D -> U: -i)
    int q = top ? (src_blk == 0 ? 1 : 3) : (w & 3);
    if (top) {
        x = 0;
        z = 0;
    }
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
        const uint32_t m = static_cast<uint32_t>(r * NT) + c.tid;
        const uint32_t k = m ^ x;
        float2 v = ld(src + k);
        if (__popc(k & z) & 1) v = float2{-v.x, -v.y};
        float2 o;
        switch (q) {
            case 0: o = v; break;
            case 1: o = float2{-v.y, v.x}; break;
            case 2: o = float2{-v.x, -v.y}; break;
            default: o = float2{v.y, -v.x}; break;
        }
        st(dst + m, o);
    }
    __syncthreads();
}

// Haar state of this job's vector: block A part into dst, normalised over the full space
template <int NT, int CHB, int L>
__device__ void haar(Ctx<NT, CHB> &c, int A, gf2 *dst) {
    constexpr int R = (1 << L) / NT;
    const uint64_t h = 1ULL << L;
    double a = 0.0;
#pragma unroll 2
    for (int r = 0; r < R; ++r) {
        const uint64_t m = static_cast<uint64_t>(r * NT + c.tid);
        const double2 u = bhaar(c.job.base, m);
        const double2 d = bhaar(c.job.base, h + m);
        a += u.x * u.x + u.y * u.y + d.x * d.x + d.y * d.y;
        const double2 s = A == 0 ? u : d;
        st(dst + m, float2{static_cast<float>(s.x), static_cast<float>(s.y)});
    }
    a = bsum1<NT>(a, c.sh, c.tid);
    const double inv = 1.0 / sqrt(a);
#pragma unroll 2
    for (int r = 0; r < R; ++r) {
        const uint64_t m = static_cast<uint64_t>(r * NT + c.tid);
        const double2 u = A == 0 ? bhaar(c.job.base, m) : bhaar(c.job.base, h + m);
        st(dst + m, float2{static_cast<float>(u.x * inv), static_cast<float>(u.y * inv)});
    }
    __syncthreads();
}

// ------------------------------------------------------------------ Lanczos
// one Lanczos iteration j: V_{j+1}, alpha_j = sh.al[j], beta_{j+1} = sh.bt[j + 1]
template <int NT, int CHB, int L>
__device__ void lanczos_step(Ctx<NT, CHB> &c, int blk, int j) {
    constexpr int R = (1 << L) / NT;
    const gf2 *vj = c.basis + static_cast<size_t>(j) * c.p.vec_stride;
    const gf2 *vp = j > 0 ? c.basis + static_cast<size_t>(j - 1) * c.p.vec_stride : nullptr;
    gf2 *vn = c.basis + static_cast<size_t>(j + 1) * c.p.vec_stride;
    // basis slots hold v_i / sc[i]; the next slot is left unnormalised (its scale 1/beta_j
    // enters wherever it is read), which saves a normalising pass per step
    const float sj = c.sh.sc[j];
    const float sp = j > 0 ? c.sh.sc[j - 1] : 0.0f;
    const double alpha = bsum1<NT>(apply_h<NT, CHB, L>(c, blk, vj, vn, sj), c.sh, c.tid);
    const double bprev = c.sh.bt[j];
    const float fa = static_cast<float>(alpha) * sj, fb = static_cast<float>(bprev) * sp;
    double w2 = 0.0;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
        const int i = r * NT + static_cast<int>(c.tid);
        const float2 q = ld(vj + i);
        float2 w = ld(vn + i);
        w.x -= fa * q.x;
        w.y -= fa * q.y;
        if (vp) {
            const float2 p = ld(vp + i);
            w.x -= fb * p.x;
            w.y -= fb * p.y;
        }
        st(vn + i, w);
        w2 += static_cast<double>(w.x) * w.x + static_cast<double>(w.y) * w.y;
    }
    const double beta = sqrt(bsum1<NT>(w2, c.sh, c.tid));
    if (c.tid == 0) {
        c.sh.al[j] = alpha;
        c.sh.bt[j + 1] = beta;
        c.sh.sc[j + 1] = beta > 0.0 ? static_cast<float>(1.0 / beta) : 0.0f;
    }
    __syncthreads();
}

// Wavefront 0 only.  c = e^{(wr + i wi) T_k} e_1 into sh.cre / sh.cim; returns |c_{k-1}|,
// or a negative value when the argument exceeds the evaluated range.
template <int NT>
__device__ double small_exp(LShared<NT> &sh, int k, double wr, double wi, uint32_t lane) {
    // Gershgorin interval of T_k (off-diagonal bt[1..k-1])
    double lo = 1e300, hi = -1e300;
    if (static_cast<int>(lane) < k) {
        const double d = sh.al[lane];
        const double e0 = lane > 0 ? fabs(sh.bt[lane]) : 0.0;
        const double e1 = static_cast<int>(lane) + 1 < k ? fabs(sh.bt[lane + 1]) : 0.0;
        lo = d - e0 - e1;
        hi = d + e0 + e1;
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    const double a = 0.5 * (hi + lo);
    const double b = fmax(0.5 * (hi - lo), 1e-300);
    const double ur = wr * b, ui = wi * b;           // argument on [-1, 1]
    if (sqrt(ur * ur + ui * ui) > kMaxArg) return -1.0;
    // samples at the Chebyshev nodes y_q = cos(pi (q + 1/2) / M)
    {
        const double y = sh.cosb[2 * lane + 1];
        const double er = exp(ur * y);
        double sn, cs;
        sincos(ui * y, &sn, &cs);
        sh.fre[lane] = er * cs;
        sh.fim[lane] = er * sn;
    }
    wave_lds_sync();
    // coefficient n = lane: (2 / M) sum_q f_q cos(pi n (2q + 1) / (2M))
    double cr = 0.0, ci = 0.0;
    for (int q = 0; q < kCheb; ++q) {
        const double cs = sh.cosb[(lane * (2 * q + 1)) & (4 * kCheb - 1)];
        cr += sh.fre[q] * cs;
        ci += sh.fim[q] * cs;
    }
    cr *= 2.0 / kCheb;
    ci *= 2.0 / kCheb;
    if (lane == 0) {
        cr *= 0.5;
        ci *= 0.5;
    }
    wave_lds_sync();
    sh.fre[lane] = cr;                                // the samples are no longer needed
    sh.fim[lane] = ci;
    wave_lds_sync();
    // sum_n a_n T_n(Y) e_1, Y = (T - a) / b, lane i = component i
    const bool in = static_cast<int>(lane) < k;
    const double d = in ? (sh.al[lane] - a) / b : 0.0;
    const double lo_off = (in && lane > 0) ? sh.bt[lane] / b : 0.0;                    // to i - 1
    const double up_off = (in && static_cast<int>(lane) + 1 < k) ? sh.bt[lane + 1] / b : 0.0;   // to i + 1
    auto applyY = [&](double u) {
        const double um = __shfl(u, (lane + 63) & 63, 64);
        const double up = __shfl(u, (lane + 1) & 63, 64);
        return in ? d * u + lo_off * um + up_off * up : 0.0;
    };
    double u0 = lane == 0 ? 1.0 : 0.0;
    double u1 = applyY(u0);
    double sr = sh.fre[0] * u0 + sh.fre[1] * u1;
    double si = sh.fim[0] * u0 + sh.fim[1] * u1;
    for (int nn = 2; nn < kCheb; ++nn) {
        const double u2 = 2.0 * applyY(u1) - u0;
        sr += sh.fre[nn] * u2;
        si += sh.fim[nn] * u2;
        u0 = u1;
        u1 = u2;
    }
    // times e^{w a}
    const double er = exp(wr * a);
    double sn, cs;
    sincos(wi * a, &sn, &cs);
    const double gr = er * cs, gi = er * sn;
    const double outr = gr * sr - gi * si, outi = gr * si + gi * sr;
    if (in) {
        sh.cre[lane] = outr;
        sh.cim[lane] = outi;
    }
    const double mag = sqrt(outr * outr + outi * outi);
    return __shfl(mag, k - 1, 64);
}

// Step decision after k Lanczos vectors (wavefront 0): ctl_i[0] = 1 if the sub-step ends
// here, ctl_d[0] = its fraction tau, ctl_i[1] = error; cre/cim hold e^{tau z T} e_1.
template <int NT>
__device__ void decide(LShared<NT> &sh, int k, int m, double remaining, double zr, double zi, double tol,
                       uint32_t lane) {
    double tn = 0.0;
    if (static_cast<int>(lane) < k) tn = fmax(fabs(sh.al[lane]), lane > 0 ? sh.bt[lane] : 0.0);
    for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_xor(tn, off, 64));
    const double bk = sh.bt[k];
    const bool breakdown = bk <= 1e-14 * fmax(tn, 1e-300);
    auto err = [&](double f) {
        const double l = small_exp<NT>(sh, k, f * zr, f * zi, lane);
        if (l < 0.0) return 1e300;
        return breakdown ? 0.0 : bk * l;
    };
    int done = 0, fail = 0;
    double tau = 0.0;
    if (!(bk == bk)) {
        fail = 6;
    } else if (err(remaining) <= tol * remaining) {
        tau = remaining;
        done = 1;
    } else if (k == m) {
        double lo = 0.0, hi = remaining;
        for (int it = 0; it < 200; ++it) {
            const double mid = (lo == 0.0) ? hi * 0.5 : sqrt(lo * hi);
            if (err(mid) <= tol * mid)
                lo = mid;
            else
                hi = mid;
            if (lo > 0.0 && hi / lo < 1.0 + 1e-3) break;
            if (lo == 0.0 && hi < 1e-14 * remaining) break;
        }
        if (lo <= 1e-12 * remaining) {
            fail = 5;
        } else {
            tau = lo;
            done = 1;
            err(tau);                                 // leaves e^{tau z T} e_1 in cre / cim
        }
    }
    if (lane == 0) {
        sh.ctl_i[0] = done;
        sh.ctl_i[1] = fail;
        sh.ctl_d[0] = tau;
    }
}

// v <- e^{z H_blk} v (in place), Lanczos with restarts and the step control of the
// single-vector path
template <int NT, int CHB, int L>
__device__ void prop(Ctx<NT, CHB> &c, int blk, double zr, double zi, gf2 *v) {
    constexpr int R = (1 << L) / NT;
    if (c.status) return;
    double nrm = sqrt(norm2<NT, CHB, L>(c, v));
    if (nrm == 0.0 || (zr == 0.0 && zi == 0.0)) return;
    if (!(nrm == nrm)) {
        c.status = 6;
        return;
    }
    const int m = c.p.m;
    double remaining = 1.0;
    for (;;) {
        if (++c.substeps > c.p.max_substeps) {
            c.status = 5;
            return;
        }
        scale_copy<NT, CHB, L>(c, v, c.basis, 1.0 / nrm);
        if (c.tid == 0) {
            c.sh.bt[0] = 0.0;
            c.sh.sc[0] = 1.0f;
        }
        __syncthreads();
        int k = 0, next = 4, done = 0;
        double tau = 0.0;
        for (int j = 0; j < m; ++j) {
            lanczos_step<NT, CHB, L>(c, blk, j);
            ++c.matvecs;
            k = j + 1;
            if (k < next && k < m) continue;
            next = k + 1;
            if (c.tid < 64) decide<NT>(c.sh, k, m, remaining, zr, zi, c.p.tol, c.tid);
            __syncthreads();
            done = c.sh.ctl_i[0];
            const int fail = c.sh.ctl_i[1];
            tau = c.sh.ctl_d[0];
            __syncthreads();
            if (fail) {
                c.status = fail;
                return;
            }
            if (done) break;
        }
        if (!done) {                                  // m == 0 cannot happen; defensive
            c.status = 5;
            return;
        }
        // v = nrm * sum_i c_i V_i
#pragma unroll 2
        for (int r = 0; r < R; ++r) {
            double sr = 0.0, si = 0.0;
            for (int i = 0; i < k; ++i) {
                const float2 q = ld(c.basis + (static_cast<size_t>(i) * c.p.vec_stride + r * NT + c.tid));
                const double cr = c.sh.cre[i] * c.sh.sc[i], ci = c.sh.cim[i] * c.sh.sc[i];
                sr += cr * q.x - ci * q.y;
                si += cr * q.y + ci * q.x;
            }
            st(v + (r * NT + c.tid), float2{static_cast<float>(nrm * sr), static_cast<float>(nrm * si)});
        }
        __syncthreads();
        remaining -= tau;
        if (remaining <= 1e-15) return;
        nrm = sqrt(norm2<NT, CHB, L>(c, v));
        if (nrm == 0.0) return;
        if (!(nrm == nrm)) {
            c.status = 6;
            return;
        }
    }
}

// the OTOC chains of one job (both blocks, all t points) into F (nt complex, accumulated)
template <int NT, int CHB, int L>
__device__ __attribute__((noinline)) void run_job(Ctx<NT, CHB> &c, double2 *F) {
    const BatchJob &jb = c.job;
    const double beta = jb.beta;
    gf2 *l = c.vec[0], *r2 = c.vec[1], *r4 = c.vec[2], *tmp = c.vec[3];
    for (int A = 0; A < 2; ++A) {
        const int B = 1 - A;
        haar<NT, CHB, L>(c, A, l);
        prop<NT, CHB, L>(c, A, -beta / 8.0, 0.0, l);                              // r0
        gamma<NT, CHB, L>(c, jb.v_top, jb.vx, jb.vz, jb.vw, A, l, r2);            // V_BA r0
        prop<NT, CHB, L>(c, B, -beta / 4.0, 0.0, r2);
        double tprev = 0.0;
        for (int k = 0; k < c.p.nt; ++k) {
            const double t = c.p.ts[k];
            const double dt = t - tprev;
            if (dt > 0.0) {
                prop<NT, CHB, L>(c, B, 0.0, -dt, r2);
                prop<NT, CHB, L>(c, A, 0.0, -dt, l);
            }
            tprev = t;
            gamma<NT, CHB, L>(c, jb.w_top, jb.wx, jb.wz, jb.ww, B, r2, r4);       // W_AB r2
            prop<NT, CHB, L>(c, A, -beta / 4.0, t, r4);
            gamma<NT, CHB, L>(c, jb.v_top, jb.vx, jb.vz, jb.vw, A, r4, tmp);      // V_BA r4
            prop<NT, CHB, L>(c, B, -beta / 4.0, -t, tmp);                         // r6
            gamma<NT, CHB, L>(c, jb.w_top, jb.wx, jb.wz, jb.ww, B, tmp, r4);      // W_AB r6
            const double2 d = dot<NT, CHB, L>(c, l, r4);
            if (c.tid == 0) {
                F[k].x += 0.25 * d.x;
                F[k].y += 0.25 * d.y;
            }
            if (c.status) return;
        }
    }
}

template <int NT, int CHB, int OCC>
__global__ void __launch_bounds__(NT, OCC * NT / 256) otoc_batch_kernel(BatchParams p) {
    __shared__ Shared<NT> sh;
    __shared__ float2 buf[1 << CHB];
    __shared__ int job_sh;
    // term staging for the job (both blocks), where LDS allows: jobs with more terms read
    // them from memory
    constexpr int TL = NT >= 512 ? 256 : 1;
    __shared__ BatchTerm tl[2][TL];
    const uint32_t tid = threadIdx.x;
    for (int j = tid; j < 4 * kCheb; j += NT) sh.cosb[j] = cos(M_PI * j / (2.0 * kCheb));
    gf2 *slot = (gf2 *)(p.ws + static_cast<size_t>(blockIdx.x) * p.slot_stride);   // address-space cast
    for (;;) {
        __syncthreads();
        if (tid == 0) job_sh = static_cast<int>(atomicAdd(p.counter, 1u));
        __syncthreads();
        const int ji = job_sh;
        if (ji >= p.n_jobs) break;
        const BatchJob &jb = p.jobs[ji];
        double2 *F = reinterpret_cast<double2 *>(p.F) + static_cast<size_t>(ji) * p.nt;
        if (tid == 0)
            for (int k = 0; k < p.nt; ++k) F[k] = double2{0.0, 0.0};
        Ctx<NT, CHB> c{p, *(LShared<NT> *)(&sh), (lf2 *)(buf), jb, slot, {slot + static_cast<size_t>(p.m + 1) * p.vec_stride,
                                               slot + static_cast<size_t>(p.m + 2) * p.vec_stride,
                                               slot + static_cast<size_t>(p.m + 3) * p.vec_stride,
                                               slot + static_cast<size_t>(p.m + 4) * p.vec_stride},
                       tid, {nullptr, nullptr}};
        if (TL > 1 && jb.K <= TL) {
            for (int blk = 0; blk < 2; ++blk)
                for (int t = static_cast<int>(tid); t < jb.K; t += NT) tl[blk][t] = p.terms[jb.term_off[blk] + t];
            __syncthreads();
            c.lterms[0] = (lterm *)(tl[0]);
            c.lterms[1] = (lterm *)(tl[1]);
        }
        // the block size is a compile-time parameter of the job code
        switch (jb.L) {
#define SYK_BL(LL)                                                       \
    case LL:                                                             \
        if constexpr ((1 << LL) >= NT && (1 << LL) <= 4 * (1 << CHB)) run_job<NT, CHB, LL>(c, F); \
        else c.status = 2;                                               \
        break;
            SYK_BL(8)
            SYK_BL(9)
            SYK_BL(10)
            SYK_BL(11)
            SYK_BL(12)
            SYK_BL(13)
            SYK_BL(14)
            SYK_BL(15)
#undef SYK_BL
            default:
                c.status = 2;
        }
        if (tid == 0) {
            p.status[ji] = c.status;
            p.matvecs[ji] = c.matvecs;
        }
    }
}

}  // namespace

bool batch_variant_supports(const BatchVariant &v, int L) {
    return L >= 8 && L <= 15 && (1 << L) >= v.nt && (1 << L) <= 4 * (1 << v.chb);
}

const std::vector<BatchVariant> &batch_variants() {
    static const std::vector<BatchVariant> v = {{1024, 14, 1}, {512, 13, 2}, {256, 12, 4}};
    return v;
}

void launch_otoc_batch(const BatchVariant &v, const BatchParams &p, int grid, hipStream_t s) {
    if (v.nt == 1024 && v.chb == 14 && v.occ == 1)
        hipLaunchKernelGGL((otoc_batch_kernel<1024, 14, 1>), dim3(grid), dim3(1024), 0, s, p);
    else if (v.nt == 512 && v.chb == 13 && v.occ == 2)
        hipLaunchKernelGGL((otoc_batch_kernel<512, 13, 2>), dim3(grid), dim3(512), 0, s, p);
    else if (v.nt == 256 && v.chb == 12 && v.occ == 4)
        hipLaunchKernelGGL((otoc_batch_kernel<256, 12, 4>), dim3(grid), dim3(256), 0, s, p);
    else
        fail(SYK_EDEVICE, "unknown batch variant");
    SYK_HIP(hipGetLastError());
}

}  // namespace syk
