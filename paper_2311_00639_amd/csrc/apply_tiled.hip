// Tiled apply_H for large parity blocks (gfx950).
//
// y[m] = sum_a c_a i^{imag_a} (-1)^{popc(m & z_a)} x[m ^ x_a]   (supplement Algorithm 1, with the
// sign parity of x_a & z_a folded into c_a).
//
// Data flow.  A workgroup owns one output tile of 2^BT consecutive amplitudes, held in
// registers: thread t keeps outputs r * NT + t, r < R.  Terms are grouped on the host by
// g = x_a >> BT, so every term of a group reads the same partner tile T ^ g.  For each
// group the partner tile is copied once into LDS by direct global-to-LDS loads (the next
// groups' tiles stream into other LDS buffers while the current one is consumed) and
// every term of the group reads it with an XOR-permuted index: the thread bits of x_a permute the lane's
// LDS address once per term, the register bits add a wave-uniform offset per read.  The
// tile and thread parts of the sign are folded into the coefficient once per term; the
// register part is a wave-uniform select per read, so an amplitude costs one LDS read,
// one address add, one select and two FMAs.  The host planner (apply_plan.cpp) maps
// workgroups to tiles so that the tiles resident on one XCD form a coset of a subspace
// that many partner offsets differ by, and orders groups class by class, so a partner
// tile fetched for one workgroup is re-read from L2 by others.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "apply_plan.hpp"

namespace syk {

namespace {

template <typename T> struct V2t;
template <> struct V2t<float> { using type = float2; };
template <> struct V2t<double> { using type = double2; };

// Per-term record (host-built, 4 + 2R dwords): thread bits of x, thread bits of z,
// z >> BT, unused, then for r < R the LDS byte offset of partner register r ^ xr and the
// sign mask (bit 31 set iff popc(r & zr) is odd) of output register r.
template <int R>
struct TermRec {
    uint32_t xt, zt, zh, pad;
    uint32_t off[R];
    uint32_t sgn[R];
};

__device__ __forceinline__ float flip_sign(float c, uint32_t m) { return __int_as_float(__float_as_int(c) ^ m); }
__device__ __forceinline__ double flip_sign(double c, uint32_t m) {
    return __longlong_as_double(__double_as_longlong(c) ^ (static_cast<long long>(m) << 32));
}

template <typename T, int BT, int RB, bool IM>
__device__ __forceinline__ void apply_terms(typename V2t<T>::type (&acc)[1 << RB], const typename V2t<T>::type *b,
                                            const TermRec<1 << RB> *__restrict__ recs, const T *__restrict__ coef,
                                            int t0, int t1, uint32_t tile, uint32_t tid) {
    using V = typename V2t<T>::type;
    constexpr int R = 1 << RB;
    if (t0 >= t1) return;
    // the next term's record is fetched while this one is applied (records are padded by one)
    TermRec<R> nxt = recs[t0];
    T cn = coef[t0];
    for (int t = t0; t < t1; ++t) {
        const TermRec<R> rec = nxt;                     // wave-uniform: scalar loads
        const T c = cn;
        nxt = recs[t + 1];
        cn = coef[t + 1];
        const uint32_t par = (__popc(tile & rec.zh) + __popc(tid & rec.zt)) & 1u;
        const T cl = flip_sign(c, par << 31);
        const char *bs = reinterpret_cast<const char *>(b + (tid ^ rec.xt));
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const V q = *reinterpret_cast<const V *>(bs + rec.off[r]);
            const T cr = flip_sign(cl, rec.sgn[r]);
            if (IM) {
                acc[r].x -= cr * q.y;
                acc[r].y += cr * q.x;
            } else {
                acc[r].x += cr * q.x;
                acc[r].y += cr * q.y;
            }
        }
    }
}

// s_waitcnt immediate (GFX9 encoding) that waits until at most `vm` vector-memory
// operations of this wave are outstanding; expcnt and lgkmcnt are left unconstrained
constexpr int waitcnt_vm(int vm) { return (vm & 15) | (7 << 4) | (15 << 8) | (((vm >> 4) & 3) << 14); }

#define SYK_LDS(p) ((__attribute__((address_space(3))) void *)(p))

// Copy partner tile `src` (2^BT amplitudes) into LDS buffer `dst` with direct
// global-to-LDS loads: 16 bytes per lane, a wave writes 1 KiB contiguous per instruction,
// so the LDS holds the tile in index order.  No VGPRs are involved.
template <typename T, int BT, int RB>
__device__ __forceinline__ void dma_tile(const typename V2t<T>::type *src, typename V2t<T>::type *dst,
                                         uint32_t tid) {
    constexpr int NT = 1 << (BT - RB);
    constexpr int BYTES = (1 << BT) * 2 * static_cast<int>(sizeof(T));
    constexpr int PER = BYTES / (NT * 16);                 // instructions per thread
    const char *g = reinterpret_cast<const char *>(src);
    char *l = reinterpret_cast<char *>(dst);
    const uint32_t wave_base = (tid & ~63u) * 16u;
#pragma unroll
    for (int j = 0; j < PER; ++j)
        __builtin_amdgcn_global_load_lds(g + (j * NT + tid) * 16, SYK_LDS(l + j * NT * 16 + wave_base), 16, 0, 0);
}

template <int K, typename V>
__device__ __forceinline__ V *pick(V *b0, V *b1, V *b2, V *b3) {
    if constexpr (K == 0) return b0;
    if constexpr (K == 1) return b1;
    if constexpr (K == 2) return b2;
    return b3;
}

// Partner tiles stream into NBUF LDS buffers by direct loads, NBUF - 1 of them in flight
// while the current one is consumed; the buffers are distinct LDS objects so that reads
// of one need not wait for copies into the others.  With NBUF = 1 the copy and the
// compute of a group alternate inside the workgroup and OCC workgroups share a CU, so one
// computes while another waits for its tile.  n_groups is a multiple of NBUF (the host
// pads with empty groups) and grp_g holds NBUF - 1 extra entries.  blockIdx maps to an
// output tile through tile_map.  The second launch bound (waves per SIMD) keeps OCC
// workgroups resident.
template <typename T, int BT, int RB, int NBUF, int OCC>
__global__ void __launch_bounds__(1 << (BT - RB), OCC * (1 << (BT - RB)) / 256) apply_h_tiled(
    const typename V2t<T>::type *__restrict__ x, typename V2t<T>::type *__restrict__ y, uint64_t ld,
    const uint32_t *__restrict__ tile_map, const uint32_t *__restrict__ grp_g,
    const uint32_t *__restrict__ grp_first, const uint32_t *__restrict__ grp_mid, int n_groups,
    const TermRec<1 << RB> *__restrict__ recs, const T *__restrict__ coef, LanczosFuse<T> lf) {
    using V = typename V2t<T>::type;
    constexpr int NT = 1 << (BT - RB);
    constexpr int R = 1 << RB;
    constexpr int TILE = 1 << BT;
    constexpr int PER = TILE * 2 * static_cast<int>(sizeof(T)) / (NT * 16);
    static_assert(NBUF >= 1 && NBUF <= 4, "1 to 4 LDS buffers");
    __shared__ V b0[TILE];
    __shared__ V b1[NBUF > 1 ? TILE : 1];
    __shared__ V b2[NBUF > 2 ? TILE : 1];
    __shared__ V b3[NBUF > 3 ? TILE : 1];

    const uint32_t tid = threadIdx.x;
    const uint32_t tile = tile_map[blockIdx.x];
    const uint64_t vo = static_cast<uint64_t>(blockIdx.y) * ld;
    const V *xv = x + vo;
    V *yv = y + vo;
    auto partner = [&](int gi) { return xv + (static_cast<uint64_t>(tile ^ grp_g[gi]) << BT); };

    V acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = V{T(0), T(0)};

    if constexpr (NBUF == 1) {
        for (int gi = 0; gi < n_groups; ++gi) {
            // the previous group's reads of b0 ended at the barrier closing its step
            dma_tile<T, BT, RB>(partner(gi), b0, tid);
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            const int t0 = static_cast<int>(grp_first[gi]);
            const int tm = static_cast<int>(grp_mid[gi]);
            const int t1 = static_cast<int>(grp_first[gi + 1]);
            apply_terms<T, BT, RB, false>(acc, b0, recs, coef, t0, tm, tile, tid);
            apply_terms<T, BT, RB, true>(acc, b0, recs, coef, tm, t1, tile, tid);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        }
    } else {
        dma_tile<T, BT, RB>(partner(0), b0, tid);
        if constexpr (NBUF > 2) dma_tile<T, BT, RB>(partner(1), b1, tid);
        if constexpr (NBUF > 3) dma_tile<T, BT, RB>(partner(2), b2, tid);
        for (int g0 = 0; g0 < n_groups; g0 += NBUF) {
            auto step = [&](auto kc) {
                constexpr int K = decltype(kc)::value;
                const int gi = g0 + K;
                // this group's copy was issued NBUF - 1 steps ago; NBUF - 2 copies are newer.
                // A bare s_barrier (no fence): each wave has waited for its own pieces of the
                // tile, LDS is coherent within the CU, and the barrier also guarantees that
                // every wave is done reading the buffer the next copy overwrites.
                __builtin_amdgcn_s_waitcnt(waitcnt_vm(PER * (NBUF - 2)));
                asm volatile("" ::: "memory");   // no LDS access or copy moves across the barrier
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                dma_tile<T, BT, RB>(partner(gi + NBUF - 1), pick<(K + NBUF - 1) % NBUF>(b0, b1, b2, b3), tid);
                const V *b = pick<K>(b0, b1, b2, b3);
                const int t0 = static_cast<int>(grp_first[gi]);
                const int tm = static_cast<int>(grp_mid[gi]);
                const int t1 = static_cast<int>(grp_first[gi + 1]);
                apply_terms<T, BT, RB, false>(acc, b, recs, coef, t0, tm, tile, tid);
                apply_terms<T, BT, RB, true>(acc, b, recs, coef, tm, t1, tile, tid);
            };
            step(std::integral_constant<int, 0>{});
            step(std::integral_constant<int, 1>{});
            if constexpr (NBUF > 2) step(std::integral_constant<int, 2>{});
            if constexpr (NBUF > 3) step(std::integral_constant<int, 3>{});
        }
    }
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));      // no copy may still target LDS at exit
    V *dst = yv + (static_cast<uint64_t>(tile) << BT);
    if (lf.partials == nullptr) {
        // outputs are not re-read by this kernel: stream them past the caches
#pragma unroll
        for (int r = 0; r < R; ++r) {
            __builtin_nontemporal_store(acc[r].x, &dst[r * NT + tid].x);
            __builtin_nontemporal_store(acc[r].y, &dst[r * NT + tid].y);
        }
        return;
    }
    // Lanczos epilogue: w = H v_j - beta_{j-1} v_{j-1}, and this tile's shares of
    // <v_j, w> (re, im), ||w||^2 and ||v_j||^2 in double
    const T bp = lf.vprev ? static_cast<T>(sqrt(lf.beta2_prev[0])) : T(0);
    const V *vp = reinterpret_cast<const V *>(lf.vprev) + (static_cast<uint64_t>(tile) << BT);
    const V *vc = reinterpret_cast<const V *>(lf.vcur) + (static_cast<uint64_t>(tile) << BT);
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    auto epilogue = [&](auto has_prev) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = r * NT + tid;
            V w = acc[r];
            if constexpr (decltype(has_prev)::value) {
                const V p = vp[i];
                w.x -= bp * p.x;
                w.y -= bp * p.y;
            }
            const V c = vc[i];
            dst[i] = w;
            sum[0] += static_cast<double>(c.x) * w.x + static_cast<double>(c.y) * w.y;
            sum[1] += static_cast<double>(c.x) * w.y - static_cast<double>(c.y) * w.x;
            sum[2] += static_cast<double>(w.x) * w.x + static_cast<double>(w.y) * w.y;
            sum[3] += static_cast<double>(c.x) * c.x + static_cast<double>(c.y) * c.y;
            // bound the loads in flight: with several workgroups per CU the register
            // budget is 64 VGPRs
            if (r % 2 == 1) __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (lf.vprev)
        epilogue(std::true_type{});
    else
        epilogue(std::false_type{});
    __shared__ double red[4][NT / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = sum[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((tid & 63) == 0) red[k][tid >> 6] = v;
    }
    __syncthreads();
    if (tid < 4) {
        double v = 0.0;
        for (int w = 0; w < NT / 64; ++w) v += red[tid][w];
        lf.partials[static_cast<size_t>(blockIdx.x) * 4 + tid] = v;
    }
}

}  // namespace

template <typename T, int BT, int RB, int NBUF, int OCC>
static void launch_variant(const ApplyPlan &pl, const T *x, T *y, int nvec, uint64_t ld, const LanczosFuse<T> &lf,
                           hipStream_t s) {
    using V = typename V2t<T>::type;
    const T *coef = nullptr;
    if constexpr (sizeof(T) == 4)
        coef = pl.c32;
    else
        coef = pl.c64;
    dim3 grid(pl.n_tiles, nvec);
    hipLaunchKernelGGL((apply_h_tiled<T, BT, RB, NBUF, OCC>), grid, dim3(1 << (BT - RB)), 0, s,
                       reinterpret_cast<const V *>(x), reinterpret_cast<V *>(y), ld, pl.tile_map, pl.grp_g,
                       pl.grp_first, pl.grp_mid, pl.n_groups,
                       reinterpret_cast<const TermRec<1 << RB> *>(pl.meta), coef, lf);
    SYK_HIP(hipGetLastError());
}

template <typename T>
void launch_apply_tiled(const ApplyPlan &pl, const T *x, T *y, int nvec, uint64_t ld, hipStream_t s,
                        const LanczosFuse<T> *lf) {
    const TiledVariant &v = tiled_variants<T>()[pl.variant];
    const LanczosFuse<T> none{};
    if (lf && nvec != 1) fail(SYK_EDEVICE, "the fused Lanczos epilogue takes one vector");
#define SYK_TV(BT, RB, NB, OC)                                                      \
    if (v.bt == BT && v.rb == RB && v.nbuf == NB && v.occ == OC) {                  \
        launch_variant<T, BT, RB, NB, OC>(pl, x, y, nvec, ld, lf ? *lf : none, s);  \
        return;                                                                     \
    }
    if constexpr (sizeof(T) == 4) {
        SYK_TV(13, 3, 2, 1)
        SYK_TV(13, 3, 1, 2)
        SYK_TV(12, 3, 1, 4)
        SYK_TV(12, 3, 2, 2)
        SYK_TV(12, 2, 4, 1)
        SYK_TV(11, 2, 2, 4)
    } else {
        SYK_TV(12, 2, 2, 1)
        SYK_TV(12, 2, 1, 2)
        SYK_TV(11, 2, 1, 4)
        SYK_TV(11, 2, 2, 2)
        SYK_TV(11, 1, 4, 1)
        SYK_TV(10, 1, 2, 4)
    }
#undef SYK_TV
    fail(SYK_EDEVICE, "unknown tiled apply_H variant");
}

template void launch_apply_tiled<float>(const ApplyPlan &, const float *, float *, int, uint64_t, hipStream_t,
                                        const LanczosFuse<float> *);
template void launch_apply_tiled<double>(const ApplyPlan &, const double *, double *, int, uint64_t, hipStream_t,
                                         const LanczosFuse<double> *);

}  // namespace syk
