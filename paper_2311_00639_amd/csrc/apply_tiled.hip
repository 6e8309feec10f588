// Tiled apply_H for large parity blocks (gfx950).
//
// y[m] = sum_a c_a i^{imag_a} (-1)^{popc(m & z_a)} x[m ^ x_a]   (supplement Algorithm 1, with the
// sign parity of x_a & z_a folded into c_a).
//
// Data flow.  A workgroup owns 2^W output tiles of 2^BT consecutive amplitudes (a coset
// t0 ^ span(h) of the tile index space), held in registers: thread t keeps outputs
// r * NT + t, r < R, of each.  Terms are grouped on the host by g = x_a >> BT, so every term
// of a group reads the same partner tile T ^ g.  The workgroup streams the union of its
// tiles' partner tiles once: each partner tile is copied into LDS by direct memory-to-LDS
// loads (buffer form, issued by four waves; the next one streams into the other buffer while
// the current one is consumed), and every term that needs it reads it with an XOR-permuted
// index: the thread bits of x_a permute the lane's LDS address once per term, the register
// bits give one address per register read.  The tile and thread parts of the sign are folded
// into the coefficient once per term, the register part is one sign operation per read, so an
// amplitude costs one LDS read, one address operation, one sign operation and two FMAs; a term
// that touches no register bit (the host puts these first in each run) reads at constant
// offsets and has no register signs.  Term data comes either from per-term records (scalar
// loads) or from per-step control blocks held in a VGPR and read with readlane (no scalar
// loads in the term loop).  The host planner (apply_plan.cpp) maps
// workgroups to tiles so that the tiles resident on one XCD form a coset of a subspace that
// many partner offsets differ by, and orders partner steps class by class, so a partner tile
// fetched for one workgroup is re-read from L2 by others.
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

// Register-static terms: a 4-dword record (thread bits of x, thread bits of z, z >> BT,
// code = (xr << RB) | zr) selects one of (2^RB)^2 compiled paths in which the partner
// register r ^ xr is a constant LDS offset and the sign of output register r (parity of
// r & zr) a constant operand sign, so an amplitude costs one LDS read and two FMAs.
struct TermRec4 {
    uint32_t xt, zt, zh, code;
};

template <typename T, int TB, int RB, int XR, int ZR, bool IM>
__device__ __forceinline__ void term_static(typename V2t<T>::type (&acc)[1 << RB], const typename V2t<T>::type *bs,
                                            T cl) {
    using V = typename V2t<T>::type;
    constexpr int R = 1 << RB;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const V q = bs[(r ^ XR) << TB];
        const T cr = (__builtin_popcount(r & ZR) & 1) ? -cl : cl;
        if (IM) {
            acc[r].x -= cr * q.y;
            acc[r].y += cr * q.x;
        } else {
            acc[r].x += cr * q.x;
            acc[r].y += cr * q.y;
        }
    }
}

template <typename T, int TB, int RB, bool IM, int C>
__device__ __forceinline__ void term_case(typename V2t<T>::type (&acc)[1 << RB], const typename V2t<T>::type *bs,
                                          T cl) {
    constexpr int R = 1 << RB;
    if constexpr (C < R * R) term_static<T, TB, RB, C / R, C % R, IM>(acc, bs, cl);
}

template <typename T, int BT, int RB, bool IM>
__device__ __forceinline__ void apply_terms_static(typename V2t<T>::type (&acc)[1 << RB],
                                                   const typename V2t<T>::type *b,
                                                   const TermRec4 *__restrict__ recs, const T *__restrict__ coef,
                                                   int t0, int t1, uint32_t tile, uint32_t tid) {
    using V = typename V2t<T>::type;
    constexpr int TB = BT - RB;
    if (t0 >= t1) return;
    TermRec4 nxt = recs[t0];
    T cn = coef[t0];
    for (int t = t0; t < t1; ++t) {
        const TermRec4 rec = nxt;                       // wave-uniform: scalar loads
        const T c = cn;
        nxt = recs[t + 1];
        cn = coef[t + 1];
        const uint32_t par = (__popc(tile & rec.zh) + __popc(tid & rec.zt)) & 1u;
        const T cl = flip_sign(c, par << 31);
        const V *bs = b + (tid ^ rec.xt);
#define SYK_C4(B)                                                  \
    case B + 0: term_case<T, TB, RB, IM, B + 0>(acc, bs, cl); break; \
    case B + 1: term_case<T, TB, RB, IM, B + 1>(acc, bs, cl); break; \
    case B + 2: term_case<T, TB, RB, IM, B + 2>(acc, bs, cl); break; \
    case B + 3: term_case<T, TB, RB, IM, B + 3>(acc, bs, cl); break;
        switch (rec.code) {
            SYK_C4(0) SYK_C4(4) SYK_C4(8) SYK_C4(12) SYK_C4(16) SYK_C4(20) SYK_C4(24) SYK_C4(28)
            SYK_C4(32) SYK_C4(36) SYK_C4(40) SYK_C4(44) SYK_C4(48) SYK_C4(52) SYK_C4(56) SYK_C4(60)
            default: break;
        }
#undef SYK_C4
    }
}

// Control-block records (record form 2): a wave holds the current partner step's 64-dword
// control block in one VGPR (lane l = dword l) and reads a record's four dwords with
// readlane into scalar registers, so the term loop issues no scalar memory load (those
// share the LDS reads' counter and would make every LDS wait also wait for them).
// Record: (thread bits of x | xr << 24, thread bits of z | sign mask << 24, z >> BT,
// coefficient: one dword for float, two for double); bit r of the sign mask is the
// parity of r & zr.
template <typename T, int BT, int RB, bool IM>
__device__ __forceinline__ void block_term(typename V2t<T>::type (&acc)[1 << RB], const typename V2t<T>::type *b,
                                           uint32_t cur, int j, uint32_t tile, uint32_t tid) {
    using V = typename V2t<T>::type;
    constexpr int R = 1 << RB;
    constexpr int TB = BT - RB;
    constexpr int SH = TB + (sizeof(T) == 4 ? 3 : 4);   // byte shift of the register index
    constexpr int RD = sizeof(T) == 4 ? 4 : 5;          // dwords per record
    const uint32_t w0 = __builtin_amdgcn_readlane(cur, RD * j);
    const uint32_t w1 = __builtin_amdgcn_readlane(cur, RD * j + 1);
    const uint32_t w2 = __builtin_amdgcn_readlane(cur, RD * j + 2);
    const uint32_t w3 = __builtin_amdgcn_readlane(cur, RD * j + 3);
    T c;
    if constexpr (sizeof(T) == 4) {
        c = __uint_as_float(w3);
    } else {
        const uint32_t w4 = __builtin_amdgcn_readlane(cur, RD * j + 4);
        c = __hiloint2double(static_cast<int>(w4), static_cast<int>(w3));
    }
    const uint32_t xt = w0 & 0xffffffu, xr = w0 >> 24;
    const uint32_t zt = w1 & 0xffffffu, sm = w1 >> 24;
    const uint32_t par = (__popc(tile & w2) + __popc(tid & zt)) & 1u;
    const T cl = flip_sign(c, par << 31);
    const uint32_t base = ((tid ^ xt) << (SH - TB)) | (xr << SH);
    const char *bb = reinterpret_cast<const char *>(b);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const V q = *reinterpret_cast<const V *>(bb + (base ^ (static_cast<uint32_t>(r) << SH)));
        // the register sign stays a scalar operand: one vector XOR per register (output
        // register 0 never changes sign: r & zr = 0)
        uint32_t sg = ((sm >> r) & 1u) << 31;
        asm("" : "+s"(sg));
        const T cr = r == 0 ? cl : flip_sign(cl, sg);
        if (IM) {
            acc[r].x -= cr * q.y;
            acc[r].y += cr * q.x;
        } else {
            acc[r].x += cr * q.x;
            acc[r].y += cr * q.y;
        }
    }
}

// A control-block term with xr = zr = 0 (the host puts these first in each run): output
// register r reads partner register r at a constant LDS offset from one address, with no
// register sign.
template <typename T, int BT, int RB, bool IM>
__device__ __forceinline__ void block_term_plain(typename V2t<T>::type (&acc)[1 << RB],
                                                 const typename V2t<T>::type *b, uint32_t cur, int j, uint32_t tile,
                                                 uint32_t tid) {
    using V = typename V2t<T>::type;
    constexpr int R = 1 << RB;
    constexpr int TB = BT - RB;
    constexpr int RD = sizeof(T) == 4 ? 4 : 5;          // dwords per record
    const uint32_t w0 = __builtin_amdgcn_readlane(cur, RD * j);
    const uint32_t w1 = __builtin_amdgcn_readlane(cur, RD * j + 1);
    const uint32_t w2 = __builtin_amdgcn_readlane(cur, RD * j + 2);
    const uint32_t w3 = __builtin_amdgcn_readlane(cur, RD * j + 3);
    T c;
    if constexpr (sizeof(T) == 4) {
        c = __uint_as_float(w3);
    } else {
        const uint32_t w4 = __builtin_amdgcn_readlane(cur, RD * j + 4);
        c = __hiloint2double(static_cast<int>(w4), static_cast<int>(w3));
    }
    const uint32_t par = (__popc(tile & w2) + __popc(tid & (w1 & 0xffffffu))) & 1u;
    const T cl = flip_sign(c, par << 31);
    const V *bs = b + (tid ^ (w0 & 0xffffffu));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const V q = bs[r << TB];
        if (IM) {
            acc[r].x -= cl * q.y;
            acc[r].y += cl * q.x;
        } else {
            acc[r].x += cl * q.x;
            acc[r].y += cl * q.y;
        }
    }
}

// one group's terms (real-phase terms [t0, tm), i-phase terms [tm, t1)) in either record form
template <typename T, int BT, int RB, int SR>
__device__ __forceinline__ void group_terms(typename V2t<T>::type (&acc)[1 << RB], const typename V2t<T>::type *b,
                                            const void *recs, const T *__restrict__ coef, int t0, int tm, int t1,
                                            uint32_t tile, uint32_t tid) {
    if constexpr (SR == 1) {
        const TermRec4 *r = static_cast<const TermRec4 *>(recs);
        apply_terms_static<T, BT, RB, false>(acc, b, r, coef, t0, tm, tile, tid);
        apply_terms_static<T, BT, RB, true>(acc, b, r, coef, tm, t1, tile, tid);
    } else {
        const TermRec<1 << RB> *r = static_cast<const TermRec<1 << RB> *>(recs);
        apply_terms<T, BT, RB, false>(acc, b, r, coef, t0, tm, tile, tid);
        apply_terms<T, BT, RB, true>(acc, b, r, coef, tm, t1, tile, tid);
    }
}

// s_waitcnt immediate (GFX9 encoding) that waits until at most `vm` vector-memory
// operations of this wave are outstanding; expcnt and lgkmcnt are left unconstrained
constexpr int waitcnt_vm(int vm) { return (vm & 15) | (7 << 4) | (15 << 8) | (((vm >> 4) & 3) << 14); }

#define SYK_LDS(p) ((__attribute__((address_space(3))) void *)(p))

// Fourth dword of a raw buffer descriptor on gfx9-family targets: 32-bit data format, no
// swizzle, no index stride.
constexpr uint32_t kBufferWord3 = 0x00020000u;

// Waves that issue the partner copies: the first four (measured on the benchmark block:
// 7.75 ms per apply with four copying waves against 8.42 with all sixteen, 8.43 with two
// and 7.93 with eight).
constexpr int copy_waves(int nt) { return nt / 64 < 4 ? nt / 64 : 4; }

// f(integral_constant<int, i>) for i = I .. N - 1 (compile-time piece index of a copy)
template <int I, int N, typename F>
__device__ __forceinline__ void static_for_j(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for_j<I + 1, N>(f);
    }
}

// direct-copy instructions per copying thread for one tile
template <typename T, int BT, int RB>
constexpr int copy_instrs() {
    return (1 << BT) * 2 * static_cast<int>(sizeof(T)) / (copy_waves(1 << (BT - RB)) * 64 * 16);
}

// Copy partner tile `src` (2^BT amplitudes) into LDS buffer `dst` with direct
// memory-to-LDS loads (buffer form) issued by the first copy_waves() waves: 16 bytes per
// lane, a wave writes 1 KiB contiguous per instruction, so the LDS holds the tile in index
// order.  No VGPRs receive data.  The buffer form, unlike the global form, lets the compiler
// count the term loop's LDS reads one by one (with a global-form copy in flight it waits for
// all eight reads of a term before the first FMA).
template <typename T, int BT, int RB>
__device__ __forceinline__ void dma_tile(const typename V2t<T>::type *src, typename V2t<T>::type *dst,
                                         uint32_t tid) {
    constexpr uint32_t CT = copy_waves(1 << (BT - RB)) * 64;   // copying threads
    constexpr int PER = copy_instrs<T, BT, RB>();
    static_assert(PER >= 1 && PER * CT * 16 == (1u << BT) * 2 * sizeof(T), "whole 1 KiB pieces per copying wave");
    char *l = reinterpret_cast<char *>(dst);
    if (tid < CT) {                                              // whole waves: a uniform branch
        // one descriptor spanning the tile; the piece offset goes in a scalar register and
        // only the lane's 16-byte slot in a VGPR
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<typename V2t<T>::type *>(src), 0, (1u << BT) * 2u * sizeof(T), kBufferWord3);
        // copying wave w moves the contiguous PER KiB from byte w * PER KiB; four 1 KiB pieces
        // share one LDS base (M0) and differ by the instruction offset, which the hardware adds
        // to the memory and the LDS address alike
        const uint32_t wbase = __builtin_amdgcn_readfirstlane((tid >> 6) * PER * 1024u);
        const uint32_t lane = tid & 63u;
        static_for_j<0, PER>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, SYK_LDS(l + wbase + (j / 4) * 4096), 16, lane * 16,
                                                     wbase + (j / 4) * 4096, (j % 4) * 1024, 0);
        });
    }
}

template <int K, typename V>
__device__ __forceinline__ V *pick(V *b0, V *b1, V *b2, V *b3) {
    if constexpr (K == 0) return b0;
    if constexpr (K == 1) return b1;
    if constexpr (K == 2) return b2;
    return b3;
}

// The output tiles of a workgroup: t0 ^ h[i], i < 2^W.
struct TileSet {
    uint32_t h[8];
};

// f(integral_constant<int, i>) for i = 0 .. n - 1, each with a compile-time index
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Partner tiles stream into NBUF LDS buffers by direct loads, NBUF - 1 of them in flight
// while the current one is consumed; the buffers are distinct LDS objects so that reads
// of one need not wait for copies into the others.  With NBUF = 1 the copy and the
// compute of a partner alternate inside the workgroup and OCC workgroups share a CU, so
// one computes while another waits for its tile.  A workgroup holds 2^W output tiles in
// registers; partner step k brings tile t0 ^ pi[k] and applies to output tile i the terms
// [ranges[3(k 2^W + i)], ...] of group pi[k] ^ h[i].  n_pi is a multiple of NBUF (the host
// pads with empty steps) and pi holds NBUF - 1 extra entries.  The second launch bound
// (waves per SIMD) keeps OCC workgroups resident.
template <typename T, int BT, int RB, int NBUF, int OCC, int SR, int W>
__global__ void __launch_bounds__(1 << (BT - RB), OCC * (1 << (BT - RB)) / 256) apply_h_tiled(
    const typename V2t<T>::type *__restrict__ x, typename V2t<T>::type *__restrict__ y, uint64_t ld,
    const uint32_t *__restrict__ tile_map, TileSet hs, const uint32_t *__restrict__ pi,
    const uint32_t *__restrict__ ranges, int n_pi, const void *__restrict__ recs, const T *__restrict__ coef,
    LanczosFuse<T> lf) {
    using V = typename V2t<T>::type;
    constexpr int NT = 1 << (BT - RB);
    constexpr int R = 1 << RB;
    constexpr int TPW = 1 << W;
    constexpr int TILE = 1 << BT;
    constexpr int PER = copy_instrs<T, BT, RB>();   // direct-copy instructions per copying thread
    static_assert(NBUF >= 1 && NBUF <= 4, "1 to 4 LDS buffers");
    static_assert(W >= 0 && W <= 3, "1 to 8 tiles per workgroup");
    __shared__ V b0[TILE];
    __shared__ V b1[NBUF > 1 ? TILE : 1];
    __shared__ V b2[NBUF > 2 ? TILE : 1];
    __shared__ V b3[NBUF > 3 ? TILE : 1];

    const uint32_t tid = threadIdx.x;
    const uint32_t t0 = tile_map[blockIdx.x];
    const uint64_t vo = static_cast<uint64_t>(blockIdx.y) * ld;
    const V *xv = x + vo;
    V *yv = y + vo;
    auto partner = [&](int k) __attribute__((always_inline)) { return xv + (static_cast<uint64_t>(t0 ^ pi[k]) << BT); };

    V acc[TPW][R];
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[i][r] = V{T(0), T(0)};   // fully unrolled: constant indices

    // the tile index must be a compile-time constant: acc[i] stays in registers
    auto terms_of = [&](const V *b, int k) __attribute__((always_inline)) {
        const uint32_t *rg = ranges + static_cast<size_t>(k) * TPW * 3;
        auto one = [&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            group_terms<T, BT, RB, SR>(acc[i], b, recs, coef, static_cast<int>(rg[3 * i]),
                                       static_cast<int>(rg[3 * i + 1]), static_cast<int>(rg[3 * i + 2]),
                                       t0 ^ hs.h[i], tid);
        };
        static_for<0, TPW>(one);
    };

    if constexpr (SR == 2) {
        // two buffers; the control block of step k + 1 is loaded during step k, just before
        // the copy of the partner of step k + 1, so the wait for that copy covers it too
        static_assert(NBUF == 2 && RB <= 3, "control blocks: 2 buffers, at most 8 registers per thread");
        const uint32_t *blocks = static_cast<const uint32_t *>(recs);
        const uint32_t lane = tid & 63u;
        dma_tile<T, BT, RB>(partner(0), b0, tid);
        uint32_t blk0 = blocks[lane], blk1 = 0;
        auto terms_blk = [&](const V *b, uint32_t cur) __attribute__((always_inline)) {
            const uint32_t cnt = __builtin_amdgcn_readlane(cur, 60);
            const uint32_t pln = __builtin_amdgcn_readlane(cur, 62);    // leading plain records per run
            int j = 0;
            static_for<0, TPW>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = decltype(ic)::value;
                const uint32_t tile = t0 ^ hs.h[i];
                const int nre = static_cast<int>((cnt >> (8 * i)) & 15u);
                const int nim = static_cast<int>((cnt >> (8 * i + 4)) & 15u);
                const int pre = static_cast<int>((pln >> (8 * i)) & 15u);
                const int pim = static_cast<int>((pln >> (8 * i + 4)) & 15u);
                // a tile without records in this step (common: about 2.8 records per step over
                // four tiles) costs one test instead of four
                if (((cnt >> (8 * i)) & 0xffu) == 0u) return;
                for (const int e = j + pre; j < e; ++j) block_term_plain<T, BT, RB, false>(acc[i], b, cur, j, tile, tid);
                for (const int e = j + nre - pre; j < e; ++j) block_term<T, BT, RB, false>(acc[i], b, cur, j, tile, tid);
                for (const int e = j + pim; j < e; ++j) block_term_plain<T, BT, RB, true>(acc[i], b, cur, j, tile, tid);
                for (const int e = j + nim - pim; j < e; ++j) block_term<T, BT, RB, true>(acc[i], b, cur, j, tile, tid);
            });
        };
        for (int k0 = 0; k0 < n_pi; k0 += 2) {
            auto step = [&](auto kc) __attribute__((always_inline)) {
                constexpr int K = decltype(kc)::value;
                const int k = k0 + K;
                __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                const uint32_t cur = K == 0 ? blk0 : blk1;
                const uint32_t nxt = blocks[static_cast<size_t>(k + 1) * 64 + lane];
                if constexpr (K == 0)
                    blk1 = nxt;
                else
                    blk0 = nxt;
                const uint32_t pn = __builtin_amdgcn_readlane(cur, 61);
                dma_tile<T, BT, RB>(xv + (static_cast<uint64_t>(t0 ^ pn) << BT), K == 0 ? b1 : b0, tid);
                terms_blk(K == 0 ? b0 : b1, cur);
            };
            step(std::integral_constant<int, 0>{});
            step(std::integral_constant<int, 1>{});
        }
    } else if constexpr (NBUF == 1) {
        for (int k = 0; k < n_pi; ++k) {
            // the previous step's reads of b0 ended at the barrier closing it
            dma_tile<T, BT, RB>(partner(k), b0, tid);
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            terms_of(b0, k);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        }
    } else {
        dma_tile<T, BT, RB>(partner(0), b0, tid);
        if constexpr (NBUF > 2) dma_tile<T, BT, RB>(partner(1), b1, tid);
        if constexpr (NBUF > 3) dma_tile<T, BT, RB>(partner(2), b2, tid);
        for (int k0 = 0; k0 < n_pi; k0 += NBUF) {
            auto step = [&](auto kc) __attribute__((always_inline)) {
                constexpr int K = decltype(kc)::value;
                const int k = k0 + K;
                // this step's copy was issued NBUF - 1 steps ago; NBUF - 2 copies are newer.
                // A bare s_barrier (no fence): each wave has waited for its own pieces of the
                // tile, LDS is coherent within the CU, and the barrier also guarantees that
                // every wave is done reading the buffer the next copy overwrites.
                __builtin_amdgcn_s_waitcnt(waitcnt_vm(PER * (NBUF - 2)));
                asm volatile("" ::: "memory");   // no LDS access or copy moves across the barrier
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                dma_tile<T, BT, RB>(partner(k + NBUF - 1), pick<(K + NBUF - 1) % NBUF>(b0, b1, b2, b3), tid);
                terms_of(pick<K>(b0, b1, b2, b3), k);
            };
            step(std::integral_constant<int, 0>{});
            step(std::integral_constant<int, 1>{});
            if constexpr (NBUF > 2) step(std::integral_constant<int, 2>{});
            if constexpr (NBUF > 3) step(std::integral_constant<int, 3>{});
        }
    }
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));      // no copy may still target LDS at exit
    if (lf.partials == nullptr) {
        // outputs are not re-read by this kernel: stream them past the caches
        auto store = [&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            V *dst = yv + (static_cast<uint64_t>(t0 ^ hs.h[i]) << BT);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                __builtin_nontemporal_store(acc[i][r].x, &dst[r * NT + tid].x);
                __builtin_nontemporal_store(acc[i][r].y, &dst[r * NT + tid].y);
            }
        };
        static_for<0, TPW>(store);
        return;
    }
    // Lanczos epilogue: w = H v_j - beta_{j-1} v_{j-1}, and this workgroup's shares of
    // <v_j, w> (re, im), ||w||^2 and ||v_j||^2 in double
    // scales of the unnormalised basis (see LanczosFuse)
    // (a zero vector after an exact breakdown stays zero)
    const double nj = lf.j >= 1 ? sqrt(lf.beta2[lf.j]) : 1.0;
    const double njm = lf.j >= 2 ? sqrt(lf.beta2[lf.j - 1]) : 1.0;
    const T sc = nj > 1e-300 ? static_cast<T>(1.0 / nj) : T(0);
    const T bp = (lf.vprev && njm > 1e-300) ? static_cast<T>(nj / njm) : T(0);
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    auto epi_tile = [&](auto has_prev, auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        {
            const uint64_t base = static_cast<uint64_t>(t0 ^ hs.h[i]) << BT;
            V *dst = yv + base;
            const V *vp = reinterpret_cast<const V *>(lf.vprev) + base;
            const V *vc = reinterpret_cast<const V *>(lf.vcur) + base;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int m = r * NT + tid;
                V w = V{sc * acc[i][r].x, sc * acc[i][r].y};
                if constexpr (decltype(has_prev)::value) {
                    const V p = vp[m];
                    w.x -= bp * p.x;
                    w.y -= bp * p.y;
                }
                const V c = V{sc * vc[m].x, sc * vc[m].y};
                dst[m] = w;
                sum[0] += static_cast<double>(c.x) * w.x + static_cast<double>(c.y) * w.y;
                sum[1] += static_cast<double>(c.x) * w.y - static_cast<double>(c.y) * w.x;
                sum[2] += static_cast<double>(w.x) * w.x + static_cast<double>(w.y) * w.y;
                sum[3] += static_cast<double>(c.x) * c.x + static_cast<double>(c.y) * c.y;
                // bound the loads in flight: with several workgroups per CU the register
                // budget is 64 VGPRs
                if (r % 2 == 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto epilogue = [&](auto has_prev) __attribute__((always_inline)) {
        static_for<0, TPW>([&](auto ic) __attribute__((always_inline)) { epi_tile(has_prev, ic); });
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

template <typename T, int BT, int RB, int NBUF, int OCC, int SR, int W>
static void launch_variant(const ApplyPlan &pl, const T *x, T *y, int nvec, uint64_t ld, const LanczosFuse<T> &lf,
                           hipStream_t s) {
    using V = typename V2t<T>::type;
    const T *coef = nullptr;
    if constexpr (sizeof(T) == 4)
        coef = pl.c32;
    else
        coef = pl.c64;
    if (pl.w != W) fail(SYK_EDEVICE, "plan and kernel disagree on tiles per workgroup");
    TileSet hs{};
    for (int i = 0; i < 8; ++i) hs.h[i] = pl.hvec[i];
    dim3 grid(pl.n_wg, nvec);
    hipLaunchKernelGGL((apply_h_tiled<T, BT, RB, NBUF, OCC, SR, W>), grid, dim3(1 << (BT - RB)), 0, s,
                       reinterpret_cast<const V *>(x), reinterpret_cast<V *>(y), ld, pl.tile_map, hs, pl.pi,
                       pl.ranges, pl.n_pi, static_cast<const void *>(pl.meta), coef, lf);
    SYK_HIP(hipGetLastError());
}

template <typename T>
void launch_apply_tiled(const ApplyPlan &pl, const T *x, T *y, int nvec, uint64_t ld, hipStream_t s,
                        const LanczosFuse<T> *lf) {
    const TiledVariant &v = tiled_variants<T>()[pl.variant];
    const LanczosFuse<T> none{};
    if (lf && nvec != 1) fail(SYK_EDEVICE, "the fused Lanczos epilogue takes one vector");
#define SYK_TV(BT, RB, NB, OC, SR, W)                                                       \
    if (v.bt == BT && v.rb == RB && v.nbuf == NB && v.occ == OC && v.sr == SR && v.w == W) {    \
        launch_variant<T, BT, RB, NB, OC, SR, W>(pl, x, y, nvec, ld, lf ? *lf : none, s);       \
        return;                                                                                 \
    }
    if constexpr (sizeof(T) == 4) {
        SYK_TV(13, 3, 2, 1, 0, 0)
        SYK_TV(13, 3, 1, 2, 0, 0)
        SYK_TV(12, 3, 2, 2, 0, 0)
        SYK_TV(12, 2, 4, 1, 0, 0)
        SYK_TV(13, 3, 2, 1, 1, 0)
        SYK_TV(13, 3, 2, 1, 0, 1)
        SYK_TV(13, 3, 2, 1, 0, 2)
        SYK_TV(12, 3, 2, 2, 0, 1)
        SYK_TV(13, 3, 2, 1, 2, 0)
        SYK_TV(13, 3, 2, 1, 2, 1)
        SYK_TV(13, 3, 2, 1, 2, 2)
        SYK_TV(11, 2, 2, 2, 2, 0)
        SYK_TV(10, 2, 2, 4, 2, 0)
        SYK_TV(11, 2, 2, 2, 2, 1)
        SYK_TV(12, 3, 2, 2, 2, 2)
        SYK_TV(12, 2, 2, 2, 2, 2)
        SYK_TV(12, 3, 2, 2, 2, 1)
    } else {
        SYK_TV(12, 2, 2, 1, 0, 0)
        SYK_TV(12, 2, 1, 2, 0, 0)
        SYK_TV(11, 2, 2, 2, 0, 0)
        SYK_TV(11, 1, 4, 1, 0, 0)
        SYK_TV(12, 2, 2, 1, 1, 0)
        SYK_TV(12, 2, 2, 1, 0, 1)
        SYK_TV(12, 2, 2, 1, 0, 2)
        SYK_TV(11, 2, 2, 2, 0, 1)
        SYK_TV(12, 2, 2, 1, 2, 0)
        SYK_TV(12, 2, 2, 1, 2, 1)
        SYK_TV(12, 2, 2, 1, 2, 2)
        SYK_TV(11, 2, 2, 2, 2, 0)
        SYK_TV(10, 2, 2, 4, 2, 0)
        SYK_TV(11, 2, 2, 2, 2, 1)
        SYK_TV(11, 2, 2, 2, 2, 2)
        SYK_TV(11, 1, 2, 2, 2, 2)
        SYK_TV(10, 1, 2, 4, 2, 2)
    }
#undef SYK_TV
    fail(SYK_EDEVICE, "unknown tiled apply_H variant");
}

template void launch_apply_tiled<float>(const ApplyPlan &, const float *, float *, int, uint64_t, hipStream_t,
                                        const LanczosFuse<float> *);
template void launch_apply_tiled<double>(const ApplyPlan &, const double *, double *, int, uint64_t, hipStream_t,
                                         const LanczosFuse<double> *);

}  // namespace syk
