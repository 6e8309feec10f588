// Launch planning of the tiled apply_H kernel (the schedule autotuner).
//
// Inputs: the terms of one parity block.  Decisions:
//  * layout rotation s: amplitude index bit b holds qubit (b + s) mod L, so the 2^BT
//    amplitudes of a tile are the qubits [s, s + BT) (mod L).  Only the vector layout
//    changes: masks are rotated the same way, so XOR/AND/parity arithmetic is unchanged.
//  * subspaces Wx (r dims, r = 5 + log2 of the workgroups resident per CU) and Wg (r + 3
//    dims) of the tile-index space: the 2^r tiles resident on one XCD at the same time
//    form a coset of Wx, those resident on the whole GPU a coset of Wg (workgroups are
//    dispatched round-robin over the 8 XCDs).  Partner tiles of two groups g, g' coincide
//    across resident workgroups iff g ^ g' lies in the subspace, so the subspaces are
//    grown greedily from the most frequent differences of partner offsets, and groups are
//    visited class by class.
//  * cost model: L2 requests scale with the number of groups D, L2 misses with the number
//    of classes modulo Wx; the rotation minimising D + 2 * classes_x + classes_g / 2 is
//    taken.
#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>
#include <unordered_map>

#include "apply_plan.hpp"

namespace syk {

uint32_t rotr_bits(uint32_t v, int s, int L) {
    if (L <= 0) return v;
    s %= L;
    const uint32_t mask = (L == 32) ? 0xFFFFFFFFu : ((1u << L) - 1u);
    v &= mask;
    if (s == 0) return v;
    return ((v >> s) | (v << (L - s))) & mask;
}

uint32_t rotl_bits(uint32_t v, int s, int L) {
    if (L <= 0) return v;
    s %= L;
    return rotr_bits(v, (L - s) % L, L);
}

namespace {

// subspace of GF(2)^n held as a reduced echelon basis: canonical coset representatives
struct Echelon {
    std::vector<uint32_t> rows;     // distinct leading bits, fully reduced, descending
    uint32_t reduce(uint32_t v) const {
        for (uint32_t r : rows) {
            const uint32_t lead = 1u << (31 - __builtin_clz(r));
            if (v & lead) v ^= r;
        }
        return v;
    }
    bool add(uint32_t v) {
        v = reduce(v);
        if (!v) return false;
        const uint32_t lead = 1u << (31 - __builtin_clz(v));
        for (auto &r : rows)
            if (r & lead) r ^= v;
        rows.push_back(v);
        std::sort(rows.begin(), rows.end(), [](uint32_t a, uint32_t b) { return a > b; });
        return true;
    }
};

int count_classes(const std::vector<uint32_t> &G, const Echelon &E) {
    std::vector<uint32_t> reps;
    reps.reserve(G.size());
    for (uint32_t g : G) reps.push_back(E.reduce(g));
    std::sort(reps.begin(), reps.end());
    return static_cast<int>(std::unique(reps.begin(), reps.end()) - reps.begin());
}

// grow `E` by up to `dims` vectors, each the most class-reducing frequent difference
std::vector<uint32_t> grow(const std::vector<uint32_t> &G, Echelon &E, int dims, int max_dim) {
    std::vector<uint32_t> picked;
    for (int d = 0; d < dims && static_cast<int>(E.rows.size()) < max_dim; ++d) {
        std::unordered_map<uint32_t, int> freq;
        for (size_t a = 0; a < G.size(); ++a)
            for (size_t b = a + 1; b < G.size(); ++b) {
                const uint32_t v = E.reduce(G[a] ^ G[b]);
                if (v) ++freq[v];
            }
        std::vector<std::pair<int, uint32_t>> cand;
        for (const auto &kv : freq) cand.push_back({-kv.second, kv.first});
        std::sort(cand.begin(), cand.end());
        if (cand.size() > 40) cand.resize(40);
        uint32_t best = 0;
        int best_c = 1 << 30;
        for (const auto &c : cand) {
            Echelon t = E;
            t.add(c.second);
            const int n = count_classes(G, t);
            if (n < best_c) {
                best_c = n;
                best = c.second;
            }
        }
        if (!best) {      // no useful difference: any unit vector outside the span
            for (int bit = 0; bit < max_dim; ++bit)
                if (E.reduce(1u << bit)) {
                    best = 1u << bit;
                    break;
                }
        }
        if (!best || !E.add(best)) break;
        picked.push_back(best);
    }
    return picked;
}

struct Candidate {
    int s = 0;
    std::vector<uint32_t> G;
    std::vector<uint32_t> wx, wg;     // basis vectors picked (wg extends wx)
    int D = 0, cx = 0, cg = 0;
    double cost = 0;
};

Candidate evaluate(const std::vector<BlockTerm> &terms, int L, int bt, int s, int res_bits) {
    Candidate c;
    c.s = s;
    const int tb = L - bt;
    for (const auto &t : terms) c.G.push_back(rotr_bits(t.x, s, L) >> bt);
    std::sort(c.G.begin(), c.G.end());
    c.G.erase(std::unique(c.G.begin(), c.G.end()), c.G.end());
    c.D = static_cast<int>(c.G.size());
    Echelon E;
    c.wx = grow(c.G, E, res_bits, tb);
    c.cx = count_classes(c.G, E);
    c.wg = grow(c.G, E, 3, tb);
    c.cg = count_classes(c.G, E);
    c.cost = c.D + 2.0 * c.cx + 0.5 * c.cg;
    return c;
}

}  // namespace

int choose_rotation(const std::vector<BlockTerm> &terms, int L, int bt, int res_bits) {
    if (L <= bt) return 0;
    // pre-select by the group count alone, then score the best few in full
    std::vector<std::pair<int, int>> byD;
    for (int s = 0; s < L; ++s) {
        std::vector<uint32_t> G;
        for (const auto &t : terms) G.push_back(rotr_bits(t.x, s, L) >> bt);
        std::sort(G.begin(), G.end());
        byD.push_back({static_cast<int>(std::unique(G.begin(), G.end()) - G.begin()), s});
    }
    std::sort(byD.begin(), byD.end());
    int best_s = 0;
    double best = 1e300;
    for (size_t i = 0; i < byD.size() && i < 4; ++i) {
        const Candidate c = evaluate(terms, L, bt, byD[i].second, res_bits);
        if (c.cost < best) {
            best = c.cost;
            best_s = c.s;
        }
    }
    return best_s;
}

HostPlan build_host_plan(const std::vector<BlockTerm> &terms, int L, int bt, int rb, int mult, int extra, int s,
                         uint32_t elem_bytes, int res_bits) {
    HostPlan hp;
    hp.rot = s;
    const int tbits = L - bt;
    hp.n_tiles = 1u << tbits;
    hp.res_bits = res_bits;
    const Candidate c = evaluate(terms, L, bt, s, res_bits);
    hp.D = c.D;
    hp.classes_xcd = c.cx;
    hp.classes_gpu = c.cg;

    // basis of the tile-index space: Wg extension (blockIdx bits [0,3): the XCD), Wx
    // (bits [3, 3 + r): XCD-local), then unit vectors completing it; blockIdx bit i selects
    // basis vector i, so the map is a bijection
    std::vector<uint32_t> basis;
    {
        Echelon E;
        std::vector<uint32_t> order;
        for (uint32_t v : c.wg) order.push_back(v);
        for (uint32_t v : c.wx) order.push_back(v);
        for (int bit = 0; bit < tbits; ++bit) order.push_back(1u << bit);
        for (uint32_t v : order)
            if (E.add(v)) basis.push_back(v);
    }
    if (static_cast<int>(basis.size()) != tbits) fail(SYK_EDEVICE, "tile basis construction failed");
    hp.tile_map.resize(hp.n_tiles);
    for (uint32_t b = 0; b < hp.n_tiles; ++b) {
        uint32_t t = 0;
        for (int i = 0; i < tbits; ++i)
            if ((b >> i) & 1u) t ^= basis[i];
        hp.tile_map[b] = t;
    }

    // group order: by class modulo Wg, then modulo Wx, then offset
    Echelon E5, E8;
    for (uint32_t v : c.wx) {
        E5.add(v);
        E8.add(v);
    }
    for (uint32_t v : c.wg) E8.add(v);
    const uint32_t low = (1u << bt) - 1u;
    const int tb = bt - rb;
    const uint32_t tmask = (1u << tb) - 1u;
    const uint32_t rmask = (1u << rb) - 1u;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::vector<int>> by;
    for (int a = 0; a < static_cast<int>(terms.size()); ++a) {
        const uint32_t g = rotr_bits(terms[a].x, s, L) >> bt;
        by[std::make_tuple(E8.reduce(g), E5.reduce(g), g)].push_back(a);
    }
    hp.grp_first.push_back(0);
    uint32_t count = 0;
    for (const auto &kv : by) {
        hp.grp_g.push_back(std::get<2>(kv.first));
        for (int pass = 0; pass < 2; ++pass) {          // real-phase terms, then i-phase terms
            if (pass == 1) hp.grp_mid.push_back(count);
            for (int a : kv.second) {
                const BlockTerm &t = terms[a];
                if (t.imag != (pass == 1)) continue;
                const uint32_t x = rotr_bits(t.x, s, L), z = rotr_bits(t.z, s, L);
                const uint32_t xl = x & low;
                const uint32_t xr = (xl >> tb) & rmask;
                const uint32_t zr = (z >> tb) & rmask;
                hp.meta.push_back(xl & tmask);
                hp.meta.push_back(z & tmask);
                hp.meta.push_back(z >> bt);
                hp.meta.push_back(0u);
                for (uint32_t r = 0; r <= rmask; ++r)          // byte offset of partner register r ^ xr
                    hp.meta.push_back(((r ^ xr) << tb) * elem_bytes);
                for (uint32_t r = 0; r <= rmask; ++r)          // sign of output register r
                    hp.meta.push_back((__builtin_popcount(r & zr) & 1) ? 0x80000000u : 0u);
                hp.c.push_back(t.c);
                ++count;
            }
        }
        hp.grp_first.push_back(count);
    }
    const uint32_t last = hp.grp_g.empty() ? 0u : hp.grp_g.back();
    while (hp.grp_g.empty() || hp.grp_g.size() % static_cast<size_t>(mult) != 0) {   // empty groups
        hp.grp_g.push_back(last);
        hp.grp_mid.push_back(count);
        hp.grp_first.push_back(count);
    }
    hp.n_groups = static_cast<int>(hp.grp_g.size());
    for (int k = 0; k < extra; ++k) hp.grp_g.push_back(last);   // targets of the last prefetches
    hp.meta.resize(hp.meta.size() + 4 + 2 * (rmask + 1), 0u);   // one padding record (term prefetch)
    hp.c.push_back(0.0);
    return hp;
}

template <typename U>
static U *upload(const std::vector<U> &v) {
    U *d = nullptr;
    const size_t n = std::max<size_t>(v.size(), 1);
    SYK_HIP(hipMalloc(reinterpret_cast<void **>(&d), n * sizeof(U)));
    if (!v.empty()) SYK_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice));
    return d;
}

void free_plan(ApplyPlan &p) {
    hipFree(p.grp_g);
    hipFree(p.grp_first);
    hipFree(p.grp_mid);
    hipFree(p.meta);
    hipFree(p.tile_map);
    hipFree(p.c32);
    hipFree(p.c64);
    p = ApplyPlan{};
}

void upload_plan(const HostPlan &hp, int bt, int rb, ApplyPlan &out) {
    ApplyPlan p;
    p.bt = bt;
    p.rb = rb;
    p.rot = hp.rot;
    p.n_tiles = hp.n_tiles;
    p.n_groups = hp.n_groups;
    try {
        p.grp_g = upload(hp.grp_g);
        p.grp_first = upload(hp.grp_first);
        p.grp_mid = upload(hp.grp_mid);
        p.meta = upload(hp.meta);
        p.tile_map = upload(hp.tile_map);
        std::vector<float> c32(hp.c.begin(), hp.c.end());
        p.c32 = upload(c32);
        p.c64 = upload(hp.c);
    } catch (...) {
        free_plan(p);
        throw;
    }
    out = p;
}

}  // namespace syk
