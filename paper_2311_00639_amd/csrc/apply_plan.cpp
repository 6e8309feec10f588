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
#include <array>
#include <cstring>
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
    std::vector<uint32_t> G;          // partner offsets of the term groups
    std::vector<uint32_t> H;          // basis of the tiles a workgroup holds (relative offsets)
    std::vector<uint32_t> Pi;         // partner offsets of a workgroup: G + span(H)
    std::vector<uint32_t> wx, wg;     // resident subspaces (modulo span(H)); wg extends wx
    int D = 0, cx = 0, cg = 0;
    double cost = 0;
};

std::vector<uint32_t> span_of(const std::vector<uint32_t> &basis) {
    std::vector<uint32_t> sp{0u};
    for (uint32_t v : basis) {
        const size_t n = sp.size();
        for (size_t i = 0; i < n; ++i) sp.push_back(sp[i] ^ v);
    }
    return sp;
}

std::vector<uint32_t> minkowski(const std::vector<uint32_t> &G, const std::vector<uint32_t> &sp) {
    std::vector<uint32_t> out;
    out.reserve(G.size() * sp.size());
    for (uint32_t g : G)
        for (uint32_t h : sp) out.push_back(g ^ h);
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

// w vectors chosen greedily among the most frequent differences of G so that G + span(H)
// (the partner tiles of a workgroup holding the tiles t0 + span(H)) stays small
std::vector<uint32_t> choose_h(const std::vector<uint32_t> &G, int w, int tb) {
    std::vector<uint32_t> H;
    if (w <= 0) return H;
    std::unordered_map<uint32_t, int> freq;
    for (size_t a = 0; a < G.size(); ++a)
        for (size_t b = a + 1; b < G.size(); ++b) ++freq[G[a] ^ G[b]];
    std::vector<std::pair<int, uint32_t>> cand;
    for (const auto &kv : freq) cand.push_back({-kv.second, kv.first});
    std::sort(cand.begin(), cand.end());
    if (cand.size() > 60) cand.resize(60);
    for (int d = 0; d < w; ++d) {
        Echelon E;
        for (uint32_t v : H) E.add(v);
        uint32_t best = 0;
        size_t best_n = ~static_cast<size_t>(0);
        for (const auto &c : cand) {
            if (!E.reduce(c.second)) continue;
            std::vector<uint32_t> t = H;
            t.push_back(c.second);
            const size_t n = minkowski(G, span_of(t)).size();
            if (n < best_n) {
                best_n = n;
                best = c.second;
            }
        }
        if (!best) {      // no useful difference (e.g. a single group): any independent vector
            for (int bit = 0; bit < tb && !best; ++bit)
                if (E.reduce(1u << bit)) best = 1u << bit;
        }
        if (!best) break;
        H.push_back(best);
    }
    return H;
}

Candidate evaluate(const std::vector<BlockTerm> &terms, int L, int bt, int s, int res_bits, int w) {
    Candidate c;
    c.s = s;
    const int tb = L - bt;
    for (const auto &t : terms) c.G.push_back(rotr_bits(t.x, s, L) >> bt);
    std::sort(c.G.begin(), c.G.end());
    c.G.erase(std::unique(c.G.begin(), c.G.end()), c.G.end());
    c.D = static_cast<int>(c.G.size());
    c.H = choose_h(c.G, std::min(w, tb), tb);
    c.Pi = minkowski(c.G, span_of(c.H));
    Echelon E;
    for (uint32_t v : c.H) E.add(v);
    c.wx = grow(c.Pi, E, res_bits, tb);
    c.cx = count_classes(c.Pi, E);
    c.wg = grow(c.Pi, E, 3, tb);
    c.cg = count_classes(c.Pi, E);
    c.cost = static_cast<double>(c.Pi.size()) / (1 << c.H.size()) + 2.0 * c.cx + 0.5 * c.cg;
    return c;
}

}  // namespace

int choose_rotation(const std::vector<BlockTerm> &terms, int L, int bt, int res_bits, int w) {
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
        const Candidate c = evaluate(terms, L, bt, byD[i].second, res_bits, w);
        if (c.cost < best) {
            best = c.cost;
            best_s = c.s;
        }
    }
    return best_s;
}

HostPlan build_host_plan(const std::vector<BlockTerm> &terms, int L, int bt, int rb, int mult, int extra, int s,
                         uint32_t elem_bytes, int res_bits, int sr, int w) {
    HostPlan hp;
    hp.rot = s;
    const int tbits = L - bt;
    hp.n_tiles = 1u << tbits;
    const Candidate c = evaluate(terms, L, bt, s, res_bits, w);
    hp.w = static_cast<int>(c.H.size());
    if (hp.w != w) fail(SYK_EDEVICE, "block too small for the tiles per workgroup of this variant");
    hp.n_wg = hp.n_tiles >> hp.w;
    hp.res_bits = res_bits + hp.w;
    hp.D = c.D;
    hp.n_partners = static_cast<int>(c.Pi.size());
    hp.classes_xcd = c.cx;
    hp.classes_gpu = c.cg;
    hp.hvec = span_of(c.H);

    // workgroup index -> first tile t0: blockIdx bits [0,3) select the Wg extension (the
    // XCD), bits [3, 3 + r) Wx (XCD-local), then vectors completing a basis of the tile
    // space modulo span(H); the tiles t0 + span(H) of all workgroups cover it once
    std::vector<uint32_t> basis;
    {
        Echelon E;
        for (uint32_t v : c.H) E.add(v);
        std::vector<uint32_t> order;
        for (uint32_t v : c.wg) order.push_back(v);
        for (uint32_t v : c.wx) order.push_back(v);
        for (int bit = 0; bit < tbits; ++bit) order.push_back(1u << bit);
        for (uint32_t v : order)
            if (E.add(v)) basis.push_back(v);
    }
    if (static_cast<int>(basis.size()) != tbits - hp.w) fail(SYK_EDEVICE, "tile basis construction failed");
    hp.tile_map.resize(hp.n_wg);
    for (uint32_t b = 0; b < hp.n_wg; ++b) {
        uint32_t t = 0;
        for (int i = 0; i < tbits - hp.w; ++i)
            if ((b >> i) & 1u) t ^= basis[i];
        hp.tile_map[b] = t;
    }

    // term records, grouped by partner offset g (real-phase terms, then i-phase terms)
    const uint32_t low = (1u << bt) - 1u;
    const int tb = bt - rb;
    const uint32_t tmask = (1u << tb) - 1u;
    const uint32_t rmask = (1u << rb) - 1u;
    std::map<uint32_t, std::vector<int>> byg;   // terms by group, in term order
    for (int a = 0; a < static_cast<int>(terms.size()); ++a) byg[rotr_bits(terms[a].x, s, L) >> bt].push_back(a);
    std::unordered_map<uint32_t, std::array<uint32_t, 3>> range;   // g -> (first, mid, end)
    std::vector<std::array<uint32_t, 5>> compact;                   // sr = 2: per-term block record
    std::vector<char> plain;                                        // sr = 2: record has xr = zr = 0
    const uint32_t rec_dw = block_record_dwords(elem_bytes), rec_max = block_records(elem_bytes);
    // sr = 2: within each (group, phase) run the terms that touch no register bit (xr = zr = 0:
    // partner register r for output register r, no register sign) come first
    auto is_plain = [&](int a) {
        const uint32_t x = rotr_bits(terms[a].x, s, L), z = rotr_bits(terms[a].z, s, L);
        return (((x & low) >> tb) & rmask) == 0 && ((z >> tb) & rmask) == 0;
    };
    uint32_t count = 0;
    for (auto &kv : byg) {
        if (sr == 2)
            std::stable_sort(kv.second.begin(), kv.second.end(),
                             [&](int a, int b) { return is_plain(a) && !is_plain(b); });
        std::array<uint32_t, 3> r{count, 0u, 0u};
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) r[1] = count;
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
                if (sr == 2) {
                    // (thread bits of x | xr << 24, thread bits of z | register sign mask << 24,
                    //  z >> bt, coefficient as float or as the two dwords of a double): bit q of the
                    //  sign mask is the parity of q & zr
                    uint32_t smask = 0;
                    for (uint32_t q = 0; q <= rmask; ++q) smask |= (__builtin_popcount(q & zr) & 1u) << q;
                    std::array<uint32_t, 5> rec{(xl & tmask) | (xr << 24), (z & tmask) | (smask << 24), z >> bt, 0u, 0u};
                    if (elem_bytes == 8) {
                        const float cf = static_cast<float>(t.c);
                        std::memcpy(&rec[3], &cf, 4);
                    } else {
                        std::memcpy(&rec[3], &t.c, 8);
                    }
                    compact.push_back(rec);
                    plain.push_back(xr == 0 && zr == 0);
                    hp.meta.resize(hp.meta.size() - 3);
                } else if (sr) {
                    hp.meta.push_back((xr << rb) | zr);        // code of the compiled register path
                } else {
                    hp.meta.push_back(0u);
                    for (uint32_t q = 0; q <= rmask; ++q)      // byte offset of partner register q ^ xr
                        hp.meta.push_back(((q ^ xr) << tb) * elem_bytes);
                    for (uint32_t q = 0; q <= rmask; ++q)      // sign of output register q
                        hp.meta.push_back((__builtin_popcount(q & zr) & 1) ? 0x80000000u : 0u);
                }
                hp.c.push_back(t.c);
                ++count;
            }
        }
        r[2] = count;
        range[kv.first] = r;
    }
    if (sr != 2) hp.meta.resize(hp.meta.size() + (sr ? 4 : 4 + 2 * (rmask + 1)), 0u);   // padding record (prefetch)
    hp.c.push_back(0.0);

    // partner schedule: class by class modulo Wg, then Wx (both with span(H)), then offset
    Echelon E5, E8;
    for (uint32_t v : c.H) {
        E5.add(v);
        E8.add(v);
    }
    for (uint32_t v : c.wx) {
        E5.add(v);
        E8.add(v);
    }
    for (uint32_t v : c.wg) E8.add(v);
    std::vector<std::tuple<uint32_t, uint32_t, uint32_t>> order;
    for (uint32_t p : c.Pi) order.push_back(std::make_tuple(E8.reduce(p), E5.reduce(p), p));
    std::sort(order.begin(), order.end());
    const size_t tpw = hp.hvec.size();
    for (const auto &o : order) {
        const uint32_t p = std::get<2>(o);
        std::vector<std::array<uint32_t, 3>> rs(tpw);
        uint32_t total = 0;
        for (size_t i = 0; i < tpw; ++i) {
            auto it = range.find(p ^ hp.hvec[i]);
            rs[i] = it == range.end() ? std::array<uint32_t, 3>{0u, 0u, 0u} : it->second;
            total += rs[i][2] - rs[i][0];
        }
        if (sr != 2 || total <= rec_max) {
            hp.pi.push_back(p);
            for (size_t i = 0; i < tpw; ++i) hp.ranges.insert(hp.ranges.end(), rs[i].begin(), rs[i].end());
            continue;
        }
        // control blocks hold at most rec_max records: split the step, repeating the
        // partner, each part taking the next records in (tile, real, imaginary) order
        std::vector<std::pair<size_t, uint32_t>> flat;
        for (size_t q = 0; q < tpw; ++q)
            for (uint32_t t = rs[q][0]; t < rs[q][2]; ++t) flat.emplace_back(q, t);
        for (size_t c0 = 0; c0 < flat.size(); c0 += rec_max) {
            const size_t c1 = std::min<size_t>(flat.size(), c0 + rec_max);
            hp.pi.push_back(p);
            for (size_t q = 0; q < tpw; ++q) {
                uint32_t lo = 0, hi = 0;
                bool any = false;
                for (size_t e = c0; e < c1; ++e)
                    if (flat[e].first == q) {
                        if (!any) lo = flat[e].second;
                        hi = flat[e].second + 1;
                        any = true;
                    }
                hp.ranges.insert(hp.ranges.end(), {lo, any ? std::min(std::max(rs[q][1], lo), hi) : 0u, hi});
            }
        }
    }
    const uint32_t last = hp.pi.empty() ? 0u : hp.pi.back();
    while (hp.pi.empty() || hp.pi.size() % static_cast<size_t>(mult) != 0) {   // empty partner steps
        hp.pi.push_back(last);
        hp.ranges.insert(hp.ranges.end(), 3 * tpw, 0u);
    }
    hp.n_pi = static_cast<int>(hp.pi.size());
    for (int k = 0; k < extra; ++k) hp.pi.push_back(last);                      // targets of the last prefetches
    if (sr == 2) {
        // one 64-dword control block per partner step (and one more for the last prefetch):
        // lanes rec_dw j .. rec_dw (j + 1) - 1 record j, lane 60 the record counts (tile i: real in bits 8i..8i+3,
        // imaginary in 8i+4..8i+7), lane 62 how many of them lead their run with xr = zr = 0 (same
        // layout), lane 61 the partner offset copied during that step
        hp.meta.assign(static_cast<size_t>(hp.n_pi + 1) * 64, 0u);
        for (int st = 0; st <= hp.n_pi; ++st) {
            uint32_t *blk = &hp.meta[static_cast<size_t>(st) * 64];
            blk[61] = hp.pi[std::min<size_t>(st + extra, hp.pi.size() - 1)];
            if (st == hp.n_pi) continue;
            uint32_t j = 0, counts = 0, plain_counts = 0;
            for (size_t i = 0; i < tpw; ++i) {
                const uint32_t *r = &hp.ranges[(static_cast<size_t>(st) * tpw + i) * 3];
                if (r[1] - r[0] > 15 || r[2] - r[1] > 15) fail(SYK_EDEVICE, "control block count overflow");
                counts |= ((r[1] - r[0]) << (8 * i)) | ((r[2] - r[1]) << (8 * i + 4));
                uint32_t pre = 0, pim = 0;      // leading plain records of each phase run
                while (r[0] + pre < r[1] && plain[r[0] + pre]) ++pre;
                while (r[1] + pim < r[2] && plain[r[1] + pim]) ++pim;
                plain_counts |= (pre << (8 * i)) | (pim << (8 * i + 4));
                for (uint32_t a = r[0]; a < r[2]; ++a, ++j) {
                    if (j >= rec_max) fail(SYK_EDEVICE, "control block record overflow");
                    for (uint32_t f = 0; f < rec_dw; ++f) blk[rec_dw * j + f] = compact[a][f];
                }
            }
            blk[60] = counts;
            blk[62] = plain_counts;
        }
    }
    return hp;
}

template <typename U>
static U *upload(const std::vector<U> &v, DeviceSlab *slab) {
    U *d = nullptr;
    const size_t n = std::max<size_t>(v.size(), 1);
    if (slab)
        d = static_cast<U *>(slab->take(n * sizeof(U), "apply plan"));
    else
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&d), n * sizeof(U)));
    if (!v.empty()) SYK_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice));
    return d;
}

void free_plan(ApplyPlan &p) {
    if (p.in_slab) {
        p = ApplyPlan{};
        return;
    }
    ignore_status(hipFree(p.pi));
    ignore_status(hipFree(p.ranges));
    ignore_status(hipFree(p.meta));
    ignore_status(hipFree(p.tile_map));
    ignore_status(hipFree(p.c32));
    ignore_status(hipFree(p.c64));
    p = ApplyPlan{};
}

void upload_plan(const HostPlan &hp, int bt, int rb, ApplyPlan &out, DeviceSlab *slab) {
    ApplyPlan p;
    p.in_slab = slab != nullptr;
    p.bt = bt;
    p.rb = rb;
    p.rot = hp.rot;
    p.w = hp.w;
    p.n_tiles = hp.n_tiles;
    p.n_wg = hp.n_wg;
    p.n_pi = hp.n_pi;
    for (size_t i = 0; i < hp.hvec.size() && i < 8; ++i) p.hvec[i] = hp.hvec[i];
    try {
        p.pi = upload(hp.pi, slab);
        p.ranges = upload(hp.ranges, slab);
        p.meta = upload(hp.meta, slab);
        p.tile_map = upload(hp.tile_map, slab);
        std::vector<float> c32(hp.c.begin(), hp.c.end());
        p.c32 = upload(c32, slab);
        p.c64 = upload(hp.c, slab);
    } catch (...) {
        free_plan(p);
        throw;
    }
    out = p;
}

}  // namespace syk
