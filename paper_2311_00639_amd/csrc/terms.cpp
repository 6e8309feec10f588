// Host-side construction of one disorder realisation of the sparse SYK Hamiltonian,
// Eq. (1), and of its parity-block term tables.
//
// Coupling ensembles (main text, "Sparse SYK Model"): exactly K = round(kN) distinct
// 4-subsets drawn uniformly (p = K/C(N,4)), or the paper's Bernoulli ensemble, every
// 4-subset kept with probability p = k N / C(N,4) (p = 1: dense SYK); J ~ N(0, sigma^2)
// with sigma^2 = 3!/(p N^3) for chi normalised to {chi_m, chi_n} = delta_mn (the printed
// 3/(8pN^3) is the variance of J/4, the coefficient of a product of four Pauli-string
// Majoranas).
//
// Term tables: every block Majorana A_n (supplement Eq. (S1), compact form) is a Pauli
// string i^w X^x Z^z; the product of four of them is formed by
// (X^a Z^b)(X^c Z^d) = (-1)^{popcount(b & c)} X^{a ^ c} Z^{b ^ d}, the XOR-and-sign product
// of spin operators described in supplement Sec. I.A.
//
// Compiled with -ffp-contract=off so that the coupling arithmetic rounds exactly as the
// written expression (one IEEE operation at a time).
#include <algorithm>
#include <cmath>
#include <set>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace syk {

static constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

namespace {

struct Stream {
    uint64_t s;
    uint64_t next() {
        s += kGamma;
        return splitmix_mix(s);
    }
};

uint64_t choose(int n, int r) {
    if (r < 0 || n < r) return 0;
    uint64_t v = 1;
    for (int i = 1; i <= r; ++i) v = v * static_cast<uint64_t>(n - r + i) / static_cast<uint64_t>(i);
    return v;
}

// idx = C(l,4) + C(k,3) + C(j,2) + C(i,1), l > k > j > i >= 0 (colex rank)
std::tuple<int, int, int, int> unrank4(uint64_t idx) {
    int sub[4];
    for (int r = 4, pos = 3; r >= 1; --r, --pos) {
        int c = r - 1;
        while (choose(c + 1, r) <= idx) ++c;
        sub[pos] = c;
        idx -= choose(c, r);
    }
    return {sub[0], sub[1], sub[2], sub[3]};
}

struct Pauli {     // i^w X^x Z^z
    uint32_t x = 0, z = 0;
    int w = 0;
};

Pauli mul(const Pauli &a, const Pauli &b) {
    Pauli r;
    r.x = a.x ^ b.x;
    r.z = a.z ^ b.z;
    r.w = (a.w + b.w + 2 * (__builtin_popcount(a.z & b.x) & 1)) & 3;
    return r;
}

}  // namespace

void block_majorana(int N, int n, uint32_t &x, uint32_t &z, int &w) {
    const int L = N / 2 - 1;
    const uint32_t all = (L == 32) ? 0xFFFFFFFFu : ((1u << L) - 1u);
    auto suffix = [&](int q) -> uint32_t { return q >= L ? 0u : (all & ~((1u << q) - 1u)); };
    if (n == 0) {
        x = all;
        z = 0;
        w = 0;
    } else if (n % 2 == 1) {          // Y_q X_{q+1..}: Y = i X Z -> i X^{suffix(q)} Z^{e_q}
        const int q = (n - 1) / 2;
        x = suffix(q);
        z = 1u << q;
        w = 1;
    } else {                          // Z_q X_{q+1..} = X^{suffix(q+1)} Z^{e_q}
        const int q = (n - 1) / 2;
        x = suffix(q + 1);
        z = 1u << q;
        w = 0;
    }
}

void build_hamiltonian(Hamiltonian &h, int N, double k, uint64_t seed, int ensemble) {
    h.N = N;
    h.L = N / 2 - 1;
    h.k = k;
    h.seed = seed;
    const uint64_t C = choose(N, 4);
    Stream rng{seed};
    std::vector<std::tuple<int, int, int, int>> chosen;
    if (ensemble == SYK_ENSEMBLE_BERNOULLI) {
        // every 4-subset, in lexicographic order, is kept with probability p = k N / C(N,4)
        // (one draw each, kept iff the [0,1) uniform is below p); p = 1 is the dense model
        const double p = k * static_cast<double>(N) / static_cast<double>(C);
        if (!(p > 0.0) || p > 1.0) fail(SYK_EINVAL, "Bernoulli ensemble needs 0 < p = k N / C(N,4) <= 1");
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j)
                for (int kk = j + 1; kk < N; ++kk)
                    for (int l = kk + 1; l < N; ++l) {
                        const double u = static_cast<double>(rng.next() >> 11) * 0x1p-53;
                        if (u < p) chosen.push_back(std::make_tuple(i, j, kk, l));
                    }
        if (chosen.empty()) fail(SYK_EINVAL, "the Bernoulli draw kept no term");
        h.p = p;
    } else {
        const double Kd = std::floor(k * static_cast<double>(N) + 0.5);
        if (!(Kd >= 1.0) || Kd > static_cast<double>(C)) fail(SYK_EINVAL, "K = round(k N) must lie in [1, C(N,4)]");
        const int Kt = static_cast<int>(Kd);
        // 2^64 - (2^64 mod C), computed in 64-bit arithmetic: (0 - C) mod C == 2^64 mod C
        const uint64_t rem = (0ULL - C) % C;
        const uint64_t limit = 0ULL - rem;           // reject r >= limit (rem == 0: never)
        std::set<std::tuple<int, int, int, int>> set;
        while (static_cast<int>(set.size()) < Kt) {
            const uint64_t r = rng.next();
            if (rem != 0 && r >= limit) continue;
            set.insert(unrank4(r % C));
        }
        chosen.assign(set.begin(), set.end());       // std::set iterates in lexicographic order
        h.p = static_cast<double>(Kt) / static_cast<double>(C);
    }
    const int K = static_cast<int>(chosen.size());
    h.K = K;
    h.ensemble = ensemble;

    // sigma^2 = 3! / (p N^3)
    const double num = 6.0;
    const double den = h.p * static_cast<double>(N * N * N);
    h.sigma = std::sqrt(num / den);
    if (ensemble != SYK_ENSEMBLE_BERNOULLI) {        // the exact-K form, kept bit-for-bit
        const double num_c = 6.0 * static_cast<double>(C);
        const double den_c = static_cast<double>(K) * static_cast<double>(N * N * N);
        h.sigma = std::sqrt(num_c / den_c);
    }
    const double two_pi = 2.0 * M_PI;

    h.ijkl.clear();
    h.J.clear();
    h.xmask.clear();
    h.zmask.clear();
    h.phase[0].clear();
    h.phase[1].clear();
    h.sum_J2 = 0.0;
    for (const auto &t : chosen) {
        h.ijkl.push_back(std::get<0>(t));
        h.ijkl.push_back(std::get<1>(t));
        h.ijkl.push_back(std::get<2>(t));
        h.ijkl.push_back(std::get<3>(t));
    }
    for (int a = 0; a < K; ++a) {
        const double u1 = static_cast<double>((rng.next() >> 11) + 1) * 0x1p-53;
        const double u2 = static_cast<double>(rng.next() >> 11) * 0x1p-53;
        const double r = std::sqrt(-2.0 * std::log(u1));
        const double Ja = h.sigma * r * std::cos(two_pi * u2);
        h.J.push_back(Ja);
        h.sum_J2 += Ja * Ja;
    }

    // block forms of gamma_i gamma_j gamma_k gamma_l
    for (int a = 0; a < K; ++a) {
        const int *s = &h.ijkl[4 * a];
        const bool top = (s[3] == N - 1);        // gamma_{N-1} = Y_parity (x) 1
        Pauli P;
        for (int c = 0; c < (top ? 3 : 4); ++c) {
            Pauli A;
            block_majorana(N, s[c], A.x, A.z, A.w);
            P = mul(P, A);
        }
        // full space: X X X X = 1 on the parity qubit; X X X Y = X Y = i Z, i.e. +i on U, -i on D
        const int wU = (P.w + (top ? 1 : 0)) & 3;
        const int wD = (P.w + (top ? 3 : 0)) & 3;
        h.xmask.push_back(P.x);
        h.zmask.push_back(P.z);
        h.phase[0].push_back(static_cast<int8_t>(wU));
        h.phase[1].push_back(static_cast<int8_t>(wD));
    }

    // kernel tables: fold (-1)^{popc(x & z)} (sign read from the source index) and the
    // real sign of i^p into c; real terms first, then imaginary terms
    for (int blk = 0; blk < 2; ++blk) {
        std::vector<BlockTerm> re, im;
        for (int a = 0; a < K; ++a) {
            const uint32_t x = static_cast<uint32_t>(h.xmask[a]);
            const uint32_t z = static_cast<uint32_t>(h.zmask[a]);
            const int p = (h.phase[blk][a] + 2 * (__builtin_popcount(x & z) & 1)) & 3;
            const double c = 0.25 * h.J[a] * ((p == 2 || p == 3) ? -1.0 : 1.0);
            BlockTerm bt{x, z, c, (p & 1) != 0};
            (bt.imag ? im : re).push_back(bt);
        }
        h.n_real[blk] = static_cast<int>(re.size());
        re.insert(re.end(), im.begin(), im.end());
        h.block_terms[blk] = std::move(re);
    }
}

}  // namespace syk
