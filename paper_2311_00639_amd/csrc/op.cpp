// General spin operators: sums of Pauli strings c X^x Z^z (Z applied first) on L qubits,
// with products, sums and adjoints formed by the XOR-and-sign rule of supplement Sec. I.A
// ((X^a Z^b)(X^c Z^d) = (-1)^{popcount(b & c)} X^{a ^ c} Z^{b ^ d}), and their conversion
// to the kernel term tables of the apply_H / Krylov path, so that other sparse models run
// through the same kernels.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <utility>
#include <vector>

#include "op.hpp"

namespace syk {

void Operator::canonicalise(double drop) {
    std::map<std::pair<uint64_t, uint64_t>, std::complex<double>> acc;
    for (const auto &t : terms) acc[{t.x, t.z}] += t.c;
    terms.clear();
    for (const auto &kv : acc)
        if (std::abs(kv.second) > drop) terms.push_back(OpTerm{kv.first.first, kv.first.second, kv.second});
}

Operator op_product(const Operator &a, const Operator &b) {
    if (a.L != b.L) fail(SYK_EINVAL, "operators act on different numbers of qubits");
    Operator r;
    r.L = a.L;
    r.terms.reserve(a.terms.size() * b.terms.size());
    for (const auto &p : a.terms)
        for (const auto &q : b.terms) {
            const double sg = (__builtin_popcountll(p.z & q.x) & 1) ? -1.0 : 1.0;
            r.terms.push_back(OpTerm{p.x ^ q.x, p.z ^ q.z, sg * p.c * q.c});
        }
    r.canonicalise(0.0);
    return r;
}

Operator op_sum(const Operator &a, const Operator &b, std::complex<double> alpha, std::complex<double> beta) {
    if (a.L != b.L) fail(SYK_EINVAL, "operators act on different numbers of qubits");
    Operator r;
    r.L = a.L;
    for (const auto &p : a.terms) r.terms.push_back(OpTerm{p.x, p.z, alpha * p.c});
    for (const auto &q : b.terms) r.terms.push_back(OpTerm{q.x, q.z, beta * q.c});
    r.canonicalise(0.0);
    return r;
}

// (c X^x Z^z)^dagger = conj(c) Z^z X^x = conj(c) (-1)^{popcount(x & z)} X^x Z^z
Operator op_adjoint(const Operator &a) {
    Operator r;
    r.L = a.L;
    for (const auto &p : a.terms) {
        const double sg = (__builtin_popcountll(p.x & p.z) & 1) ? -1.0 : 1.0;
        r.terms.push_back(OpTerm{p.x, p.z, sg * std::conj(p.c)});
    }
    r.canonicalise(0.0);
    return r;
}

bool op_is_hermitian(const Operator &a, double tol) {
    const Operator d = op_sum(a, op_adjoint(a), 1.0, -1.0);
    double scale = 0.0;
    for (const auto &t : a.terms) scale = std::max(scale, std::abs(t.c));
    for (const auto &t : d.terms)
        if (std::abs(t.c) > tol * std::max(scale, 1e-300)) return false;
    return true;
}

// Canonical terms J i^p X^x Z^z (p = 0 for the real part of c, 1 for the imaginary part),
// then the kernel form y[m] += c' (-1)^{popc(m & z)} x[m ^ x] with c' = J (-1)^{popc(x & z)}
// (the sign read at the source index moved to the output index) and an i factor for
// p = 1.  Real terms first, then i terms.
void build_operator_hamiltonian(Hamiltonian &h, const Operator &op) {
    if (op.L < 1 || op.L > 31) fail(SYK_EINVAL, "operators need 1 <= L <= 31 qubits");
    h.N = 2 * (op.L + 1);
    h.L = op.L;
    h.k = 0.0;
    h.p = 0.0;
    h.sigma = 0.0;
    h.seed = 0;
    h.ensemble = -1;
    h.hermitian = op_is_hermitian(op, 1e-13);
    h.sum_J2 = 0.0;
    h.ijkl.clear();
    h.J.clear();
    h.xmask.clear();
    h.zmask.clear();
    h.phase[0].clear();
    h.phase[1].clear();
    std::vector<BlockTerm> re, im;
    auto add = [&](uint64_t x, uint64_t z, double J, int p) {
        const double sg = (__builtin_popcountll(x & z) & 1) ? -1.0 : 1.0;
        (p ? im : re).push_back(BlockTerm{static_cast<uint32_t>(x), static_cast<uint32_t>(z), sg * J, p == 1});
        for (int q = 0; q < 4; ++q) h.ijkl.push_back(-1);
        h.J.push_back(J);
        h.sum_J2 += J * J;
        h.xmask.push_back(x);
        h.zmask.push_back(z);
        h.phase[0].push_back(static_cast<int8_t>(p));
        h.phase[1].push_back(static_cast<int8_t>(p));
    };
    for (const auto &t : op.terms) {
        if (t.c.real() != 0.0) add(t.x, t.z, t.c.real(), 0);
        if (t.c.imag() != 0.0) add(t.x, t.z, t.c.imag(), 1);
    }
    if (h.J.empty()) fail(SYK_EINVAL, "operator has no terms");
    h.K = static_cast<int>(h.J.size());
    for (int blk = 0; blk < 2; ++blk) {      // both "blocks" hold the operator
        h.n_real[blk] = static_cast<int>(re.size());
        std::vector<BlockTerm> all = re;
        all.insert(all.end(), im.begin(), im.end());
        h.block_terms[blk] = std::move(all);
    }
}

}  // namespace syk
