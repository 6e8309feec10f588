// General spin operators (sums of Pauli strings) and their kernel term tables.
#pragma once

#include <complex>
#include <vector>

#include "internal.hpp"

namespace syk {

struct OpTerm {
    uint64_t x, z;                 // c X^x Z^z, Z applied first; qubit q = bit q
    std::complex<double> c;
};

struct Operator {
    int L = 0;
    std::vector<OpTerm> terms;     // canonical: sorted by (x, z), no duplicates
    void canonicalise(double drop);
};

Operator op_product(const Operator &a, const Operator &b);
Operator op_sum(const Operator &a, const Operator &b, std::complex<double> alpha, std::complex<double> beta);
Operator op_adjoint(const Operator &a);
bool op_is_hermitian(const Operator &a, double tol);
// term tables of a handle that applies `op` (on both block slots) through apply_H / Krylov
void build_operator_hamiltonian(Hamiltonian &h, const Operator &op);

}  // namespace syk
