"""Closed forms for Hamiltonians whose terms commute pairwise, at any N the full vector fits.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

H = sum_b J_b chi_i chi_j chi_k chi_l = sum_b (J_b / 4) P_b (Eq. (1), chi = gamma / sqrt 2),
with P_b = gamma_i gamma_j gamma_k gamma_l for the sorted subset b.  Each P_b is Hermitian
with P_b^2 = 1 (four distinct anticommuting gammas squaring to 1), and two such products
commute exactly when their subsets share an even number of indices, because moving one
gamma product of length 4 past another picks up (-1)^(16 - |a & b|).  When every pair
commutes:

* e^{zH} = prod_b e^{z J_b P_b / 4} = prod_b (cosh(z J_b / 4) + sinh(z J_b / 4) P_b);
* the spectrum has up to 2^K distinct levels sum_b (J_b / 4) s_b, s_b = +-1, so a Krylov
  basis started from a random state keeps growing well past a handful of vectors;
* for W = chi_i and V = chi_j, i != j, both in term a and in no other term, W and V
  anticommute with P_a and commute with every other P_b.  Moving them to the left through
  the exponentials of the random-state estimator of the supplement (the one of Eq. (2) with
  the symmetric split of the last e^{-beta H / 4}) flips the sign of the H_a part each time
  and leaves the rest alone; the H_a exponents add to 4 i t, the rest to -beta, and
  chi_i chi_j chi_i chi_j = -1/4, so

      F_psi(t) = -(1/4) <psi| e^{-beta H_rest} (cos(J_a t) + i sin(J_a t) P_a) |psi>,

  H_rest = sum_{b != a} (J_b / 4) P_b.

Vectors live on the full space of N/2 qubits (index bit q = qubit q, the parity qubit the
most significant), and a Pauli string acts on them as the tensor product of its 2x2
single-qubit matrices, one tensor axis at a time: the plain definition of a Kronecker
product applied to a vector, no bit tricks.
"""
import numpy as np

from . import pauli


def apply_string(s, v: np.ndarray) -> np.ndarray:
    """P v for the Pauli string s = (labels, p) on n qubits and v of length 2^n.

    The vector is viewed as an n-dimensional 2 x ... x 2 tensor; in C order the first axis
    is the most significant index bit, so qubit q is axis n - 1 - q.  Each non-identity
    label contracts its 2x2 matrix with that axis."""
    labels, p = s
    n = len(labels)
    if v.shape != (1 << n,):
        raise ValueError("vector length must be 2^(number of qubits)")
    T = v.astype(np.complex128).reshape((2,) * n)
    for q, lab in enumerate(labels):
        if lab == pauli.I:
            continue
        ax = n - 1 - q
        T = np.moveaxis(np.tensordot(pauli.SIGMA[lab], T, axes=([1], [ax])), 0, ax)
    return (1j ** p) * T.reshape(-1)


def term_string(N: int, subset):
    """gamma_i gamma_j gamma_k gamma_l on the full space (N/2 qubits), as a Pauli string."""
    L = N // 2 - 1
    s = (tuple([pauli.I] * (L + 1)), 0)
    for n in subset:
        s = pauli.multiply(s, pauli.full_majorana(N, n))
    return s


def commute(a, b) -> bool:
    """Whether the products of the gammas of 4-subsets a and b commute."""
    return len(set(a) & set(b)) % 2 == 0


def all_commute(subsets) -> bool:
    subsets = [tuple(s) for s in subsets]
    return all(commute(subsets[x], subsets[y]) for x in range(len(subsets)) for y in range(x))


def expm_apply(N: int, subsets, J, z: complex, v: np.ndarray) -> np.ndarray:
    """e^{zH} v on the full space for pairwise commuting terms."""
    if not all_commute(subsets):
        raise ValueError("the terms do not commute pairwise")
    out = np.asarray(v, dtype=np.complex128)
    for s, Jb in zip(subsets, J):
        w = z * Jb / 4.0
        out = np.cosh(w) * out + np.sinh(w) * apply_string(term_string(N, s), out)
    return out


def lone_pair_term(subsets, i: int, j: int) -> int:
    """Index a of the only term that contains i and j, with neither in any other term
    (-1 if there is none)."""
    hits = [a for a, s in enumerate(subsets) if i in s or j in s]
    if len(hits) != 1 or i not in subsets[hits[0]] or j not in subsets[hits[0]]:
        return -1
    return hits[0]


def otoc_state(N: int, subsets, J, i: int, j: int, beta: float, ts, psi: np.ndarray) -> np.ndarray:
    """F_psi(t) of the random-state estimator (complex) for W = chi_i, V = chi_j, by the
    closed form above.  Requires pairwise commuting terms, i != j, both in exactly one term
    and in no other."""
    if not all_commute(subsets):
        raise ValueError("the terms do not commute pairwise")
    if i == j:
        raise ValueError("i and j must differ")
    a = lone_pair_term(subsets, i, j)
    if a < 0:
        raise ValueError("i and j must both lie in one term and in no other")
    rest = [s for b, s in enumerate(subsets) if b != a]
    Jrest = [Jb for b, Jb in enumerate(J) if b != a]
    u = expm_apply(N, rest, Jrest, -beta, psi) if rest else np.asarray(psi, dtype=np.complex128)
    c0 = np.vdot(psi, u)                                       # <psi| e^{-beta H_rest} |psi>
    c1 = np.vdot(psi, apply_string(term_string(N, subsets[a]), u))   # ... P_a ...
    Ja = J[a]
    return np.array([-0.25 * (np.cos(Ja * t) * c0 + 1j * np.sin(Ja * t) * c1) for t in ts], dtype=np.complex128)
