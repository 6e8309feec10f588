"""Rows of y = H_blk x for sampled output indices, at any N, without a dense matrix.

Each term of Eq. (1) restricted to a parity block is a Pauli string
(``oracle.pauli.term_blocks``).  Row m of a Pauli string P has exactly one nonzero
entry, in column n = m with every X/Y qubit flipped, equal to the phase times the
product over qubits of the single-qubit matrix elements <m_q| sigma |n_q>:
X -> 1, Y -> -i if m_q = 0 else +i, Z -> +1 if m_q = 0 else -1.  So

    y[m] = sum_a (J_a / 4) i^{p_a} prod_q <m_q| sigma_{a,q} |n_q> x[n]

with the 1/4 = (1/sqrt 2)^4 from chi = gamma / sqrt 2.  This is the definition of a
matrix-vector product row by row; it shares nothing with the bit-mask encoding of
supplement Algorithm 1 that the library uses.
"""
import numpy as np

from . import pauli


def block_terms(N: int, subsets, J, block: int):
    """[(labels, coefficient)] for block 0 (U) or 1 (D): coefficient = (J/4) i^p."""
    out = []
    for s, Ja in zip(subsets, J):
        (lab, p) = pauli.term_blocks(N, s)[block]
        out.append((lab, (Ja / 4.0) * (1j ** p)))
    return out


def apply_rows(terms, x_at, rows: np.ndarray) -> np.ndarray:
    """y[rows] for y = H_blk x.  ``x_at(idx)`` returns x at uint64 indices ``idx``."""
    rows = np.asarray(rows, dtype=np.uint64)
    y = np.zeros(rows.shape, dtype=np.complex128)
    for labels, coef in terms:
        src = rows.copy()
        elem = np.ones(rows.shape, dtype=np.complex128)
        for q, lab in enumerate(labels):
            if lab == pauli.I:
                continue
            bit = ((rows >> np.uint64(q)) & np.uint64(1)).astype(bool)
            if lab == pauli.X:
                src ^= np.uint64(1 << q)
            elif lab == pauli.Y:
                src ^= np.uint64(1 << q)
                elem *= np.where(bit, 1j, -1j)
            else:
                elem *= np.where(bit, -1.0, 1.0)
        y += coef * elem * x_at(src)
    return y
