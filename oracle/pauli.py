"""Pauli strings and the Jordan-Wigner Majorana representation (supplement, Sec. I,
Eq. (S1) and its compact form; Pauli matrices defined right after it).

A Pauli string on n qubits is held as (labels, p): labels[q] in {0:I, 1:X, 2:Y, 3:Z}
acts on qubit q, which is bit q of the basis index, and p is the power of i of an
overall phase.  Products are taken qubit by qubit with the single-qubit table
sigma_a sigma_b = delta_ab I + i eps_abc sigma_c.

Readings adopted:
* sigma_y = [[0, -i], [i, 0]] (the textbook sign; the supplement prints the other
  sign, which only relabels J signs and leaves the ensemble unchanged);
* block Majoranas on L = N/2 - 1 qubits, from the compact form of Eq. (S1):
  A_0 = prod_{q<L} X_q, and for 1 <= n <= N-2,
  A_n = (Y if n odd else Z)_{floor((n-1)/2)} * prod_{q >= floor((n+1)/2)} X_q;
* full space of L+1 qubits, the parity qubit being the most significant:
  gamma_n = X_parity (x) A_n for n <= N-2 and gamma_{N-1} = Y_parity (x) 1, so that
  gamma_{N-1}'s UD block is -i 1 and gamma_{N-2}'s blocks are Z_{L-1}, as the
  supplement states.
"""
import numpy as np

I, X, Y, Z = 0, 1, 2, 3

# single-qubit products: _MUL[a][b] = (c, p) with sigma_a sigma_b = i^p sigma_c
_MUL = {}
for _a in range(4):
    _MUL[(_a, I)] = (_a, 0)
    _MUL[(I, _a)] = (_a, 0)
    _MUL[(_a, _a)] = (I, 0)
for (_a, _b, _c) in ((X, Y, Z), (Y, Z, X), (Z, X, Y)):       # cyclic: i eps_abc = +i
    _MUL[(_a, _b)] = (_c, 1)
    _MUL[(_b, _a)] = (_c, 3)

SIGMA = [
    np.array([[1, 0], [0, 1]], dtype=np.complex128),
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def multiply(s1, s2):
    """Product of two Pauli strings (labels, p) qubit by qubit."""
    l1, p1 = s1
    l2, p2 = s2
    assert len(l1) == len(l2)
    out = []
    p = p1 + p2
    for a, b in zip(l1, l2):
        c, q = _MUL[(a, b)]
        out.append(c)
        p += q
    return (tuple(out), p % 4)


def block_majorana(N: int, n: int):
    """A_n on L = N/2 - 1 qubits (0 <= n <= N-2)."""
    L = N // 2 - 1
    if not 0 <= n <= N - 2:
        raise ValueError("block Majorana index out of range")
    labels = [I] * L
    if n == 0:
        for q in range(L):
            labels[q] = X
        return (tuple(labels), 0)
    q0 = (n - 1) // 2
    labels[q0] = Y if n % 2 == 1 else Z
    for q in range((n + 1) // 2, L):
        labels[q] = X
    return (tuple(labels), 0)


def full_majorana(N: int, n: int):
    """gamma_n on L+1 qubits; qubit L is the parity qubit."""
    L = N // 2 - 1
    if n == N - 1:
        return (tuple([I] * L + [Y]), 0)
    labels, p = block_majorana(N, n)
    return (tuple(list(labels) + [X]), p)


def dense(s) -> np.ndarray:
    """Dense matrix of a Pauli string: kron over qubits, most significant qubit first."""
    labels, p = s
    M = np.array([[1.0 + 0j]])
    for q in reversed(range(len(labels))):
        M = np.kron(M, SIGMA[labels[q]])
    return (1j ** p) * M


def canonical(s):
    """(x, z, w) with string = i^w X^x Z^z (Z applied first), x and z as bit masks.

    Y = i X Z, so each Y contributes one factor of i (the supplement's coeff = lambda * i^{#Y})."""
    labels, p = s
    x = z = 0
    ny = 0
    for q, a in enumerate(labels):
        if a in (X, Y):
            x |= 1 << q
        if a in (Y, Z):
            z |= 1 << q
        if a == Y:
            ny += 1
    return x, z, (p + ny) % 4


def term_blocks(N: int, subset):
    """Parity-block forms of gamma_i gamma_j gamma_k gamma_l.

    Returns ((labels_U, p_U), (labels_D, p_D)): the UU and DD blocks as Pauli strings on
    L qubits.  The full-space product is formed qubit by qubit on L+1 qubits; its parity
    qubit label must be I or Z (the product of four Majoranas is block diagonal), and
    Z contributes +1 on the U block and -1 (= i^2) on the D block."""
    L = N // 2 - 1
    s = (tuple([I] * (L + 1)), 0)
    for n in subset:
        s = multiply(s, full_majorana(N, n))
    labels, p = s
    top = labels[L]
    if top not in (I, Z):
        raise AssertionError("product of four Majoranas is not block diagonal")
    blk = tuple(labels[:L])
    pU = p % 4
    pD = (p + (2 if top == Z else 0)) % 4
    return (blk, pU), (blk, pD)


def from_xz(L: int, x: int, z: int):
    """The Pauli string X^x Z^z (Z applied first) on L qubits as (labels, p): per qubit
    X Z = -i Y, so each qubit with both bits set contributes a factor i^-1."""
    labels = []
    ny = 0
    for q in range(L):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        if bx and bz:
            labels.append(Y)
            ny += 1
        elif bx:
            labels.append(X)
        elif bz:
            labels.append(Z)
        else:
            labels.append(I)
    return tuple(labels), (-ny) % 4


def operator_dense(L: int, xs, zs, cs) -> np.ndarray:
    """Dense matrix of sum_a c_a X^{x_a} Z^{z_a}."""
    M = np.zeros((1 << L, 1 << L), dtype=np.complex128)
    for x, z, c in zip(xs, zs, cs):
        M += c * dense(from_xz(L, int(x), int(z)))
    return M


def to_xz(labels):
    """Inverse of from_xz: a label string P = (x) sigma_q as (x, z, p) with P = i^p X^x Z^z
    (per qubit Y = i X Z)."""
    x = z = 0
    ny = 0
    for q, lab in enumerate(labels):
        if lab in (X, Y):
            x |= 1 << q
        if lab in (Y, Z):
            z |= 1 << q
        ny += lab == Y
    return x, z, ny % 4
