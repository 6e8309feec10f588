"""Dense definitions (complex128) for small N (N <= 20, full dimension <= 1024).

Everything here is the plain definition written out:
* Majoranas chi_n = gamma_n / sqrt(2), gamma_n the dense Pauli strings of supplement
  Eq. (S1) (see ``oracle.pauli`` for the convention), so {chi_m, chi_n} = delta_mn as
  in the main text;
* H = sum_a J_a chi_i chi_j chi_k chi_l, Eq. (1), as a sum of dense matrix products;
* parity blocks H_UU = H[:h, :h], H_DD = H[h:, h:] (supplement, parity-block form);
* e^{zH} v through the eigendecomposition H = U diag(E) U^dagger;
* the regularised OTOC of Eq. (2), once as the exact trace
  Tr[y W(t) y V y W(t) y V] / dim with y = e^{-beta H/4}, W(t) = e^{iHt} W e^{-iHt}
  (cyclically equal to the trace in Eq. (2)), and once as the random-state estimator of
  the supplement, <psi| e^{(it-b/8)H} W e^{-(it+b/4)H} V e^{(it-b/4)H} W e^{-(it+b/4)H}
  V e^{-bH/8} |psi>, evaluated on the full space (not in block form);
* the Green function of the supplement,
  G(t) = <psi| e^{(it-b/2)H} gamma e^{-iHt} gamma e^{-bH/2} |psi>.
"""
import numpy as np

from . import pauli


def dimension(N: int) -> int:
    return 1 << (N // 2)


def gammas(N: int):
    """Dense gamma_n (Pauli-string normalisation, gamma^2 = 1), n = 0..N-1."""
    return [pauli.dense(pauli.full_majorana(N, n)) for n in range(N)]


def chis(N: int):
    """Dense chi_n = gamma_n / sqrt(2): {chi_m, chi_n} = delta_mn."""
    s = 1.0 / np.sqrt(2.0)
    return [g * s for g in gammas(N)]


def hamiltonian(N: int, subsets, J) -> np.ndarray:
    """H = sum_a J_a chi_i chi_j chi_k chi_l (Eq. (1)), dense on the full space."""
    ch = chis(N)
    d = dimension(N)
    H = np.zeros((d, d), dtype=np.complex128)
    for (i, j, k, l), Ja in zip(subsets, J):
        H += Ja * (ch[i] @ ch[j] @ ch[k] @ ch[l])
    return H


def parity_operator(N: int) -> np.ndarray:
    """Gamma = Z on the parity qubit (the most significant qubit)."""
    d = dimension(N)
    return np.diag(np.where(np.arange(d) < d // 2, 1.0, -1.0)).astype(np.complex128)


def blocks(H: np.ndarray):
    """(H_UU, H_DD): U is the first half of the index range (parity bit 0)."""
    h = H.shape[0] // 2
    return H[:h, :h], H[h:, h:]


class Eig:
    """Eigendecomposition H = U diag(E) U^dagger of a Hermitian matrix."""

    def __init__(self, H: np.ndarray):
        self.E, self.U = np.linalg.eigh(H)

    def expm(self, z: complex) -> np.ndarray:
        """Dense e^{zH}."""
        return (self.U * np.exp(z * self.E)) @ self.U.conj().T

    def expm_apply(self, z: complex, v: np.ndarray) -> np.ndarray:
        """e^{zH} v."""
        return self.U @ (np.exp(z * self.E)[:, None] * (self.U.conj().T @ v.reshape(len(self.E), -1))).reshape(v.shape)

    def to_eig(self, A: np.ndarray) -> np.ndarray:
        return self.U.conj().T @ A @ self.U


def otoc_trace(H: np.ndarray, W: np.ndarray, V: np.ndarray, beta: float, ts) -> np.ndarray:
    """Exact Tr[y W(t) y V y W(t) y V] / dim, y = e^{-beta H/4}, for each t (complex)."""
    eg = Eig(H)
    We = eg.to_eig(W)
    Ve = eg.to_eig(V)
    y = np.exp(-beta * eg.E / 4.0)
    d = H.shape[0]
    out = []
    for t in ts:
        ph = np.exp(1j * eg.E * t)
        Wt = (ph[:, None] * We) * ph.conj()[None, :]          # e^{iEt} W e^{-iEt}
        A = (y[:, None] * Wt) @ (y[:, None] * Ve)             # y W(t) y V
        out.append(np.trace(A @ A) / d)
    return np.array(out, dtype=np.complex128)


def otoc_state(H: np.ndarray, W: np.ndarray, V: np.ndarray, beta: float, ts, psi: np.ndarray) -> np.ndarray:
    """Random-state estimator of the supplement on the full space (complex, one psi)."""
    eg = Eig(H)
    out = []
    for t in ts:
        e1 = eg.expm(1j * t - beta / 8.0)
        e2 = eg.expm(-(1j * t + beta / 4.0))
        e3 = eg.expm(1j * t - beta / 4.0)
        e5 = eg.expm(-beta / 8.0)
        chain = e1 @ W @ e2 @ V @ e3 @ W @ e2 @ V @ e5
        out.append(np.vdot(psi, chain @ psi))
    return np.array(out, dtype=np.complex128)


def green_state(H: np.ndarray, G: np.ndarray, beta: float, ts, psi: np.ndarray) -> np.ndarray:
    """G(t) = <psi| e^{(it-b/2)H} gamma e^{-iHt} gamma e^{-bH/2} |psi> (complex)."""
    eg = Eig(H)
    out = []
    for t in ts:
        chain = eg.expm(1j * t - beta / 2.0) @ G @ eg.expm(-1j * t) @ G @ eg.expm(-beta / 2.0)
        out.append(np.vdot(psi, chain @ psi))
    return np.array(out, dtype=np.complex128)


def normalise_curves(F: np.ndarray):
    """Average over random vectors (axis 0) and normalise by t = 0.

    Returns (F_raw, F_norm, F_imag): F_raw = mean_v Re F_v(t), F_norm = F_raw / F_raw[0]
    (a ratio of sums over vectors), F_imag = mean_v Im F_v(t)."""
    F = np.atleast_2d(F)
    raw = F.real.mean(axis=0)
    return raw, raw / raw[0], F.imag.mean(axis=0)
