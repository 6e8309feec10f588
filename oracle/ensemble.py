"""The sparse coupling ensemble of Eq. (1) (main text, "Sparse SYK Model").

H = sum over kept 4-subsets i<j<k<l of J_ijkl chi_i chi_j chi_k chi_l, with Gaussian
J of zero mean.  The paper's sparsity parameter is k = (p/N) C(N,4), so the mean
number of kept terms is kN.  Readings adopted:

* exactly K = round(kN) distinct 4-subsets are kept, drawn uniformly, and the
  keep-probability entering the variance is p = K / C(N,4);
* with chi normalised so that {chi_m, chi_n} = delta_mn (chi = Pauli string / sqrt 2),
  the coupling variance is sigma^2 = 3! / (p N^3).  The paper's printed variance
  3/(8 p N^3) is exactly the variance of J/4, the coefficient of the product of
  four Pauli-string Majoranas, so both statements describe the same ensemble.

Random draws follow a fixed recipe on one SplitMix64 stream seeded with ``seed``:
rejection-sampled subset ranks unranked in the colex combinatorial number system,
duplicates skipped, the K subsets sorted lexicographically, then one Box-Muller
normal per subset, in sorted order.
"""
import math

from .splitmix import SplitMix64, unit_open0, unit_open1


def n_terms(N: int, k: float) -> int:
    """K = round-half-away-from-zero(k N)."""
    return int(math.floor(k * N + 0.5))


def coupling_sigma(N: int, K: int) -> float:
    """sigma = sqrt(3! C(N,4) / (K N^3)), i.e. variance 3!/(p N^3) with p = K / C(N,4)."""
    num = 6.0 * float(math.comb(N, 4))
    den = float(K) * float(N * N * N)
    return math.sqrt(num / den)


def unrank_colex4(idx: int):
    """Inverse of idx = C(l,4) + C(k,3) + C(j,2) + C(i,1) with l > k > j > i >= 0."""
    out = []
    for r in (4, 3, 2, 1):
        c = r - 1
        while math.comb(c + 1, r) <= idx:
            c += 1
        out.append(c)
        idx -= math.comb(c, r)
    l, k, j, i = out
    return (i, j, k, l)


def sample_terms(N: int, k: float, seed: int):
    """Return (subsets, J, sigma): K sorted distinct 4-subsets of range(N) and their couplings."""
    if N % 2 or N < 6:
        raise ValueError("N must be even and >= 6")
    K = n_terms(N, k)
    C = math.comb(N, 4)
    if K < 1 or K > C:
        raise ValueError("K out of range")
    rng = SplitMix64(seed)
    limit = (1 << 64) - ((1 << 64) % C)      # reject r >= limit so r mod C is uniform
    chosen = set()
    while len(chosen) < K:
        r = rng.next()
        if r >= limit:
            continue
        chosen.add(unrank_colex4(r % C))
    subsets = sorted(chosen)
    sigma = coupling_sigma(N, K)
    J = []
    for _ in subsets:
        u1 = unit_open0(rng.next())
        u2 = unit_open1(rng.next())
        J.append(sigma * math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2))
    return subsets, J, sigma


def sample_terms_bernoulli(N: int, k: float, seed: int):
    """The Bernoulli ensemble of Eq. (1): each 4-subset i<j<k<l is kept independently
    with probability p = k N / C(N,4) (p = 1: the dense model), J ~ N(0, 3!/(p N^3)).

    Draws on one SplitMix64 stream seeded with ``seed``: one uniform (r >> 11) 2^-53 per
    subset in lexicographic order, kept iff it is below p; then one Box-Muller normal per
    kept subset, in order.  Returns (subsets, J, sigma)."""
    if N % 2 or N < 6:
        raise ValueError("N must be even and >= 6")
    p = k * N / math.comb(N, 4)
    if not (0.0 < p <= 1.0):
        raise ValueError("p out of range")
    rng = SplitMix64(seed)
    subsets = []
    for i in range(N):
        for j in range(i + 1, N):
            for kk in range(j + 1, N):
                for l in range(kk + 1, N):
                    if unit_open1(rng.next()) < p:
                        subsets.append((i, j, kk, l))
    if not subsets:
        raise ValueError("no term kept")
    sigma = math.sqrt(6.0 / (p * N ** 3))
    J = []
    for _ in subsets:
        u1 = unit_open0(rng.next())
        u2 = unit_open1(rng.next())
        J.append(sigma * math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2))
    return subsets, J, sigma
