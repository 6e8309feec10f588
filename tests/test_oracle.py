"""Pins of the oracle against the paper and against mathematics (no GPU).

Each test ties an oracle function to something other than itself: an algebraic
identity the paper states, a closed form, a library routine, a hand-derived fixture,
or a statistical law.  A plausible mistake (dropped term, wrong sign or index,
transposed operand) in the oracle fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import commuting, dense, ensemble, haar, lyapunov, matfree, pauli, splitmix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- Majoranas
@pytest.mark.parametrize("N", [6, 8, 10, 12, 14])
def test_clifford_algebra(N):
    """{chi_m, chi_n} = delta_mn (main text, Clifford algebra below Eq. (1))."""
    ch = dense.chis(N)
    d = ch[0].shape[0]
    for m in range(N):
        for n in range(N):
            ac = ch[m] @ ch[n] + ch[n] @ ch[m]
            ref = np.eye(d) if m == n else np.zeros((d, d))
            assert np.abs(ac - ref).max() < 1e-15
        assert np.allclose(ch[m], ch[m].conj().T)


@pytest.mark.parametrize("N", [6, 10, 14])
def test_block_forms_stated_in_supplement(N):
    """Majoranas are block off-diagonal; gamma_{N-1}^UD = -gamma_{N-1}^DU = -i 1 and
    gamma_{N-2}^UD = gamma_{N-2}^DU = sigma_z on block qubit N/2-2 (supplement, Sec. I)."""
    g = dense.gammas(N)
    d = g[0].shape[0]
    h = d // 2
    L = N // 2 - 1
    for gn in g:
        assert np.abs(gn[:h, :h]).max() == 0 and np.abs(gn[h:, h:]).max() == 0
    assert np.array_equal(g[N - 1][:h, h:], -1j * np.eye(h))
    assert np.array_equal(g[N - 1][h:, :h], 1j * np.eye(h))
    z_top = np.diag([(-1.0) ** ((b >> (L - 1)) & 1) for b in range(h)])
    assert np.array_equal(g[N - 2][:h, h:], z_top)
    assert np.array_equal(g[N - 2][h:, :h], z_top)


def test_pauli_table_matches_matrices():
    """sigma_a sigma_b = i^p sigma_c from the table equals the 2x2 matrix product, and the
    matrices are the textbook ones (sigma_x sigma_y = i sigma_z)."""
    S = pauli.SIGMA
    assert np.array_equal(S[1] @ S[2], 1j * S[3])
    for a in range(4):
        for b in range(4):
            (c,), p = pauli.multiply(((a,), 0), ((b,), 0))
            assert np.array_equal(S[a] @ S[b], (1j ** p) * S[c])


def test_canonical_readoff_matches_dense():
    """canonical(s) = (x, z, w) means s|m> = i^w (-1)^{popc(m & z)} |m ^ x> for every m."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        s = (tuple(int(a) for a in rng.integers(0, 4, n)), int(rng.integers(0, 4)))
        M = pauli.dense(s)
        x, z, w = pauli.canonical(s)
        for m in range(1 << n):
            col = np.zeros(1 << n, dtype=np.complex128)
            col[m ^ x] = (1j ** w) * (-1) ** bin(m & z).count("1")
            assert np.allclose(M[:, m], col)


def test_hand_derived_terms_N8():
    """Hand-derived block forms (tests/golden/hand_terms_N8.txt) from Eq. (S1)."""
    rows = []
    with open(os.path.join(GOLDEN, "hand_terms_N8.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 3
    for r in rows:
        sub = tuple(int(v) for v in r[:4])
        x, z, pU, pD = int(r[4], 2), int(r[5], 2), int(r[6]), int(r[7])
        (lu, qu), (ld, qd) = pauli.term_blocks(8, sub)
        assert pauli.canonical((lu, qu)) == (x, z, pU)
        assert pauli.canonical((ld, qd)) == (x, z, pD)
        # and the dense blocks of the full product agree
        g = dense.gammas(8)
        P = g[sub[0]] @ g[sub[1]] @ g[sub[2]] @ g[sub[3]]
        assert np.array_equal(P[:8, :8], pauli.dense((lu, qu)))
        assert np.array_equal(P[8:, 8:], pauli.dense((ld, qd)))


@pytest.mark.parametrize("N", [8, 10, 12])
def test_term_blocks_equal_dense_blocks(N):
    """term_blocks (qubit-by-qubit products) equals the dense blocks of gamma_i gamma_j gamma_k gamma_l,
    and the phase is real iff popcount(x & z) is even (Hermitian terms)."""
    g = dense.gammas(N)
    h = g[0].shape[0] // 2
    rng = np.random.default_rng(N)
    for _ in range(30):
        sub = tuple(sorted(rng.choice(N, 4, replace=False).tolist()))
        P = g[sub[0]] @ g[sub[1]] @ g[sub[2]] @ g[sub[3]]
        (lu, pu), (ld, pd) = pauli.term_blocks(N, sub)
        assert np.array_equal(P[:h, :h], pauli.dense((lu, pu)))
        assert np.array_equal(P[h:, h:], pauli.dense((ld, pd)))
        x, z, w = pauli.canonical((lu, pu))
        assert (w % 2 == 0) == (bin(x & z).count("1") % 2 == 0)


# --------------------------------------------------------------------------- ensemble
def test_unrank_is_a_bijection():
    N = 11
    seen = set()
    for idx in range(math.comb(N, 4)):
        s = ensemble.unrank_colex4(idx)
        assert 0 <= s[0] < s[1] < s[2] < s[3] < N
        seen.add(s)
    assert len(seen) == math.comb(N, 4)


def test_sample_terms_structure():
    subs, J, sigma = ensemble.sample_terms(16, 4, 1)
    assert len(subs) == 64 and len(set(subs)) == 64
    assert subs == sorted(subs)
    assert all(0 <= s[0] < s[1] < s[2] < s[3] < 16 for s in subs)
    # sigma^2 = 3!/(p N^3), p = K/C(N,4); dense limit p = 1 gives 6/N^3
    assert abs(ensemble.coupling_sigma(10, math.comb(10, 4)) ** 2 - 6.0 / 1000) < 1e-18
    assert abs(sigma ** 2 - 6.0 / ((64 / math.comb(16, 4)) * 16 ** 3)) < 1e-15
    assert ensemble.n_terms(56, 4) == 224 and ensemble.n_terms(48, 4) == 192
    assert ensemble.n_terms(56, 1.0 / 56) == 1


def test_subsets_uniform():
    """K=1 draws over many seeds are uniform over the C(8,4) = 70 subsets (chi-square)."""
    counts = {}
    n = 7000
    for seed in range(n):
        (s,), _, _ = ensemble.sample_terms(8, 1.0 / 8, seed)
        counts[s] = counts.get(s, 0) + 1
    assert len(counts) == 70
    exp = n / 70
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 69 + 5 * math.sqrt(2 * 69)          # mean 69, sd ~11.7


def test_coupling_law_moments():
    """J ~ N(0, sigma^2): mean, variance and kurtosis over many draws."""
    J = []
    for seed in range(200):
        _, Js, sigma = ensemble.sample_terms(12, 4, 1000 + seed)   # K = 48, sigma fixed
        J.extend(Js)
    J = np.array(J) / sigma
    n = len(J)
    assert abs(J.mean()) < 4 / math.sqrt(n)
    assert abs(J.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(np.mean(J ** 4) - 3) < 5 * math.sqrt(96 / n)


def test_splitmix_finaliser_is_bijective():
    """The finaliser inverts with the modular inverses of its multipliers."""
    M = splitmix.MASK64

    def unxorshift(y, s):
        x = y
        for _ in range(64 // s + 1):
            x = y ^ (x >> s)
        return x

    inv1 = pow(splitmix._M1, -1, 1 << 64)
    inv2 = pow(splitmix._M2, -1, 1 << 64)
    rng = np.random.default_rng(3)
    for v in rng.integers(0, 2 ** 63, 50, dtype=np.int64):
        z0 = int(v) * 2 + 1
        y = splitmix.mix(z0)
        y = unxorshift(y, 31)
        y = (y * inv2) & M
        y = unxorshift(y, 27)
        y = (y * inv1) & M
        y = unxorshift(y, 30)
        assert y == z0
    # the stream is mix(seed + n GAMMA) and the vectorised finaliser agrees
    g = splitmix.SplitMix64(12345)
    outs = [g.next() for _ in range(5)]
    assert outs == [splitmix.mix(12345 + (n + 1) * splitmix.GAMMA) for n in range(5)]
    arr = splitmix.mix_array(np.array([(12345 + (n + 1) * splitmix.GAMMA) & M for n in range(5)], dtype=np.uint64))
    assert [int(a) for a in arr] == outs


def test_splitmix_bits_balanced():
    g = splitmix.SplitMix64(99)
    ones = np.zeros(64)
    n = 20000
    for _ in range(n):
        r = g.next()
        ones += [(r >> b) & 1 for b in range(64)]
    assert np.all(np.abs(ones / n - 0.5) < 5 * 0.5 / math.sqrt(n))


# --------------------------------------------------------------------------- Hamiltonian
@pytest.mark.parametrize("N,k,seed", [(10, 3, 1), (12, 2, 2), (16, 4, 1)])
def test_hamiltonian_invariants(N, k, seed):
    """H Hermitian, Tr H = 0, Tr H^2/dim = sum J^2 / 16, [H, Gamma] = 0, Gamma ~ prod gamma."""
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    H = dense.hamiltonian(N, subs, J)
    d = H.shape[0]
    assert np.abs(H - H.conj().T).max() < 1e-15
    assert abs(np.trace(H)) < 1e-13
    assert abs(np.trace(H @ H).real / d - sum(x * x for x in J) / 16) < 1e-14
    Gm = dense.parity_operator(N)
    assert np.abs(H @ Gm - Gm @ H).max() < 1e-15
    g = dense.gammas(N)
    P = np.eye(d, dtype=np.complex128)
    for gn in g:
        P = P @ gn
    ratio = P[0, 0] / Gm[0, 0]
    assert abs(abs(ratio) - 1) < 1e-14 and np.allclose(P, ratio * Gm)


def test_hamiltonian_two_terms_by_hand():
    """H for two hand-picked terms equals the explicit sum of chi products."""
    ch = dense.chis(8)
    H = dense.hamiltonian(8, [(0, 1, 2, 3), (1, 2, 5, 7)], [0.5, -1.25])
    ref = 0.5 * ch[0] @ ch[1] @ ch[2] @ ch[3] - 1.25 * ch[1] @ ch[2] @ ch[5] @ ch[7]
    assert np.abs(H - ref).max() < 1e-16
    # (0,1,2,3) is -Z1 on each block (hand fixture) and chi^4 carries 1/4
    assert np.allclose(dense.hamiltonian(8, [(0, 1, 2, 3)], [1.0])[:8, :8],
                       -0.25 * pauli.dense(((0, 3, 0), 0)))


@pytest.mark.parametrize("N", [10, 12, 14, 16])
def test_bott_periodicity_spectra(N):
    """Parity-block spectra by N mod 8 (the Bott periodicity invoked in the main text):
    N = 2, 6 mod 8: spec H_UU = spec H_DD; N = 4 mod 8: every level doubly degenerate
    within each block; N = 0 mod 8: no pairing and no degeneracy."""
    subs, J, _ = ensemble.sample_terms(N, 3, 5)
    HU, HD = dense.blocks(dense.hamiltonian(N, subs, J))
    eU = np.linalg.eigvalsh(HU)
    eD = np.linalg.eigvalsh(HD)
    r = N % 8
    tol = 1e-12
    if r in (2, 6):
        assert np.abs(eU - eD).max() < tol
    elif r == 4:
        assert np.abs(eU[0::2] - eU[1::2]).max() < tol
        assert np.abs(eD[0::2] - eD[1::2]).max() < tol
    else:
        assert np.abs(eU - eD).max() > 1e-3
        assert np.min(np.diff(eU)) > 1e-10


def test_parity_blocks_are_the_only_nonzero_blocks():
    subs, J, _ = ensemble.sample_terms(12, 3, 3)
    H = dense.hamiltonian(12, subs, J)
    h = H.shape[0] // 2
    assert np.abs(H[:h, h:]).max() == 0 and np.abs(H[h:, :h]).max() == 0


# --------------------------------------------------------------------------- expm
def test_expm_matches_scipy():
    subs, J, _ = ensemble.sample_terms(12, 3, 4)
    H = dense.hamiltonian(12, subs, J)
    eg = dense.Eig(H)
    v = np.random.default_rng(1).standard_normal(H.shape[0]) + 0j
    for z in (-0.7j, 0.3 - 2.5j, -1.25, 2j - 0.5):
        ref = scipy.linalg.expm(z * H) @ v
        assert np.abs(eg.expm_apply(z, v) - ref).max() < 1e-12 * max(1, np.abs(ref).max())
    # unitarity and composition
    u = eg.expm_apply(-3.0j, v)
    assert abs(np.linalg.norm(u) - np.linalg.norm(v)) < 1e-12
    a = eg.expm_apply(0.4 - 1j, eg.expm_apply(-0.1 + 2j, v))
    assert np.abs(a - eg.expm_apply(0.3 + 1j, v)).max() < 1e-12


# --------------------------------------------------------------------------- OTOC
def test_otoc_t0_beta0_is_minus_quarter():
    """chi_i chi_j chi_i chi_j = -1/4 for i != j: F(0) = -1/4 at beta = 0 for any psi."""
    N = 12
    subs, J, _ = ensemble.sample_terms(N, 3, 9)
    H = dense.hamiltonian(N, subs, J)
    ch = dense.chis(N)
    for (i, j) in ((1, 2), (N - 1, N - 2), (0, 7)):
        assert abs(dense.otoc_trace(H, ch[i], ch[j], 0.0, [0.0])[0] + 0.25) < 1e-14
        psi = haar.haar_state(N, 77, i)
        assert abs(dense.otoc_state(H, ch[i], ch[j], 0.0, [0.0], psi)[0] + 0.25) < 1e-14


@pytest.mark.parametrize("beta", [0.0, 5.0])
def test_otoc_single_term_closed_forms(beta):
    """H = J chi_a chi_b chi_c chi_d = (J/4) P with P^2 = 1.  chi_n anticommutes with P iff n
    is in the term, which gives: both i, j in the term -> Re F = -cos(Jt)/4 for every psi
    and every beta; exactly one in the term -> F = -1/4; neither -> t-independent."""
    N = 12
    Jv = 0.7
    term = (1, 2, 5, 11)
    H = dense.hamiltonian(N, [term], [Jv])
    ch = dense.chis(N)
    ts = np.linspace(0, 6, 13)
    psi = haar.haar_state(N, 5, 0)
    Fs = dense.otoc_state(H, ch[1], ch[2], beta, ts, psi)
    Ft = dense.otoc_trace(H, ch[1], ch[2], beta, ts)
    assert np.abs(Fs.real + np.cos(Jv * ts) / 4).max() < 1e-13
    assert np.abs(Ft + np.cos(Jv * ts) / 4).max() < 1e-13
    Fs = dense.otoc_state(H, ch[11], ch[3], beta, ts, psi)
    assert np.abs(Fs + 0.25).max() < 1e-13
    Fs = dense.otoc_state(H, ch[0], ch[3], beta, ts, psi)
    assert np.abs(Fs - Fs[0]).max() < 1e-13


def test_otoc_trace_is_real_and_state_average_converges():
    """The trace is real (it equals its own conjugate by cyclicity) and the random-state
    estimator averages to it (typicality, supplement Sec. I)."""
    N = 10
    subs, J, _ = ensemble.sample_terms(N, 3, 11)
    H = dense.hamiltonian(N, subs, J)
    ch = dense.chis(N)
    ts = [0.0, 0.8, 2.0]
    Ft = dense.otoc_trace(H, ch[N - 1], ch[N - 2], 2.0, ts)
    assert np.abs(Ft.imag).max() < 1e-15
    Fs = np.mean([dense.otoc_state(H, ch[N - 1], ch[N - 2], 2.0, ts, haar.haar_state(N, 3, v))
                  for v in range(400)], axis=0)
    # spread of one estimate ~ |F| / sqrt(dim); 400 vectors -> ~ 0.25/sqrt(32*400)
    assert np.abs(Fs - Ft).max() < 0.02


def test_otoc_equals_sum_of_parity_block_chains():
    """The supplement's block form: <psi|O|psi> = <psi_U|O_UU|psi_U> + <psi_D|O_DD|psi_D>, where
    every Majorana maps U <-> D.  Computed with dense blocks and compared with the full space."""
    N = 12
    subs, J, _ = ensemble.sample_terms(N, 3, 13)
    H = dense.hamiltonian(N, subs, J)
    ch = dense.chis(N)
    h = H.shape[0] // 2
    HU, HD = dense.blocks(H)
    eU, eD = dense.Eig(HU), dense.Eig(HD)
    i, j, beta, t = 3, 8, 4.0, 1.3
    W, V = ch[i], ch[j]
    psi = haar.haar_state(N, 21, 0)
    full = dense.otoc_state(H, W, V, beta, [t], psi)[0]
    tot = 0
    for (eA, eB, WAB, VBA, ps) in (
            (eU, eD, W[:h, h:], V[h:, :h], psi[:h]),
            (eD, eU, W[h:, :h], V[:h, h:], psi[h:])):
        r = eA.expm_apply(-beta / 8, ps)
        r = VBA @ r
        r = eB.expm_apply(-(1j * t + beta / 4), r)
        r = WAB @ r
        r = eA.expm_apply(1j * t - beta / 4, r)
        r = VBA @ r
        r = eB.expm_apply(-(1j * t + beta / 4), r)
        r = WAB @ r
        r = eA.expm_apply(1j * t - beta / 8, r)
        tot += np.vdot(ps, r)
    assert abs(tot - full) < 1e-13


def test_normalise_curves():
    F = np.array([[-0.25 + 0.1j, -0.2], [-0.25 - 0.1j, -0.1]])
    raw, nrm, im = dense.normalise_curves(F)
    assert np.allclose(raw, [-0.25, -0.15]) and np.allclose(nrm, [1.0, 0.6]) and np.allclose(im, [0, 0])


# --------------------------------------------------------------------------- Green function
def test_green_function_single_term():
    """G(t) with gamma = gamma_n in the single term: gamma e^{-iHt} = e^{iHt} gamma, so
    G(t) = <psi|e^{(2it - beta) H}|psi> and Re G at beta = 0 is cos(Jt/2)."""
    N = 10
    Jv = 0.9
    H = dense.hamiltonian(N, [(0, 4, 6, 9)], [Jv])
    g = dense.gammas(N)
    psi = haar.haar_state(N, 8, 0)
    ts = np.linspace(0, 5, 11)
    G = dense.green_state(H, g[9], 0.0, ts, psi)
    assert np.abs(G.real - np.cos(Jv * ts / 2)).max() < 1e-13
    G0 = dense.green_state(H, g[9], 3.0, [0.0], psi)[0]
    assert abs(G0 - np.vdot(psi, dense.Eig(H).expm_apply(-3.0, psi))) < 1e-13


# --------------------------------------------------------------------------- Haar states
def test_haar_state_properties():
    N = 16
    psi = haar.haar_state(N, 1001, 0)
    d = 1 << (N // 2)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-14
    raw = haar.raw_amplitudes(1001, 0, np.arange(d, dtype=np.uint64))
    assert np.allclose(psi, raw / np.linalg.norm(raw))
    assert abs(haar.raw_norm2(N, 1001, 0, chunk=64) - np.sum(np.abs(raw) ** 2)) < 1e-9
    # independent vectors are nearly orthogonal; amplitudes are standard complex normals
    psi2 = haar.haar_state(N, 1001, 1)
    assert abs(np.vdot(psi, psi2)) < 5 / math.sqrt(d)
    big = haar.raw_amplitudes(5, 3, np.arange(1 << 18, dtype=np.uint64))
    n = big.size
    assert abs(big.real.mean()) < 5 / math.sqrt(n) and abs(big.imag.mean()) < 5 / math.sqrt(n)
    assert abs(big.real.var() - 1) < 5 * math.sqrt(2 / n) and abs(big.imag.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(np.mean(big.real * big.imag)) < 5 / math.sqrt(n)


# --------------------------------------------------------------------------- matrix-free rows
@pytest.mark.parametrize("N,blk", [(12, 0), (12, 1), (16, 0), (16, 1)])
def test_matfree_rows_match_dense(N, blk):
    subs, J, _ = ensemble.sample_terms(N, 4, 17)
    H = dense.hamiltonian(N, subs, J)
    Hb = dense.blocks(H)[blk]
    h = Hb.shape[0]
    x = np.random.default_rng(2).standard_normal(h) + 1j * np.random.default_rng(3).standard_normal(h)
    y = matfree.apply_rows(matfree.block_terms(N, subs, J, blk), lambda idx: x[idx.astype(np.int64)],
                           np.arange(h, dtype=np.uint64))
    assert np.abs(y - Hb @ x).max() < 1e-14


def test_matfree_hermitian_at_large_N():
    """<e_m, H e_n> = conj <e_n, H e_m> for sampled pairs at N = 48 (rows of unit vectors)."""
    N = 48
    subs, J, _ = ensemble.sample_terms(N, 4, 48)
    terms = matfree.block_terms(N, subs, J, 0)
    rng = np.random.default_rng(0)
    h = 1 << (N // 2 - 1)
    for _ in range(20):
        m = int(rng.integers(0, h))
        # H e_n has row m nonzero only for n = m ^ x_a: probe each such n
        for labels, _c in terms[:10]:
            n = m
            for q, lab in enumerate(labels):
                if lab in (pauli.X, pauli.Y):
                    n ^= 1 << q
            e = lambda idx, k=n: (idx == k).astype(np.complex128)
            hmn = matfree.apply_rows(terms, e, np.array([m], dtype=np.uint64))[0]
            f = lambda idx, k=m: (idx == k).astype(np.complex128)
            hnm = matfree.apply_rows(terms, f, np.array([n], dtype=np.uint64))[0]
            assert abs(hmn - np.conj(hnm)) < 1e-15


# --------------------------------------------------------------------------- Bernoulli ensemble
def test_bernoulli_dense_limit_keeps_every_subset():
    """p = 1 (k = C(N,4)/N) is the dense model: every 4-subset, in lexicographic order."""
    N = 10
    subs, J, sigma = ensemble.sample_terms_bernoulli(N, math.comb(N, 4) / N, 3)
    assert subs == list(itertools.combinations(range(N), 4))
    assert abs(sigma - math.sqrt(6.0 / N ** 3)) < 1e-15 and len(J) == len(subs)


def test_bernoulli_counts_and_coupling_moments():
    """K ~ Binomial(C(N,4), p) with p = kN / C(N,4); J ~ N(0, 3!/(p N^3))."""
    N, k = 14, 3.0
    C = math.comb(N, 4)
    p = k * N / C
    Ks, Js = [], []
    for seed in range(60):
        subs, J, sigma = ensemble.sample_terms_bernoulli(N, k, 1000 + seed)
        assert subs == sorted(set(subs)) and all(s[0] < s[1] < s[2] < s[3] < N for s in subs)
        Ks.append(len(subs))
        Js.extend(np.asarray(J) / sigma)
    mean, sd = C * p, math.sqrt(C * p * (1 - p))
    assert abs(np.mean(Ks) - mean) < 4 * sd / math.sqrt(len(Ks))
    assert abs(np.std(Ks) / sd - 1) < 0.35
    Js = np.asarray(Js)
    assert abs(Js.mean()) < 4 / math.sqrt(Js.size) and abs(Js.var() - 1) < 6 * math.sqrt(2 / Js.size)
    assert abs(sigma ** 2 * p * N ** 3 - 6.0) < 1e-12


def test_bernoulli_hamiltonian_invariants():
    N = 12
    subs, J, _ = ensemble.sample_terms_bernoulli(N, 6.0, 11)
    H = dense.hamiltonian(N, subs, J)
    d = H.shape[0]
    assert np.allclose(H, H.conj().T, atol=1e-14)
    assert abs(np.trace(H)) < 1e-12
    assert abs(np.trace(H @ H).real / d - np.sum(np.asarray(J) ** 2) / 16) < 1e-12


# --------------------------------------------------------------------------- spin operators
def test_from_xz_round_trip_and_textbook_products():
    """X^x Z^z from per-qubit labels: canonical() inverts it, and on one qubit X Z = -i Y
    is the product of the textbook matrices."""
    rng = np.random.default_rng(4)
    for _ in range(40):
        L = int(rng.integers(1, 7))
        x, z = int(rng.integers(0, 1 << L)), int(rng.integers(0, 1 << L))
        assert pauli.canonical(pauli.from_xz(L, x, z)) == (x, z, 0)
    Xm, Zm = pauli.SIGMA[pauli.X], pauli.SIGMA[pauli.Z]
    assert np.allclose(pauli.dense(pauli.from_xz(1, 1, 1)), Xm @ Zm)
    # two qubits: X^x Z^z = (X^x1 Z^z1) (x) (X^x0 Z^z0), qubit 1 the most significant
    M = pauli.dense(pauli.from_xz(2, 0b01, 0b11))
    assert np.allclose(M, np.kron(Zm, Xm @ Zm))


def test_operator_dense_is_linear():
    L = 3
    a = pauli.operator_dense(L, [1, 6], [2, 5], [0.5, -1j])
    b = pauli.operator_dense(L, [1], [2], [0.5]) + pauli.operator_dense(L, [6], [5], [-1j])
    assert np.allclose(a, b)


# ---------------------------------------------------------------- t*(N) and lambda_L

def test_crossing_time_piecewise_linear_is_exact():
    t = [0.0, 1.0, 2.0, 3.0]
    F = [1.0, 0.9, 0.7, 0.4]
    assert lyapunov.crossing_time(t, F, 0.8)[0] == pytest.approx(1.5, abs=1e-15)
    assert lyapunov.crossing_time(t, F, 0.85)[0] == pytest.approx(1.25, abs=1e-15)
    assert lyapunov.crossing_time(t, F, 0.9)[0] == 1.0           # a sample equal to F0
    assert math.isnan(lyapunov.crossing_time(t, F, 0.3)[0])      # never reached
    # the first crossing counts, not a later one after a revival
    assert lyapunov.crossing_time([0, 1, 2, 3, 4], [1.0, 0.7, 0.9, 0.6, 0.5], 0.8)[0] == pytest.approx(0.6667, abs=1e-4)


def test_crossing_time_error_of_a_straight_line():
    # F = 1 - s t with a constant standard error: sigma_t = sigma_F / s
    s, sig = 0.2, 0.01
    t = np.linspace(0.0, 3.0, 7)
    ts, err = lyapunov.crossing_time(t, 1.0 - s * t, 0.75, np.full(7, sig))
    assert ts == pytest.approx(1.25, abs=1e-14) and err == pytest.approx(sig / s, rel=1e-14)


def test_crossing_time_on_a_smooth_curve_within_interpolation_bound():
    # F = 1 - c1 e^{lam t}/N is concave, so the chord lies below it and crosses F0 first;
    # the time error is at most (h^2/8) max|F''| / min|F'| over the bracketing segment
    lam, c1, N, F0 = 1.1, 0.3, 30.0, 0.8
    exact = (math.log(N) + math.log((1 - F0) / c1)) / lam
    for h in (0.1, 0.05, 0.025, 0.0125):
        t = np.arange(0.0, 6.0 + h / 2, h)
        err = lyapunov.crossing_time(t, 1 - c1 * np.exp(lam * t) / N, F0)[0] - exact
        lo = math.floor(exact / h) * h
        bound = h * h / 8 * c1 * lam ** 2 * math.exp(lam * (lo + h)) / N / (c1 * lam * math.exp(lam * lo) / N)
        assert -bound <= err <= 0.0, (h, err, bound)


def test_inverse_slope_of_pure_logarithm_is_lambda():
    # t* = gamma_0 + log N / lambda: the log difference quotient gives lambda exactly
    lam, g0 = 0.73, -1.2
    N = np.array([14.0, 22.0, 30.0, 38.0, 46.0, 54.0])
    Nm, y, e = lyapunov.slope_points(N, g0 + np.log(N) / lam)
    assert np.allclose(y, lam, rtol=1e-13) and np.all(np.isnan(e))
    assert np.allclose(Nm, np.sqrt(N[:-1] * N[1:]))
    Nm4, _, _ = lyapunov.slope_points(N, g0 + np.log(N) / lam, dN=16)
    assert len(Nm4) == 4
    assert len(lyapunov.slope_points([14.0, 30.0], [1.0, 2.0])[0]) == 0   # no pair 8 apart


def test_fit_slope_two_parameters_matches_textbook_regression():
    rng = np.random.default_rng(4)
    x = 1.0 / np.array([17.0, 25.7, 33.8, 41.8, 49.8])
    sig = rng.uniform(0.01, 0.05, x.size)
    y = 0.8 - 3.0 * x + sig * rng.standard_normal(x.size)
    w = 1 / sig ** 2
    S, Sx, Sy, Sxx, Sxy = w.sum(), (w * x).sum(), (w * y).sum(), (w * x * x).sum(), (w * x * y).sum()
    D = S * Sxx - Sx ** 2
    r = lyapunov.fit_slope(1.0 / x, y, sig, a1=True, a2=False)
    assert r["lambda"] == pytest.approx((Sxx * Sy - Sx * Sxy) / D, rel=1e-12)
    assert r["alpha1"] == pytest.approx((S * Sxy - Sx * Sy) / D, rel=1e-12)
    assert r["lambda_err"] == pytest.approx(math.sqrt(Sxx / D), rel=1e-12)
    assert r["alpha1_err"] == pytest.approx(math.sqrt(S / D), rel=1e-12)
    assert r["dof"] == 3 and r["alpha2"] == 0.0


def test_fit_slope_constant_is_weighted_mean():
    y = np.array([0.7, 0.9, 0.8])
    sig = np.array([0.1, 0.2, 0.05])
    r = lyapunov.fit_slope([20.0, 30.0, 40.0], y, sig, a1=False)
    w = 1 / sig ** 2
    assert r["lambda"] == pytest.approx((w * y).sum() / w.sum(), rel=1e-13)
    assert r["lambda_err"] == pytest.approx(1 / math.sqrt(w.sum()), rel=1e-13)
    ru = lyapunov.fit_slope([20.0, 30.0, 40.0], y, None, a1=False)
    assert ru["lambda"] == pytest.approx(0.8, rel=1e-14)
    assert ru["lambda_err"] == pytest.approx(y.std(ddof=1) / math.sqrt(3), rel=1e-12)


@pytest.mark.parametrize("g1,g2", [(True, False), (False, True), (True, True)])
def test_fit_global_recovers_model_parameters(g1, g2):
    lam, g0, c1, c2 = 0.62, -0.9, 3.5 if g1 else 0.0, -40.0 if g2 else 0.0
    N = np.array([14.0, 22.0, 30.0, 38.0, 46.0, 54.0])
    ts = g0 + np.log(N) / lam * (1 + c1 / N + c2 / N ** 2)
    r = lyapunov.fit_global(N, ts, None, g1=g1, g2=g2)
    assert r["lambda"] == pytest.approx(lam, rel=1e-9) and r["gamma0"] == pytest.approx(g0, abs=1e-8)
    assert r["gamma1"] == pytest.approx(c1, abs=1e-6) and r["gamma2"] == pytest.approx(c2, abs=1e-4)


def test_fit_global_matches_nonlinear_least_squares():
    # the linear reparametrisation has the same optimum and, by first-order propagation,
    # the same covariance as a direct non-linear fit in (gamma_0, lambda, gamma_1)
    import scipy.optimize
    rng = np.random.default_rng(9)
    N = np.array([14.0, 22.0, 30.0, 38.0, 46.0, 54.0])
    sig = rng.uniform(0.02, 0.06, N.size)
    ts = -0.5 + np.log(N) / 0.7 * (1 + 2.0 / N) + sig * rng.standard_normal(N.size)
    r = lyapunov.fit_global(N, ts, sig, g1=True)
    f = lambda n, a, lam, c: a + np.log(n) / lam * (1 + c / n)            # noqa: E731
    p, cov = scipy.optimize.curve_fit(f, N, ts, p0=[0.0, 0.5, 0.0], sigma=sig, absolute_sigma=True,
                                     xtol=1e-15, ftol=1e-15, gtol=1e-15)
    e = np.sqrt(np.diag(cov))
    assert r["gamma0"] == pytest.approx(p[0], abs=1e-6) and r["lambda"] == pytest.approx(p[1], rel=1e-6)
    assert r["gamma1"] == pytest.approx(p[2], abs=1e-5)
    assert r["lambda_err"] == pytest.approx(e[1], rel=1e-4) and r["gamma1_err"] == pytest.approx(e[2], rel=1e-4)
    assert r["gamma0_err"] == pytest.approx(e[0], rel=1e-4)
    chi2 = float((((ts - f(N, *p)) / sig) ** 2).sum())
    assert r["chi2"] == pytest.approx(chi2, rel=1e-6)


def test_lyapunov_chain_on_curves_with_the_scaling_form():
    # F_N(t) = 1 - c1 e^{lambda t} / N (the form of Eqs. (3)-(4) with g0 = 1, g linear):
    # t*(N) = (log N + log((1 - F0)/c1)) / lambda, so both fits return lambda
    lam, c1 = 0.9, 0.25
    t = np.arange(0.0, 8.0, 0.01)
    N = np.array([14.0, 22.0, 30.0, 38.0, 46.0, 54.0])
    for F0 in (0.75, 0.85):
        ts = np.array([lyapunov.crossing_time(t, 1 - c1 * np.exp(lam * t) / n, F0)[0] for n in N])
        assert np.allclose(ts, (np.log(N) + math.log((1 - F0) / c1)) / lam, atol=2e-5)
        Nm, y, _ = lyapunov.slope_points(N, ts)
        assert lyapunov.fit_slope(Nm, y)["lambda"] == pytest.approx(lam, rel=1e-3)
        g = lyapunov.fit_global(N, ts, g1=False)
        assert g["lambda"] == pytest.approx(lam, rel=1e-4)
        assert g["gamma0"] == pytest.approx(math.log((1 - F0) / c1) / lam, abs=1e-3)


def test_ensemble_mean_and_standard_error():
    import scipy.stats
    rng = np.random.default_rng(2)
    rows = 1 + 0.1 * rng.standard_normal((7, 5))
    m, s = lyapunov.ensemble_mean(rows)
    assert np.allclose(m, rows.mean(axis=0)) and np.allclose(s, scipy.stats.sem(rows, axis=0), rtol=1e-13)
    assert np.all(lyapunov.ensemble_mean(rows[:1])[1] == 0.0)


# --------------------------------------------------------------------------- commuting terms
# Two sets of 4-subsets of range(12) whose gamma products commute pairwise (every pair shares
# 0 or 2 indices), each with a term holding a pair (i, j) that no other term touches; the
# second puts the pair on chi_{N-1}, chi_{N-2}.
COMMUTING_N12 = [
    ([(0, 1, 2, 3), (2, 3, 4, 5), (4, 5, 6, 7), (6, 7, 8, 9), (2, 3, 8, 9), (8, 9, 10, 11), (4, 5, 10, 11)], (0, 1)),
    ([(0, 1, 2, 3), (0, 1, 8, 9), (2, 3, 4, 5), (4, 5, 6, 7), (6, 7, 8, 9), (8, 9, 10, 11)], (11, 10)),
]


def test_apply_string_matches_dense_kron():
    """P v by one 2x2 contraction per tensor axis equals the dense Kronecker matrix times v."""
    rng = np.random.default_rng(4)
    n = 5
    for _ in range(20):
        s = (tuple(int(a) for a in rng.integers(0, 4, n)), int(rng.integers(0, 4)))
        v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        assert np.abs(commuting.apply_string(s, v) - pauli.dense(s) @ v).max() < 1e-14


def test_commutation_rule_matches_dense_products():
    """gamma products of two 4-subsets commute iff the subsets share an even number of indices."""
    N = 10
    g = dense.gammas(N)
    rng = np.random.default_rng(8)
    seen = set()
    for _ in range(60):
        a, b = (tuple(sorted(rng.choice(N, 4, replace=False))) for _ in range(2))
        Pa, Pb = g[a[0]] @ g[a[1]] @ g[a[2]] @ g[a[3]], g[b[0]] @ g[b[1]] @ g[b[2]] @ g[b[3]]
        comm = np.abs(Pa @ Pb - Pb @ Pa).max() < 1e-12
        assert comm == commuting.commute(a, b)
        seen.add(comm)
    assert seen == {True, False}


@pytest.mark.parametrize("case", range(len(COMMUTING_N12)))
def test_commuting_expm_matches_eigendecomposition(case):
    """prod_b (cosh(z J_b/4) + sinh(z J_b/4) P_b) v equals e^{zH} v from the dense H by eigh."""
    N = 12
    subs, _ = COMMUTING_N12[case]
    assert commuting.all_commute(subs)
    J = np.random.default_rng(case).standard_normal(len(subs)) * 1.3
    eg = dense.Eig(dense.hamiltonian(N, subs, J))
    v = haar.haar_state(N, 31, case)
    for z in (-2.5j, -1.7, 0.8 - 3.0j):
        assert np.abs(commuting.expm_apply(N, subs, J, z, v) - eg.expm_apply(z, v)).max() < 1e-12


@pytest.mark.parametrize("case", range(len(COMMUTING_N12)))
@pytest.mark.parametrize("beta", [0.0, 3.0])
def test_commuting_otoc_matches_dense_chain(case, beta):
    """The closed form of the random-state OTOC equals the dense full-space chain of the
    supplement's estimator (itself pinned above) for commuting terms and a lone pair."""
    N = 12
    subs, (i, j) = COMMUTING_N12[case]
    J = np.random.default_rng(10 + case).standard_normal(len(subs)) * 1.3
    H = dense.hamiltonian(N, subs, J)
    ch = dense.chis(N)
    psi = haar.haar_state(N, 7, case)
    ts = [0.0, 0.3, 1.1, 2.6, 5.0]
    ref = dense.otoc_state(H, ch[i], ch[j], beta, ts, psi)
    got = commuting.otoc_state(N, subs, J, i, j, beta, ts, psi)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
    if beta == 0.0:
        assert abs(got[0] + 0.25) < 1e-13


def test_commuting_closed_form_refuses_what_it_does_not_cover():
    N = 12
    subs, (i, j) = COMMUTING_N12[0]
    J = np.ones(len(subs))
    psi = haar.haar_state(N, 1, 0)
    with pytest.raises(ValueError):
        commuting.expm_apply(N, subs + [(0, 4, 6, 8)], list(J) + [1.0], -1.0, psi)   # shares 1 with (0,1,2,3)
    with pytest.raises(ValueError):
        commuting.otoc_state(N, subs, J, 2, 3, 0.0, [0.0], psi)                      # 2, 3 in several terms


@pytest.mark.parametrize("N,K,seed,i,j", [(40, 6, 91, 39, 5), (40, 8, 188076, 39, 19)])
def test_commuting_realisations_used_by_the_gpu_tests(N, K, seed, i, j):
    """The seeds of the large-N commuting checks draw pairwise commuting terms with (i, j) a
    lone pair, and at beta = 0, t = 0 the closed form is -1/4."""
    subs, J, _ = ensemble.sample_terms(N, K / N, seed)
    assert len(subs) == K and commuting.all_commute(subs)
    assert commuting.lone_pair_term(subs, i, j) >= 0


def test_splitmix64_reference_streams():
    """The oracle's SplitMix64 reproduces the generator's published reference outputs
    (tests/golden/splitmix64_reference.txt): seed 0 and seed 1234567, five outputs each."""
    from oracle.splitmix import SplitMix64
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_reference.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for row in rows:
        g = SplitMix64(int(row[0]))
        assert [g.next() for _ in range(len(row) - 1)] == [int(v) for v in row[1:]]
