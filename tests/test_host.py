"""Host-side library logic, no GPU: the C ABI loads and exports every declared symbol,
the term tables equal the oracle's bit for bit, the small exponential matches a library
routine, and argument errors come back as status codes."""
import math
import os
import re

import numpy as np
import pytest
import scipy.linalg

import paper_2311_00639_amd as syk
from oracle import ensemble, lyapunov, pauli

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "syk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(syk_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(syk.library_path())
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("N,k,seed", [(6, 1, 5), (8, 1 / 8, 3), (10, 21, 2), (16, 4, 1), (24, 2, 3000),
                                      (48, 4, 48), (56, 4, 56), (64, 8, 50000)])
def test_term_tables_bit_exact(N, k, seed):
    """Subsets, J (bitwise), x/z masks and block phases equal the oracle's, which are
    derived by qubit-by-qubit Pauli products rather than XOR algebra."""
    h = syk.create_hamiltonian(N, 4, k, seed)
    T = h.terms()
    inf = h.info()
    subs, J, sigma = ensemble.sample_terms(N, k, seed)
    assert inf["K"] == len(subs) == ensemble.n_terms(N, k)
    assert [tuple(int(v) for v in r) for r in T["ijkl"]] == subs
    assert np.array_equal(T["J"], np.array(J))             # bitwise
    assert inf["sigma"] == sigma and inf["L"] == N // 2 - 1 and inf["block_dim"] == 1 << (N // 2 - 1)
    assert abs(inf["p"] - len(subs) / math.comb(N, 4)) < 1e-18
    for a, s in enumerate(subs):
        (lu, pu), (ld, pd) = pauli.term_blocks(N, s)
        xu, zu, wu = pauli.canonical((lu, pu))
        xd, zd, wd = pauli.canonical((ld, pd))
        assert (xu, zu) == (xd, zd)
        assert int(T["xmask"][a]) == xu and int(T["zmask"][a]) == zu
        assert int(T["phase_U"][a]) == wu and int(T["phase_D"][a]) == wd


def test_tridiag_expm_matches_scipy():
    rng = np.random.default_rng(4)
    for n in (1, 2, 5, 30, 60):
        a = rng.standard_normal(n)
        b = np.abs(rng.standard_normal(n - 1)) + 0.1
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        for z in (-0.3j, 2.0 - 5j, -4.0, 0.5 + 0.5j):
            ref = scipy.linalg.expm(z * T)[:, 0]
            got = syk.tridiag_expm(a, b, z)
            assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_tridiag_expm_degenerate():
    """Repeated eigenvalues and a zero off-diagonal (split matrix)."""
    a = np.array([1.0, 1.0, -2.0, 0.5])
    b = np.array([0.0, 0.3, 0.0])
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ref = scipy.linalg.expm(-1.5j * T)[:, 0]
    assert np.abs(syk.tridiag_expm(a, b, -1.5j) - ref).max() < 1e-13


@pytest.mark.parametrize("args,status", [
    ((7, 4, 4.0, 1), syk.SykError),
    ((66, 4, 4.0, 1), syk.SykError),
    ((16, 2, 4.0, 1), syk.SykError),
    ((16, 4, 0.0, 1), syk.SykError),
    ((8, 4, 100.0, 1), syk.SykError),      # K = 800 > C(8,4) = 70
])
def test_create_rejects_bad_arguments(args, status):
    with pytest.raises(status) as e:
        syk.create_hamiltonian(*args)
    assert e.value.status in (1, 2)


def test_error_codes():
    with pytest.raises(syk.SykError) as e:
        syk.create_hamiltonian(16, 3, 4.0, 1)
    assert e.value.status == 2                      # SYK_EUNSUPPORTED
    with pytest.raises(syk.SykError) as e:
        syk.workspace_bytes(16, 1, syk.C64)
    assert e.value.status == 1
    with pytest.raises(syk.SykError):
        syk.tridiag_expm(np.zeros(0), np.zeros(0), 1.0)


def test_workspace_bytes_model():
    """(m + 5) vectors (Krylov basis m+1, chain vectors l, r2, r4, tmp) plus scalars; the
    supplement's minimum for Krylov dimension v is (v + 3) vectors."""
    for N, m, dt, es in ((56, 60, syk.C64, 8), (48, 40, syk.C128, 16), (16, 30, syk.C128, 16)):
        b = syk.workspace_bytes(N, m, dt)
        vec = (1 << (N // 2 - 1)) * es
        assert (m + 5) * vec <= b <= (m + 5) * vec + 8 * 1024 * 1024


def test_sigma_and_sumJ2_consistent():
    h = syk.create_hamiltonian(20, 4, 3, 11)
    inf = h.info()
    T = h.terms()
    assert abs(inf["sum_J2"] - float(np.sum(T["J"] ** 2))) < 1e-14


@pytest.mark.parametrize("N,k,dt", [(40, 4, syk.C64), (48, 4, syk.C128), (56, 4, syk.C64), (64, 8, syk.C64)])
def test_plan_describe(N, k, dt):
    """Planner invariants (host-only): bijective tile map and complete grouping are checked
    inside the call; the planner's layout groups no worse than the standard order."""
    h = syk.create_hamiltonian(N, 4, k, N)
    auto = syk.plan_describe(h, 0, dt, -1)
    std = syk.plan_describe(h, 0, dt, 0)
    assert auto["tiled"] == 1 and std["tiled"] == 1
    L = N // 2 - 1
    assert auto["n_tiles"] == 1 << (L - auto["tile_bits"]) and 0 <= auto["rot"] < L
    assert 1 <= auto["classes_gpu"] <= auto["classes_xcd"] <= auto["n_groups"] <= h.info()["K"]
    cost = lambda d: d["n_groups"] + 2 * d["classes_xcd"] + 0.5 * d["classes_gpu"]
    assert cost(auto) <= cost(std) + 1e-9
    # the D block shares the x masks: same grouping
    assert syk.plan_describe(h, 1, dt, auto["rot"])["n_groups"] == auto["n_groups"]


def test_plan_describe_small_block_not_tiled():
    h = syk.create_hamiltonian(16, 4, 4, 1)
    assert syk.plan_describe(h, 0, syk.C64)["tiled"] == 0


def test_batch_argument_checks_without_gpu():
    """Argument errors of the batched call are reported before any device work."""
    ts = [0.0, 1.0]
    for items, kw in [([(34, 2, 1, 33, 32, 1)], {}), ([(24, 2, 1, 5, 5, 1)], {}), ([(24, 2, 1, 23, 22, 1)], {"m": 61}),
                      ([(23, 2, 1, 22, 21, 1)], {}), ([(24, 2, 1, 23, 22, 1)], {"nvec": 0})]:
        with pytest.raises(syk.SykError) as e:
            syk.otoc_batch(items, 1.0, ts, **kw)
        assert e.value.status == 1
    with pytest.raises(syk.SykError) as e:
        syk.otoc_batch([(24, 2, 1, 23, 22, 1)], 1.0, [1.0, 0.5])
    assert e.value.status == 1


@pytest.mark.parametrize("dt", [syk.C64, syk.C128])
def test_plan_describe_every_variant_N56(dt):
    """Every compiled tiled variant plans the N = 56 block: the consistency checks inside
    the call (tiles covered once, every term applied once per tile) pass, and holding
    several tiles per workgroup streams fewer partner tiles per output tile."""
    h = syk.create_hamiltonian(56, 4, 4, 56)
    per_tile = {}
    for v in range(14):
        syk.select_variant(h, dt, v)
        d = syk.plan_describe(h, 0, dt, -1)
        assert d["variant"] == v and d["tiled"] == 1
        assert d["n_tiles"] == 1 << (27 - d["tile_bits"])
        assert d["n_groups"] <= d["n_partners"] <= d["n_groups"] * d["tiles_per_wg"]
        per_tile.setdefault(d["tile_bits"], {})[d["tiles_per_wg"]] = d["n_partners"] / d["tiles_per_wg"]
    for bt, m in per_tile.items():
        for tpw, p in m.items():
            if tpw > 1:
                assert p < m.get(1, 1e9)


@pytest.mark.parametrize("N,k,seed", [(12, 5.0, 3), (16, 4.0, 7), (16, 1820 / 16, 1), (20, 2.5, 9)])
def test_bernoulli_tables_match_oracle_bitwise(N, k, seed):
    """The library's Bernoulli draw (subsets, J, sigma, K) equals the oracle's bit for bit."""
    h = syk.create_hamiltonian(N, 4, k, seed, syk.BERNOULLI)
    T = h.terms()
    subs, J, sigma = ensemble.sample_terms_bernoulli(N, k, seed)
    assert h.info()["K"] == len(subs)
    assert np.array_equal(T["ijkl"], np.asarray(subs, dtype=np.int32))
    assert np.array_equal(T["J"], np.asarray(J)) and h.info()["sigma"] == sigma


def test_bernoulli_argument_errors():
    for args in [(16, 4, 200.0, 1, syk.BERNOULLI), (16, 4, 2.0, 1, 7)]:
        with pytest.raises(syk.SykError) as e:
            syk.create_hamiltonian(*args)
        assert e.value.status == 1


def _random_op(L, n, rng):
    x = rng.integers(0, 1 << L, n).astype(np.uint64)
    z = rng.integers(0, 1 << L, n).astype(np.uint64)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return x, z, c


def test_operator_algebra_matches_dense():
    """Products, linear combinations and adjoints of Pauli sums (host) equal the dense
    matrix operations of the oracle's Kronecker-built matrices."""
    rng = np.random.default_rng(21)
    L = 4
    xa, za, ca = _random_op(L, 7, rng)
    xb, zb, cb = _random_op(L, 5, rng)
    A = syk.Operator(L, xa, za, ca)
    B = syk.Operator(L, xb, zb, cb)
    dA = pauli.operator_dense(L, xa, za, ca)
    dB = pauli.operator_dense(L, xb, zb, cb)
    dense_of = lambda op: pauli.operator_dense(L, *op.terms())
    assert np.allclose(dense_of(A), dA, atol=1e-13)
    assert np.allclose(dense_of(A @ B), dA @ dB, atol=1e-12)
    assert np.allclose(dense_of(A.combine(B, 0.5 - 2j, 3.0)), (0.5 - 2j) * dA + 3.0 * dB, atol=1e-12)
    assert np.allclose(dense_of(A.adjoint()), dA.conj().T, atol=1e-13)
    H = A + A.adjoint()
    assert H.is_hermitian() and not A.is_hermitian()
    # merged terms: A - A has no terms
    assert (A - A).terms()[0].size == 0


def test_operator_argument_errors():
    with pytest.raises(syk.SykError):
        syk.Operator(3, [8], [0], [1.0])           # beyond qubit L-1
    with pytest.raises(syk.SykError):
        syk.Operator(0, [], [], [])
    with pytest.raises(syk.SykError):
        syk.Operator(3, [1], [0], [float("nan")])
    with pytest.raises(syk.SykError):
        syk.Operator(3, [1], [0], [1.0]) @ syk.Operator(4, [1], [0], [1.0])


# ---------------------------------------------------------------- t*(N) and lambda_L (host code)

def test_crossing_time_matches_oracle():
    rng = np.random.default_rng(11)
    for trial in range(30):
        nt = int(rng.integers(2, 40))
        t = np.cumsum(rng.uniform(0.0, 0.3, nt))
        F = 1.0 - np.cumsum(rng.uniform(-0.02, 0.08, nt))
        err = rng.uniform(0.0, 0.01, nt)
        F0 = float(rng.uniform(0.5, 1.0))
        a = syk.crossing_time(t, F, F0, err)
        b = lyapunov.crossing_time(t, F, F0, err)
        if math.isnan(b[0]):
            assert math.isnan(a[0]) and math.isnan(a[1])
        else:
            assert a[0] == pytest.approx(b[0], rel=1e-14, abs=1e-14)
            assert a[1] == pytest.approx(b[1], rel=1e-12, abs=1e-15)
    ts, e = syk.crossing_time([0.0, 1.0, 2.0], [1.0, 0.9, 0.7], 0.8)
    assert ts == pytest.approx(1.5) and math.isnan(e)


@pytest.mark.parametrize("terms", [0, 1, 2, 3])
@pytest.mark.parametrize("weighted", [False, True])
def test_lyapunov_fits_match_oracle(terms, weighted):
    rng = np.random.default_rng(terms + 5 * weighted)
    N = np.array([54.0, 14.0, 30.0, 22.0, 46.0, 38.0, 62.0])     # unsorted on purpose
    sig = rng.uniform(0.02, 0.06, N.size)
    ts = -0.4 + np.log(N) / 0.65 * (1 + 1.5 / N) + sig * rng.standard_normal(N.size)
    e = sig if weighted else None
    a = syk.lyapunov_fit(N, ts, e, method=syk.FIT_SLOPE, terms=terms)
    Nm, y, ye = lyapunov.slope_points(N, ts, e)
    b = lyapunov.fit_slope(Nm, y, ye if weighted else None, a1=bool(terms & 1), a2=bool(terms & 2))
    for key in ("lambda", "lambda_err", "alpha1", "alpha1_err", "alpha2", "alpha2_err", "chi2"):
        assert a[key] == pytest.approx(b[key], rel=1e-9, abs=1e-12), key
    assert a["dof"] == b["dof"] and a["n_points"] == len(y) == 6
    order = np.argsort(a["points"][0])
    assert np.allclose(a["points"][0][order], np.sort(Nm)) and np.allclose(a["points"][1][order], y[np.argsort(Nm)])
    a = syk.lyapunov_fit(N, ts, e, method=syk.FIT_GLOBAL, terms=terms)
    b = lyapunov.fit_global(N, ts, e, g1=bool(terms & 1), g2=bool(terms & 2))
    for key in ("lambda", "lambda_err", "gamma0", "gamma0_err", "gamma1", "gamma1_err", "gamma2", "gamma2_err",
                "chi2"):
        assert a[key] == pytest.approx(b[key], rel=1e-8, abs=1e-12), key
    assert a["dof"] == b["dof"] == N.size - 2 - bin(terms).count("1")


def test_lyapunov_fit_recovers_scaling_form_exactly():
    lam = 0.81
    N = np.array([22.0, 30.0, 38.0, 46.0, 54.0])
    r = syk.lyapunov_fit(N, 0.3 + np.log(N) / lam, method=syk.FIT_SLOPE, terms=0)
    assert r["lambda"] == pytest.approx(lam, rel=1e-13) and r["lambda_err"] == pytest.approx(0.0, abs=1e-12)
    r = syk.lyapunov_fit(N, 0.3 + np.log(N) / lam * (1 - 2.0 / N), method=syk.FIT_GLOBAL, terms=1)
    assert r["lambda"] == pytest.approx(lam, rel=1e-11) and r["gamma1"] == pytest.approx(-2.0, abs=1e-8)
    assert r["gamma0"] == pytest.approx(0.3, abs=1e-9)


def test_lyapunov_fit_errors():
    N = np.array([14.0, 22.0, 30.0])
    ts = np.array([1.0, 1.5, 1.8])
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit(N, ts, method=syk.FIT_SLOPE, terms=3)               # 2 pairs, 3 parameters
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit([14.0, 30.0], [1.0, 2.0], method=syk.FIT_SLOPE)      # no pair 8 apart
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit(N, [1.0, 1.0, 1.8], method=syk.FIT_SLOPE)            # equal t* in a pair
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit(N, [1.0, np.nan, 1.8], method=syk.FIT_GLOBAL)
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit(N, ts, [0.1, 0.0, 0.1], method=syk.FIT_GLOBAL)        # zero error
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit(N, ts, method=5)
    with pytest.raises(syk.SykError):
        syk.lyapunov_fit([30.0, 30.0, 30.0], ts, method=syk.FIT_GLOBAL, terms=0)   # dependent columns
    r = syk.lyapunov_fit(N, ts, method=syk.FIT_GLOBAL, terms=1)                # dof = 0: no errors
    assert r["dof"] == 0 and math.isnan(r["lambda_err"])
    with pytest.raises(syk.SykError):
        syk.crossing_time([0.0, 1.0], [1.0, 0.5], math.inf)
    with pytest.raises(syk.SykError):
        syk.crossing_time([1.0, 0.0], [1.0, 0.5], 0.8)
    with pytest.raises(syk.SykError):
        syk.crossing_time([0.0], [1.0], 0.8)


def test_otoc_ensemble_argument_checks_without_gpu():
    ts = [0.0, 1.0]
    with pytest.raises(syk.SykError):
        syk.otoc_ensemble(24, 4, 1, 0, 23, 22, 1.0, ts)            # n_real < 1
    with pytest.raises(syk.SykError):
        syk.otoc_ensemble(24, 4, 1, 2, 23, 23, 1.0, ts)            # i == j
    with pytest.raises(syk.SykError) as e:
        syk.otoc_ensemble(40, 4, 1, 2, 39, 38, 1.0, ts, path=0)    # batched path cannot serve N = 40
    assert e.value.status == 2
    with pytest.raises(syk.SykError):
        syk.otoc_ensemble(24, 4, 1, 2, 23, 22, 1.0, ts, ensemble=7)


def test_full_sector_argument_checks_without_gpu():
    """SYK_FULL takes 2^(N/2) amplitudes and is refused for operator handles, before any
    device work."""
    import ctypes as ct
    from paper_2311_00639_amd import _lib
    h = syk.create_hamiltonian(12, 4, 3, 1)
    n = 1 << 5
    st = _lib._lib.syk_apply_H(h.handle, syk.FULL, syk.C64, ct.c_void_p(1), ct.c_void_p(2), n, 1, n, None)
    assert st == 1                                                   # EINVAL: 2^L is not the full size
    op = syk.Operator(4, [1], [0], [1.0]).to_hamiltonian()
    st = _lib._lib.syk_apply_H(op.handle, syk.FULL, syk.C64, ct.c_void_p(1), ct.c_void_p(2), 1 << 5, 1, 1 << 5, None)
    assert st == 2                                                   # EUNSUPPORTED


def test_planner_rotation_is_cached_per_precision_and_variant():
    """The planner's layout is remembered per (precision, variant): planning every variant
    in one precision first leaves the other precision's choices unchanged, and each equals
    the choice a fresh handle makes for that variant alone."""
    mixed = syk.create_hamiltonian(56, 4, 4, 57)
    for first, second in [(syk.C128, syk.C64), (syk.C64, syk.C128)]:
        for dt in (first, second):
            for v in range(14):
                syk.select_variant(mixed, dt, v)
                got = syk.plan_describe(mixed, 0, dt, -1)["rot"]
                fresh = syk.create_hamiltonian(56, 4, 4, 57)
                syk.select_variant(fresh, dt, v)
                assert got == syk.plan_describe(fresh, 0, dt, -1)["rot"], (dt, v)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more, it exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_gather_kernel_groups_terms_by_x_mask():
    """Blocks below the tiled size: the gather kernel loads each distinct x mask once per
    amplitude; its group count is the number of distinct masks of the block's terms, about
    K / 19 for dense SYK and about K for sparse Hamiltonians."""
    for N, k, ens, dense in [(16, math.comb(16, 4) / 16, syk.BERNOULLI, True), (30, math.comb(30, 4) / 30,
                                                                            syk.BERNOULLI, True),
                             (16, 4, syk.EXACT_K, False), (30, 40, syk.EXACT_K, False)]:
        h = syk.create_hamiltonian(N, 4, k, 3, ens)
        masks = len(set(int(v) for v in h.terms()["xmask"]))
        for blk in (0, 1):
            d = syk.plan_describe(h, blk, syk.C64, -1)
            assert d["tiled"] == 0 and d["n_groups"] == masks
        assert (h.info()["K"] >= 10 * masks) == dense


def test_binding_refuses_bad_vectors_before_the_library():
    """The binding checks every state-vector tensor (dtype, agreement of dtypes, contiguity,
    length, device) before a pointer reaches the library: no kernel ever sees a short,
    strided, mismatched or host buffer."""
    import torch
    h = syk.create_hamiltonian(12, 4, 3, 1)
    n = 1 << 5
    good = torch.zeros(n, dtype=torch.complex64)                     # right shape, but on the host
    with pytest.raises(TypeError, match="GPU"):
        syk.apply_H(h, 0, good, good.clone())
    with pytest.raises(ValueError, match="elements"):
        syk.apply_H(h, 0, good, torch.zeros(n - 1, dtype=torch.complex64))
    with pytest.raises(ValueError, match="elements"):
        syk.apply_H(h, 0, torch.zeros(2, n, dtype=torch.complex64), torch.zeros(2, n, dtype=torch.complex64),
                    nvec=2, ld=n + 8)                                # (nvec - 1) ld + n > 2 n
    with pytest.raises(TypeError, match="dtype"):
        syk.apply_H(h, 0, good, torch.zeros(n, dtype=torch.complex128))
    with pytest.raises(TypeError):
        syk.apply_H(h, 0, good, torch.zeros(n, dtype=torch.float32))
    with pytest.raises(ValueError, match="contiguous"):
        syk.apply_H(h, 0, good, torch.zeros(2 * n, dtype=torch.complex64)[::2])
    with pytest.raises(ValueError, match="elements"):
        syk.krylov_expm(h, syk.FULL, -1j, good, good.clone())        # the full space needs 2^(N/2)
    with pytest.raises(TypeError, match="GPU"):
        syk.krylov_expm(h, 0, -1j, good, good.clone())
    with pytest.raises(ValueError, match="elements"):
        syk.haar_state(12, 1, 0, good, torch.zeros(3, dtype=torch.complex64))
    with pytest.raises(TypeError, match="dtype"):
        syk.apply_majorana(12, 3, 0, good, torch.zeros(n, dtype=torch.complex128))
    with pytest.raises(TypeError, match="torch tensor"):
        syk.apply_majorana(12, 3, 0, good, 12345)


def _rotr(v, s, L):
    s %= L
    m = (1 << L) - 1
    return ((v >> s) | (v << (L - s))) & m if s else v


@pytest.mark.parametrize("N,k,blk,dt", [(40, 4.0, 0, "c64"), (56, 4.0, 0, "c64"), (56, 8.0, 1, "c64"),
                                        (44, 4.0, 0, "c128"), (52, 4.0, 1, "c128")])
def test_control_blocks_hold_every_term_plain_records_first(N, k, blk, dt):
    """The control blocks of variant 10 (complex64: 2^13-amplitude tiles, 8 registers per
    thread; complex128: 2^12-amplitude tiles, 4 registers; 4 tiles per workgroup), decoded
    word by word and compared with the Hamiltonian's own block terms (J, x and z masks,
    phases): every (tile, term) pair appears once, with its layout-rotated masks, register
    sign mask and coefficient, in the right phase; the records that touch no register bit
    lead each run and lane 62 counts exactly them."""
    import numpy as np
    code = syk.C64 if dt == "c64" else syk.C128
    h = syk.create_hamiltonian(N, 4, k, N)
    syk.select_variant(h, code, 10)
    d = syk.plan_describe(h, blk, code, -1)
    bt, rb = (13, 3) if dt == "c64" else (12, 2)
    assert d["tiled"] == 1 and d["tile_bits"] == bt and d["tiles_per_wg"] == 4
    blocks = syk.plan_blocks(h, blk, code, -1)
    L = N // 2 - 1
    tpw, s = 4, d["rot"]
    rd = 4 if dt == "c64" else 5                  # words per record
    rec_max = 60 // rd
    tb = bt - rb
    tmask, rmask = (1 << tb) - 1, (1 << rb) - 1
    # expected records from the terms: the coefficient folds J/4, the sign of i^p and the
    # parity of x & z (the sign read from the source index); odd p is the i phase
    T = h.terms()
    phase = T["phase_U"] if blk == 0 else T["phase_D"]
    want = {}
    n_plain = 0
    for a in range(len(T["J"])):
        x, z = int(T["xmask"][a]), int(T["zmask"][a])
        p = (int(phase[a]) + 2 * (bin(x & z).count("1") & 1)) & 3
        cd = 0.25 * T["J"][a] * (-1.0 if p in (2, 3) else 1.0)
        cw = tuple(int(v) for v in np.frombuffer((np.float32(cd) if dt == "c64" else np.float64(cd)).tobytes(),
                                                  dtype=np.uint32))
        xr_, zr_ = _rotr(x, s, L), _rotr(z, s, L)
        xr = (xr_ >> tb) & rmask
        zr = (zr_ >> tb) & rmask
        sm = sum(((bin(q & zr).count("1") & 1) << q) for q in range(rmask + 1))
        key = ((xr_ & tmask) | (xr << 24), (zr_ & tmask) | (sm << 24), zr_ >> bt) + cw + (p & 1,)
        want[key] = want.get(key, 0) + tpw
        n_plain += tpw if (xr == 0 and zr == 0) else 0
    got = {}
    plain_total = 0
    for b in blocks[:-1]:
        cnt, pln = int(b[60]), int(b[62])
        j = 0
        for i in range(tpw):
            for imag in (0, 1):
                n = (cnt >> (8 * i + 4 * imag)) & 15
                pre = (pln >> (8 * i + 4 * imag)) & 15
                assert pre <= n
                for r in range(n):
                    w = [int(v) for v in b[rd * j:rd * j + rd]]
                    is_plain = (w[0] >> 24) == 0 and (w[1] >> 24) == 0
                    assert is_plain == (r < pre), (i, imag, r, pre, n)
                    key = tuple(w) + (imag,)
                    got[key] = got.get(key, 0) + 1
                    j += 1
                plain_total += pre
        assert j <= rec_max
        assert not b[rd * j:60].any()         # nothing after the last record
    assert got == want
    assert plain_total == n_plain
    h.close()
