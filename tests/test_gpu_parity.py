"""GPU parity: the HIP path (through the C ABI) against the oracle on the same seeded inputs.

Tolerances:
* complex128 apply_H: ||y - y_ref|| / ||y_ref|| <= 1e-10 (stated target; observed ~1e-16).
* complex64 apply_H: the input is rounded to complex64 first and the oracle evaluates the
  rounded input in float64, so only the float32 accumulation of <= K terms differs:
  per row |err| <= K u sum_a |c_a x[m^x_a]| with u = 2^-24; the test uses the norm-wise
  bound 4e-6 relative and the row-wise bound K u sum_a |c_a x|.
* Krylov propagators: requested tolerance 1e-12 (c128) or 1e-7 (c64) per propagation.
* OTOC: 1e-9 absolute on F (c128), 1e-5 absolute on F (c64 states, double reductions).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2311_00639_amd as syk  # noqa: E402
from oracle import dense, ensemble, haar, matfree, pauli  # noqa: E402
from tests import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


def dev(a, dtype):
    t = torch.from_numpy(np.ascontiguousarray(a.astype(np.complex128)))
    return t.to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy().astype(np.complex128)


def cdt(dt):
    return torch.complex64 if dt == syk.C64 else torch.complex128


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------------- apply_H, small N
@pytest.mark.parametrize("N,k,seed", [(6, 1, 5), (10, 21, 2), (12, 3, 7), (16, 4, 1), (20, 4, 20)])
@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
@pytest.mark.parametrize("blk", [0, 1])
def test_apply_h_vs_dense(N, k, seed, dt, blk):
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    Hb = dense.blocks(dense.hamiltonian(N, subs, J))[blk]
    h = syk.create_hamiltonian(N, 4, k, seed)
    n = Hb.shape[0]
    x = inputs.complex_vector(n, seed + 100)[0]
    xd = dev(x, cdt(dt))
    xr = host(xd)                           # the rounded input the GPU sees
    yd = torch.empty_like(xd)
    syk.apply_H(h, blk, xd, yd)
    y = host(yd)
    yref = Hb @ xr
    if dt == syk.C128:
        assert rel(y, yref) <= 1e-10
        assert np.abs(y - yref).max() <= 1e-13 * np.abs(yref).max()
    else:
        assert rel(y, yref) <= 4e-6
        bound = len(subs) * U24 * (np.abs(Hb) @ np.abs(xr)) + 1e-30
        assert np.all(np.abs(y - yref) <= bound)


def test_apply_h_many_vectors_with_stride():
    """nvec > 1 with a leading dimension larger than the block (a ragged stride)."""
    N, k, seed = 14, 3, 9
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    HU = dense.blocks(dense.hamiltonian(N, subs, J))[0]
    h = syk.create_hamiltonian(N, 4, k, seed)
    n = HU.shape[0]
    nvec, ld = 5, n + 37
    X = np.zeros((nvec, ld), dtype=np.complex128)
    X[:, :n] = inputs.complex_vector(n, 5, nvec)
    X[:, n:] = 7.0                      # padding must be ignored and left untouched
    xd = dev(X, torch.complex128)
    yd = torch.full_like(xd, 3.0 + 0j)
    syk.apply_H(h, 0, xd, yd, nvec=nvec, ld=ld)
    Y = host(yd)
    for v in range(nvec):
        assert rel(Y[v, :n], HU @ X[v, :n]) <= 1e-13
    assert np.all(Y[:, n:] == 3.0)


def test_apply_h_repeatable_bitwise():
    h = syk.create_hamiltonian(24, 4, 2, 1)
    n = 1 << 11
    xd = dev(inputs.complex_vector(n, 3)[0], torch.complex128)
    a = torch.empty_like(xd)
    b = torch.empty_like(xd)
    syk.apply_H(h, 1, xd, a)
    syk.apply_H(h, 1, xd, b)
    assert torch.equal(a, b)


# --------------------------------------------------------------------------- apply_H, large N
def _sampled_rows_check(N, k, seed, dt, blk, nrows=3000, variant=None):
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    h = syk.create_hamiltonian(N, 4, k, seed)
    if variant is not None:
        syk.select_variant(h, dt, variant)
    n = 1 << (N // 2 - 1)
    x = inputs.complex_vector(n, seed + 1)[0]
    xd = dev(x, cdt(dt))
    del x
    yd = torch.empty_like(xd)
    syk.apply_H(h, blk, xd, yd)
    rows = inputs.row_sample(n, nrows, seed + 2)
    xr = host(xd)
    del xd
    rows_t = torch.from_numpy(rows.astype(np.int64)).to("cuda")
    y = host(yd[rows_t])
    terms = matfree.block_terms(N, subs, J, blk)
    yref = matfree.apply_rows(terms, lambda idx: xr[idx.astype(np.int64)], rows)
    # sum_a |c_a| |x[m ^ x_a]|: same flips, all matrix-element phases dropped (Y -> X, Z -> I)
    flips = [(tuple(pauli.X if lab in (pauli.X, pauli.Y) else pauli.I for lab in labels), abs(c))
             for labels, c in terms]
    mag = matfree.apply_rows(flips, lambda idx: np.abs(xr[idx.astype(np.int64)]), rows).real
    return y, yref, mag, len(subs)


@pytest.mark.parametrize("blk", [0, 1])
def test_apply_h_sampled_rows_N48_c128(blk):
    y, yref, mag, K = _sampled_rows_check(48, 4, 48, syk.C128, blk)
    assert rel(y, yref) <= 1e-10
    assert np.all(np.abs(y - yref) <= K * 2.0 ** -52 * mag)


def test_apply_h_sampled_rows_N56_c64():
    """The N = 56, k = 4 (K = 224) block of the benchmark, complex64, same launch path."""
    y, yref, mag, K = _sampled_rows_check(56, 4, 56, syk.C64, 0, nrows=2000)
    assert rel(y, yref) <= 4e-6
    assert np.all(np.abs(y - yref) <= K * U24 * mag)


@pytest.mark.parametrize("N,dt,blk", [(36, syk.C128, 0), (38, syk.C128, 0), (38, syk.C128, 1), (38, syk.C64, 0),
                                       (40, syk.C64, 0), (40, syk.C64, 1), (44, syk.C128, 1)])
def test_apply_h_tiled_smallest_sizes(N, dt, blk):
    """Blocks on both sides of the gather/tiled switch (the tiled kernel serves 2^5 tiles
    and up: N >= 38 in complex128, N >= 40 in complex64), sampled rows."""
    y, yref, mag, K = _sampled_rows_check(N, 3, N + 1, dt, blk, nrows=6000)
    if dt == syk.C128:
        assert np.all(np.abs(y - yref) <= K * 2.0 ** -52 * mag)
    else:
        assert np.all(np.abs(y - yref) <= K * U24 * mag)


N_VARIANTS = 17


@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
@pytest.mark.parametrize("variant", range(N_VARIANTS))
def test_every_tiled_variant(dt, variant):
    """Each compiled tiled variant (tile size, LDS buffering, workgroups per CU), pinned:
    sampled rows of apply_H against the oracle, and the fused Lanczos step against full
    re-orthogonalisation with separate kernels."""
    N = 40
    y, yref, mag, K = _sampled_rows_check(N, 4, 400 + variant, dt, variant % 2, nrows=4000, variant=variant)
    u = 2.0 ** -52 if dt == syk.C128 else U24
    assert np.all(np.abs(y - yref) <= K * u * mag)
    h = syk.create_hamiltonian(N, 4, 4, 400 + variant)
    syk.select_variant(h, dt, variant)
    n = 1 << (N // 2 - 1)
    vd = dev(inputs.complex_vector(n, 50 + variant)[0], cdt(dt))
    a = torch.empty_like(vd)
    b = torch.empty_like(vd)
    syk.krylov_expm(h, 0, 1.5j - 0.6, vd, a, m=30, reorth=0)
    syk.krylov_expm(h, 0, 1.5j - 0.6, vd, b, m=30, reorth=2)
    err = (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()
    assert err <= (1e-10 if dt == syk.C128 else 2e-6)


@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
@pytest.mark.parametrize("variant", [8, 9, 10])
def test_control_block_variants_split_partner_steps(dt, variant):
    """Control-block variants on a Hamiltonian with many terms per partner tile (N = 40,
    K = 1600): partner steps carrying more records than one block holds are split on the
    host; sampled rows against the oracle, both blocks."""
    for blk in (0, 1):
        y, yref, mag, K = _sampled_rows_check(40, 40, 900 + variant, dt, blk, nrows=1500, variant=variant)
        u = 2.0 ** -52 if dt == syk.C128 else U24
        assert np.all(np.abs(y - yref) <= K * u * mag)


def test_select_variant_rejects_out_of_range():
    h = syk.create_hamiltonian(40, 4, 4, 1)
    with pytest.raises(syk.SykError):
        syk.select_variant(h, syk.C64, N_VARIANTS)
    n = len(syk.autotune(h, syk.C64)[1])
    assert n == N_VARIANTS


@pytest.mark.parametrize("variant", [None, 8, 10])
def test_apply_h_tiled_many_vectors_padded(variant):
    """nvec = 3 vectors at a padded leading dimension through the tiled kernel (N = 40):
    the default variant and control-block variants with one and four tiles per workgroup."""
    N, k, seed = 40, 4, 12
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    h = syk.create_hamiltonian(N, 4, k, seed)
    if variant is not None:
        syk.select_variant(h, syk.C64, variant)
    n = 1 << (N // 2 - 1)
    nvec, ld = 3, n + 1000
    X = torch.zeros(nvec, ld, dtype=torch.complex64, device="cuda")
    for v in range(nvec):
        X[v, :n] = dev(inputs.complex_vector(n, 30 + v)[0], torch.complex64)
    X[:, n:] = 5.0
    Y = torch.full_like(X, 2.0)
    syk.apply_H(h, 0, X, Y, nvec=nvec, ld=ld)
    rows = inputs.row_sample(n, 3000, 9)
    terms = matfree.block_terms(N, subs, J, 0)
    Xh = host(X)
    Yh = host(Y)
    for v in range(nvec):
        xr = Xh[v, :n]
        yref = matfree.apply_rows(terms, lambda idx: xr[idx.astype(np.int64)], rows)
        assert rel(Yh[v, rows.astype(np.int64)], yref) <= 4e-6
    assert np.all(Yh[:, n:] == 2.0)


def _device_sampled_rows(N, k, seed, dt, nrows, blk=0):
    """apply_H at large N on a device-generated vector; rows recomputed by the oracle from
    the vector's entries gathered at the partner indices."""
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    h = syk.create_hamiltonian(N, 4, k, seed)
    n = 1 << (N // 2 - 1)
    g = torch.Generator(device="cuda").manual_seed(seed)
    xd = torch.randn(n, dtype=cdt(dt), device="cuda", generator=g)
    yd = torch.empty_like(xd)
    syk.apply_H(h, blk, xd, yd)
    torch.cuda.synchronize()
    rows = inputs.row_sample(n, nrows, seed + 2)
    y = host(yd[torch.from_numpy(rows.astype(np.int64)).to("cuda")])
    del yd

    def x_at(idx):
        return host(xd[torch.from_numpy(np.asarray(idx, dtype=np.int64)).to("cuda")])

    terms = matfree.block_terms(N, subs, J, blk)
    yref = matfree.apply_rows(terms, x_at, rows)
    flips = [(tuple(pauli.X if lab in (pauli.X, pauli.Y) else pauli.I for lab in labels), abs(c))
             for labels, c in terms]
    mag = matfree.apply_rows(flips, lambda idx: np.abs(x_at(idx)), rows).real
    del xd
    torch.cuda.empty_cache()
    return y, yref, mag, len(subs)


def test_apply_h_largest_block_N64_c64():
    """The largest block the library takes: N = 64, 2^31 complex64 amplitudes (16 GiB per
    vector), k = 4 (K = 256), tiled kernel, on sampled rows with the accumulation bound."""
    y, yref, mag, K = _device_sampled_rows(64, 4, 64, syk.C64, 300)
    assert np.all(np.abs(y - yref) <= K * U24 * mag)
    assert rel(y, yref) <= 4e-6


def test_apply_h_large_block_N60_c128():
    """N = 60 in complex128 (2^29 amplitudes, 8 GiB per vector), block D, sampled rows."""
    y, yref, mag, K = _device_sampled_rows(60, 2, 60, syk.C128, 300, blk=1)
    assert np.all(np.abs(y - yref) <= K * 2.0 ** -52 * mag)
    assert rel(y, yref) <= 1e-12


def test_apply_h_hermitian_N40():
    """<u, H v> = conj <v, H u> for Haar-like u, v (exact up to rounding)."""
    h = syk.create_hamiltonian(40, 4, 4, 40)
    n = 1 << 19
    U = dev(inputs.complex_vector(n, 1)[0], torch.complex128)
    V = dev(inputs.complex_vector(n, 2)[0], torch.complex128)
    HU = torch.empty_like(U)
    HV = torch.empty_like(V)
    syk.apply_H(h, 0, U, HU)
    syk.apply_H(h, 0, V, HV)
    a = torch.vdot(U, HV).item()
    b = torch.vdot(V, HU).item()
    assert abs(a - b.conjugate()) <= 1e-12 * abs(a)
    # ||H v||^2 concentrates at (sum J^2 / 16) ||v||^2
    r = torch.vdot(HV, HV).real.item() / torch.vdot(V, V).real.item()
    assert abs(r / (h.info()["sum_J2"] / 16) - 1) < 0.05


# --------------------------------------------------------------------------- Haar states
@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_haar_state_vs_oracle_N16(dt):
    N = 16
    n = 1 << (N // 2 - 1)
    pu = torch.empty(n, dtype=cdt(dt), device="cuda")
    pd = torch.empty_like(pu)
    syk.haar_state(N, 1001, 3, pu, pd)
    ref = haar.haar_state(N, 1001, 3)
    got = np.concatenate([host(pu), host(pd)])
    tol = 1e-14 if dt == syk.C128 else 2e-7
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_haar_state_sampled_N48():
    N = 48
    n = 1 << (N // 2 - 1)
    pu = torch.empty(n, dtype=torch.complex128, device="cuda")
    pd = torch.empty_like(pu)
    syk.haar_state(N, 4800, 0, pu, pd)
    nrm = math.sqrt(haar.raw_norm2(N, 4800, 0))
    idx = inputs.row_sample(2 * n, 2000, 1)
    full = torch.cat([pu, pd])
    got = host(full[torch.from_numpy(idx.astype(np.int64)).to("cuda")])
    ref = haar.raw_amplitudes(4800, 0, idx) / nrm
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    assert abs(torch.vdot(full, full).real.item() - 1) < 1e-12


# --------------------------------------------------------------------------- Majorana insertions
@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_majorana_blocks_vs_dense(dt):
    N = 12
    g = dense.gammas(N)
    h2 = g[0].shape[0] // 2
    x = inputs.complex_vector(h2, 8)[0]
    xd = dev(x, cdt(dt))
    xr = host(xd)
    tol = 1e-15 if dt == syk.C128 else 1e-6
    for n in range(N):
        for src in (0, 1):
            yd = torch.empty_like(xd)
            syk.apply_majorana(N, n, src, xd, yd, scale=0.5 - 0.25j)
            block = g[n][h2:, :h2] if src == 0 else g[n][:h2, h2:]
            assert np.abs(host(yd) - (0.5 - 0.25j) * block @ xr).max() <= tol


# --------------------------------------------------------------------------- Krylov propagator
@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
@pytest.mark.parametrize("z", [-0.3j, -7.0j, -1.25, 3j - 0.7, -20j - 5.0])
def test_krylov_expm_vs_eigh(dt, z):
    N, k, seed = 16, 4, 1
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    HD = dense.blocks(dense.hamiltonian(N, subs, J))[1]
    h = syk.create_hamiltonian(N, 4, k, seed)
    v = inputs.complex_vector(HD.shape[0], 4)[0]
    vd = dev(v, cdt(dt))
    vr = host(vd)
    out = torch.empty_like(vd)
    st = syk.krylov_expm(h, 1, z, vd, out, m=30)
    ref = dense.Eig(HD).expm_apply(z, vr)
    tol = 1e-10 if dt == syk.C128 else 1e-5
    assert rel(host(out), ref) <= tol
    assert st["matvecs"] >= 1 and st["substeps"] >= 1


@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
@pytest.mark.parametrize("reorth", [0, 1, 2, 3])
def test_krylov_reorthogonalisation_modes_vs_eigh(dt, reorth):
    """Every reorthogonalisation mode (none, local, full CGS2, partial after Simon) on a
    long Lanczos run (N = 20: 512-dimensional blocks, m = 128, |z| far beyond one short
    sub-step) against the eigendecomposition; full mode reorthogonalises every step, partial
    mode some but not all, the others none."""
    N, k, seed = 20, 4, 8
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    HD = dense.blocks(dense.hamiltonian(N, subs, J))[0]
    h = syk.create_hamiltonian(N, 4, k, seed)
    v = inputs.complex_vector(HD.shape[0], 12)[0]
    vd = dev(v, cdt(dt))
    out = torch.empty_like(vd)
    z = -120.0j
    st = syk.krylov_expm(h, 0, z, vd, out, m=128, reorth=reorth)
    ref = dense.Eig(HD).expm_apply(z, host(vd))
    assert rel(host(out), ref) <= (1e-10 if dt == syk.C128 else 1e-5), st
    if reorth == 2:
        assert st["reorths"] == st["matvecs"]
    elif reorth == 3:
        assert 1 <= st["reorths"] < st["matvecs"], st
    else:
        assert st["reorths"] == 0


def test_krylov_in_place_and_unitary():
    h = syk.create_hamiltonian(30, 4, 4, 3)
    n = 1 << 14
    vd = dev(inputs.complex_vector(n, 6)[0], torch.complex128)
    n0 = torch.linalg.vector_norm(vd).item()
    w = vd.clone()
    syk.krylov_expm(h, 0, -4.0j, w, w, m=30)
    assert abs(torch.linalg.vector_norm(w).item() / n0 - 1) < 1e-11
    # composition: e^{-2iH} e^{-2iH} v = e^{-4iH} v
    a = vd.clone()
    syk.krylov_expm(h, 0, -2.0j, a, a)
    syk.krylov_expm(h, 0, -2.0j, a, a)
    assert (torch.linalg.vector_norm(a - w) / n0).item() < 1e-10


@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_krylov_fused_step_matches_full_reorth_N40(dt):
    """N = 40 runs the fused tiled Lanczos step (reorth = 0); full re-orthogonalisation
    (reorth = 2, separate kernels) must give the same propagator to the tolerance."""
    h = syk.create_hamiltonian(40, 4, 4, 40)
    n = 1 << 19
    vd = dev(inputs.complex_vector(n, 21)[0], cdt(dt))
    tol = 1e-10 if dt == syk.C128 else 2e-6
    for z in (-2.5j, 1.5j - 0.6, -9.0j):
        a = torch.empty_like(vd)
        b = torch.empty_like(vd)
        sa = syk.krylov_expm(h, 1, z, vd, a, m=40, reorth=0)
        sb = syk.krylov_expm(h, 1, z, vd, b, m=40, reorth=2)
        err = (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()
        assert err <= tol, (z, err, sa, sb)
    # unitary evolution keeps the norm
    syk.krylov_expm(h, 0, -7.0j, vd, a, m=40)
    r = (torch.linalg.vector_norm(a) / torch.linalg.vector_norm(vd)).item()
    assert abs(r - 1) <= (1e-11 if dt == syk.C128 else 2e-6)


def test_krylov_single_term_breakdown_N48():
    """H = (J/4) P with P^2 = 1: e^{-iHt} v = cos(Jt/4) v - i sin(Jt/4) P v exactly; the
    Krylov space has dimension 2 (breakdown)."""
    N = 48
    h = syk.create_hamiltonian(N, 4, 1.0 / N, 77)
    Jv = float(h.terms()["J"][0])
    n = 1 << (N // 2 - 1)
    vd = dev(inputs.complex_vector(n, 9)[0], torch.complex128)
    Hv = torch.empty_like(vd)
    syk.apply_H(h, 0, vd, Hv)
    t = 3.7
    a = Jv / 4
    out = torch.empty_like(vd)
    st = syk.krylov_expm(h, 0, -1j * t, vd, out, m=10)
    ref = math.cos(a * t) * vd - 1j * math.sin(a * t) * (Hv / a)
    assert (torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref)).item() < 1e-12
    assert st["breakdown"] == 1 and st["matvecs"] <= 10


# --------------------------------------------------------------------------- OTOC
def _oracle_otoc(N, k, seed, i, j, beta, ts, state_seed, nvec=1):
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    H = dense.hamiltonian(N, subs, J)
    ch = dense.chis(N)
    F = np.array([dense.otoc_state(H, ch[i], ch[j], beta, ts, haar.haar_state(N, state_seed, v))
                  for v in range(nvec)])
    return dense.normalise_curves(F)


@pytest.mark.parametrize("i,j", [(1, 2), (15, 14)])
@pytest.mark.parametrize("beta", [0.0, 5.0])
@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_otoc_config_N16_vs_oracle(i, j, beta, dt):
    """N = 16, k = 4 (K = 64), one realisation, one Haar state, m = 30, t = 0:0.1:10."""
    ts = np.round(np.arange(101) * 0.1, 10)
    raw, nrm, im = _oracle_otoc(16, 4, 1, i, j, beta, ts, 1001)
    h = syk.create_hamiltonian(16, 4, 4, 1)
    g_raw, g_nrm, g_im, st = syk.otoc(h, i, j, beta, ts, nvec=1, state_seed=1001, dtype=dt, m=30)
    tol = 1e-9 if dt == syk.C128 else 1e-5
    assert np.abs(g_raw - raw).max() <= tol
    assert np.abs(g_nrm - nrm).max() <= tol
    assert np.abs(g_im - im).max() <= tol
    assert st["matvecs"] > 0


def test_otoc_two_vectors_ratio_of_sums():
    ts = [0.0, 0.5, 1.5]
    raw, nrm, im = _oracle_otoc(12, 3, 5, 11, 10, 2.0, ts, 77, nvec=2)
    h = syk.create_hamiltonian(12, 4, 3, 5)
    g_raw, g_nrm, g_im, _ = syk.otoc(h, 11, 10, 2.0, ts, nvec=2, state_seed=77, dtype=syk.C128)
    assert np.abs(g_raw - raw).max() < 1e-10 and np.abs(g_nrm - nrm).max() < 1e-9


def test_otoc_t_grid_without_zero():
    """F_norm is normalised by t = 0 even when the grid does not start at 0."""
    ts = [0.4, 0.9]
    raw, nrm, _ = _oracle_otoc(12, 3, 6, 1, 4, 1.0, [0.0] + ts, 5)
    h = syk.create_hamiltonian(12, 4, 3, 6)
    g_raw, g_nrm, _, _ = syk.otoc(h, 1, 4, 1.0, ts, state_seed=5, dtype=syk.C128)
    assert np.abs(g_raw - raw[1:]).max() < 1e-10 and np.abs(g_nrm - nrm[1:]).max() < 1e-9


@pytest.mark.parametrize("N,dt", [(48, syk.C128), (56, syk.C64)])
def test_otoc_single_term_closed_forms_large_N(N, dt):
    """K = 1: Re F = -cos(J t)/4 when both Majoranas are in the term (any beta, any psi),
    F = -1/4 when exactly one is, F_norm = 1 when neither is."""
    h = syk.create_hamiltonian(N, 4, 1.0 / N, 5)
    T = h.terms()
    term = [int(v) for v in T["ijkl"][0]]
    Jv = float(T["J"][0])
    ts = np.array([0.0, 0.7, 2.5, 6.0])
    tol = 1e-9 if dt == syk.C128 else 1e-5
    others = [n for n in range(N) if n not in term]
    raw, nrm, _, _ = syk.otoc(h, term[0], term[2], 4.0, ts, state_seed=3, dtype=dt, m=8)
    assert np.abs(raw + np.cos(Jv * ts) / 4).max() <= tol
    raw, _, _, _ = syk.otoc(h, term[1], others[0], 4.0, ts, state_seed=3, dtype=dt, m=8)
    assert np.abs(raw + 0.25).max() <= tol
    _, nrm, _, _ = syk.otoc(h, others[0], others[1], 4.0, ts, state_seed=3, dtype=dt, m=8)
    assert np.abs(nrm - 1).max() <= 2 * tol


@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_otoc_rotated_layout_matches_standard_N40(dt):
    """The planner's rotated vector layout gives the same OTOC as the standard layout
    (whose apply_H, Haar and Majorana kernels are checked against the oracle above)."""
    h = syk.create_hamiltonian(40, 4, 4, 41)
    plan = syk.plan_describe(h, 0, dt)
    assert plan["tiled"] == 1
    ts = [0.0, 0.5, 1.5]
    a = syk.otoc(h, 39, 38, 3.0, ts, state_seed=2, dtype=dt, m=30, layout=-1)
    b = syk.otoc(h, 39, 38, 3.0, ts, state_seed=2, dtype=dt, m=30, layout=0)
    c = syk.otoc(h, 39, 38, 3.0, ts, state_seed=2, dtype=dt, m=30, layout=7)
    tol = 1e-9 if dt == syk.C128 else 1e-5
    for other in (b, c):
        assert np.abs(a[0] - other[0]).max() <= tol * max(1.0, np.abs(a[0]).max())
        assert np.abs(a[1] - other[1]).max() <= tol


def test_otoc_beta0_t0_minus_quarter_N40():
    h = syk.create_hamiltonian(40, 4, 4, 8)
    raw, _, im, _ = syk.otoc(h, 39, 38, 0.0, [0.0], state_seed=1, dtype=syk.C128)
    assert abs(raw[0] + 0.25) < 1e-12 and abs(im[0]) < 1e-12


def test_otoc_benchmark_configuration_c64_against_c128_N56():
    """The benchmark's own configuration (N = 56, k = 4, seed 56, state 5600, chi_55 and
    chi_54, Krylov dimension 60, complex64 at tol 3e-6 on the autotuned tiled kernel with the
    fused Lanczos step) on a short t grid, against the complex128 path on the same
    realisation and state (itself pinned to the oracle at small N).  A consistency check at
    full size: F(0) at beta = 0 is -1/4 exactly, and the normalised curves agree to the
    mixed-precision bound 1e-5."""
    N = 56
    torch.cuda.empty_cache()
    h = syk.create_hamiltonian(N, 4, 4, 56)
    syk.autotune(h, syk.C64)
    ts = [0.0, 0.25, 0.5]
    a = syk.otoc(h, N - 1, N - 2, 5.0, ts, state_seed=5600, dtype=syk.C64, m=60, tol=3e-6)
    syk.release_workspace()
    b = syk.otoc(h, N - 1, N - 2, 5.0, ts, state_seed=5600, dtype=syk.C128, m=60)
    syk.release_workspace()
    assert np.abs(a[1] - b[1]).max() <= 1e-5
    assert abs(a[0][0] - b[0][0]) <= 1e-5 * abs(b[0][0])
    c = syk.otoc(h, N - 1, N - 2, 0.0, [0.0], state_seed=5600, dtype=syk.C64)
    syk.release_workspace()
    assert abs(c[0][0] + 0.25) <= 1e-6


def test_otoc_plain_complex128_configuration_N48():
    """The plain complex128 single-realisation configuration as configured (N = 48, k = 4,
    so K = 192, seed 48, Krylov dimension 40, beta = 10, 16 Haar vectors of state seed
    4800, chi_47 and chi_46) on a short t grid.  Per vector: F(0) at beta = 0 is -1/4
    exactly (chi_i chi_j chi_i chi_j = -1/4 for any normalised state).  The 16-vector curve
    at beta = 10 through complex64 states agrees with the complex128 one to the
    mixed-precision bound 1e-5 on F_norm (and on F_raw relative to |F_raw(0)|)."""
    N = 48
    torch.cuda.empty_cache()
    h = syk.create_hamiltonian(N, 4, 4, 48)
    assert h.info()["K"] == 192
    for v in range(16):
        raw, nrm, im, _ = syk.otoc(h, N - 1, N - 2, 0.0, [0.0], nvec=1, state_seed=4800 + v, dtype=syk.C128, m=40)
        assert abs(raw[0] + 0.25) <= 1e-12, (v, raw[0])
        assert abs(im[0]) <= 1e-12
    ts = [0.0, 0.25, 0.5]
    b = syk.otoc(h, N - 1, N - 2, 10.0, ts, nvec=16, state_seed=4800, dtype=syk.C128, m=40)
    syk.release_workspace()
    a = syk.otoc(h, N - 1, N - 2, 10.0, ts, nvec=16, state_seed=4800, dtype=syk.C64, m=40)
    syk.release_workspace()
    h.close()
    print(f"C2 shape: F_norm c128 {b[1]}, |c64 - c128| {np.abs(a[1] - b[1]).max():.2e}", flush=True)
    assert np.abs(a[1] - b[1]).max() <= 1e-5
    assert np.abs(a[0] - b[0]).max() <= 1e-5 * abs(b[0][0])
    assert b[3]["matvecs"] > 0 and a[3]["matvecs"] > 0


@pytest.mark.parametrize("N,k,seed", [(24, 4, 31), (40, 2, 32)])
def test_otoc_precision_check_reports_the_complex128_deviation(N, k, seed):
    """precision_check: the complex64 result's error against a complex128 re-evaluation on
    the same Haar vectors (relative F_raw at t = 0, F_norm at the last t) equals the error
    against a separate complex128 call, and meets the mixed-precision bound 1e-5; the
    gather path (N = 24) and the tiled path with the fused Lanczos step (N = 40)."""
    h = syk.create_hamiltonian(N, 4, k, seed)
    ts = [0.0, 0.5, 1.5]
    a = syk.otoc(h, N - 1, N - 2, 4.0, ts, nvec=2, state_seed=77, dtype=syk.C64, m=30, precision_check=True)
    b = syk.otoc(h, N - 1, N - 2, 4.0, [0.0, ts[-1]], nvec=2, state_seed=77, dtype=syk.C128, m=30)
    c = syk.otoc(h, N - 1, N - 2, 4.0, ts, nvec=2, state_seed=77, dtype=syk.C64, m=30)
    syk.release_workspace()
    h.close()
    want = max(abs(a[0][0] - b[0][0]) / abs(b[0][0]), abs(a[1][-1] - b[1][-1]))
    st = a[3]
    print(f"N={N}: mp_err {st['mp_err']:.3e} (separate c128 call {want:.3e}), {st['mp_seconds']:.2f} s", flush=True)
    assert abs(st["mp_err"] - want) <= 1e-9
    assert 0.0 <= st["mp_err"] <= 1e-5
    assert c[3]["mp_err"] == -1.0                      # not requested: not evaluated
    assert np.array_equal(a[0], c[0])                 # the check does not change the result
    assert st["matvecs"] == c[3]["matvecs"]


def test_otoc_rejects_bad_arguments():
    h = syk.create_hamiltonian(12, 4, 3, 5)
    for args in ((3, 3, 1.0, [0.0]), (0, 12, 1.0, [0.0]), (0, 1, -1.0, [0.0]), (0, 1, 1.0, [0.5, 0.2])):
        with pytest.raises(syk.SykError) as e:
            syk.otoc(h, *args, dtype=syk.C128)
        assert e.value.status == 1


@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_full_sector_apply_and_propagator_vs_dense(dt):
    """SYK_FULL: the whole 2^(N/2) space (U block, then D) against the oracle's full dense H
    (N = 12): y = H x, and e^{zH} v for a complex z."""
    N, k, seed = 12, 4, 21
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    H = dense.hamiltonian(N, subs, J)
    h = syk.create_hamiltonian(N, 4, k, seed)
    d = H.shape[0]
    x = inputs.complex_vector(d, 61)[0]
    xd = dev(x, cdt(dt))
    yd = torch.empty_like(xd)
    syk.apply_H(h, syk.FULL, xd, yd)
    ref = H @ host(xd)
    assert rel(host(yd), ref) <= (1e-13 if dt == syk.C128 else 2e-7)
    z = -0.3 - 1.7j
    out = torch.empty_like(xd)
    st = syk.krylov_expm(h, syk.FULL, z, xd, out, m=30)
    w, U = np.linalg.eigh(H)
    ref = U @ (np.exp(z * w) * (U.conj().T @ host(xd)))
    assert rel(host(out), ref) <= (1e-10 if dt == syk.C128 else 1e-5)
    assert st["matvecs"] >= 2


def test_full_sector_is_the_two_blocks_N40():
    """SYK_FULL at a tiled size (N = 40) equals the U and D applies on the two halves, bitwise."""
    h = syk.create_hamiltonian(40, 4, 4, 77)
    n = 1 << 19
    g = torch.Generator(device="cuda").manual_seed(77)
    x = torch.randn(2 * n, dtype=torch.complex64, device="cuda", generator=g)
    y = torch.empty_like(x)
    syk.apply_H(h, syk.FULL, x, y)
    yu = torch.empty(n, dtype=torch.complex64, device="cuda")
    yv = torch.empty_like(yu)
    syk.apply_H(h, syk.BLOCK_U, x[:n].contiguous(), yu)
    syk.apply_H(h, syk.BLOCK_D, x[n:].contiguous(), yv)
    torch.cuda.synchronize()
    assert torch.equal(y[:n], yu) and torch.equal(y[n:], yv)


def test_handle_shared_by_threads_on_streams():
    """One handle used at once from four host threads, each on its own stream (plans are
    built concurrently on first use): apply_H and krylov_expm give the results of the same
    calls made one after another, bitwise."""
    import threading
    N = 44
    h = syk.create_hamiltonian(N, 4, 4, 404)
    n = 1 << (N // 2 - 1)
    xs = [dev(inputs.complex_vector(n, 800 + i)[0], torch.complex64) for i in range(4)]
    outs = [[None, None] for _ in range(4)]
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                y = torch.empty_like(xs[i])
                syk.apply_H(h, i % 2, xs[i], y, stream=s)
                e = torch.empty_like(xs[i])
                syk.krylov_expm(h, i % 2, -0.5j, xs[i], e, m=20, stream=s)
            s.synchronize()
            outs[i] = [y, e]
        except Exception as ex:          # reported by the main thread
            errors.append(ex)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for i in range(4):
        y = torch.empty_like(xs[i])
        syk.apply_H(h, i % 2, xs[i], y)
        e = torch.empty_like(xs[i])
        syk.krylov_expm(h, i % 2, -0.5j, xs[i], e, m=20)
        torch.cuda.synchronize()
        assert torch.equal(outs[i][0], y) and torch.equal(outs[i][1], e)
