"""General spin operators (Pauli sums) through the apply_H / Krylov kernels.

* apply of complex, non-Hermitian operators against the oracle's dense matrices (L = 6, 10),
  both precisions; an L = 18 operator through the tiled kernel on sampled rows.
* e^{-iHt} for the transverse-field Ising chain H = sum Z_q Z_{q+1} + g sum X_q (L = 10)
  against the dense exponential; non-Hermitian operators are refused by the propagator.
"""
import numpy as np
import pytest
import scipy.linalg

torch = pytest.importorskip("torch")

import paper_2311_00639_amd as syk  # noqa: E402
from oracle import matfree, pauli  # noqa: E402
from tests import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex128))).to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy().astype(np.complex128)


@pytest.mark.parametrize("L,n", [(6, 9), (10, 40)])
@pytest.mark.parametrize("dt", [syk.C128, syk.C64])
def test_operator_apply_vs_dense(L, n, dt):
    rng = np.random.default_rng(L + n)
    x = rng.integers(0, 1 << L, n).astype(np.uint64)
    z = rng.integers(0, 1 << L, n).astype(np.uint64)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    op = syk.Operator(L, x, z, c)
    M = pauli.operator_dense(L, x, z, c)
    h = op.to_hamiltonian()
    cd = torch.complex64 if dt == syk.C64 else torch.complex128
    xd = dev(inputs.complex_vector(1 << L, 5)[0], cd)
    xr = host(xd)
    for blk in (0, 1):
        yd = torch.empty_like(xd)
        syk.apply_H(h, blk, xd, yd)
        ref = M @ xr
        tol = 1e-13 if dt == syk.C128 else 1e-6
        assert np.linalg.norm(host(yd) - ref) / np.linalg.norm(ref) <= tol


def test_operator_tiled_sampled_rows_L18():
    L, n = 18, 60
    rng = np.random.default_rng(3)
    x = rng.integers(0, 1 << L, n).astype(np.uint64)
    z = rng.integers(0, 1 << L, n).astype(np.uint64)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    h = syk.Operator(L, x, z, c).to_hamiltonian()
    xd = dev(inputs.complex_vector(1 << L, 6)[0], torch.complex128)
    yd = torch.empty_like(xd)
    syk.apply_H(h, 0, xd, yd)
    rows = inputs.row_sample(1 << L, 500, 7)
    xr = host(xd)
    y = host(yd)[rows.astype(np.int64)]
    terms = []
    for xa, za, ca in zip(x, z, c):
        labels, p = pauli.from_xz(L, int(xa), int(za))
        terms.append((labels, ca * (1j ** p)))
    ref = matfree.apply_rows(terms, lambda idx: xr[idx.astype(np.int64)], rows)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) <= 1e-13


def test_ising_chain_propagator_vs_expm():
    L, g, t = 10, 0.7, 1.3
    xs, zs, cs = [], [], []
    for q in range(L - 1):
        xs.append(0), zs.append((1 << q) | (1 << (q + 1))), cs.append(1.0)
    for q in range(L):
        xs.append(1 << q), zs.append(0), cs.append(g)
    op = syk.Operator(L, xs, zs, cs)
    assert op.is_hermitian()
    H = pauli.operator_dense(L, xs, zs, cs)
    h = op.to_hamiltonian()
    v = inputs.complex_vector(1 << L, 8)[0]
    vd = dev(v, torch.complex128)
    out = torch.empty_like(vd)
    syk.krylov_expm(h, 0, -1j * t, vd, out, m=30)
    ref = scipy.linalg.expm(-1j * t * H) @ v
    assert np.linalg.norm(host(out) - ref) / np.linalg.norm(ref) <= 1e-10
    with pytest.raises(syk.SykError):
        syk.otoc(h, 1, 2, 1.0, [0.0, 1.0])
    nh = syk.Operator(L, [1], [1], [1.0]).to_hamiltonian()      # X Z is not Hermitian
    with pytest.raises(syk.SykError):
        syk.krylov_expm(nh, 0, -1j, vd, out)
