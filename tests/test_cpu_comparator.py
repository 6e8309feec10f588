"""The plain CPU matrix-free comparator (oracle/cpu_lanczos.c) against the oracle.

* pauli.to_xz inverts from_xz and reproduces the dense label strings (with the i^p phase).
* cpu_apply equals the oracle's row-by-row products on every row (N = 14, both blocks) and
  on sampled rows at N = 24; and the dense block at N = 12.
* cpu_lanczos gives the alpha, beta of a three-term Lanczos on the dense block (N = 12).
"""
import numpy as np
import pytest

from oracle import cpu_lanczos, dense, ensemble, matfree, pauli


def test_to_xz_inverts_from_xz_and_matches_dense():
    rng = np.random.default_rng(0)
    L = 4
    for _ in range(30):
        labels = tuple(int(v) for v in rng.integers(0, 4, L))
        x, z, p = pauli.to_xz(labels)
        back, q = pauli.from_xz(L, x, z)
        assert back == labels and (p + q) % 4 == 0
        P = pauli.dense((labels, 0))
        assert np.allclose(P, (1j ** p) * pauli.operator_dense(L, [x], [z], [1.0]))


@pytest.mark.parametrize("blk", [0, 1])
def test_cpu_apply_every_row_N14(blk):
    N, k, seed = 14, 4, 3
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    terms = matfree.block_terms(N, subs, J, blk)
    L = N // 2 - 1
    v = np.random.default_rng(1).standard_normal(1 << L) + 1j * np.random.default_rng(2).standard_normal(1 << L)
    y = cpu_lanczos.apply(L, cpu_lanczos.xz_terms(terms), v)
    rows = np.arange(1 << L, dtype=np.uint64)
    ref = matfree.apply_rows(terms, lambda idx: v[idx.astype(np.int64)], rows)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_cpu_apply_sampled_rows_N24_and_dense_N12():
    N = 24
    subs, J, _ = ensemble.sample_terms(N, 4, 8)
    terms = matfree.block_terms(N, subs, J, 1)
    L = N // 2 - 1
    v = np.random.default_rng(3).standard_normal(1 << L) + 0.5j
    y = cpu_lanczos.apply(L, cpu_lanczos.xz_terms(terms), v)
    rows = np.random.default_rng(4).integers(0, 1 << L, 500).astype(np.uint64)
    ref = matfree.apply_rows(terms, lambda idx: v[idx.astype(np.int64)], rows)
    assert np.abs(y[rows.astype(np.int64)] - ref).max() <= 1e-13 * np.abs(ref).max()
    N = 12
    subs, J, _ = ensemble.sample_terms(N, 5, 2)
    HU, _ = dense.blocks(dense.hamiltonian(N, subs, J))
    v = np.random.default_rng(5).standard_normal(HU.shape[0]) + 1j
    y = cpu_lanczos.apply(N // 2 - 1, cpu_lanczos.xz_terms(matfree.block_terms(N, subs, J, 0)), v)
    assert np.abs(y - HU @ v).max() <= 1e-13 * np.abs(HU @ v).max()


def test_cpu_lanczos_matches_dense_three_term_recurrence():
    N = 12
    subs, J, _ = ensemble.sample_terms(N, 5, 4)
    HU, _ = dense.blocks(dense.hamiltonian(N, subs, J))
    v0 = np.random.default_rng(6).standard_normal(HU.shape[0]) + 1j * np.random.default_rng(7).standard_normal(
        HU.shape[0])
    steps = 8
    a, b, t_apply, t_total, thr = cpu_lanczos.lanczos(N // 2 - 1, cpu_lanczos.xz_terms(
        matfree.block_terms(N, subs, J, 0)), v0, steps)
    assert thr >= 1 and 0.0 <= t_apply <= t_total
    # the recurrence written out on the dense block
    v = v0 / np.linalg.norm(v0)
    vp = np.zeros_like(v)
    bp = 0.0
    for j in range(steps):
        w = HU @ v - bp * vp
        al = np.vdot(v, w).real
        w = w - al * v
        be = np.linalg.norm(w)
        assert a[j] == pytest.approx(al, abs=1e-12) and b[j] == pytest.approx(be, rel=1e-12)
        vp, v, bp = v, w / be, be
