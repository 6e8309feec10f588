"""Batched OTOC (one persistent launch over many realisations and vectors), through the C ABI.

* Against the oracle's chain with dense propagators on the same Haar states (N = 18-22,
  every launch shape that serves the block sizes), complex64 states: 1e-5 on F.
* Against the single-request path (syk_otoc, complex64) at N = 24, 28, 32: 1e-5 on the
  normalised F, 1e-5 relative to F(0) on the raw values (beta = 10).
* Single-term Hamiltonian (K = 1) at N = 32: Re F = -cos(Jt)/4 when both Majoranas are in
  the term, -1/4 when one is, for every state; beta = 0, t = 0 gives -1/4.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2311_00639_amd as syk  # noqa: E402
from oracle import dense, ensemble, haar  # noqa: E402

pytestmark = pytest.mark.gpu

TS = [0.0, 0.5, 1.5, 3.0]


def oracle_curve(N, k, seed, i, j, ss, beta, ts, nvec):
    subs, J, _ = ensemble.sample_terms(N, k, seed)
    H = dense.hamiltonian(N, subs, J)
    ch = dense.chis(N)
    F = np.stack([dense.otoc_state(H, ch[i], ch[j], beta, ts, haar.haar_state(N, ss, v)) for v in range(nvec)])
    return dense.normalise_curves(F)


@pytest.mark.parametrize("variant,items", [
    (2, [(18, 2, 1, 17, 16, 11), (20, 4, 2, 3, 7, 12), (20, 8, 3, 19, 18, 13)]),
    (1, [(20, 4, 4, 19, 18, 14), (22, 2, 5, 21, 20, 15)]),
    (0, [(22, 4, 6, 21, 20, 16), (22, 3, 7, 1, 2, 17)]),
])
def test_batch_vs_oracle(variant, items):
    torch.cuda.set_device(0)
    beta, nvec = 2.0, 2
    raw, nrm, im, st = syk.otoc_batch(items, beta, TS, nvec=nvec, m=30, tol=1e-7, variant=variant)
    assert st["variant"] == variant and st["n_jobs"] == nvec * len(items) and st["matvecs"] > 0
    for r, (N, k, seed, i, j, ss) in enumerate(items):
        ref_raw, ref_nrm, ref_im = oracle_curve(N, k, seed, i, j, ss, beta, TS, nvec)
        assert np.abs(raw[r] - ref_raw).max() <= 1e-5, (r, raw[r], ref_raw)
        assert np.abs(im[r] - ref_im).max() <= 1e-5
        assert np.abs(nrm[r] - ref_nrm).max() <= 1e-5


def test_batch_vs_single_request_path():
    torch.cuda.set_device(0)
    items = [(24, 2, 21, 23, 22, 31), (28, 4, 22, 27, 26, 32), (32, 8, 23, 31, 30, 33), (28, 8, 24, 5, 9, 34)]
    ts = [0.0, 0.75, 2.0, 5.0]
    beta = 10.0
    raw, nrm, im, st = syk.otoc_batch(items, beta, ts, nvec=1, m=30, tol=1e-7)
    for r, (N, k, seed, i, j, ss) in enumerate(items):
        h = syk.create_hamiltonian(N, 4, k, seed)
        a_raw, a_nrm, a_im, _ = syk.otoc(h, i, j, beta, ts, nvec=1, state_seed=ss, dtype=syk.C64, m=30,
                                         autotune=False)
        # the mixed-precision bound 1e-5 applies to the normalised OTOC; the raw values
        # carry the e^{-beta H} weights, so they are compared relative to F(0)
        scale = abs(a_raw[0])
        assert np.abs(nrm[r] - a_nrm).max() <= 1e-5, (r, nrm[r], a_nrm)
        assert np.abs(raw[r] - a_raw).max() <= 1e-5 * scale, (r, raw[r], a_raw)
        assert np.abs(im[r] - a_im).max() <= 1e-5 * scale


def test_batch_single_term_closed_forms_N32():
    torch.cuda.set_device(0)
    N = 32
    h = syk.create_hamiltonian(N, 4, 1.0 / N, 5)
    term = [int(v) for v in h.terms()["ijkl"][0]]
    Jv = float(h.terms()["J"][0])
    out = next(m for m in range(N) if m not in term)
    ts = np.linspace(0.0, 4.0, 5)
    items = [(N, 1.0 / N, 5, term[3], term[1], 7), (N, 1.0 / N, 5, term[0], out, 8)]
    raw, nrm, im, _ = syk.otoc_batch(items, 0.0, ts, nvec=2, m=10)
    assert np.abs(raw[0] + np.cos(Jv * ts) / 4).max() <= 1e-5
    assert np.abs(raw[1] + 0.25).max() <= 1e-5
    assert abs(raw[0][0] + 0.25) <= 1e-6


def test_batch_rejects_bad_arguments():
    with pytest.raises(syk.SykError):
        syk.otoc_batch([(34, 2, 1, 33, 32, 1)], 1.0, TS)          # block too large for the batch
    with pytest.raises(syk.SykError):
        syk.otoc_batch([(24, 2, 1, 5, 5, 1)], 1.0, TS)            # i == j
    with pytest.raises(syk.SykError):
        syk.otoc_batch([(24, 2, 1, 23, 22, 1)], 1.0, TS, m=61)
    with pytest.raises(syk.SykError):
        syk.otoc_batch([(18, 2, 1, 17, 16, 1)], 1.0, TS, variant=0)   # 2^8 amplitudes < 1024 threads
