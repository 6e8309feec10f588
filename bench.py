"""Benchmark of the sparse-SYK OTOC hot path on one MI355X.

Workload (mixed precision at scale): N = 56 Majoranas (parity blocks of 2^27 amplitudes),
q = 4, k = 4 (K = 224 terms), one disorder realisation (seed 56), complex64 state
vectors with double Lanczos reductions and tridiagonal exponential, Krylov dimension 60,
per-propagation tolerance 3e-6 (complex64 rounding, not the tolerance, sets the error of F;
the mixed_precision leg reports it), one Haar state (state_seed 5600), W = chi_55,
V = chi_54, t = 0, 0.25, ..., 20 (81 points); a realisation is the three curves at
beta = 5, 10 and 20.

Timed region: the whole beta = 10 curve, one library call (both parity-block chains,
2 x 81 = 162 chain points, each ending in a synchronising overlap).  A step is one of
`--steps` consecutive segments of those chain points (about 8 of them at the default 20
steps); the library reports each chain point through its progress callback, which dates
the step boundaries.  `--warmup` W runs the first ceil(81 W / steps) t points of the same
curve beforehand.  value = realisations per hour = 3600 / (3 x curve seconds x c), with
c = 1.027 the measured cost of the beta = 5, 10 and 20 curves together relative to three
beta = 10 curves (`--all-betas` times the three: beta = 20 costs 9% more than beta = 10,
beta = 5 1% less; the longest propagations have |z| = |it -+ beta/4|).

Printed: one JSON line with the roofline of the dominant kernel (apply_H), taken from
HIP-event timings of every apply_H launch in the timed region, and cpu_baseline = the
oracle's matrix-free row evaluation timed on a bounded sample, scaled by the
term-amplitudes one realisation needs.

Secondary legs, outside the timed region, each run only while its estimated cost fits in
the wall budget (`--budget`, seconds from start, default 440), in this order:
* mixed_precision: the same realisation, Haar state and beta = 10 evaluated with
  complex128 states at t = 0, 5, 10, 20, and the complex64 curve's deviation from it
  there (the error of the mixed-precision path, per result); it also times the complex64
  path on the same four points, giving the speed ratio over the plain complex128 path at
  equal OTOC accuracy;
* serving: the request engine under a Poisson stream of OTOC requests at a fixed offered
  rate for a fixed window, with p50/p99 submit-to-finish latency and completed
  realisations per hour;
* serving_c5: a burst of ten requests spanning the serving sizes N = 32 ... 64 (N = 64 blocks
  hold 2^31 amplitudes, 16 GiB per complex64 vector) into an engine whose arena is 85% of
  free device memory: admission by footprint, the N = 64 request at a reduced Krylov
  dimension, p50/p99 latency and each request's complex64 error against complex128;
* batched: the persistent batched launch on a sample of the many-small-realisations
  workload (realisations of N uniform in {24, 28, 32}, k uniform in {2, 4, 8}, seed
  3000 + r, 4 Haar states each, complex64, beta = 10, t = 0:0.25:15, Krylov dim 30), with
  realisations per hour;
* apply_k1: apply_H at N = 56 with k = 1 (K = 56), where HBM bandwidth binds, with its
  algorithmic HBM fraction;
* cpu_baseline.plain_cpu_lanczos: a plain C/OpenMP complex128 matrix-free Lanczos
  iteration on the same block (oracle/cpu_lanczos.c), projected to realisations/hour;
* other_entry_points: the Green function of chi_55 on the benchmark realisation (beta = 10,
  t = 0:0.25:5), one dense-SYK apply_H at N = 38 (K = 73815), and a transverse-field Ising
  chain on 27 qubits as a general spin operator (one apply_H, one e^{-iH} propagation);
* lyapunov_pipeline: disorder averages at N = 14, 22, 30 (128 realisations each, beta = 5,
  k = 4), crossing times at F0 = 0.75 and 0.85 and the Eq. (5) / Eq. (6) fits: the analysis
  pipeline end to end and its cost, not a Table I estimate.
Derived figures of the timed curve: the VALU-floor fraction of apply_H (one lane
instruction per term-amplitude), the measured HBM rate (hardware-counter bytes over the
event-timed launch), and the algorithmic HBM fraction of a whole Lanczos iteration (7
vector passes: x read, y written and v_{j-1}, v_j read by the fused epilogue, then y, u_j
read and u_{j+1} written by the residual pass).

--pmc-sample runs a short chain (t = 0, 0.25, 0.5) in the identical launch configuration
plus a 1 GiB device copy, for hardware-counter passes.  --all-betas times the whole
realisation (the three curves, about 7 minutes) and prints their costs, the source of the
pricing factor above.  --plain-c128 times the plain complex128 single-realisation
configuration (N = 48, 16 Haar states, Krylov dimension 40, beta = 10, t = 0:0.25:20) and the
same through complex64 states (about 8 minutes).
"""
import argparse
import json
import math
import os
import sys
import time

T_START = time.perf_counter()

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K_SPARSITY, SEED, STATE_SEED = 56, 4, 56, 5600
BETAS = (5.0, 10.0, 20.0)
BETA_TIMED = 10.0
CHAIN_POINTS = 2 * 81                     # parity-block chains x t points of one curve
M_KRYLOV = 60
TOL_C64 = 3e-6
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3          # published, counts packed FP32 (two lanes per FMA issue)
FP32_NONPACKED_PEAK_TFLOPS = 78.6        # one FP32 FMA per lane per clock (packed FP32 is disabled here)
SERVING_WINDOW_S, SERVING_DRAIN_S = 30.0, 45.0
# Cost of a whole realisation (the beta = 5, 10 and 20 curves) relative to three beta = 10 curves,
# measured with all three curves timed by `bench.py --all-betas` on one MI355X (119.0 s, 120.6 s
# and 131.8 s; profiles/otoc_realisation_three_curves_N56_k4_c64.txt).  The timed region is
# the beta = 10 curve; value divides its time by this factor's worth of the other two curves.
REALISATION_COST_FACTOR = (119.0 + 120.6 + 131.8) / (3 * 120.6)

# HBM traffic of one apply_H launch of this workload, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes over `bench.py --pmc-sample`, each scaled by the same counter's reading for a
# plain device copy of known size (profiles/apply_h_tiled_N56_k4_c64_traffic.txt).  Valid
# only for the kernel revision it was measured on.
TRAFFIC = {"kernel_rev": "tiled-block-14", "variant": 10, "fetch_bytes": 28039795806, "write_bytes": 1073872896}


def log(msg):
    print(f"[bench {time.perf_counter() - T_START:6.1f} s] {msg}", file=sys.stderr, flush=True)


def t_grid():
    return [0.25 * n for n in range(81)]


def cpu_baseline(term_amps_per_realisation: float, seconds_target: float = 12.0):
    """Oracle (numpy, float64) matrix-free rows of H_UU at N = 56 on a bounded row sample."""
    import numpy as np

    from oracle import ensemble, matfree
    subs, J, _ = ensemble.sample_terms(N, K_SPARSITY, SEED)
    terms = matfree.block_terms(N, subs, J, 0)
    n = 1 << (N // 2 - 1)
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(n, dtype=np.float32) + 1j * rng.standard_normal(n, dtype=np.float32)).astype(np.complex64)
    xat = lambda idx: x[idx.astype(np.int64)].astype(np.complex128)
    rows_per_call = 1 << 16
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds_target:
        rows = rng.integers(0, n, rows_per_call, dtype=np.uint64)
        matfree.apply_rows(terms, xat, rows)
        done += rows_per_call
    dt = time.perf_counter() - t0
    rate = done * len(terms) / dt                       # term-amplitudes per second
    return {"value": 3600.0 * rate / term_amps_per_realisation, "unit": "realisations/h", "cores": 1,
            "kind": "oracle",
            "sample": f"oracle.matfree.apply_rows on {done} random rows of the N=56 K=224 U block "
                      f"({dt:.1f} s, {rate:.3e} term-amps/s, single-threaded numpy), scaled by "
                      f"{term_amps_per_realisation:.3e} term-amps per realisation measured on the GPU"}


def mixed_precision_check(syk, curve_c64, stream):
    """complex128 reference of the timed beta = 10 curve at a few t points."""
    t_check = [0.0, 5.0, 10.0, 20.0]
    h = syk.create_hamiltonian(N, 4, K_SPARSITY, SEED)
    syk.autotune(h, syk.C128, stream=stream)
    t0 = time.perf_counter()
    raw, nrm, im, st = syk.otoc(h, N - 1, N - 2, 10.0, t_check, nvec=1, state_seed=STATE_SEED, dtype=syk.C128,
                                m=M_KRYLOV, stream=stream)
    secs = time.perf_counter() - t0
    h.close()
    # the same four points through the complex64 path, for the speed ratio at equal accuracy
    h64 = syk.create_hamiltonian(N, 4, K_SPARSITY, SEED)
    syk.autotune(h64, syk.C64, stream=stream)
    t1 = time.perf_counter()
    _, _, _, st64 = syk.otoc(h64, N - 1, N - 2, 10.0, t_check, nvec=1, state_seed=STATE_SEED, dtype=syk.C64,
                             m=M_KRYLOV, tol=TOL_C64, stream=stream)
    secs64 = time.perf_counter() - t1
    h64.close()
    ts = t_grid()
    idx = [ts.index(t) for t in t_check]
    c_raw, c_nrm, c_im = (curve_c64[0][idx], curve_c64[1][idx], curve_c64[2][idx])
    scale = abs(float(raw[0]))
    return {"t": t_check, "F_norm_c128": [float(v) for v in nrm], "F_norm_c64": [float(v) for v in c_nrm],
            "F_raw0_c128": float(raw[0]),
            "abs_err_F_norm": [float(abs(a - b)) for a, b in zip(c_nrm, nrm)],
            "rel_err_F_raw": [float(abs(a - b)) / scale for a, b in zip(c_raw, raw)],
            "rel_err_F_imag": [float(abs(a - b)) / scale for a, b in zip(c_im, im)],
            "max_abs_err_F_norm": float(max(abs(a - b) for a, b in zip(c_nrm, nrm))),
            "tolerance_F_norm": 1e-5, "c128_seconds": secs, "c128_matvecs": st["matvecs"],
            "c64_seconds_same_points": secs64, "c64_matvecs_same_points": st64["matvecs"],
            "c64_speedup_over_c128": secs / secs64,
            "note": "raw F carries the e^{-beta H} weights of an unnormalised state; errors of F_raw and F_imag "
                    "are relative to |F_raw(0)|"}


def apply_k1_leg(syk, stream):
    """apply_H at N = 56 with k = 1 (K = 56), where HBM bandwidth binds: the autotuner's
    per-variant times of a plain apply, best variant."""
    h = syk.create_hamiltonian(N, 4, 1.0, SEED)
    syk.autotune(h, syk.C64, stream=stream)
    variant, ms = syk.autotune(h, syk.C64, stream=stream)
    info = h.info()
    h.close()
    best = min(m for m in ms if m > 0)
    n = info["block_dim"]
    alg = 2.0 * n * 8
    return {"K": info["K"], "variant": variant, "ms": best, "term_amps_per_s": info["K"] * n / (best * 1e-3),
            "algorithmic_hbm_TBps": alg / (best * 1e-3) / 1e12,
            "algorithmic_hbm_frac": alg / (best * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "variant_ms": ms, "note": "plain apply (read x once, write y once), complex64, seed 56"}


def cpu_lanczos_leg(matvecs_per_realisation: float, steps: int = 1):
    """Plain C/OpenMP matrix-free complex128 Lanczos (oracle/cpu_lanczos.c) on the N = 56 U
    block: one iteration timed, the realisation rate projected from the per-iteration time."""
    import numpy as np

    from oracle import cpu_lanczos, ensemble, matfree
    subs, J, _ = ensemble.sample_terms(N, K_SPARSITY, SEED)
    xzc = cpu_lanczos.xz_terms(matfree.block_terms(N, subs, J, 0))
    L = N // 2 - 1
    rng = np.random.default_rng(2)
    v0 = np.empty(1 << L, dtype=np.complex128)
    v0.real = rng.standard_normal(1 << L)
    v0.imag = rng.standard_normal(1 << L)
    a, b, t_apply, t_total, thr = cpu_lanczos.lanczos(L, xzc, v0, steps)
    del v0
    t_iter = t_total / steps
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value_projected": 3600.0 / (matvecs_per_realisation * t_iter), "unit": "realisations/h",
            "threads": thr, "nproc": os.cpu_count(), "cpu_model": model,
            "seconds_per_matvec": t_apply / steps, "seconds_per_iteration": t_iter,
            "term_amps_per_s": len(xzc[0]) * (1 << L) / (t_apply / steps),
            "sample": f"{steps} Lanczos iterations on the N=56 K=224 U block in complex128 (plain C, OpenMP, "
                      f"no tiling), projected by {matvecs_per_realisation:.0f} matvecs per realisation "
                      f"measured on the GPU"}


def lyapunov_leg(syk, n_real=128, beta=5.0, k=4.0):
    """The t*(N) / lambda_L pipeline end to end on a small ensemble: disorder-averaged
    normalised OTOCs at N = 14, 22, 30 (batched path where it serves, else single-request),
    crossing times at F0 = 0.75 and 0.85, and the fits of Eq. (5) (slope pairs N, N + 8) and
    Eq. (6).  A demonstration of the pipeline and its cost, not a Table I estimate (that needs
    ~10^4 realisations per point and N up to 54)."""
    ts = [0.1 * n for n in range(81)]
    Ns = (14, 22, 30)
    t0 = time.perf_counter()
    curves, paths = {}, {}
    for n_maj in Ns:
        mean, sem, st = syk.otoc_ensemble(n_maj, k, 20000 + 1000 * n_maj, n_real, n_maj - 1, n_maj - 2, beta, ts,
                                          nvec=1, state_seed=30000 + 1000 * n_maj, dtype=syk.C64, m=30, tol=1e-7)
        curves[n_maj] = (mean, sem)
        paths[n_maj] = "batched" if st["path"] == 0 else "single-request"
    wall = time.perf_counter() - t0
    out = {"N": list(Ns), "realisations_per_N": n_real, "beta": beta, "k": k, "t_grid": "0:0.1:8", "paths": paths,
           "wall_s": wall, "realisations_per_h": 3600.0 * n_real * len(Ns) / wall, "F0": {}}
    for F0 in (0.75, 0.85):
        tst, ter = [], []
        for n_maj in Ns:
            a, b = syk.crossing_time(ts, curves[n_maj][0], F0, curves[n_maj][1])
            tst.append(a)
            ter.append(b)
        rec = {"tstar": tst, "tstar_err": ter}
        if all(x == x for x in tst):                     # every curve crossed F0
            sl = syk.lyapunov_fit(Ns, tst, ter, method=syk.FIT_SLOPE, terms=0)
            gl = syk.lyapunov_fit(Ns, tst, ter, method=syk.FIT_GLOBAL, terms=0)
            rec["lambda_slope_eq5"] = [sl["lambda"], sl["lambda_err"]]
            rec["inverse_slopes"] = [list(map(float, sl["points"][0])), list(map(float, sl["points"][1]))]
            rec["lambda_global_eq6"] = [gl["lambda"], gl["lambda_err"]]
        out["F0"][str(F0)] = rec
    return out


def next_rows_leg(syk, h, stream):
    """Costs of the other entry points on this GPU, outside the timed region:
    * green: the Green function G_R(t) of chi_55 on the benchmark realisation (N = 56,
      k = 4, beta = 10, t = 0:0.25:5, complex64, Krylov dim 60, tol 3e-6);
    * dense: one apply_H of dense SYK (p = 1, K = C(38,4) = 73815) at N = 38, best
      autotuned variant, with its VALU-floor fraction; dense_gather: the same at N = 30
      (K = 27405), below the tiled size, where the gather kernel groups terms by x mask;
    * spin_operator: a transverse-field Ising chain on 27 qubits (sum Z_q Z_{q+1} + 0.7 sum X_q)
      through syk_op_to_hamiltonian: one apply_H (best variant) and one e^{-iH} propagation."""
    import math

    import torch
    out = {}
    ts = [0.25 * n for n in range(21)]
    t0 = time.perf_counter()
    raw, nrm, im, st = syk.green(h, N - 1, 10.0, ts, nvec=1, state_seed=STATE_SEED, dtype=syk.C64, m=M_KRYLOV,
                                 tol=TOL_C64, stream=stream)
    wall = time.perf_counter() - t0
    out["green"] = {"n": N - 1, "beta": 10.0, "t_grid": "0:0.25:5", "wall_s": wall, "matvecs": st["matvecs"],
                    "ms_per_matvec": wall * 1e3 / max(st["matvecs"], 1),
                    "G_norm": {str(ts[i]): float(nrm[i]) for i in (0, 4, 8, 20)}}
    syk.release_workspace()

    nd = 38
    hd = syk.create_hamiltonian(nd, 4, math.comb(nd, 4) / nd, 2, syk.BERNOULLI)
    info = hd.info()
    variant, ms = syk.autotune(hd, syk.C64, stream=stream)
    best = min(m for m in ms if m > 0)
    ta = info["K"] * info["block_dim"]
    out["dense"] = {"N": nd, "K": info["K"], "variant": variant, "ms": best, "term_amps_per_s": ta / (best * 1e-3),
                    "valu_floor_frac": ta / 3.93e13 / (best * 1e-3), "variant_ms": ms}
    hd.close()
    # below the tiled size: the gather kernel with terms grouped by x mask
    ng = 30
    hg = syk.create_hamiltonian(ng, 4, math.comb(ng, 4) / ng, 2, syk.BERNOULLI)
    info = hg.info()
    x = torch.randn(info["block_dim"], dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    syk.apply_H(hg, 0, x, y, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        syk.apply_H(hg, 0, x, y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / 20
    ta = info["K"] * info["block_dim"]
    out["dense_gather"] = {"N": ng, "K": info["K"], "x_mask_groups": syk.plan_describe(hg, 0, syk.C64, -1)["n_groups"],
                           "ms": gms, "term_amps_per_s": ta / (gms * 1e-3)}
    del x, y
    hg.close()

    L, g = 27, 0.7
    xs, zs, cs = [], [], []
    for q in range(L - 1):
        xs.append(0), zs.append((1 << q) | (1 << (q + 1))), cs.append(1.0)
    for q in range(L):
        xs.append(1 << q), zs.append(0), cs.append(g)
    op = syk.Operator(L, xs, zs, cs)
    ho = op.to_hamiltonian()
    variant, ms = syk.autotune(ho, syk.C64, stream=stream)
    best = min(m for m in ms if m > 0)
    v = torch.randn(1 << L, dtype=torch.complex64, device="cuda")
    v /= torch.linalg.vector_norm(v)
    w = torch.empty_like(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kst = syk.krylov_expm(ho, 0, -1j, v, w, m=M_KRYLOV, tol=TOL_C64, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["spin_operator"] = {"L": L, "terms": len(xs), "apply_variant": variant, "apply_ms": best,
                            "apply_term_amps_per_s": len(xs) * (1 << L) / (best * 1e-3),
                            "apply_algorithmic_hbm_frac": 2.0 * (1 << L) * 8 / (best * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "expm_wall_s": wall, "expm_stats": kst,
                            "norm_after": float(torch.linalg.vector_norm(w))}
    del v, w
    ho.close()
    op.close()
    syk.release_workspace()
    return out


def batched_leg(syk, n_real=512, seed=3000):
    """Persistent batched launch over n_real small-N realisations (4 Haar states each)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    items = []
    for r in range(n_real):
        n_maj = int(rng.choice([24, 28, 32]))
        k = int(rng.choice([2, 4, 8]))
        items.append((n_maj, k, seed + r, n_maj - 1, n_maj - 2, 100000 + r))
    ts = [0.25 * n for n in range(61)]
    t0 = time.perf_counter()
    raw, nrm, im, st = syk.otoc_batch(items, 10.0, ts, nvec=4, m=30, tol=1e-7)
    wall = time.perf_counter() - t0
    return {"realisations": n_real, "vectors_per_realisation": 4, "jobs": st["n_jobs"], "wall_s": wall,
            "kernel_s": st["kernel_ms"] / 1e3, "realisations_per_h": 3600.0 * n_real / wall,
            "matvecs": st["matvecs"], "launch_shape": st["variant"], "tuned_ms": st["tuned_ms"],
            "slots": st["slots"],
            "mix": "N in {24,28,32}, k in {2,4,8}, seed 3000+r, 4 Haar states, c64, beta=10, t=0:0.25:15, m=30"}


def serving_leg(syk, rate_hz=4.0, window_s=SERVING_WINDOW_S, drain_s=SERVING_DRAIN_S, seed=500):
    """Poisson stream of OTOC requests into the engine (continuous batching)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    Ns, ks = (32, 36, 40, 44, 48), (1, 2, 4, 8)
    ts = [0.5 * n for n in range(11)]
    arrivals, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > window_s:
            break
        arrivals.append((t, int(rng.choice(Ns)), int(rng.choice(ks))))
    eng = syk.Engine(budget_bytes=64 << 30, max_active=4)
    start = time.perf_counter()
    done, i, failed = 0, 0, 0
    while done < len(arrivals):
        now = time.perf_counter() - start
        while i < len(arrivals) and arrivals[i][0] <= now:
            _, n_maj, k = arrivals[i]
            eng.submit(n_maj, k, 50000 + i, 10.0, ts, state_seed=50000 + i, dtype=syk.C64, m=30)
            i += 1
        if now > window_s + drain_s:
            break
        nxt = arrivals[i][0] - now if i < len(arrivals) else 0.5
        r = eng.poll(max(1, int(1000 * min(nxt, 0.5))))
        if r is not None:
            done += 1
            failed += r["status"] != 0
            if done % 25 == 0:
                log(f"serving: {done}/{len(arrivals)} requests done, {now:.0f} s")
    wall = time.perf_counter() - start
    st = eng.stats()
    eng.close()
    return {"requests": len(arrivals), "completed": st["completed"], "failed": st["failed"] + failed,
            "offered_rate_per_s": rate_hz, "window_s": window_s, "wall_s": wall,
            "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
            "realisations_per_h": 3600.0 * st["completed"] / wall,
            "busy_s": st["busy_seconds"], "peak_bytes": st["peak_bytes"], "max_active": 4,
            "mix": "N in {32,36,40,44,48}, k in {1,2,4,8}, beta=10, t=0:0.5:5, c64, m=30, 1 Haar state"}


def serving_c5_leg(syk, seed=5005):
    """A burst of OTOC requests spanning the serving configuration's sizes, N in
    {32, 40, 48, 56, 60, 64} (N = 64: parity blocks of 2^31 amplitudes, 16 GiB per complex64
    vector), submitted at once into an engine whose arena is 85% of free device memory, so
    admission by footprint decides what runs together and the largest requests run at a
    reduced Krylov dimension.  Short chains (beta = 10, t = 0 and 0.5) keep the burst within
    a minute; k is 1 at N >= 60 and drawn from {1, 2, 4, 8} below.  Every request asks for
    its complex64 error against complex128 (precision_check)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ts = [0.0, 0.5]
    reqs = []
    for n_maj in (64, 60, 56, 56, 48, 48, 40, 40, 32, 32):
        k = 1 if n_maj >= 60 else int(rng.choice([1, 2, 4, 8]))
        reqs.append((n_maj, k))
    eng = syk.Engine(budget_bytes=0, max_active=4)
    t0 = time.perf_counter()
    ids = {}
    for i, (n_maj, k) in enumerate(reqs):
        ids[eng.submit(n_maj, k, 70000 + i, 10.0, ts, state_seed=70000 + i, dtype=syk.C64, m=30, m_min=8,
                       precision_check=n_maj <= 56)] = (n_maj, k)
    out = []
    for _ in reqs:
        r = eng.poll(300000)
        if r is None:
            break
        n_maj, k = ids[r["id"]]
        out.append({"N": n_maj, "k": k, "status": r["status"], "m_used": r["m_used"],
                    "footprint_GiB": r["footprint_bytes"] / 2 ** 30, "latency_s": r["t_end"] - r["t_submit"],
                    "run_s": r["t_end"] - r["t_start"], "matvecs": r["stats"]["matvecs"],
                    "mp_err": r["stats"]["mp_err"]})
        log(f"serving_c5: N={n_maj} k={k} done in {out[-1]['latency_s']:.1f} s (m={r['m_used']})")
    wall = time.perf_counter() - t0
    st = eng.stats()
    eng.close()
    lat = sorted(o["latency_s"] for o in out if o["status"] == 0)
    errs = [o["mp_err"] for o in out if o["mp_err"] >= 0]
    return {"requests": len(reqs), "completed": st["completed"], "failed": st["failed"], "wall_s": wall,
            "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
            "budget_GiB": st["budget_bytes"] / 2 ** 30, "peak_GiB": st["peak_bytes"] / 2 ** 30,
            "realisations_per_h": 3600.0 * st["completed"] / wall, "max_mp_err": max(errs) if errs else None,
            "latency_s_sorted": lat, "per_request": out,
            "mix": "burst of 10: N 64, 60, 56, 56, 48, 48, 40, 40, 32, 32; k = 1 at N >= 60, else from {1,2,4,8}; "
                   "beta=10, t=(0, 0.5), c64, m=30 (m_min 8), precision_check at N <= 56"}


def plain_c128_leg(syk, stream):
    """The plain complex128 single-realisation configuration (N = 48, k = 4 so K = 192, seed 48,
    16 Haar states of seed 4800, Krylov dimension 40, beta = 10, t = 0:0.25:20, chi_47 and chi_46),
    timed as one library call in complex128 (tolerance 1e-12) and again with complex64 states
    (FP64 reductions, tolerance 3e-6) on the same realisation and states: realisations per hour
    of each and the largest difference of their normalised curves."""
    import numpy as np
    n_maj = 48
    h = syk.create_hamiltonian(n_maj, 4, 4, 48)
    ts = t_grid()
    res = {}
    for dt, name, kw in ((syk.C128, "c128", dict(m=40)), (syk.C64, "c64", dict(m=40, tol=TOL_C64))):
        syk.autotune(h, dt, stream=stream)

        def progress(done, total, name=name):
            if done % 256 == 0 or done == total:
                log(f"plain_c128: {name} {done}/{total} chain points")

        t0 = time.perf_counter()
        raw, nrm, im, st = syk.otoc(h, n_maj - 1, n_maj - 2, 10.0, ts, nvec=16, state_seed=4800, dtype=dt,
                                    progress=progress, stream=stream, **kw)
        sec = time.perf_counter() - t0
        syk.release_workspace()
        res[name] = {"seconds": sec, "matvecs": st["matvecs"], "realisations_per_h": 3600.0 / sec,
                     "F_norm": {str(ts[i]): float(nrm[i]) for i in (20, 40, 80)}, "_nrm": nrm}
        log(f"plain_c128: {name} {sec:.1f} s, {st['matvecs']} matvecs")
    err = float(np.abs(res["c64"]["_nrm"] - res["c128"]["_nrm"]).max())
    for r in res.values():
        del r["_nrm"]
    h.close()
    return {"plain_c128": True, "config": "N=48, k=4 (K=192), seed 48, 16 Haar states (seed 4800), Krylov dim 40, "
                                          "beta=10, t=0:0.25:20, chi_47 / chi_46",
            "c128": res["c128"], "c64": res["c64"], "max_abs_err_F_norm_c64_vs_c128": err,
            "speedup_c64_over_c128": res["c128"]["seconds"] / res["c64"]["seconds"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--budget", type=float, default=440.0,
                    help="wall seconds from start within which the secondary legs must end")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-sample", action="store_true")
    ap.add_argument("--all-betas", action="store_true",
                    help="time the whole realisation (the beta = 5, 10 and 20 curves) and print their costs")
    ap.add_argument("--plain-c128", action="store_true",
                    help="time the plain complex128 single-realisation configuration (N = 48, k = 4, 16 Haar "
                         "states, Krylov dim 40, beta = 10, t = 0:0.25:20) and the same through complex64")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip every secondary leg except cpu_baseline")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: realisations of the sparse-SYK OTOC are independent jobs "
              "and shard across GPUs with no communication; run one process per GPU with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if not 1 <= args.steps <= CHAIN_POINTS or args.warmup < 0:
        print(f"--steps must lie in [1, {CHAIN_POINTS}] (a step is a segment of one OTOC curve's "
              f"{CHAIN_POINTS} chain points) and --warmup must be >= 0", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2311_00639_amd as syk

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.plain_c128:
        print(json.dumps(plain_c128_leg(syk, stream)), flush=True)
        return
    h = syk.create_hamiltonian(N, 4, K_SPARSITY, SEED)
    info = h.info()
    # one-time setup outside the timed region: plans for every kernel variant, autotuning
    variant, variant_ms = syk.autotune(h, syk.C64, stream=stream)
    plan = syk.plan_describe(h, 0, syk.C64, -1)
    log(f"setup done: variant {variant}, {min(m for m in variant_ms if m > 0):.3f} ms per apply")

    if args.pmc_sample:
        raw, nrm, im, st = syk.otoc(h, N - 1, N - 2, BETA_TIMED, [0.0, 0.25, 0.5], state_seed=STATE_SEED,
                                    dtype=syk.C64, m=M_KRYLOV, tol=TOL_C64, profile=True, stream=stream)
        x = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")
        x.zero_()
        y = x.clone()                     # calibration: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print(json.dumps({"pmc_sample": True, "apply_launches": st["apply_launches"],
                          "apply_ms_avg": st["apply_ms"] / st["apply_launches"], "copy_bytes": x.numel() * 8,
                          "variant": variant, "plan": plan}), flush=True)
        del x, y
        return

    if args.all_betas:
        ts = t_grid()
        out = {"all_betas": True, "curves": {}}
        for beta in BETAS:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            raw, nrm, im, st = syk.otoc(h, N - 1, N - 2, beta, ts, nvec=1, state_seed=STATE_SEED, dtype=syk.C64,
                                        m=M_KRYLOV, tol=TOL_C64, stream=stream)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            out["curves"][str(beta)] = {"seconds": sec, "matvecs": st["matvecs"],
                                        "F_norm": {str(ts[i]): float(nrm[i]) for i in (20, 40, 80)}}
            log(f"beta {beta}: {sec:.1f} s, {st['matvecs']} matvecs")
        tot = sum(c["seconds"] for c in out["curves"].values())
        out["realisation_seconds"] = tot
        out["realisations_per_h"] = 3600.0 / tot
        out["cost_factor_vs_three_beta10"] = tot / (3.0 * out["curves"]["10.0"]["seconds"])
        print(json.dumps(out), flush=True)
        return

    ts = t_grid()
    K_steps = args.steps
    # step s ends at chain point bounds[s] (chain points are counted 1..CHAIN_POINTS)
    bounds = [round((s + 1) * CHAIN_POINTS / K_steps) for s in range(K_steps)]

    if args.warmup:
        # W steps' worth of chain points: the first ceil(nt * W / K) t points, both blocks
        n_warm = min(len(ts), max(1, math.ceil(len(ts) * args.warmup / K_steps)))
        syk.otoc(h, N - 1, N - 2, BETA_TIMED, ts[:n_warm], nvec=1, state_seed=STATE_SEED, dtype=syk.C64,
                 m=M_KRYLOV, tol=TOL_C64, stream=stream)
        log(f"warmup done ({n_warm} t points, both blocks)")

    stamps = []
    t0 = None

    def progress(done, total):
        now = time.perf_counter()
        stamps.append(now)
        k = len(stamps)
        if k in bounds:
            s = bounds.index(k)
            log(f"step {s + 1}/{K_steps} done ({k}/{total} chain points, {now - t0:.1f} s)")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    raw, nrm, im, st = syk.otoc(h, N - 1, N - 2, BETA_TIMED, ts, nvec=1, state_seed=STATE_SEED, dtype=syk.C64,
                                m=M_KRYLOV, tol=TOL_C64, profile=True, progress=progress, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    curve10 = (raw, nrm, im)
    ends = [stamps[b - 1] for b in bounds]
    step_s = [e - s for s, e in zip([t0] + ends[:-1], ends)]

    K = info["K"]
    n = info["block_dim"]
    launches = st["apply_launches"]
    avg_s = st["apply_ms"] / 1e3 / max(launches, 1)
    matvecs = st["matvecs"]
    term_amps = K * n
    flops = 4.0 * term_amps                   # complex amplitude times real coefficient: 2 FMA
    alg_bytes = 2.0 * n * 8                   # read x once, write y once (complex64)
    achieved_tflops = flops / avg_s / 1e12
    value = 3600.0 / (3.0 * elapsed * REALISATION_COST_FACTOR)   # a realisation is the three curves
    t_iter = elapsed / max(matvecs, 1)        # wall time per Lanczos iteration
    valu_floor_s = term_amps / 3.93e13        # one VALU lane-instruction per term-amp
    term_amps_per_real = 3.0 * matvecs * REALISATION_COST_FACTOR * term_amps   # the three curves' matvecs
    lib_rev = syk.kernel_revision()
    traffic = None
    if TRAFFIC["fetch_bytes"] and TRAFFIC["kernel_rev"] == lib_rev and TRAFFIC["variant"] == variant:
        traffic = TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]

    rec = {
        "metric": "apply_H term-amps/s & % HBM peak; OTOC realisations/h N=56 k=4; p50/p99",
        "value": value,
        "unit": "realisations/h",
        "n_gpus": 1,
        "steps": K_steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / K_steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sparse SYK OTOC, mixed precision at scale: N=56, q=4, k=4 (K=224), seed 56, "
                               "complex64 states with double Lanczos reductions and tridiagonal exponential, "
                               "Krylov dim 60, tol 3e-6, t=0:0.25:20, 1 Haar state (seed 5600), W=chi_55, "
                               "V=chi_54; timed: the whole beta=10 curve (2 parity-block chains x 81 t points = "
                               f"{CHAIN_POINTS} chain points), one step = {CHAIN_POINTS}/steps consecutive chain "
                               "points; a realisation = the curves at beta 5, 10 and 20, priced as 3x the "
                               "beta=10 curve times their measured cost factor 1.027",
                   "N": N, "K": K, "block_amps": n, "krylov_m": M_KRYLOV, "krylov_tol": TOL_C64,
                   "beta_timed": BETA_TIMED, "betas_per_realisation": list(BETAS), "nt": len(ts),
                   "parallelism": "single GPU"},
        "step_seconds": {"min": min(step_s), "max": max(step_s)},
        "curve_seconds": elapsed,
        "realisation_cost_factor": REALISATION_COST_FACTOR,
        "value_three_beta10_curves": 3600.0 / (3.0 * elapsed),
        "apply_H_term_amps_per_s": term_amps / avg_s,
        "apply_H_ms": avg_s * 1e3,
        "apply_H_algorithmic_hbm_frac": alg_bytes / avg_s / 1e9 / HBM_PEAK_GBS,
        "apply_H_valu_floor_frac": valu_floor_s / avg_s,
        "apply_H_measured_hbm_TBps": (traffic / avg_s / 1e12) if traffic else None,
        "lanczos_iteration_ms": t_iter * 1e3,
        "lanczos_iteration_algorithmic_hbm_frac": 7.0 * n * 8 / t_iter / 1e9 / HBM_PEAK_GBS,
        "matvecs_per_curve": matvecs,
        "kernel": {"revision": lib_rev, "variant": variant, "variant_ms": variant_ms, "plan": plan},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "frac_of_nonpacked_fp32": achieved_tflops / FP32_NONPACKED_PEAK_TFLOPS,
                     "algorithmic_hbm_frac": alg_bytes / avg_s / 1e9 / HBM_PEAK_GBS,
                     "measured_hbm_frac": (traffic / avg_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "kernel": "apply_h_tiled", "launches_timed": launches,
                     "per_launch": {"term_amps": term_amps, "flop": flops, "algorithmic_bytes": alg_bytes}},
        "otoc_F_norm": {str(ts[i]): float(nrm[i]) for i in (4, 20, 40, 80)},
    }
    log(f"timed curve: {elapsed:.1f} s, {matvecs} matvecs, apply {avg_s * 1e3:.3f} ms; "
        f"{value:.3f} realisations/h")

    # every leg below runs only if its estimated cost still fits in the wall budget
    def fits(name, est_s):
        left = args.budget - (time.perf_counter() - T_START)
        if est_s > left:
            rec.setdefault("legs_skipped", []).append(name)
            log(f"{name}: skipped ({est_s:.0f} s estimated, {left:.0f} s of the budget left)")
            return False
        log(f"{name} ({left:.0f} s of the budget left)")
        return True

    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(term_amps_per_real, seconds_target=10.0)
    extras = not args.no_extras
    if extras and not args.no_precision and fits("mixed_precision", 70):
        syk.release_workspace()
        rec["mixed_precision"] = mixed_precision_check(syk, curve10, stream)
        syk.release_workspace()
    if extras and not args.no_serving and fits("serving", SERVING_WINDOW_S + SERVING_DRAIN_S + 15):
        rec["serving"] = serving_leg(syk)
        syk.release_workspace()
    if extras and not args.no_serving and fits("serving_c5", 95):
        rec["serving_c5"] = serving_c5_leg(syk)
        syk.release_workspace()
    if extras and not args.no_batched and fits("batched", 30):
        rec["batched"] = batched_leg(syk)
    if extras and not args.no_precision and fits("apply_k1", 20):
        rec["apply_k1"] = apply_k1_leg(syk, stream)
        syk.release_workspace()
    if extras and not args.no_cpu_baseline and fits("plain_cpu_lanczos", 45):
        rec["cpu_baseline"]["plain_cpu_lanczos"] = cpu_lanczos_leg(3.0 * matvecs * REALISATION_COST_FACTOR)
    if extras and not args.no_precision and fits("other_entry_points", 30):
        rec["other_entry_points"] = next_rows_leg(syk, h, stream)
    if extras and not args.no_batched and fits("lyapunov_pipeline", 45):
        rec["lyapunov_pipeline"] = lyapunov_leg(syk)
    rec["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
