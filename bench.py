"""Benchmark of the sparse-SYK OTOC hot path on one MI355X.

Workload (mixed precision at scale): N = 56 Majoranas (parity blocks of 2^27 amplitudes),
q = 4, k = 4 (K = 224 terms), one disorder realisation (seed 56), complex64 state
vectors with double Lanczos reductions and tridiagonal exponential, Krylov dimension 60,
one Haar state (state_seed 5600), W = chi_55, V = chi_54, beta in {5, 10, 20},
t = 0, 0.25, ..., 20 (81 points).  One step is one OTOC realisation: the three beta
curves, both parity-block chains, every t point.

Printed: one JSON line.  value = OTOC realisations per hour; roofline of the dominant
kernel (apply_H) from HIP-event timings of every apply_H launch in the timed region;
cpu_baseline = the oracle's matrix-free row evaluation timed on a bounded sample and
scaled by the term-amplitudes one realisation needs.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K_SPARSITY, SEED, STATE_SEED = 56, 4, 56, 5600
BETAS = (5.0, 10.0, 20.0)
M_KRYLOV = 60
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


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
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the sparse-SYK OTOC path here is single-GPU "
              "(realisations shard across GPUs as independent jobs); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2311_00639_amd as syk

    torch.cuda.set_device(0)
    h = syk.create_hamiltonian(N, 4, K_SPARSITY, SEED)
    info = h.info()
    ts = t_grid()
    stream = torch.cuda.current_stream()

    def step(profile):
        out = []
        for beta in BETAS:
            raw, nrm, im, st = syk.otoc(h, N - 1, N - 2, beta, ts, nvec=1, state_seed=STATE_SEED, dtype=syk.C64,
                                        m=M_KRYLOV, profile=profile, stream=stream)
            out.append((raw, nrm, im, st))
        return out

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step(True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    apply_ms = sum(st["apply_ms"] for r in results for (_, _, _, st) in r)
    launches = sum(st["apply_launches"] for r in results for (_, _, _, st) in r)
    matvecs = sum(st["matvecs"] for r in results for (_, _, _, st) in r)
    K = info["K"]
    n = info["block_dim"]
    avg_s = apply_ms / 1e3 / max(launches, 1)
    term_amps = K * n
    flops = 4.0 * term_amps                   # complex amplitude times real coefficient: 2 FMA
    alg_bytes = 2.0 * n * 8                   # read x once, write y once (complex64)
    achieved_tflops = flops / avg_s / 1e12
    value = args.steps * 3600.0 / elapsed
    term_amps_per_real = matvecs / args.steps * term_amps

    rec = {
        "metric": "apply_H term-amps/s & % HBM peak; OTOC realisations/h N=56 k=4; p50/p99",
        "value": value,
        "unit": "realisations/h",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sparse SYK OTOC realisation: N=56, q=4, k=4 (K=224), complex64 states, "
                               "double Lanczos reductions, Krylov dim 60, beta in {5,10,20}, t=0:0.25:20, "
                               "1 Haar state, W=chi_55, V=chi_54",
                   "N": N, "K": K, "block_amps": n, "krylov_m": M_KRYLOV, "betas": list(BETAS), "nt": len(ts),
                   "parallelism": "single GPU"},
        "apply_H_term_amps_per_s": term_amps / avg_s,
        "apply_H_ms": avg_s * 1e3,
        "apply_H_algorithmic_hbm_frac": alg_bytes / avg_s / 1e9 / HBM_PEAK_GBS,
        "matvecs_per_realisation": matvecs / args.steps,
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "apply_H", "launches_timed": launches},
        "otoc_F_norm_t1": {str(b): float(r[1][4]) for b, r in zip(BETAS, results[-1])},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(term_amps_per_real)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
