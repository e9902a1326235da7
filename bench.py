"""Benchmark of the hybrid tree force path on one MI355X.

One step = one soft step of the two-timestep leapfrog on the N = 2^20
Plummer sphere (eps = 0.01, theta = 0.5, cutoff for ~64 neighbours,
R1 = R2/2, 4 hard substeps of 1/64): four tree builds, one soft force, four
hard forces and the kicks and drifts, all inside libhtree on the GPU.

Prints one JSON line.  ``value`` is the whole-job interaction rate: (soft
interactions + accepted hard pairs) per step divided by the step time.  The
``roofline`` object describes the dominant kernel (the soft walk+interaction
kernel), timed with HIP events recorded by the library on its stream over the
timed steps; ``cpu_baseline`` times the FP64 oracle on the host cores on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 flops per interaction: a monopole or far
# particle term is 3 sub, 3 fma (r^2 + eps^2), 1 rsqrt, 3 mul, 3 fma (FMA = 2
# flops) = 19; a near particle term adds the unsoftened r^2 (5), sqrt (1) and
# the (1 - K) polynomial and weight (7) = 32.
FLOPS_FAR = 19
FLOPS_NEAR = 32
# MI355X vector peaks derived from the unit counts: 256 CUs x 4 SIMD x 16 lanes
# x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for non-packed FP32 (the build
# disables packed FP32); the published packed figure is 157.3 TFLOP/s.
PEAK_FP32 = 78.6
PEAK_FP32_PACKED = 157.3


def cpu_baseline(wl, x, m64, seconds_hint=20.0):
    """Oracle soft force (tree walk + FP64 interactions) over a sample of
    sink groups of the same tree, on all host threads."""
    import numpy as np

    import oracle
    import synth
    t0 = time.perf_counter()
    T = oracle.Tree(x, m64, n_crit=wl.n_crit, theta=wl.theta)
    t_build = time.perf_counter() - t0
    ng = T.ngroups
    k = 16
    groups = synth.sample_indices(ng, k, 7)
    t0 = time.perf_counter()
    _, _, inter = T.soft(1.0, wl.eps, wl.R1, wl.R2, 1, groups=groups)
    dt = time.perf_counter() - t0
    # grow the sample to fill about seconds_hint of CPU time
    k2 = int(min(ng, max(k, k * seconds_hint / max(dt, 1e-3))))
    groups = synth.sample_indices(ng, k2, 8)
    t0 = time.perf_counter()
    _, _, inter = T.soft(1.0, wl.eps, wl.R1, wl.R2, 1, groups=groups)
    dt = time.perf_counter() - t0
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 oracle soft force (walk + interactions) for %d of %d sink groups "
                      "of the N=2^20 Plummer tree (%d interactions, %.1f s; tree build %.1f s "
                      "not included)" % (k2, ng, inter, dt, t_build)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the force path is single-GPU by design "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1406_6158_amd as P
    import synth

    wl = synth.WORKLOADS["plummer1m"]
    x, v, m = wl.make()
    v32 = v.astype(np.float32)
    m32 = m.astype(np.float32)
    params = P.default_params(eps=wl.eps, theta=wl.theta, R1=wl.R1, R2=wl.R2,
                              dt_soft=wl.dt_soft, n_sub=wl.n_sub, hybrid=1, n_crit=wl.n_crit,
                              flags=P.F_TIMING)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = P.HTree(wl.n, params, device=dev)
    t.set_state(torch.from_numpy(x), torch.from_numpy(v32), torch.from_numpy(m32))
    print("bench: %s N=%d, warmup %d, steps %d" % (wl.name, wl.n, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    for k in range(args.warmup):
        t.step(1)
        t.sync()
        print("bench: warmup step %d done" % k, file=sys.stderr, flush=True)
    t.stats()                                # reset counters and event timings
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        t.step(1)
    t.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = t.stats()
    K = args.steps
    ms_step = 1e3 * wall / K
    soft_inter = st["soft_interactions"] / K
    hard_pairs = st["hard_pairs"] / K
    value = (soft_inter + hard_pairs) / (wall / K)

    # dominant kernel: the soft walk + interaction kernel
    calls = max(st["calls_soft"], 1)
    soft_ms = st["ms_soft"] / calls
    near_frac = st["soft_near"] / max(st["soft_cells"] + st["soft_far"] + st["soft_near"], 1)
    flops = soft_inter * (FLOPS_FAR * (1 - near_frac) + FLOPS_NEAR * near_frac)
    achieved = flops / (soft_ms * 1e-3) / 1e12
    line = {
        "metric": "interactions/s + s/step at N=2^20 Plummer; batched p50/p99 solve latency",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "s_per_step": ms_step / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plummer N=2^20 eps=0.01 theta=0.5 ngb~64 n_sub=4 dt_h=1/64",
                   "n": wl.n, "theta": wl.theta, "eps": wl.eps, "R2": wl.R2, "n_sub": wl.n_sub,
                   "group": 64, "n_crit": wl.n_crit},
        "soft_interactions_per_step": soft_inter,
        "hard_pairs_per_step": hard_pairs,
        "hard_candidates_per_step": st["hard_candidates"] / K,
        "soft_kernel_interactions_per_s": soft_inter / (soft_ms * 1e-3),
        "phase_ms_per_step": {"build": st["ms_build"] / K, "soft": st["ms_soft"] / K,
                              "hard": st["ms_hard"] / K},
        "roofline": {"kernel": "k_soft (walk + FP32 interactions)", "bound": "alu",
                     "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32,
                     "frac_of_packed_fp32_peak": achieved / PEAK_FP32_PACKED,
                     "traffic": None},
        "cpu_baseline": None,
    }
    t.close()
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, x, m32.astype(np.float64))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
