"""Benchmark of the hybrid tree force path on one MI355X.

One step = one soft step of the two-timestep leapfrog on the N = 2^20
Plummer sphere (eps = 0.01, theta = 0.5, cutoff for ~64 neighbours,
R1 = R2/2, 4 hard substeps of 1/64): one tree build, three refits of the
node boxes, one soft force, four hard forces and the kicks and drifts, all
inside libhtree on the GPU.

Prints one JSON line.  ``value`` is the whole-job interaction rate: (soft
interactions + accepted hard pairs) per step divided by the step time.  The
``roofline`` object describes the dominant kernel by time (the hard kernel:
FP64 pair tests and pair forces), ``roofline_interaction`` the soft walk +
FP32 interaction kernel; both are timed with HIP events recorded by the
library on its stream around each launch over the timed steps.
``cpu_baseline`` times the FP64 oracle on the host cores on a bounded sample
of the same workload, and compares the library's forces of the benchmarked
configuration (same positions, same launch configuration) with the
oracle's on that sample: ``parity`` repeats the p99 errors.

Two further sections run after the timed steps and are reported beside
them: ``ensemble`` (512 independent Plummer clusters, N log-uniform in
[2^10, 2^16], one batched context after autotuning (g, n_crit) per size
class, against the same 512 systems run one after another as single
contexts) and ``serving`` (Poisson arrivals at 500/s of force solves with N
log-uniform in [2^12, 2^20], admitted by HBM footprint into the request
server, p50/p99 latency).

    python bench.py [--gpus 1] [--steps 16] [--warmup 1] [--no-cpu-baseline]
                    [--no-ensemble] [--no-serve] [--serve-requests 20000]
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
# the (1 - K) polynomial and weight (7) = 32.  Beyond R2 the weight is 1 by
# the definition of K, so a stricter count gives 32 only to the near pairs
# within R2 (the hard kernel's pairs, plus each sink with itself) and 19 to
# every other entry; both are reported.
FLOPS_FAR = 19
FLOPS_NEAR = 32
# Algorithmic FP64 flops of the hard force (section II.C eqs. 7-10): a
# candidate pair test is 3 sub, 1 mul, 2 fma (r^2) = 8; an accepted pair adds
# r = sqrt(r^2) (1), r^2 + eps^2 (1), its inverse 3/2 power (rsqrt and two
# mul, 3), K(r) (Y: sub and mul, Y^2, two fma, Y^6 by two mul, product: 10),
# the factor m K / (r^2 + eps^2)^{3/2} (2) and the three fma of the sum (6)
# = 23, whatever instructions an implementation spends on them.
FLOPS_HARD_TEST = 8
FLOPS_HARD_PAIR = 23
PEAK_FP64 = 78.6
# MI355X vector peaks derived from the unit counts: 256 CUs x 4 SIMD x 16 lanes
# x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for non-packed FP32 (the build
# disables packed FP32); the published packed figure is 157.3 TFLOP/s.
PEAK_FP32 = 78.6
PEAK_FP32_PACKED = 157.3

# HBM bytes per launch at this workload, from rocprofv3 counters: reads from
# the L2-to-memory read requests counted by size (32, 64, 128 bytes: exact;
# FETCH_SIZE counts a 128-byte request as 64 bytes on this GPU, which a plain
# copy and a random gather calibrate), writes from WRITE_SIZE (exact on a plain
# copy).  The hard figure is the mean of a step's four launches (one after the
# build that records the searches, three after refits that replay them).  The
# summary with commands is profiles/counters_plummer1m_step.txt.  Valid only
# for the kernel source it was measured on: reported as null once force.hip or
# htree_dev.h differ from that source.
SOFT_TRAFFIC = {"bytes": 1872.6e6, "source_hash": "8807390a0a87b499"}
HARD_TRAFFIC = {"bytes": 1618.8e6, "source_hash": "8807390a0a87b499"}


def _kernel_source_hash():
    """Hash of the soft kernel's sources with comments and blank lines
    dropped (comment edits do not change the kernel)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1406_6158_amd", "csrc")
    h = hashlib.sha256()
    for name in ("force.hip", "htree_dev.h"):
        with open(os.path.join(csrc, name)) as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def cpu_baseline(wl, x, m64, gpu=None, seconds_hint=20.0):
    """Oracle soft force (tree walk + FP64 interactions) over a sample of
    sink groups of the same tree, on all host threads.  With ``gpu`` (the
    library's soft and hard forces and neighbour counts of the benchmarked
    configuration at the same positions, caller order), also the parity of
    those results against the oracle on the sampled groups and sinks."""
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
    o_soft, _, inter = T.soft(1.0, wl.eps, wl.R1, wl.R2, 1, groups=groups)
    dt = time.perf_counter() - t0
    # the other phases, for context: the hard force (direct neighbour sums) on
    # a sample of sinks, and the direct force on a sample, both scaled to N
    n = x.shape[1]
    hs = synth.sample_indices(n, 4096, 9)
    t0 = time.perf_counter()
    o_hard, _, o_ngb = oracle.split_direct(x, m64, 1.0, wl.eps, wl.R1, wl.R2, sinks=hs, soft=False)
    t_hard = (time.perf_counter() - t0) * n / len(hs)
    parity = None
    if gpu is not None:
        perm, _, _ = T.sorted()
        st = T.group_starts()
        sinks = np.concatenate([perm[st[k]:st[k + 1]] for k in groups])

        def rel(a, ref):
            # sinks without neighbours have a zero hard force; they are masked out below
            with np.errstate(invalid="ignore", divide="ignore"):
                return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)

        es = rel(gpu["soft"][:, sinks], o_soft[:, sinks])
        hm = o_ngb > 0
        eh = rel(gpu["hard"][:, hs], o_hard)[hm]
        parity = {
            "reference": "FP64 oracle on the same tree and lists (soft: every sink of the %d "
                         "sampled groups; hard: %d sampled sinks, brute-force neighbour sets)"
                         % (len(groups), len(hs)),
            "soft_p50": float(np.percentile(es, 50)), "soft_p99": float(np.percentile(es, 99)),
            "soft_max": float(es.max()), "soft_sinks": int(sinks.size),
            "hard_p50": float(np.percentile(eh, 50)), "hard_p99": float(np.percentile(eh, 99)),
            "hard_max": float(eh.max()),
            "hard_ngb_exact": bool(np.array_equal(gpu["ngb"][hs], o_ngb)),
            "tolerance_p99": 1e-5,
        }
    ds = synth.sample_indices(n, 1024, 10)
    t0 = time.perf_counter()
    oracle.direct(x, m64, 1.0, wl.eps, sinks=ds)
    t_direct = (time.perf_counter() - t0) * n / len(ds)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    # the same soft interaction loops on the host's SIMD units and threads
    # (paper_1406_6158_amd/cpu: the CPU/GPU comparison of section IV.C), on
    # synthetic groups with this tree's mean list lengths per group
    host = None
    try:
        from paper_1406_6158_amd import cpu_compare
        pc, far, near = T.walk_counts(wl.R2, 1)
        nf = int(round(float(np.mean(pc + far))))
        nn = int(round(float(np.mean(near))))
        hrate, hthreads = cpu_compare.rate(nf, nn, wl.eps * wl.eps, wl.R2, 1.0 / (wl.R2 - wl.R1),
                                           groups=2048, threads=oracle.threads(), repeat=3)
        host = {"value": hrate, "unit": "interactions/s", "threads": hthreads,
                "kind": "host SIMD soft interaction loops (AVX2 FP32, compensated tiles)",
                "lists": "2048 synthetic groups of 64 sinks with this tree's mean lists per "
                         "group: %d far (cells + far particles) and %d near sources" % (nf, nn)}
    except (RuntimeError, OSError) as e:
        host = {"value": None, "error": str(e)}
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu, "host_simd_kernels": host,
            "sample": "FP64 oracle soft force (walk + interactions) for %d of %d sink groups "
                      "of the N=2^20 Plummer tree (%d interactions, %.1f s; tree build %.1f s "
                      "not included)" % (k2, ng, inter, dt, t_build),
            "phases_s": {"tree_build": t_build,
                         "soft_all_groups_extrapolated": dt * ng / k2,
                         "hard_extrapolated_from_4096_sinks": t_hard,
                         "direct_extrapolated_from_1024_sinks": t_direct},
            "parity": parity}


def _log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def direct_sample(torch, X, M, idx, G, eps, chunk=128):
    """FP64 direct sum of the softened force (plain torch arithmetic on the
    GPU, independent of the library) on the sinks `idx`: the accuracy
    reference of the comparator."""
    out = torch.empty(3, len(idx), dtype=torch.float64, device=X.device)
    for c0 in range(0, len(idx), chunk):
        xi = X[:, idx[c0:c0 + chunk]]
        d = X[:, None, :] - xi[:, :, None]
        r2 = (d * d).sum(0) + eps * eps
        w = M[None, :] * r2.rsqrt() ** 3
        out[:, c0:c0 + chunk] = G * (d * w[None]).sum(-1)
    return out


def comparator(P, torch, wl, x, v32, m32, hyb_ms_step, hard_ms_call, steps):
    """The plain tree (hybrid = 0, one force per dt_h) at the same force
    accuracy: theta bisected until its p99 force error on 2^14 sampled sinks
    equals that of the hybrid force (soft at theta = 0.5 plus hard), both
    against an FP64 direct sum.  Reports R_hybrid = T_hybrid(dt_s) /
    (n T_tree) and T_hard / T_tree."""
    import numpy as np

    import synth
    n = wl.n
    idx = torch.from_numpy(synth.sample_indices(n, wl.sample, wl.sample_seed)).cuda()
    X = torch.from_numpy(x).cuda()
    V = torch.from_numpy(v32).cuda()
    M = torch.from_numpy(m32).cuda()
    ref = direct_sample(torch, X, M.double(), idx, 1.0, wl.eps)
    refn = ref.norm(dim=0)

    def p99(theta, hybrid, **kw):
        p = P.default_params(eps=wl.eps, theta=theta, R1=wl.R1, R2=wl.R2, hybrid=hybrid,
                             n_crit=wl.n_crit, **kw)
        t = P.HTree(n, p)
        t.set_state(X, V, M)
        t.build_tree()
        a = t.soft_force()
        if hybrid:
            h, _ = t.hard_force()
            a = a + h
        t.sync()
        e = (a[:, idx].double() - ref).norm(dim=0) / refn
        t.close()
        return float(torch.quantile(e, 0.99))

    e_h = p99(wl.theta, 1)
    lo, hi = 0.05, 1.5
    e_lo, e_hi = p99(lo, 0), p99(hi, 0)
    for _ in range(10):
        mid = 0.5 * (lo + hi)
        e = p99(mid, 0)
        if e > e_h:
            hi, e_hi = mid, e
        else:
            lo, e_lo = mid, e
    theta_eq = lo
    _log("comparator: hybrid p99 %.3e; plain tree theta %.4f gives %.3e" % (e_h, lo, e_lo))
    p = P.default_params(eps=wl.eps, theta=theta_eq, hybrid=0, n_sub=1,
                         dt_soft=wl.dt_soft / wl.n_sub, n_crit=wl.n_crit, flags=P.F_TIMING)
    t = P.HTree(n, p)
    t.set_state(X, V, M)
    t.step(1)
    t.sync()
    t.stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        t.step(1)
    t.sync()
    ms_tree = 1e3 * (time.perf_counter() - t0) / steps
    st = t.stats()
    t.close()
    # the paper's own opening rule (section II.B absolute MAC, a_err = 2^-8 as
    # in section IV.A, groups measured by their nearest sink) in the same
    # hybrid step: its force error on the same sample and its step time
    mac = dict(a_err=2.0 ** -8, group_mac=1)
    e_mac = p99(wl.theta, 1, **mac)
    p = P.default_params(eps=wl.eps, R1=wl.R1, R2=wl.R2, dt_soft=wl.dt_soft, n_sub=wl.n_sub,
                         hybrid=1, n_crit=wl.n_crit, flags=P.F_TIMING | P.F_REUSE, **mac)
    t = P.HTree(n, p)
    t.set_state(X, V, M)
    t.step(1)
    t.sync()
    t.stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        t.step(1)
    t.sync()
    ms_mac = 1e3 * (time.perf_counter() - t0) / steps
    sm = t.stats()
    t.close()
    _log("paper MAC: p99 %.3e, %.3f ms per step" % (e_mac, ms_mac))
    paper_mac = {"a_err": 2.0 ** -8, "group_rule": "minimum over sinks",
                 "p99_force_error": e_mac, "ms_per_step": ms_mac,
                 "soft_interactions_per_step": sm["soft_interactions"] / steps,
                 "phase_ms_per_step": {"build": sm["ms_build"] / steps,
                                       "soft": sm["ms_soft"] / steps,
                                       "hard": sm["ms_hard"] / steps}}
    return {
        "what": "plain tree (hybrid=0, one force per dt_h=1/64) at the hybrid's force accuracy",
        "reference": "FP64 direct sum on %d sampled sinks (seed %d)" % (wl.sample, wl.sample_seed),
        "hybrid_p99_force_error": e_h, "plain_theta": theta_eq, "plain_p99_force_error": e_lo,
        "T_tree_ms": ms_tree,
        "T_tree_phase_ms": {"build": st["ms_build"] / steps, "soft": st["ms_soft"] / steps},
        "T_hybrid_ms": hyb_ms_step,
        "R_hybrid": hyb_ms_step / (wl.n_sub * ms_tree),
        "T_hard_over_T_tree": hard_ms_call / ms_tree,
        "paper_context": "the paper reports R_hybrid 0.8-0.9 and 0.7 and T_hard about 0.4 of a "
                         "tree force on its GPU cluster (different hardware)",
        "hybrid_with_paper_mac": paper_mac,
    }


def ensemble(P, torch, steps, count=512):
    """Batched context over `count` Plummer clusters (sizes log-uniform in
    [2^10, 2^16], eps = 4 / N^(1/3), theta = 0.5, cutoff for ~32 neighbours,
    4 hard substeps of 1/64 per soft step) against the same systems stepped one
    after another as single contexts on one stream."""
    import numpy as np

    import synth
    from paper_1406_6158_amd import autotune
    sizes = [int(n) for n in synth.ensemble_sizes(count)]
    _log("ensemble: %d systems, %d particles" % (len(sizes), sum(sizes)))
    systems = []
    for k, n in enumerate(sizes):
        x, v, m = synth.plummer(n, 4000 + k)
        systems.append(dict(n=n, x=torch.from_numpy(x).cuda(),
                            v=torch.from_numpy(v.astype(np.float32)).cuda(),
                            m=torch.from_numpy(m.astype(np.float32)).cuda()))

    def mk(k, g, nc, flags=P.F_TIMING | P.F_REUSE):
        n = sizes[k]
        R2 = synth.r2_for_neighbours("plummer", n, 32)
        return P.default_params(eps=4.0 / n ** (1.0 / 3.0), theta=0.5, R1=R2 / 2, R2=R2,
                                dt_soft=1.0 / 16.0, n_sub=4, hybrid=1, n_crit=nc,
                                group_size=g, flags=flags)

    table, times = autotune.tune(P, torch, systems, mk, log=_log)
    params = [mk(k, *table[autotune.size_class(n)], flags=P.F_REUSE) for k, n in enumerate(sizes)]
    x = torch.cat([s["x"] for s in systems], dim=1)
    v = torch.cat([s["v"] for s in systems], dim=1)
    m = torch.cat([s["m"] for s in systems])
    t = P.HTree(sizes, params)
    t.set_state(x, v, m)
    t.step(1)
    t.sync()
    t.stats()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(t.stream)
        t.step(1)
        e1.record(t.stream)
    t.sync()
    st = t.stats()
    step_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    inter = (st["soft_interactions"] + st["hard_pairs"]) / steps
    t.close()
    del x, v, m
    _log("ensemble: batched step %.3f ms (p50)" % _pct(step_ms, 50))
    # the same systems as single contexts, one after another on one stream
    singles = []
    for k, s in enumerate(systems):
        h = P.HTree(s["n"], params[k])
        h.set_state(s["x"], s["v"], s["m"])
        singles.append(h)
    for h in singles:
        h.step(1)
    torch.cuda.synchronize()
    stream = singles[0].stream
    start = torch.cuda.Event(enable_timing=True)
    done = [torch.cuda.Event(enable_timing=True) for _ in singles]
    start.record(stream)
    for h, e in zip(singles, done):
        h.step(1)
        e.record(stream)
    torch.cuda.synchronize()
    lat = [start.elapsed_time(e) for e in done]
    for h in singles:
        h.close()
    _log("ensemble: sequential total %.3f ms" % lat[-1])
    return {
        "workload": "%d Plummer clusters, N log-uniform in [2^10, 2^16] (seed 4), eps=4/N^(1/3), "
                    "theta=0.5, ngb~32, n_sub=4, dt_h=1/64" % len(sizes),
        "systems": len(sizes), "particles": sum(sizes),
        "autotune": {"2^%d" % c: {"g": g, "n_crit": nc, "ms": times[c][(g, nc)]}
                     for c, (g, nc) in table.items()},
        "batched_ms_per_step": {"p50": _pct(step_ms, 50), "p99": _pct(step_ms, 99),
                                "mean": float(np.mean(step_ms)), "steps": steps},
        "batched_interactions_per_s": inter / (np.mean(step_ms) * 1e-3),
        "sequential_latency_ms": {"p50": _pct(lat, 50), "p99": _pct(lat, 99),
                                  "total": lat[-1]},
        "sequential_over_batched": lat[-1] / float(np.mean(step_ms)),
    }


def serving(P, torch, n_req, warm, arena_bytes, label, pool_per_model=2):
    """Poisson arrivals (500/s) of hybrid force solves, N log-uniform in
    [2^12, 2^20], Plummer or cold cube, theta in [0.4, 0.7]; eps =
    0.01 (2^20/N)^(1/3), cutoff for ~64 neighbours.  Each request's
    positions are the first N particles of one of a few pre-drawn 2^20-particle
    sets of its model (an i.i.d. sample's prefix is an i.i.d. sample); their
    masses are 2^-20 each with G = 2^20/N, which gives the accelerations of N
    equal masses of total mass 1."""
    import numpy as np

    import synth
    nmax = 1 << 20
    reqs = synth.serving_requests(n_req + warm)
    pool = {}
    for model, gen in (("plummer", synth.plummer), ("cube", synth.cold_cube)):
        pool[model] = [torch.from_numpy(gen(nmax, 7000 + 10 * j + (model == "cube"))[0]).cuda()
                       for j in range(pool_per_model)]
    m_pool = torch.full((nmax,), 1.0 / nmax, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    def params(r):
        n = r["n"]
        R2 = synth.r2_for_neighbours(r["model"], n, 64)
        return P.default_params(G=nmax / n, eps=0.01 * (nmax / n) ** (1.0 / 3.0),
                                theta=r["theta"], R1=R2 / 2, R2=R2, hybrid=1)

    arrive = np.array([r["t"] for r in reqs])
    done_t = np.full(len(reqs), np.nan)
    inter = np.zeros(len(reqs))
    idx = {}
    srv = P.Server(arena_bytes, n_streams=4, per_stream=2)
    k = 0
    n_done = 0
    max_pending = 0
    _log("serving[%s]: %d requests (+%d warm-up), arena %.1f GiB"
         % (label, n_req, warm, arena_bytes / 2 ** 30))
    t0 = time.perf_counter()
    while n_done < len(reqs):
        now = time.perf_counter() - t0
        while k < len(reqs) and arrive[k] <= now:
            r = reqs[k]
            x = pool[r["model"]][k % pool_per_model][:, :r["n"]]
            idx[srv.submit(params(r), x, m_pool[:r["n"]])] = k
            k += 1
        fin = srv.poll()
        if fin:
            tnow = time.perf_counter() - t0
            for rid in fin:
                j = idx.pop(rid)
                inf = srv.info(rid)
                if inf["status"] != 0:
                    raise RuntimeError("request %d failed with status %d" % (j, inf["status"]))
                done_t[j] = tnow
                inter[j] = inf["soft_interactions"] + inf["hard_pairs"]
                srv.release(rid)
                n_done += 1
                if n_done % 2000 == 0:
                    _log("serving[%s]: %d done" % (label, n_done))
        max_pending = max(max_pending, k - n_done)
    st = srv.stats()
    srv.close()
    sel = slice(warm, None)
    lat = (done_t - arrive)[sel] * 1e3
    span = np.nanmax(done_t[sel]) - arrive[warm]
    ns = np.array([r["n"] for r in reqs])[sel]
    return {
        "workload": "Poisson arrivals 500/s (seed 5), N log-uniform in [2^12, 2^20], Plummer or "
                    "cold cube, theta U[0.4, 0.7], eps=0.01(2^20/N)^(1/3), ngb~64, hybrid "
                    "build+soft+hard per request",
        "arena_gib": arena_bytes / 2 ** 30, "requests": n_req, "warmup_requests": warm,
        "streams": 4, "per_stream": 2,
        "latency_ms": {"p50": _pct(lat, 50), "p99": _pct(lat, 99), "max": float(np.max(lat)),
                       "mean": float(np.mean(lat))},
        "latency_ms_large_n": {"p50": _pct(lat[ns >= 1 << 18], 50),
                               "p99": _pct(lat[ns >= 1 << 18], 99)},
        "served_requests_per_s": n_req / span,
        "served_interactions_per_s": float(inter[sel].sum() / span),
        "peak_in_flight": st["peak_in_flight"], "max_outstanding": int(max_pending),
        "arena_peak_gib": st["bytes_peak"] / 2 ** 30,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=8)
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--paper-mac", action="store_true",
                    help="time the same step with the paper's opening rule (absolute MAC, "
                         "a_err = 2^-8, groups measured by their nearest sink) instead of "
                         "theta = 0.5; the step line only (for kernel profiles of that rule)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the reference kernels for scaling HBM byte counters and "
                         "exit: a plain 512 MiB device copy and a gather of 2^24 records of "
                         "32 bytes in random order, five times each")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        # the force kernels gather records of particles (x, y, z, m: 32 bytes)
        # by index, so the counters are also calibrated on a gather of 32-byte
        # rows in random order
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        rows = 1 << 24
        src = torch.ones(rows, 4, dtype=torch.float64, device="cuda")
        idx = torch.randperm(rows, device="cuda", generator=g)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.index_select(src, 0, idx, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": (1 << 27) * 4, "copy_bytes_written": (1 << 27) * 4,
                          "gather_rows": rows, "gather_row_bytes": 32,
                          "gather_bytes_read": rows * 32 + rows * 8,
                          "gather_bytes_written": rows * 32, "launches": 5}))
        return
    if args.paper_mac:
        # the parity, ensemble, serving and comparator legs are defined for the
        # theta rule
        args.no_cpu_baseline = args.no_ensemble = args.no_serve = args.no_comparator = True
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
    # the hard searches recorded after each build are replayed on the three
    # refitted substeps (exact neighbour sets; measured faster than walking
    # from the root every substep)
    opening = dict(a_err=2.0 ** -8, group_mac=1) if args.paper_mac else {}
    params = P.default_params(eps=wl.eps, theta=wl.theta, R1=wl.R1, R2=wl.R2,
                              dt_soft=wl.dt_soft, n_sub=wl.n_sub, hybrid=1, n_crit=wl.n_crit,
                              flags=P.F_TIMING | P.F_REUSE, **opening)
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
    gpu_forces = None
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(t.stream)
        t.step(1)
        evs[k][1].record(t.stream)
    t.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = t.stats()
    K = args.steps
    ms_step = 1e3 * wall / K
    step_ms = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    ms_median = step_ms[len(step_ms) // 2]
    soft_inter = st["soft_interactions"] / K
    hard_pairs = st["hard_pairs"] / K
    value = (soft_inter + hard_pairs) / (wall / K)

    # the soft walk + interaction kernel
    calls = max(st["calls_soft"], 1)
    soft_ms = st["ms_soft"] / calls
    near_frac = st["soft_near"] / max(st["soft_cells"] + st["soft_far"] + st["soft_near"], 1)
    flops = soft_inter * (FLOPS_FAR * (1 - near_frac) + FLOPS_NEAR * near_frac)
    achieved = flops / (soft_ms * 1e-3) / 1e12
    within_r2 = st["hard_pairs"] / max(st["calls_hard"], 1) + wl.n
    flops_strict = soft_inter * FLOPS_FAR + within_r2 * (FLOPS_NEAR - FLOPS_FAR)
    achieved_strict = flops_strict / (soft_ms * 1e-3) / 1e12
    # the dominant kernel by time: the hard kernel (one launch per substep)
    hcalls = max(st["calls_hard"], 1)
    hard_ms = st["ms_hard"] / hcalls
    hflops = (FLOPS_HARD_TEST * st["hard_candidates"] + FLOPS_HARD_PAIR * st["hard_pairs"]) / hcalls
    hachieved = hflops / (hard_ms * 1e-3) / 1e12
    src_ok = _kernel_source_hash() == SOFT_TRAFFIC["source_hash"]
    # the measured soft traffic is that of the theta-rule instance of the kernel
    soft_ok = src_ok and not args.paper_mac
    line = {
        "metric": "interactions/s + s/step at N=2^20 Plummer; batched p50/p99 solve latency",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "s_per_step": ms_step / 1e3,
        "s_per_step_median": ms_median / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plummer N=2^20 eps=0.01 %s ngb~64 n_sub=4 dt_h=1/64"
                               % ("abs-MAC a_err=2^-8 nearest-sink" if args.paper_mac
                                  else "theta=0.5"),
                   "n": wl.n, "theta": None if args.paper_mac else wl.theta,
                   "a_err": 2.0 ** -8 if args.paper_mac else None, "eps": wl.eps, "R2": wl.R2,
                   "n_sub": wl.n_sub, "group": 64, "n_crit": wl.n_crit,
                   "hard_search_reuse": True},
        "soft_interactions_per_step": soft_inter,
        "hard_pairs_per_step": hard_pairs,
        "hard_candidates_per_step": st["hard_candidates"] / K,
        "soft_kernel_interactions_per_s": soft_inter / (soft_ms * 1e-3),
        "phase_ms_per_step": {"build": st["ms_build"] / K, "soft": st["ms_soft"] / K,
                              "hard": st["ms_hard"] / K},
        "roofline": {"kernel": "k_hard (R2 walk + exact FP64 pair tests + FP64 pair forces)",
                     "bound": "alu", "achieved": hachieved, "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": hachieved / PEAK_FP64,
                     "traffic": HARD_TRAFFIC["bytes"] if src_ok else None,
                     "traffic_unit": "bytes per launch (HBM, counter-measured)",
                     "launch_ms": hard_ms, "share_of_step": st["ms_hard"] / K / ms_step},
        "roofline_interaction": {"kernel": "k_soft (walk + FP32 interactions)", "bound": "alu",
                                 "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                                 "frac": achieved / PEAK_FP32,
                                 "frac_of_packed_fp32_peak": achieved / PEAK_FP32_PACKED,
                                 "achieved_weight_within_R2_only": achieved_strict,
                                 "frac_weight_within_R2_only": achieved_strict / PEAK_FP32,
                                 "traffic": SOFT_TRAFFIC["bytes"] if soft_ok else None,
                                 "traffic_unit": "bytes per launch (HBM, counter-measured)",
                                 "launch_ms": soft_ms, "share_of_step": st["ms_soft"] / K / ms_step},
        "cpu_baseline": None,
    }
    t.close()
    if not args.no_cpu_baseline:
        # the benchmarked configuration's forces at the initial positions, for
        # the parity statement of the CPU-baseline leg
        tp = P.HTree(wl.n, params, device=dev)
        tp.set_state(torch.from_numpy(x), torch.from_numpy(v32), torch.from_numpy(m32))
        tp.build_tree()
        a_s = tp.soft_force()
        a_h, ngb = tp.hard_force()
        tp.sync()
        gpu_forces = {"soft": a_s.cpu().numpy().astype(np.float64),
                      "hard": a_h.cpu().numpy().astype(np.float64),
                      "ngb": ngb.cpu().numpy().astype(np.int64)}
        tp.close()
    if not args.no_comparator:
        hard_call = st["ms_hard"] / max(st["calls_hard"], 1)
        line["comparator"] = comparator(P, torch, wl, x, v32, m32, ms_step, hard_call,
                                        max(args.steps, 3))
    if not args.no_ensemble:
        line["ensemble"] = ensemble(P, torch, args.ensemble_steps)
    if not args.no_serve and args.serve_requests > 0:
        nr = args.serve_requests
        line["serving"] = [
            serving(P, torch, nr, max(nr // 20, 50), 32 << 30, "32 GiB"),
            serving(P, torch, max(nr // 4, 100), max(nr // 80, 25), 2 << 30, "2 GiB"),
        ]
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, x, m32.astype(np.float64), gpu=gpu_forces)
        hk = line["cpu_baseline"].get("host_simd_kernels") or {}
        if hk.get("value"):
            hk["gpu_soft_kernel_over_host"] = line["soft_kernel_interactions_per_s"] / hk["value"]
        par = line["cpu_baseline"]["parity"]
        line["parity"] = {k: par[k] for k in ("soft_p99", "hard_p99", "hard_ngb_exact",
                                              "tolerance_p99")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
