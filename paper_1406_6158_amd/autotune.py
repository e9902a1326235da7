"""Autotuner for batched contexts: picks the sink-group size g and the leaf
threshold n_crit per size class of systems.

Systems are put in classes by floor(log2 N).  For each class, every
candidate (g, n_crit) is timed on a batched context holding all systems of
that class (so the GPU sees the same amount of work as in the real batch),
one full soft step each (build, soft force, n_sub hard forces, kicks), with
the library's own HIP event timings.  The candidate with the least summed
phase time wins.  The force definition does not depend on g or n_crit beyond
which cells the opening test sees; every candidate is a valid setting of the
method.
"""
from __future__ import annotations

import math

DEFAULT_CANDIDATES = ((64, 16), (64, 8), (64, 32), (32, 16), (32, 8), (48, 16), (16, 8))


def size_class(n: int) -> int:
    return int(math.floor(math.log2(max(int(n), 1))))


def _time_batch(P, torch, systems, params, reps):
    t = P.HTree([s["n"] for s in systems], params)
    x = torch.cat([s["x"] for s in systems], dim=1)
    v = torch.cat([s["v"] for s in systems], dim=1)
    m = torch.cat([s["m"] for s in systems])
    t.set_state(x, v, m)
    t.step(1)                       # warm-up
    t.sync()
    t.stats()
    best = float("inf")
    for _ in range(reps):
        t.step(1)
        t.sync()
        st = t.stats()
        best = min(best, st["ms_build"] + st["ms_soft"] + st["ms_hard"])
    t.close()
    return best


def tune(P, torch, systems, make_params, candidates=DEFAULT_CANDIDATES, reps=2, log=None):
    """``systems``: list of dicts with device tensors x [3,n] f64, v [3,n] f32,
    m [n] f32 and ``n``; ``make_params(k, g, n_crit)`` returns the Params of
    system k (with HTREE_F_TIMING) for a candidate.  Returns
    ({size class: (g, n_crit)}, {size class: {candidate: ms}})."""
    classes = {}
    for k, s in enumerate(systems):
        classes.setdefault(size_class(s["n"]), []).append(k)
    table, times = {}, {}
    for c in sorted(classes):
        ks = classes[c]
        times[c] = {}
        for g, nc in candidates:
            ms = _time_batch(P, torch, [systems[k] for k in ks],
                             [make_params(k, g, nc) for k in ks], reps)
            times[c][(g, nc)] = ms
        table[c] = min(times[c], key=times[c].get)
        if log:
            log("autotune: class 2^%d (%d systems) -> g=%d n_crit=%d (%.3f ms; worst %.3f ms)"
                % (c, len(ks), table[c][0], table[c][1], times[c][table[c]],
                   max(times[c].values())))
    return table, times
