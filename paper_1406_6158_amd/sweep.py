"""Energy-error sweep over the hybrid method's parameters (n, R1, R2).

The paper chooses the number of hard substeps n and the changeover radii R1,
R2 by the error in total energy after test runs of its Plummer model
(section IV.A; it settles on n = 4, R2 = 2 R1).  This module repeats that
selection procedure with this library: for each setting it advances the same
initial state over the same time with the nested kick-drift-kick of
``HTree.step`` (hard substep dt_h fixed, soft step n dt_h) and reports the
relative change of the total energy and the time per soft step.

The energy is evaluated on the GPU too: the potential of every particle is
the unsplit softened potential summed over all other particles, taken from a
plain-tree context with theta = 0 (every cell opened, so it is the direct
sum) and the potential flag; E = sum m v^2 / 2 + sum m phi / 2 is reduced
in FP64.  The paper prints no energy errors for comparison (reported values
only).

    python -m paper_1406_6158_amd.sweep [--n 1048576] [--time 1.0]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import F_POT, HTree, default_params


def total_energy(x, v, m, G, eps, device="cuda"):
    """Kinetic + potential energy of (x [3][n] f64, v [3][n] f32, m [n] f32)
    tensors on the device; the potential is the direct sum (theta = 0 plain
    tree on the GPU)."""
    import torch
    n = int(m.shape[0])
    p = default_params(G=G, eps=eps, theta=0.0, hybrid=0, flags=F_POT)
    t = HTree(n, p, device=device)
    t.set_state(x, v, m)
    t.build_tree()
    _, pot = t.soft_force(want_pot=True)
    t.sync()
    m64 = m.to(torch.float64)
    kin = 0.5 * float((m64 * (v.to(torch.float64) ** 2).sum(0)).sum())
    pe = 0.5 * float((m64 * pot.to(torch.float64)).sum())
    t.close()
    return kin, pe


def run_setting(x, v, m, eps, theta, n_sub, R1, R2, dt_h, t_end, hybrid=1, device="cuda"):
    """Advances (x, v, m) to t_end with n_sub hard substeps of dt_h per soft
    step (plain tree: hybrid = 0, one force per dt_h); returns the relative
    energy change and the time per soft step."""
    import torch
    n = int(m.shape[0])
    dt_s = dt_h * (n_sub if hybrid else 1)
    steps = int(round(t_end / dt_s))
    p = default_params(eps=eps, theta=theta, R1=R1, R2=R2 if hybrid else 2 * R1,
                       dt_soft=dt_s, n_sub=n_sub if hybrid else 1, hybrid=hybrid)
    e0 = sum(total_energy(x, v, m, 1.0, eps, device))
    t = HTree(n, p, device=device)
    t.set_state(x, v, m)
    t.step(0)                  # initial forces
    t.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t.step(steps)
    t.sync()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(steps, 1)
    xe, ve = t.get_state()
    t.sync()
    t.close()
    e1 = sum(total_energy(xe, ve, m, 1.0, eps, device))
    return {"n_sub": n_sub if hybrid else 1, "R1": R1, "R2": R2 if hybrid else None,
            "hybrid": hybrid, "dt_h": dt_h, "soft_steps": steps,
            "dE_rel": (e1 - e0) / abs(e0), "ms_per_soft_step": ms,
            "ms_per_unit_time": ms * steps / t_end}


def sweep(x, v, m, eps, theta, dt_h, t_end, n_subs, ngbs, r2_of, device="cuda"):
    """All (n_sub, R2 for a mean neighbour count) settings with R1 = R2 / 2,
    plus the plain tree at the same dt_h."""
    import torch
    xd = torch.as_tensor(x, dtype=torch.float64, device=device)
    vd = torch.as_tensor(v, dtype=torch.float32, device=device)
    md = torch.as_tensor(m, dtype=torch.float32, device=device)
    out = []
    for ngb in ngbs:
        R2 = r2_of(ngb)
        for ns in n_subs:
            r = run_setting(xd, vd, md, eps, theta, ns, R2 / 2, R2, dt_h, t_end, 1, device)
            r["ngb"] = ngb
            out.append(r)
    r = run_setting(xd, vd, md, eps, theta, 1, r2_of(ngbs[0]) / 2, None, dt_h, t_end, 0, device)
    out.append(r)
    return out


def main():
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--time", type=float, default=1.0)
    ap.add_argument("--dt-h", type=float, default=1.0 / 64.0)
    ap.add_argument("--seed", type=int, default=2)
    a = ap.parse_args()
    x, v, m = synth.plummer(a.n, a.seed)
    eps = 0.01 * (float(1 << 20) / a.n) ** (1.0 / 3.0)
    rows = sweep(x, v, m.astype(np.float32), eps, 0.5, a.dt_h, a.time, [1, 2, 4, 8],
                 [32.0, 64.0, 128.0], lambda k: synth.r2_for_neighbours("plummer", a.n, k))
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
