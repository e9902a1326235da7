"""The static-scratch context (htree_create_static) against the context on
a caller workspace (htree_create): same inputs, same kernels, so the same
group tables, list sizes and neighbour counts bit for bit and forces within
the parity tolerance (they are expected to be identical).  Two contexts in a
row, the second on a smaller system, so the second runs on the contents the
first left in the scratch; then the capacity and one-holder checks."""
import numpy as np
import pytest

import synth
from tests._gpu import as_inputs, make_tree, need_gpu, rel_err

pytestmark = pytest.mark.gpu

TOL_P99 = 1e-5


def _solve(P, torch, x, v32, m32, static, **kw):
    p = P.default_params(flags=P.F_POT, **kw)
    t = P.HTree(x.shape[1], p, static=static)
    t.set_state(torch.from_numpy(x), torch.from_numpy(v32), torch.from_numpy(m32))
    t.build_tree()
    a_s, pot = t.soft_force(want_pot=True)
    a_h, ngb = t.hard_force()
    t.step(1)
    xs, vs = t.get_state()
    t.sync()
    out = dict(a_s=a_s.cpu().numpy(), pot=pot.cpu().numpy(), a_h=a_h.cpu().numpy(),
               ngb=ngb.cpu().numpy(), starts=t.group_starts(), counts=t.group_counts(),
               stats=t.stats(), x=xs.cpu().numpy(), v=vs.cpu().numpy())
    t.close()
    return out


def _cases():
    n1 = 1 << 16
    x1, v1, _ = synth.plummer(n1, 71)
    R2a = synth.r2_for_neighbours("plummer", n1, 48)
    n2 = 3001
    x2, v2, _ = synth.plummer(n2, 72)
    R2b = synth.r2_for_neighbours("plummer", n2, 32)
    return [((x1, v1, synth.lognormal_masses(n1, 73)), dict(G=2.5, eps=0.01, R1=R2a / 2, R2=R2a)),
            ((x2, v2, np.full(n2, 1.0 / n2)), dict(eps=1.0 / 64, R1=R2b / 2, R2=R2b, theta=0.7))]


def test_static_scratch_matches_workspace_context_twice():
    torch, P = need_gpu()
    for (x, v, m), kw in _cases():
        x, v32, m32, _, _ = as_inputs(x, v, m)
        print("static scratch: n", x.shape[1], kw, flush=True)
        ref = _solve(P, torch, x, v32, m32, False, **kw)
        got = _solve(P, torch, x, v32, m32, True, **kw)
        assert np.array_equal(got["starts"], ref["starts"])
        for a, b in zip(got["counts"], ref["counts"]):
            assert np.array_equal(a, b)
        assert np.array_equal(got["ngb"], ref["ngb"])
        for k in ("soft_interactions", "hard_candidates", "hard_pairs"):
            assert got["stats"][k] == ref["stats"][k], k
        for k in ("a_s", "a_h"):
            e = rel_err(got[k].astype(np.float64), ref[k].astype(np.float64))
            e = e[np.linalg.norm(ref[k], axis=0) > 0]
            assert np.percentile(e, 99) <= TOL_P99, k
        assert np.percentile(np.abs(got["pot"] - ref["pot"]) / np.abs(ref["pot"]), 99) <= TOL_P99
        assert np.allclose(got["x"], ref["x"], rtol=0, atol=1e-12)
        assert np.allclose(got["v"], ref["v"], rtol=1e-5, atol=1e-7)
        same = all(np.array_equal(got[k], ref[k]) for k in ("a_s", "a_h", "pot", "x", "v"))
        print("  bit-identical to the workspace context:", same, flush=True)


def test_static_scratch_capacity_and_single_holder():
    torch, P = need_gpu()
    p = P.default_params()
    with pytest.raises(P.HTreeError) as ei:
        P.HTree(1 << 17, p, static=True)
    assert ei.value.code == P.HTREE_ENOMEM
    t = P.HTree(1000, p, static=True)
    with pytest.raises(P.HTreeError) as ei:
        P.HTree(500, p, static=True)
    assert ei.value.code == P.HTREE_ESTATE
    t.close()
    t2 = P.HTree(500, p, static=True)   # free again once the holder is destroyed
    t2.close()
