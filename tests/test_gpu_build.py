"""GPU tree build vs the oracle: keys, permutation, frame, topology and
centres of mass must agree bit for bit."""
import numpy as np
import pytest

import synth
from tests._gpu import as_inputs, make_tree, need_gpu

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "plummer4k":
        return synth.plummer(4096, 1)
    if name == "ragged1000":
        return synth.plummer(1000, 41)
    if name == "cube3001":
        return synth.cold_cube(3001, 42)
    if name == "tiny1":
        return synth.plummer(1, 43)
    if name == "small15":
        return synth.plummer(15, 44)
    if name == "dups":
        x, v, m = synth.plummer(5000, 45)
        x[:, 1000:1100] = x[:, 999:1000]       # 101 coincident particles: depth-21 leaves
        return x, v, m
    if name == "hernquist20k":
        return synth.hernquist(20000, 46)
    if name == "lognormal4k":
        x, v, _ = synth.plummer(4096, 1)
        return x, v, synth.lognormal_masses(4096, 49)
    if name == "dups_lognormal":
        x, v, _ = _case("dups")
        return x, v, synth.lognormal_masses(5000, 50)
    raise KeyError(name)


CASES = ["plummer4k", "ragged1000", "cube3001", "tiny1", "small15", "dups", "hernquist20k",
         "lognormal4k", "dups_lognormal"]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("n_crit", [16, 1, 5])
def test_build_bit_exact(orc, case, n_crit):
    torch, P = need_gpu()
    x, v, m = _case(case)
    x, v32, m32, v64, m64 = as_inputs(x, v, m)
    print("case", case, "n_crit", n_crit, "n", x.shape[1], flush=True)
    t = make_tree(P, torch, x, v32, m32, n_crit=n_crit, theta=0.6)
    t.build_tree()
    t.sync()
    keys, perm, lo, side = t.export_keys()
    T = orc.Tree(x, m64, n_crit=n_crit, theta=0.6)
    olo, oside = T.frame()
    operm, okey, ou = T.sorted()
    assert np.array_equal(lo, olo) and side == oside
    assert np.array_equal(keys, okey)
    assert np.array_equal(perm.astype(np.int64), operm)
    g = t.export_nodes()
    o = T.nodes()
    assert len(g["level"]) == T.nnodes
    gk = np.lexsort((g["first"], g["level"]))
    ok = np.lexsort((o["first"], o["level"]))
    for f in ("level", "first", "count"):
        assert np.array_equal(g[f][gk].astype(np.int64), o[f][ok].astype(np.int64)), f
    assert np.array_equal(g["M"][gk], o["M"][ok])
    assert np.array_equal(g["com"][:, gk], o["com"][:, ok])
    assert np.array_equal(t.group_starts().astype(np.int64), T.group_starts())


def test_build_deterministic():
    torch, P = need_gpu()
    x, v, m = synth.plummer(50000, 47)
    x, v32, m32, _, _ = as_inputs(x, v, m)
    out = []
    for _ in range(2):
        t = make_tree(P, torch, x, v32, m32)
        t.build_tree()
        t.sync()
        out.append(t.export_nodes())
    for f in out[0]:
        assert np.array_equal(out[0][f], out[1][f])


def test_nonfinite_input_reported():
    torch, P = need_gpu()
    x, v, m = synth.plummer(1000, 48)
    x[1, 10] = np.nan
    x, v32, m32, _, _ = as_inputs(x, v, m)
    t = make_tree(P, torch, x, v32, m32)
    t.build_tree()
    with pytest.raises(P.HTreeError) as ei:
        t.sync()
    assert ei.value.code == P.HTREE_EINVAL


def _brute_boxes(xs, first, count):
    """Per-axis minima and maxima of the sorted positions xs [3][n] over each
    node's range [first, first + count), one node at a time."""
    lo = np.empty((3, first.size))
    hi = np.empty((3, first.size))
    for k in range(first.size):
        seg = xs[:, first[k]:first[k] + count[k]]
        lo[:, k] = seg.min(axis=1)
        hi[:, k] = seg.max(axis=1)
    return lo, hi


def _boxes_through_refits(P, torch, x, v32, m32, nodes_of, **kw):
    """Builds, then drifts three times with a refit after each drift; after
    the build and after every refit the exported node boxes must equal the
    exact minima and maxima of the nodes' particles (nodes_of picks which
    nodes to check); between a drift and its refit they are refused."""
    t = make_tree(P, torch, x, v32, m32, **kw)
    t.build_tree()
    t.soft_force()
    t.hard_force()          # the drift goes through the kick, which needs forces
    _, perm, _, _ = t.export_keys()
    nd = t.export_nodes()
    sel = nodes_of(nd["count"])
    first, count = nd["first"][sel], nd["count"][sel]
    for k in range(4):
        if k:
            t.kick_drift(0.0, dt_drift=0.15)
            with pytest.raises(P.HTreeError):
                t.export_node_boxes()
            t.refit()
        xd, _ = t.get_state()
        t.sync()
        lo, hi = t.export_node_boxes()
        blo, bhi = _brute_boxes(xd.cpu().numpy()[:, perm], first, count)
        assert np.array_equal(lo[:, sel], blo) and np.array_equal(hi[:, sel], bhi), k
    t.close()


@pytest.mark.parametrize("case", ["plummer4k", "dups", "hernquist20k"])
def test_node_boxes_after_refits(case):
    """Every node's box, from the level pass and from the chunk-cover refit."""
    torch, P = need_gpu()
    x, v, m = _case(case)
    x, v32, m32, _, _ = as_inputs(x, v, m)
    print("node boxes", case, flush=True)
    _boxes_through_refits(P, torch, x, v32, m32, lambda c: np.arange(c.size),
                          eps=0.01, R1=0.025, R2=0.05)


def test_node_boxes_after_refits_2e20():
    """At N = 2^20 (the refit's chunks of 32, 1024 and 32768 particles all in
    use): every node above 1024 particles and 4096 sampled others."""
    torch, P = need_gpu()
    wl = synth.WORKLOADS["plummer1m"]
    x, v, m = wl.make()
    x, v32, m32, _, _ = as_inputs(x, v, m)
    print("node boxes plummer 2^20", flush=True)
    rng = np.random.default_rng(7)

    def pick(count):
        big = np.flatnonzero(count > 1024)
        rest = rng.choice(np.flatnonzero(count <= 1024), 4096, replace=False)
        return np.concatenate([big, rest])

    _boxes_through_refits(P, torch, x, v32, m32, pick, eps=wl.eps, R1=wl.R1, R2=wl.R2,
                          n_crit=wl.n_crit)
