"""Batches of independent systems in one context (one launch per phase).

Each system of a batch must match the oracle run on that system alone, and
must give bit-for-bit the same results as the library run on that system
alone: a system's result does not depend on what it is batched with."""
import numpy as np
import pytest

import synth
from tests._gpu import need_gpu, rel_err, report

pytestmark = pytest.mark.gpu


def _systems(count, seed, lo=8.0, hi=12.0):
    rng = np.random.default_rng(seed)
    sizes = np.rint(2.0 ** rng.uniform(lo, hi, count)).astype(int)
    out = []
    for k, n in enumerate(sizes):
        model = "plummer" if k % 3 else "cube"
        x, v, m = (synth.plummer if model == "plummer" else synth.cold_cube)(int(n), seed * 1000 + k)
        R2 = synth.r2_for_neighbours(model, int(n), 24 + 8 * (k % 3))
        out.append(dict(x=x, v=v.astype(np.float32), m=m.astype(np.float32),
                        eps=0.005 * (1 + k % 4), theta=0.35 + 0.1 * (k % 5), R1=R2 / 2, R2=R2,
                        n_crit=(16, 8, 32)[k % 3], group=(64, 32, 48, 16)[k % 4]))
    return out


def _params(P, s, **kw):
    return P.default_params(eps=s["eps"], theta=s["theta"], R1=s["R1"], R2=s["R2"],
                            n_crit=s.get("n_crit", 16), group_size=s.get("group", 64), **kw)


def _run(P, torch, systems, batch, **kw):
    if batch:
        t = P.HTree([s["x"].shape[1] for s in systems], [_params(P, s, **kw) for s in systems])
    else:
        s = systems[0]
        t = P.HTree(s["x"].shape[1], _params(P, s, **kw))
    x = np.concatenate([s["x"] for s in systems], axis=1)
    v = np.concatenate([s["v"] for s in systems], axis=1)
    m = np.concatenate([s["m"] for s in systems])
    t.set_state(torch.from_numpy(x), torch.from_numpy(v), torch.from_numpy(m))
    return t


def test_batch_matches_oracle(orc):
    torch, P = need_gpu()
    systems = _systems(24, 5)
    t = _run(P, torch, systems, True, flags=P.F_POT)
    t.build_tree()
    a_s, pot = t.soft_force(want_pot=True)
    a_h, ngb = t.hard_force()
    t.sync()
    a_s, pot, a_h, ngb = (u.cpu().numpy() for u in (a_s, pot, a_h, ngb))
    gst = t.group_starts()
    cnt = t.group_counts()
    off, goff = 0, 0
    worst = 0.0
    for k, s in enumerate(systems):
        n = s["x"].shape[1]
        m64 = s["m"].astype(np.float64)
        # n_crit and the group size differ between the systems of the batch
        T = orc.Tree(s["x"], m64, n_crit=s["n_crit"], theta=s["theta"], group=s["group"])
        og = T.group_starts()
        ng = len(og) - 1
        assert np.array_equal(gst[goff:goff + ng + 1].astype(np.int64) - off, og), k
        oc = T.walk_counts(s["R2"], 1)
        for j in range(3):
            assert np.array_equal(cnt[j][goff:goff + ng], oc[j]), (k, j)
        oa, opot, _ = T.soft(1.0, s["eps"], s["R1"], s["R2"], 1, potential=True)
        e = rel_err(a_s[:, off:off + n].astype(np.float64), oa)
        worst = max(worst, np.percentile(e, 99))
        oh, _, ongb = orc.split_direct(s["x"], m64, 1.0, s["eps"], s["R1"], s["R2"], soft=False)
        assert np.array_equal(ngb[off:off + n], ongb), k
        if (ongb > 0).any():
            eh = rel_err(a_h[:, off:off + n].astype(np.float64), oh)[ongb > 0]
            assert np.percentile(eh, 99) <= 1e-5, k
        off += n
        goff += ng
    print("batch soft worst p99 %.3e" % worst)
    assert worst <= 1e-5


@pytest.mark.parametrize("hybrid", [1, 0])
def test_batch_equals_single_bit_exact(hybrid):
    torch, P = need_gpu()
    systems = _systems(6, 6, 9.0, 11.0)
    tb = _run(P, torch, systems, True, hybrid=hybrid, flags=P.F_POT)
    tb.build_tree()
    ab, pb = tb.soft_force(want_pot=True)
    if hybrid:
        hb, nb = tb.hard_force()
    tb.sync()
    off = 0
    for k, s in enumerate(systems):
        n = s["x"].shape[1]
        t1 = _run(P, torch, [s], False, hybrid=hybrid, flags=P.F_POT)
        t1.build_tree()
        a1, p1 = t1.soft_force(want_pot=True)
        assert torch.equal(a1, ab[:, off:off + n]) and torch.equal(p1, pb[off:off + n]), k
        if hybrid:
            h1, n1 = t1.hard_force()
            assert torch.equal(h1, hb[:, off:off + n]) and torch.equal(n1, nb[off:off + n]), k
        off += n


def test_batch_step_equals_single():
    torch, P = need_gpu()
    systems = _systems(5, 7, 9.0, 11.0)
    kw = dict(dt_soft=1.0 / 32, n_sub=2)
    tb = _run(P, torch, systems, True, **kw)
    tb.step(2)
    tb.sync()
    xb, vb = tb.get_state()
    off = 0
    for s in systems:
        n = s["x"].shape[1]
        t1 = _run(P, torch, [s], False, **kw)
        t1.step(2)
        t1.sync()
        x1, v1 = t1.get_state()
        assert torch.equal(x1, xb[:, off:off + n]) and torch.equal(v1, vb[:, off:off + n])
        off += n


def test_many_small_systems(orc):
    # more than 256 systems: two-pass system ordering and node partition
    torch, P = need_gpu()
    rng = np.random.default_rng(8)
    sizes = rng.integers(1, 120, 300)
    systems = []
    for k, n in enumerate(sizes):
        x, v, m = synth.plummer(int(n), 8000 + k)
        R2 = synth.r2_for_neighbours("plummer", max(int(n), 2), 16)
        systems.append(dict(x=x, v=v.astype(np.float32), m=m.astype(np.float32), eps=0.01,
                            theta=0.5, R1=R2 / 2, R2=R2))
    t = _run(P, torch, systems, True)
    t.build_tree()
    t.soft_force()
    _, ngb = t.hard_force()
    t.sync()
    ngb = ngb.cpu().numpy()
    cnt = t.group_counts()
    off, goff = 0, 0
    for k, s in enumerate(systems):
        n = s["x"].shape[1]
        m64 = s["m"].astype(np.float64)
        T = orc.Tree(s["x"], m64, n_crit=16, theta=0.5)
        ng = T.ngroups
        oc = T.walk_counts(s["R2"], 1)
        for j in range(3):
            assert np.array_equal(cnt[j][goff:goff + ng], oc[j]), (k, j)
        _, _, ongb = orc.split_direct(s["x"], m64, 1.0, 0.01, s["R1"], s["R2"], soft=False)
        assert np.array_equal(ngb[off:off + n], ongb), k
        off += n
        goff += ng
