"""The oracle's absolute MAC (section II.B, eqs. 5-6; a_err as in section
IV.A) and the minimum-over-sinks group rule (section III.A.2, eq. 11).

Pins: B2 and b_max of a hand-placed cluster from exact rational arithmetic,
r_b assembled from them with correctly rounded square roots in decimal;
B2 (parallel-axis sums over children) and b_max^2 of every node of a random
tree against the direct particle sums; the walk's lists against a
node-by-node brute-force derivation of the accepted set under both group
rules; monotonicity in a_err; the limit a_err -> 0 (every cell opened) equal
to the direct sum.  The tree force error at a_err = 2^-8 is reported (the
paper prints none: parity unpinned)."""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import synth


def test_cluster_closed_form(orc):
    # four particles with unequal masses inside one leaf (n < n_crit)
    pts = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.5, 0.0), (0.25, 0.25, 0.75)]
    ms = [0.5, 0.25, 0.125, 0.125]
    x = np.array(pts, dtype=np.float64).T.copy()
    m = np.array(ms)
    G, aerr = 2.5, 2.0 ** -8
    T = orc.Tree(x, m, n_crit=16, theta=0.5).set_mac(aerr, G)
    B2, bm = T.node_mac()
    rb2 = T.nodes()["rb2"]
    assert T.nnodes == 1
    # exact: COM and sum m |x - COM|^2 (the build frame's shift cancels)
    M = sum(Fraction(v) for v in ms)
    com = [sum(Fraction(w) * Fraction(p[a]) for w, p in zip(ms, pts)) / M for a in range(3)]
    d2 = [sum((Fraction(p[a]) - com[a]) ** 2 for a in range(3)) for p in pts]
    B2x = sum(Fraction(w) * q for w, q in zip(ms, d2))
    bmx = max(d2)
    assert B2[0] == pytest.approx(float(B2x), rel=1e-15)
    assert bm[0] == pytest.approx(float(bmx), rel=1e-15)
    # eq. 5 with these moments, square roots in 40-digit decimal
    getcontext().prec = 40
    b = Decimal(bmx.numerator) / Decimal(bmx.denominator)
    B2d = Decimal(B2x.numerator) / Decimal(B2x.denominator)
    rb = b.sqrt() / 2 + (b / 4 + (3 * Decimal(G) * B2d / Decimal(aerr)).sqrt()).sqrt()
    assert rb2[0] == pytest.approx(float(rb * rb), rel=1e-15)
    ref = float(np.loadtxt(synth.__file__.replace("synth/__init__.py", "tests/golden/abs_mac.txt")))
    assert rb2[0] == pytest.approx(ref, rel=1e-15)


def test_moments_vs_particle_sums(orc):
    x, v, m = synth.plummer(3000, 31)
    m = synth.lognormal_masses(3000, 32)
    T = orc.Tree(x, m, n_crit=8, theta=0.5)
    nd = T.nodes()
    B2, bm = T.node_mac()
    perm, key, u = T.sorted()
    ms = m[perm]
    inner = 0
    for c in range(T.nnodes):
        b, e = nd["first"][c], nd["first"][c] + nd["count"][c]
        d = u[:, b:e] - nd["com"][:, c:c + 1]
        q = (d * d).sum(axis=0)
        assert B2[c] == pytest.approx((ms[b:e] * q).sum(), rel=1e-11, abs=1e-300)
        assert bm[c] == pytest.approx(q.max(), rel=4e-16, abs=1e-300)
        inner += nd["nchild"][c] > 0
    assert inner > 50


def _brute_lists(T, k, R2, hybrid, min_sinks):
    """Accepted cells / far / near leaves node by node: listed iff accepted
    (or a leaf) while every proper ancestor was opened; a cell is measured by
    the minimum over the group's sinks or the group's box distance."""
    nd = T.nodes()
    perm, key, u = T.sorted()
    st = T.group_starts()
    b, e = st[k], st[k + 1]
    s = u[:, b:e]
    glo, ghi = s.min(axis=1), s.max(axis=1)

    def box2(lo, hi):
        gap = np.maximum(np.maximum(glo - hi, lo - ghi), 0.0)
        return (gap ** 2).sum()

    status = []
    for c in range(T.nnodes):
        com = nd["com"][:, c]
        D1 = ((s - com[:, None]) ** 2).sum(axis=0).min() if min_sinks else box2(com, com)
        D2 = box2(nd["blo"][:, c], nd["blo"][:, c] + nd["l"][c])
        sep = D2 >= R2 * R2 if hybrid else D2 > 0
        if D1 >= nd["rb2"][c] and sep:
            status.append("pc")
        elif nd["nchild"][c] == 0:
            status.append("near" if hybrid and D2 < R2 * R2 else "far")
        else:
            status.append("open")
    out = {"pc": set(), "far": set(), "near": set()}
    for c in range(T.nnodes):
        if status[c] == "open":
            continue
        p, ok = nd["parent"][c], True
        while p >= 0:
            ok &= status[p] == "open"
            p = nd["parent"][p]
        if ok:
            out[status[c]].add(c)
    return out


@pytest.mark.parametrize("aerr,min_sinks", [(2.0 ** -8, False), (2.0 ** -8, True), (0.0, True)])
@pytest.mark.parametrize("hybrid", [0, 1])
def test_walk_vs_bruteforce(orc, aerr, min_sinks, hybrid):
    x, v, m = synth.plummer(512, 33)
    T = orc.Tree(x, m, n_crit=8, theta=0.6, group=32).set_mac(aerr, 1.0, min_sinks)
    for k in range(T.ngroups):
        pc, far, near = T.walk_group(k, 0.25, hybrid)
        ref = _brute_lists(T, k, 0.25, hybrid, min_sinks)
        assert set(pc.tolist()) == ref["pc"]
        assert set(far.tolist()) == ref["far"]
        assert set(near.tolist()) == ref["near"]


def test_lists_shrink_with_aerr_and_min_rule(orc):
    x, v, m = synth.plummer(8192, 34)
    tot = []
    for aerr in (2.0 ** -12, 2.0 ** -8, 2.0 ** -4):
        T = orc.Tree(x, m, n_crit=16, theta=0.5).set_mac(aerr)
        c = T.walk_counts(0.05, 1)
        tot.append(c[0] + c[1] + c[2])
    assert np.all(tot[1] <= tot[0]) and np.all(tot[2] <= tot[1])
    assert tot[0].sum() > tot[2].sum()
    # the minimum over sinks is never below the box distance: no group's
    # list grows, and some shrink
    T = orc.Tree(x, m, n_crit=16, theta=0.5).set_mac(2.0 ** -8, 1.0, True)
    c = T.walk_counts(0.05, 1)
    tmin = c[0] + c[1] + c[2]
    assert np.all(tmin <= tot[1]) and tmin.sum() < tot[1].sum()


@pytest.mark.parametrize("min_sinks", [False, True])
def test_tiny_aerr_is_direct(orc, min_sinks):
    wl = synth.WORKLOADS["plummer4k"]
    x, v, m = wl.make()
    T = orc.Tree(x, m, n_crit=16, theta=0.5).set_mac(1e-290, 1.0, min_sinks)
    acc, _, inter = T.soft(1.0, wl.eps, wl.R1, wl.R2, 0)
    assert inter == 4096 * 4096
    ref = orc.direct(x, m, 1.0, wl.eps)
    assert np.abs(acc - ref).max() < 1e-12 * np.linalg.norm(ref, axis=0).max()


def test_abs_mac_force_error_reported(orc):
    wl = synth.WORKLOADS["plummer4k"]
    x, v, m = wl.make()
    ref = orc.direct(x, m, 1.0, wl.eps)
    for min_sinks in (False, True):
        T = orc.Tree(x, m, n_crit=16, theta=0.5).set_mac(2.0 ** -8, 1.0, min_sinks)
        acc, _, inter = T.soft(1.0, wl.eps, wl.R1, wl.R2, 0)
        e = np.linalg.norm(acc - ref, axis=0) / np.linalg.norm(ref, axis=0)
        print("a_err 2^-8 min_sinks %d: interactions %d, force error p50 %.2e p99 %.2e"
              % (min_sinks, inter, np.percentile(e, 50), np.percentile(e, 99)))
        assert np.percentile(e, 99) < 3e-2
