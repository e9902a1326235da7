"""Pins of the oracle's particle-cell (monopole) term and of the cell moments
it uses, with unequal masses and G != 1.

* Every cell's mass and centre of mass against a brute-force mass-weighted
  mean of its particles (log-normal masses: an unweighted mean fails).
* Clusters of coincident particles: a cell whose particles all sit at one
  point has its monopole equal to the sum of their pair terms, so a tree
  walk that accepts only such cells must reproduce the direct sum to
  rounding.  The opening angle is chosen so that no cell holding two
  clusters can ever be accepted, while single-cluster cells are accepted at
  some depth; the test checks that particle-cell terms were really used.
"""
import numpy as np
import pytest

import synth

G = 2.5


def _clusters(seed, n_side=4, spacing=1.0, jitter=0.15, kmax=40):
    """Coincident clusters on a jittered n_side^3 lattice; returns (x, m, cid)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(n_side, dtype=np.float64) * spacing
    c = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    c = c + rng.uniform(-jitter, jitter, c.shape)
    k = rng.integers(1, kmax + 1, c.shape[1])
    cid = np.repeat(np.arange(c.shape[1]), k)
    x = np.ascontiguousarray(c[:, cid])
    perm = rng.permutation(cid.size)           # clusters interleaved in input order
    x, cid = np.ascontiguousarray(x[:, perm]), cid[perm]
    m = synth.lognormal_masses(cid.size, seed + 1)
    return x, m, cid


def test_every_node_com_is_mass_weighted(orc):
    x, v, _ = synth.plummer(6000, 31)
    m = synth.lognormal_masses(6000, 32)
    T = orc.Tree(x, m, n_crit=8, theta=0.6)
    perm, key, u = T.sorted()
    nd = T.nodes()
    ms = m[perm]
    for k in range(T.nnodes):
        f, c = nd["first"][k], nd["count"][k]
        w = ms[f:f + c]
        M = w.sum()
        com = (u[:, f:f + c] * w).sum(axis=1) / M
        assert nd["M"][k] == pytest.approx(M, rel=1e-13)
        assert np.all(np.abs(nd["com"][:, k] - com) <= 1e-12 * nd["l"][k])
    # an unweighted mean would differ by far more than the tolerance
    f, c = nd["first"][0], nd["count"][0]
    assert np.abs(u[:, f:f + c].mean(axis=1) - nd["com"][:, 0]).max() > 1e-4 * nd["l"][0]


@pytest.mark.parametrize("hybrid", [0, 1])
def test_particle_cell_term_equals_direct_on_coincident_clusters(orc, hybrid):
    x, m, cid = _clusters(41)
    n = x.shape[1]
    eps, R1, R2 = 0.05, 0.15, 0.3
    lo = x.min(axis=1)
    side = 2.0 ** np.ceil(np.log2((x - lo[:, None]).max()))
    # separation of distinct clusters >= 1 - 2 * 0.15 * sqrt(3) > 0.45: a cell
    # holding two of them has side > 0.45 / sqrt(3); it could be accepted only
    # from a distance >= side / theta > sqrt(3) * root side
    theta = 0.45 / np.sqrt(3) / (np.sqrt(3) * side) * 0.99
    T = orc.Tree(x, m, n_crit=2, theta=theta, group=16)
    acc, pot, _ = T.soft(G, eps, R1, R2, hybrid, potential=True)
    if hybrid:
        _, ref, _ = orc.split_direct(x, m, G, eps, R1, R2)
    else:
        ref = orc.direct(x, m, G, eps)
    # scale of the terms: sum_j G m_j / (r^2 + eps^2) per sink
    d = x[:, None, :] - x[:, :, None]
    scale = (G * m[None, :] / ((d * d).sum(0) + eps * eps)).sum(axis=1)
    err = np.linalg.norm(acc - ref, axis=0)
    assert np.all(err <= 1e-14 * scale), err.max() / scale[np.argmax(err)]
    _, pref = orc.direct(x, m, G, eps, potential=True)
    assert np.all(np.abs(pot - pref) <= 1e-14 * np.abs(pref))
    # the particle-cell branch was used, with cells of several particles
    npc, nfar, nnear = T.walk_counts(R2, hybrid)
    assert np.all(npc > 0)
    nd = T.nodes()
    multi = 0
    for k in range(0, T.ngroups, 3):
        pc, _, _ = T.walk_group(k, R2, hybrid)
        multi += int((nd["count"][pc] > 1).sum())
        # every accepted cell holds one cluster only
        perm, _, _ = T.sorted()
        for c in pc:
            f, cnt = nd["first"][c], nd["count"][c]
            assert np.unique(cid[perm[f:f + cnt]]).size == 1
    assert multi > 100


def test_monopole_error_shrinks_with_distance(orc):
    """Non-coincident sources: the monopole about the centre of mass has no
    dipole error, so its error falls as (b/r)^2 relative to the force."""
    rng = np.random.Generator(np.random.PCG64(5))
    src = rng.uniform(-0.5, 0.5, (3, 50))
    ms = synth.lognormal_masses(50, 6)
    errs = []
    for dist in (8.0, 16.0, 32.0):
        x = np.concatenate([src, np.array([[dist], [0.3], [-0.2]])], axis=1)
        m = np.concatenate([ms, [1e-3]])
        # theta large enough that the cluster's top cell is accepted from the sink
        T = orc.Tree(x, m, n_crit=2, theta=0.9, group=1)
        acc, _, _ = T.soft(G, 1e-9, 0.0, 0.0, 0)
        ref = orc.direct(x, m, G, 1e-9)
        npc, _, _ = T.walk_counts(0.0, 0)
        st = T.group_starts()
        perm, _, _ = T.sorted()
        k = int(np.nonzero(perm[st[:-1]] == 50)[0][0])
        assert npc[k] >= 1
        errs.append(np.linalg.norm(acc[:, 50] - ref[:, 50]) / np.linalg.norm(ref[:, 50]))
    # quadrupole-order error: x4 smaller per doubling of the distance
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0
