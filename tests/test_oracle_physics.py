"""Pins of the oracle's pair force, direct sum, changeover split and energies.

Each check compares the oracle with something fixed outside it: hand-evaluated
rationals, closed forms, invariants of the equations, or a library routine.
"""
import math
from pathlib import Path

import numpy as np
import pytest

import synth

GOLD = Path(__file__).parent / "golden"


def _golden_K():
    rows = []
    for line in (GOLD / "changeover_K.txt").read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            a, b, c, d = (int(t) for t in line.split())
            rows.append((a / b, c / d))
    return rows


def test_K_exact_dyadic_values(orc):
    # section II.C eq. (10), values evaluated by hand in rationals
    for Y, K in _golden_K():
        assert orc.K(Y) == K, (Y, orc.K(Y), K)


def test_K_shape(orc):
    # K(Y) = S(Y^2) with S the quintic smoothstep, S(1 - s) = 1 - S(s): K = 1/2 at Y^2 = 1/2
    assert abs(orc.K(math.sqrt(0.5)) - 0.5) < 4e-16
    Y = np.linspace(0.0, 1.0, 2001)
    K = np.array([orc.K(y) for y in Y])
    assert np.all(np.diff(K) >= 0.0)            # monotone across the band
    h = 1e-4                                    # flat at both ends (C^2 joins)
    assert orc.K(h) < 1e-20 and 1.0 - orc.K(1.0 - h) < 1e-6
    # derivative 60 Y^5 (1 - Y^2)^2 by finite differences (derived by hand)
    for y in (0.3, 0.5, 0.8):
        fd = (orc.K(y + 1e-6) - orc.K(y - 1e-6)) / 2e-6
        assert abs(fd - 60 * y ** 5 * (1 - y * y) ** 2) < 1e-7


def test_two_body_closed_form(orc):
    # section II.A eq. (2): a_1 = G m_2 d / (d^2 + eps^2)^{3/2}
    x = np.array([[0.1, 0.1 + 0.6], [0.2, 0.2 - 0.8], [-0.3, -0.3]])
    m = np.array([0.25, 0.75])
    G, eps = 2.0, 0.3
    acc, pot = orc.direct(x, m, G, eps, potential=True)
    d = x[:, 1] - x[:, 0]
    s = (1.0 + eps * eps) ** 1.5          # |d| = 1
    np.testing.assert_allclose(acc[:, 0], G * m[1] * d / s, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(acc[:, 1], -G * m[0] * d / s, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(pot, [-G * m[1] / math.sqrt(1.09), -G * m[0] / math.sqrt(1.09)],
                               rtol=1e-15)


def test_direct_momentum(orc):
    x, v, m = synth.plummer(2048, 7)
    m = m * (1.0 + 0.5 * np.sin(np.arange(m.size)))     # unequal masses
    acc = orc.direct(x, m, 1.0, 0.01)
    p = (acc * m).sum(axis=1)
    assert np.abs(p).max() < 1e-14 * np.abs(acc * m).sum()


def test_direct_vs_numpy_bruteforce(orc):
    # plain numpy evaluation of eq. (2) on a tiny set
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3, 40))
    m = rng.uniform(0.5, 1.5, 40)
    acc = orc.direct(x, m, 1.3, 0.05)
    d = x[:, None, :] - x[:, :, None]          # d[:, i, j] = x_j - x_i
    r2 = (d ** 2).sum(0) + 0.05 ** 2
    w = 1.3 * m[None, :] * r2 ** -1.5
    np.fill_diagonal(w, 0.0)
    ref = (d * w[None]).sum(2)
    np.testing.assert_allclose(acc, ref, rtol=1e-12, atol=1e-14)


def _mean_pe(orc, gen, n, seeds):
    w = []
    for s in seeds:
        x, v, m = gen(n, s)
        w.append(orc.energy(x, None, m, 1.0, 0.0)[1] / (1.0 - 1.0 / n))
    return np.mean(w), np.std(w, ddof=1) / math.sqrt(len(w))


@pytest.mark.parametrize("model,closed", [
    ("plummer", -3.0 * math.pi / 32.0),       # -3 pi G M^2 / (32 a)
    ("hernquist", -0.18),                      # truncated at 50a, renormalised
])
def test_potential_energy_closed_form(orc, model, closed):
    gen = synth.plummer if model == "plummer" else synth.hernquist
    mean, se = _mean_pe(orc, gen, 4096, range(100, 108))
    assert abs(mean - closed) < 4.0 * se + 1e-3 * abs(closed), (mean, se, closed)


def test_cube_potential_energy(orc):
    # W = -(G M^2 / 2) <1/r>; for the cube [-1,1]^3, <1/r> = E_unit[1/r] / 2 where
    # E_unit[1/r] = 8 int_{[0,1]^3} (1-x)(1-y)(1-z)/|r| (triangular difference density)
    from scipy import integrate
    eu, _ = integrate.tplquad(lambda z, y, x: 8 * (1 - x) * (1 - y) * (1 - z) /
                              math.sqrt(x * x + y * y + z * z), 0, 1, 0, 1, 0, 1,
                              epsabs=1e-9, epsrel=1e-9)
    closed = -0.5 * eu / 2.0
    mean, se = _mean_pe(orc, synth.cold_cube, 4096, range(200, 206))
    assert abs(mean - closed) < 4.0 * se + 1e-3 * abs(closed), (mean, se, closed)


def test_plummer_virial(orc):
    x, v, m = synth.plummer(4096, 11)
    kin, pot = orc.energy(x, v, m, 1.0, 0.0)
    assert abs(2.0 * kin / abs(pot) - 1.0) < 0.06


def test_split_sums_to_direct(orc):
    x, v, m = synth.plummer(4096, 1)
    wl = synth.WORKLOADS["plummer4k"]
    a = orc.direct(x, m, 1.0, wl.eps)
    ah, aso, ngb = orc.split_direct(x, m, 1.0, wl.eps, wl.R1, wl.R2)
    scale = np.linalg.norm(a, axis=0).max()
    assert np.abs(ah + aso - a).max() < 1e-14 * scale
    # the neighbour relation is symmetric, so the hard force conserves momentum
    assert np.abs((ah * m).sum(axis=1)).max() < 1e-15 * np.abs(ah * m).sum()


def test_neighbour_sets_vs_kdtree(orc):
    from scipy.spatial import cKDTree
    x, v, m = synth.plummer(4096, 1)
    wl = synth.WORKLOADS["plummer4k"]
    _, _, ngb = orc.split_direct(x, m, 1.0, wl.eps, wl.R1, wl.R2, soft=False)
    kd = cKDTree(x.T)
    ref = np.array([len(kd.query_ball_point(p, wl.R2)) - 1 for p in x.T])
    np.testing.assert_array_equal(ngb, ref)
    # the R2 formula for ~32 neighbours lands close to its target
    assert 25.0 < ngb.mean() < 40.0


def test_hard_force_limit_cases(orc):
    # R1 -> R2 makes K a step: hard = direct restricted to r < R2
    x, v, m = synth.cold_cube(500, 4)
    R2 = 0.4
    ah, _, ngb = orc.split_direct(x, m, 1.0, 0.01, R2 * (1 - 1e-12), R2, soft=False)
    d = x[:, None, :] - x[:, :, None]
    r2 = (d ** 2).sum(0)
    msk = (r2 < R2 * R2) & ~np.eye(500, dtype=bool)
    w = m[None, :] * (r2 + 1e-4) ** -1.5 * msk
    ref = (d * w[None]).sum(2)
    np.testing.assert_allclose(ah, ref, rtol=1e-6, atol=1e-12)
