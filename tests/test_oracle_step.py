"""Pins of the oracle's two-timestep leapfrog (nested kick-drift-kick).

n = 1 must reduce to the plain leapfrog of section II.A; the scheme is time
reversible; a softened circular binary returns to its start after one period.
"""
import math

import numpy as np
import pytest

import synth


def _plain_kdk(orc, x, v, m, G, eps, dt, steps):
    """Textbook kick-drift-kick with direct forces (section II.A eqs. 3-4)."""
    x, v = x.copy(), v.copy()
    a = orc.direct(x, m, G, eps)
    for _ in range(steps):
        v += 0.5 * dt * a
        x += dt * v
        a = orc.direct(x, m, G, eps)
        v += 0.5 * dt * a
    return x, v


def test_single_substep_is_plain_leapfrog(orc):
    # theta = 0: soft + hard = direct, so n = 1 must give the plain leapfrog
    x, v, m = synth.plummer(512, 31)
    G, eps, dt = 1.0, 1.0 / 64, 1.0 / 128
    R2 = synth.r2_for_neighbours("plummer", 512, 32)
    xr, vr = _plain_kdk(orc, x, v, m, G, eps, dt, 5)
    for hybrid in (0, 1):
        xh, vh = orc.step(x, v, m, G, eps, 0.0, R2 / 2, R2, 16, 64, hybrid, dt, 1, 5)
        assert np.abs(xh - xr).max() < 1e-12
        assert np.abs(vh - vr).max() < 1e-11


@pytest.mark.parametrize("hybrid,n_sub", [(0, 1), (1, 1), (1, 4)])
def test_time_reversible(orc, hybrid, n_sub):
    x, v, m = synth.plummer(256, 32)
    R2 = synth.r2_for_neighbours("plummer", 256, 32)
    args = (1.0, 1.0 / 64, 0.5, R2 / 2, R2, 16, 64, hybrid, 1.0 / 32, n_sub)
    x1, v1 = orc.step(x, v, m, *args, 6)
    x2, v2 = orc.step(x1, -v1, m, *args, 6)
    assert np.abs(x2 - x).max() < 1e-11
    assert np.abs(-v2 - v).max() < 1e-11


def test_circular_binary(orc):
    # relative orbit of a softened binary: omega^2 = G (m1 + m2) / (d^2 + eps^2)^{3/2}
    G, eps, d = 1.0, 0.1, 1.0
    m = np.array([0.3, 0.7])
    om = math.sqrt(G * m.sum() / (d * d + eps * eps) ** 1.5)
    x = np.array([[-0.7 * d, 0.3 * d], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-0.7 * d * om, 0.3 * d * om], [0.0, 0.0]])
    period = 2 * math.pi / om
    errs = []
    for steps in (200, 400):
        dt = period / steps
        for hybrid, R2 in ((0, 0.5), (1, 2.0)):       # R2 > d: binary fully hard
            x1, v1 = orc.step(x, v, m, G, eps, 0.0, R2 / 2, R2, 16, 64, hybrid, dt, 1, steps)
            errs.append(np.abs(x1 - x).max())
    assert max(errs) < 2e-3
    # second order: halving dt cuts the phase error about fourfold
    assert errs[2] < errs[0] / 3.0


def test_energy_error_reported(orc):
    """Energy drift of the small Plummer case over ten steps of 1/128 (the
    paper gives no value to compare with: parity unpinned; loose bound only)."""
    wl = synth.WORKLOADS["plummer4k"]
    x, v, m = wl.make()
    k0, w0 = orc.energy(x, v, m, 1.0, wl.eps)
    x1, v1 = orc.step(x, v, m, 1.0, wl.eps, wl.theta, wl.R1, wl.R2, 16, 64, 1,
                      2.0 / 128, 2, 5)
    k1, w1 = orc.energy(x1, v1, m, 1.0, wl.eps)
    assert abs((k1 + w1) - (k0 + w0)) / abs(k0 + w0) < 1e-3
