"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This module only draws particle sets (positions, velocities, masses) and names
the workloads; it holds none of the force method's arithmetic, so both the GPU
library and the FP64 oracle can be fed from it without sharing any code.

Every generator takes an integer seed and uses numpy's PCG64 bit generator, so
the same call gives the same bytes on any machine.

Model choices (the paper's test problem is a Plummer sphere, section IV.A):

* ``plummer``   -- Plummer sphere, G = M = a = 1, untruncated; radii by the
  inverse of the cumulative mass M(r) = r^3/(1+r^2)^{3/2}; speeds by rejection
  sampling of the isotropic distribution function (Aarseth, Henon & Wielen
  1974); isotropic directions; shifted to the centre-of-mass frame.
* ``hernquist`` -- Hernquist profile M(r) = r^2/(r+a)^2 truncated at 50a and
  renormalised to M = 1, at rest.
* ``cold_cube`` -- uniform cube [-1, 1]^3, M = 1, at rest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "plummer", "hernquist", "cold_cube", "lognormal_masses", "sample_indices",
    "r2_for_neighbours", "Workload", "WORKLOADS", "ensemble_sizes",
    "serving_requests",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere, shape (3, n)."""
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth])


def _com_shift(x: np.ndarray, v: np.ndarray, m: np.ndarray):
    mt = m.sum()
    x = x - (x * m).sum(axis=1, keepdims=True) / mt
    v = v - (v * m).sum(axis=1, keepdims=True) / mt
    return x, v


def plummer(n: int, seed: int, a: float = 1.0, G: float = 1.0, M: float = 1.0):
    """Plummer sphere with ``n`` equal-mass particles.

    Returns ``(x, v, m)``: x and v are float64 arrays of shape (3, n) (structure
    of arrays), m is float64 of shape (n,) with every entry M/n.
    """
    rng = _rng(seed)
    # radius from the enclosed-mass fraction X in (0, 1)
    X = rng.uniform(0.0, 1.0, n)
    X = np.clip(X, 1e-12, 1.0 - 1e-12)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    x = _isotropic(rng, n) * r
    # speed q * v_esc with q drawn from g(q) = q^2 (1-q^2)^{7/2}, g <= 0.1
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    v = _isotropic(rng, n) * (q * vesc)
    m = np.full(n, M / n)
    x, v = _com_shift(x, v, m)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def hernquist(n: int, seed: int, a: float = 1.0, rt_over_a: float = 50.0, M: float = 1.0):
    """Hernquist halo truncated at ``rt_over_a * a``, total mass M, at rest."""
    rng = _rng(seed)
    xmax = (rt_over_a / (rt_over_a + 1.0)) ** 2
    X = rng.uniform(0.0, xmax, n)
    s = np.sqrt(X)
    r = a * s / (1.0 - s)
    x = _isotropic(rng, n) * r
    v = np.zeros((3, n))
    m = np.full(n, M / n)
    x, v = _com_shift(x, v, m)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def cold_cube(n: int, seed: int, half: float = 1.0, M: float = 1.0):
    """Uniform cube [-half, half]^3 at rest."""
    rng = _rng(seed)
    x = rng.uniform(-half, half, (3, n))
    v = np.zeros((3, n))
    m = np.full(n, M / n)
    return np.ascontiguousarray(x), v, m


def lognormal_masses(n: int, seed: int, sigma: float = 1.0, M: float = 1.0) -> np.ndarray:
    """``n`` masses exp(N(0, sigma^2)) scaled to total M (float64)."""
    rng = _rng(seed)
    m = np.exp(rng.normal(0.0, sigma, n))
    return m * (M / m.sum())


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """``k`` distinct particle indices out of ``n`` (sorted, int64)."""
    rng = _rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# Mean number of other particles within distance R of a particle, in the
# small-R limit, is N * (4 pi / 3) R^3 * (integral of rho^2 dV) / M^2.  The
# integrals below are properties of the input distributions only.
_RHO2 = {
    # Plummer, a = M = 1: (3/(4 pi))^2 * 4 pi * (15 pi / 768) = 45 / 1024
    "plummer": 45.0 / 1024.0,
    # Hernquist truncated at 50a, renormalised: c^2/(5 pi) (1 - (1/51)^5), c = (51/50)^2
    "hernquist": (51.0 / 50.0) ** 4 / (5.0 * math.pi) * (1.0 - 51.0 ** -5),
    # uniform cube of side 2, M = 1: rho = 1/8
    "cube": 1.0 / 8.0,
}


def r2_for_neighbours(model: str, n: int, n_ngb: float) -> float:
    """Cutoff radius whose sphere holds ``n_ngb`` other particles on average."""
    return (n_ngb / (n * (4.0 * math.pi / 3.0) * _RHO2[model])) ** (1.0 / 3.0)


@dataclass(frozen=True)
class Workload:
    """One named problem: input model plus the force and integrator settings."""
    name: str
    model: str
    n: int
    seed: int
    eps: float
    theta: float
    n_ngb: float            # target mean neighbour count inside R2
    n_sub: int = 4          # hard substeps per soft step
    dt_soft: float = 1.0 / 16.0
    n_crit: int = 16
    group: int = 64
    soft_steps: int = 1
    sample: int = 1 << 14   # sinks checked against the oracle at full size
    sample_seed: int = 22

    @property
    def R2(self) -> float:
        return r2_for_neighbours(self.model, self.n, self.n_ngb)

    @property
    def R1(self) -> float:
        return 0.5 * self.R2

    def make(self):
        if self.model == "plummer":
            return plummer(self.n, self.seed)
        if self.model == "hernquist":
            return hernquist(self.n, self.seed)
        if self.model == "cube":
            return cold_cube(self.n, self.seed)
        raise ValueError(self.model)


WORKLOADS = {
    # small Plummer case: N = 4096, eps = 1/64, theta = 0.5, ~32 neighbours,
    # ten leapfrog steps of 1/128
    "plummer4k": Workload("plummer4k", "plummer", 4096, 1, 1.0 / 64.0, 0.5, 32.0,
                          n_sub=1, dt_soft=1.0 / 128.0, soft_steps=10,
                          sample=4096),
    # headline Plummer case: N = 2^20, eps = 0.01, theta = 0.5, ~64
    # neighbours, 4 hard substeps of 1/64 per soft step
    "plummer1m": Workload("plummer1m", "plummer", 1 << 20, 2, 0.01, 0.5, 64.0,
                          n_sub=4, dt_soft=1.0 / 16.0, soft_steps=16),
    # Hernquist halo: N = 2^23, eps = 0.005, force only
    "hernquist8m": Workload("hernquist8m", "hernquist", 1 << 23, 3, 0.005, 0.6, 64.0,
                            sample_seed=33),
}


def ensemble_sizes(count: int = 512, seed: int = 4, lo: float = 10.0, hi: float = 16.0):
    """Particle counts log-uniform in [2^lo, 2^hi] for a batch of systems."""
    rng = _rng(seed)
    return np.rint(2.0 ** rng.uniform(lo, hi, count)).astype(np.int64)


def serving_requests(count: int, seed: int = 5, rate: float = 500.0,
                     lo: float = 12.0, hi: float = 20.0):
    """Poisson arrivals of force-solve requests.

    Returns a list of dicts with arrival time (s), N, model, theta and a
    per-request seed; the particle sets are drawn lazily with ``make_request``.
    """
    rng = _rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    n = np.rint(2.0 ** rng.uniform(lo, hi, count)).astype(np.int64)
    cube = rng.uniform(0.0, 1.0, count) < 0.5
    theta = rng.uniform(0.4, 0.7, count)
    out = []
    for k in range(count):
        out.append({"t": float(t[k]), "n": int(n[k]),
                    "model": "cube" if cube[k] else "plummer",
                    "theta": float(theta[k]), "seed": 5000 + k})
    return out
