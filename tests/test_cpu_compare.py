"""The host comparison loops (paper_1406_6158_amd/cpu/soft_cpu.cpp: the soft
interaction loops on CPU threads, for the CPU/GPU comparison of section IV.C)
against the oracle.  Groups are 64 particles consecutive in the oracle tree's
key order (so each is compact, as the library's groups are) of a 512-particle
Plummer sample with log-normal masses, each sink and source taken as an FP32
offset from its group's box centre.  With every particle as a far source of
every group the loops must give the direct sum (oracle.direct, eq. 1 with
softening); with every particle as a near source, the soft part of the
direct split (oracle.split_direct, eqs. 7-9).  FP32 with compensated tile
sums: p99 relative error within 1e-5."""
import numpy as np
import pytest

import oracle
import synth
from paper_1406_6158_amd import build as hb
from paper_1406_6158_amd import cpu_compare as cc

N = 512
TOL_P99 = 1e-5


@pytest.fixture(scope="module")
def case():
    if not cc.LIB_PATH.exists():
        hb.build_cpu()
    x, _, _ = synth.plummer(N, 61)
    m = synth.lognormal_masses(N, 62).astype(np.float32).astype(np.float64)
    R2 = synth.r2_for_neighbours("plummer", N, 32)
    eps = 1.0 / 64
    perm, _, _ = oracle.Tree(x, m).sorted()
    x, m = x[:, perm], m[perm]            # key order: compact groups
    ng = N // cc.SINKS
    sinks = np.zeros((ng, 3, cc.SINKS))
    src = np.zeros((ng, N, 4))
    for g in range(ng):
        part = x[:, g * cc.SINKS:(g + 1) * cc.SINKS]
        c = 0.5 * (part.min(axis=1) + part.max(axis=1))
        sinks[g] = part - c[:, None]
        src[g, :, :3] = (x - c[:, None]).T
        src[g, :, 3] = m
    return x, m, eps, R2, sinks, src


def _rel(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


def _flat(out):
    return np.concatenate(list(out.astype(np.float64)), axis=1)   # [3][N] in particle order


def test_far_sources_give_the_direct_sum(case):
    x, m, eps, R2, sinks, src = case
    out = cc.soft(sinks, src, None, eps * eps, R2, 1.0 / (R2 - R2 / 2), threads=4)
    ref = oracle.direct(x, m, 1.0, eps)
    e = _rel(_flat(out), ref)
    assert np.percentile(e, 99) <= TOL_P99 and e.max() <= 1e-4


def test_near_sources_give_the_soft_split(case):
    x, m, eps, R2, sinks, src = case
    out = cc.soft(sinks, None, src, eps * eps, R2, 1.0 / (R2 - R2 / 2), threads=3)
    _, ref, _ = oracle.split_direct(x, m, 1.0, eps, R2 / 2, R2, soft=True)
    e = _rel(_flat(out), ref)
    assert np.percentile(e, 99) <= TOL_P99 and e.max() <= 1e-4


def test_far_and_near_add_and_threads_agree(case):
    x, m, eps, R2, sinks, src = case
    k = dict(eps2=eps * eps, R2=R2, invdR=1.0 / (R2 - R2 / 2))
    both = cc.soft(sinks, src[:, :200], src[:, 200:], threads=1, **k)
    again = cc.soft(sinks, src[:, :200], src[:, 200:], threads=5, **k)
    assert np.array_equal(both, again)            # groups are independent of the split
    far = cc.soft(sinks, src[:, :200], None, threads=2, **k)
    near = cc.soft(sinks, None, src[:, 200:], threads=2, **k)
    assert np.allclose(both, far + near, rtol=1e-5, atol=1e-6 * np.abs(both).max())


def test_rejects_bad_shapes(case):
    _, _, eps, R2, sinks, src = case
    with pytest.raises(ValueError):
        cc.soft(sinks[:, :, :32], src, None, eps * eps, R2, 1.0)
    with pytest.raises(ValueError):
        cc.soft(sinks, src[:3], None, eps * eps, R2, 1.0)
