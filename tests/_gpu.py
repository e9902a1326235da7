"""Shared helpers of the GPU parity tests (inputs go to both sides unchanged)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_6158_amd as P
    P.lib()   # raises when the HIP library is missing: no fallback
    return torch, P


def as_inputs(x, v, m):
    """float64 positions, float32 velocities and masses for the library; the
    oracle gets the same values widened to float64."""
    v32 = v.astype(np.float32)
    m32 = m.astype(np.float32)
    return x, v32, m32, v32.astype(np.float64), m32.astype(np.float64)


def make_tree(P, torch, x, v32, m32, **kw):
    p = P.default_params(**kw)
    t = P.HTree(x.shape[1], p)
    t.set_state(torch.from_numpy(x), torch.from_numpy(v32), torch.from_numpy(m32))
    return t


def rel_err(a, ref):
    """Per-sink relative error |a - ref| / |ref| of (3, n) arrays."""
    num = np.linalg.norm(a - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return num / np.maximum(den, 1e-300)


def report(tag, e):
    print("%s: p50 %.3e p99 %.3e max %.3e" % (tag, np.percentile(e, 50), np.percentile(e, 99),
                                              e.max()), flush=True)
