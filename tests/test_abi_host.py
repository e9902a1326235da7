"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, sizes workspaces exactly and rejects bad parameters.
No device work is launched."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def abi():
    import paper_1406_6158_amd as P
    try:
        P.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return P


def _declared():
    txt = (ROOT / "include" / "htree.h").read_text()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(htree_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_path(abi):
    names = _declared()
    for need in ("htree_build_tree", "htree_soft_force", "htree_hard_force", "htree_kick_drift",
                 "htree_step", "htree_create", "htree_workspace_bytes", "htree_destroy"):
        assert need in names


def test_every_declared_symbol_is_exported(abi):
    L = abi.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_params(abi):
    p = abi.default_params()
    assert p.G == 1.0 and p.theta == 0.5 and p.n_crit == 16 and p.group_size == 64
    assert p.hybrid == 1 and p.n_sub == 4 and p.precision == 0


def test_workspace_monotone_and_aligned(abi):
    p = abi.default_params()
    prev = 0
    for n in (1, 63, 64, 65, 4096, 100000, 1 << 20):
        b = abi.workspace_bytes(p, n)
        assert b > prev and b % 256 == 0
        prev = b
    # roughly linear in n at large n
    b1, b2 = abi.workspace_bytes(p, 1 << 20), abi.workspace_bytes(p, 1 << 21)
    assert 1.9 < b2 / b1 < 2.1


@pytest.mark.parametrize("field,value", [
    ("eps", 0.0), ("eps", float("nan")), ("G", -1.0), ("theta", -0.1), ("n_crit", 0),
    ("group_size", 0), ("group_size", 65), ("precision", 2), ("n_sub", 0), ("R1", 0.2), ("hybrid", 3),
    ("flags", 64), ("dt_soft", float("inf")),
])
def test_invalid_params_rejected(abi, field, value):
    p = abi.default_params()
    setattr(p, field, value)
    assert abi.workspace_bytes(p, 1000) == 0
    assert abi.lib().htree_last_error()


def test_invalid_n_rejected(abi):
    p = abi.default_params()
    assert abi.workspace_bytes(p, 0) == 0
    assert abi.workspace_bytes(p, (1 << 27) + 1) == 0


def test_plain_mode_ignores_band(abi):
    p = abi.default_params(hybrid=0, R1=0.0, R2=0.0)
    assert abi.workspace_bytes(p, 1000) > 0


def test_create_rejects_small_or_misaligned_workspace(abi):
    p = abi.default_params()
    n = 1000
    need = abi.workspace_bytes(p, n)
    h = C.c_void_p()
    L = abi.lib()
    # these fail before any device call
    assert L.htree_create(C.byref(h), C.byref(p), n, C.c_void_p(256), need - 256, None) == \
        abi.HTREE_ENOMEM
    assert L.htree_create(C.byref(h), C.byref(p), n, C.c_void_p(257), need, None) == \
        abi.HTREE_EINVAL
    assert L.htree_create(C.byref(h), C.byref(p), n, None, need, None) == abi.HTREE_EINVAL
    assert not h.value


def test_batch_workspace_and_validation(abi):
    ps = [abi.default_params(eps=0.01 * (k + 1), theta=0.4 + 0.1 * k) for k in range(3)]
    sizes = [1000, 1, 5000]
    b = abi.batch_workspace_bytes(ps, sizes)
    singles = sum(abi.workspace_bytes(p, n) for p, n in zip(ps, sizes))
    assert b > 0 and b % 256 == 0
    assert 0.5 * singles < b < 1.5 * singles
    assert abi.batch_workspace_bytes(ps[:1], [6001]) < b * 1.2
    # integrator and layout settings must agree across systems
    bad = [abi.default_params(), abi.default_params(n_sub=2)]
    assert abi.batch_workspace_bytes(bad, [10, 10]) == 0
    assert b"n_sub" in abi.lib().htree_last_error()
    assert abi.batch_workspace_bytes([], []) == 0
    bad = [abi.default_params(), abi.default_params(eps=-1.0)]
    assert abi.batch_workspace_bytes(bad, [10, 10]) == 0
    assert abi.batch_workspace_bytes(ps[:2], [10, 0]) == 0


def test_precision_fp64_accepted(abi):
    p = abi.default_params(precision=1)
    assert abi.workspace_bytes(p, 1000) > 0


def test_create_static_rejects_before_any_device_call(abi):
    """The static-scratch context refuses sizes whose workspace exceeds the
    scratch (ENOMEM) and bad arguments (EINVAL) before touching a device."""
    p = abi.default_params()
    L = abi.lib()
    h = C.c_void_p()
    assert abi.workspace_bytes(p, 1 << 16) <= abi.STATIC_SCRATCH_BYTES
    big = 1 << 17
    assert abi.workspace_bytes(p, big) > abi.STATIC_SCRATCH_BYTES
    assert L.htree_create_static(C.byref(h), C.byref(p), big, None) == abi.HTREE_ENOMEM
    assert b"static scratch" in L.htree_last_error()
    assert L.htree_create_static(None, C.byref(p), 1000, None) == abi.HTREE_EINVAL
    assert L.htree_create_static(C.byref(h), C.byref(p), 0, None) == abi.HTREE_EINVAL
    assert not h.value
