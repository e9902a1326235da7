"""Host-side checks of the request server: the arena allocator (compiled
with the host compiler, no HIP) and the footprint that admission uses.  No
device work is launched."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def test_arena_allocator(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "arena_check"
    subprocess.run([cxx, "-std=c++17", "-O2", "-o", str(exe), str(ROOT / "tests" / "arena_check.cpp")],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


@pytest.fixture(scope="module")
def abi():
    import paper_1406_6158_amd as P
    try:
        P.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return P


def _r(b):
    return (b + 255) // 256 * 256


@pytest.mark.parametrize("hybrid,flags", [(1, 0), (0, 0), (1, 1), (0, 1)])
def test_footprint_is_workspace_plus_outputs(abi, hybrid, flags):
    for n in (1, 100, 4097, 1 << 20):
        p = abi.default_params(hybrid=hybrid, flags=flags, R1=0.01, R2=0.02)
        ws = abi.workspace_bytes(p, n)
        want = _r(ws) + _r(12 * n)
        if hybrid:
            want += _r(12 * n) + _r(4 * n)
        if flags & abi.F_POT:
            want += _r(4 * n)
        assert abi.solve_footprint(p, n) == want


def test_footprint_invalid_is_zero(abi):
    assert abi.solve_footprint(abi.default_params(eps=0.0), 100) == 0
    assert abi.solve_footprint(abi.default_params(), 0) == 0


def test_server_argument_errors(abi):
    """Argument checks that come before any device call."""
    import ctypes as C
    L = abi.lib()
    h = C.c_void_p()
    streams = (C.c_void_p * 1)(None)
    # NULL or misaligned arena
    assert L.htree_server_create(C.byref(h), None, 1 << 20, streams, 1, 1) == abi.HTREE_EINVAL
    assert L.htree_server_create(C.byref(h), C.c_void_p(0x1001), 1 << 20, streams, 1, 1) == abi.HTREE_EINVAL
    # stream and depth limits
    assert L.htree_server_create(C.byref(h), C.c_void_p(0x1000), 1 << 20, streams, 0, 1) == abi.HTREE_EINVAL
    assert L.htree_server_create(C.byref(h), C.c_void_p(0x1000), 1 << 20, streams, 1, 17) == abi.HTREE_EINVAL
    assert L.htree_server_create(C.byref(h), C.c_void_p(0x1000), 1 << 20, None, 1, 1) == abi.HTREE_EINVAL
    # calls on a NULL server
    rid = C.c_int64()
    p = abi.default_params()
    assert L.htree_server_submit(None, C.byref(p), 10, None, 10, None, None,
                                 C.byref(rid)) == abi.HTREE_EINVAL
    nd = C.c_int32()
    assert L.htree_server_poll(None, None, 0, C.byref(nd)) == abi.HTREE_EINVAL
    assert L.htree_server_release(None, 1) == abi.HTREE_EINVAL
    L.htree_server_destroy(None)
