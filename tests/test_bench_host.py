"""Host checks of the benchmark driver and the autotuner's bookkeeping (no
device work)."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    import bench
    h = bench._kernel_source_hash()
    assert len(h) == 16 and h == bench._kernel_source_hash()
    # a copy of the sources with an extra comment and blank line hashes the same
    csrc = tmp_path / "paper_1406_6158_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("force.hip", "htree_dev.h"):
        txt = (ROOT / "paper_1406_6158_amd" / "csrc" / name).read_text()
        (csrc / name).write_text("// an added comment\n\n" + txt.replace("\n", "  // note\n", 3))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._kernel_source_hash() == h
    (csrc / "force.hip").write_text((csrc / "force.hip").read_text() + "\nint x;\n")
    assert bench._kernel_source_hash() != h


def test_traffic_pin_matches_a_hash_format():
    import bench
    assert set(bench.SOFT_TRAFFIC) == {"bytes", "source_hash"}
    assert len(bench.SOFT_TRAFFIC["source_hash"]) == 16 and bench.SOFT_TRAFFIC["bytes"] > 0


def test_percentile_helper():
    import bench
    assert bench._pct([1.0, 2.0, 3.0], 50) == 2.0
    assert bench._pct([], 50) is None


def test_size_classes():
    from paper_1406_6158_amd import autotune
    assert autotune.size_class(1024) == 10
    assert autotune.size_class(1025) == 10
    assert autotune.size_class(2047) == 10
    assert autotune.size_class(2048) == 11
    assert autotune.size_class(1) == 0
    # every candidate is a valid setting of the library
    for g, nc in autotune.DEFAULT_CANDIDATES:
        assert 1 <= g <= 64 and 1 <= nc <= 4096
