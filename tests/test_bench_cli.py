"""The benchmark's command line without a GPU: more than one GPU is refused
with a message and a non-zero status (the solver has no multi-GPU path), the
gradient byte count that the gradient benches report against matches its
terms, the hash that ties the committed traffic counters to the kernel
covers the sources and their per-source build flags, and a counted byte
figure is reported only for the kernel it was counted for."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_gradient_bytes_terms():
    sys.path.insert(0, str(ROOT))
    import bench
    # one segment (interval >= nt): forward 16 + 4 (its accelerations), no
    # recomputation, adjoint 16, one separately imaged term 16 and nt - 1
    # fused ones 12, flushes 16 every 32 terms
    nt = 64
    assert bench.gradient_bytes(nt, nt) == 16 * nt + 4 * nt + 16 * nt + 12 * (nt - 1) + 16 + 16 * 2
    # interval 1: every step its own segment, none fused; the last segment's
    # single step is not recomputed
    assert bench.gradient_bytes(10, 1) == 16 * 10 + 4 + 20 * 9 + 16 * 10 + 16 * 10 + 16


def test_kernel_hash_covers_sources_and_build_flags():
    sys.path.insert(0, str(ROOT))
    import bench
    from paper_1608_03984_amd import _build

    # every per-source flag set names a source the build compiles
    assert set(_build.EXTRA) <= set(_build.SOURCES)
    # the hashed sources exist and are compiled by the build
    names = [f.name for f in bench.KERNEL_SOURCES]
    assert all(f.exists() for f in bench.KERNEL_SOURCES)
    assert {n for n in names if n.endswith(".hip")} <= set(_build.SOURCES)
    h = bench.kernel_source_hash()
    saved = dict(_build.EXTRA)
    try:
        _build.EXTRA["fd_acoustic_hi.hip"] = ["-O2"]
        assert bench.kernel_source_hash() != h
    finally:
        _build.EXTRA.clear()
        _build.EXTRA.update(saved)
    assert bench.kernel_source_hash() == h


def test_traffic_is_used_only_for_the_launched_kernel():
    """A committed per-order byte count is reported only when it was counted
    for the kernel the context launches (radius, waves and rows of its tile)."""
    sys.path.insert(0, str(ROOT))
    import bench

    t = {4: ("acoustic3d_tiled<2, 12, 2, 1, false, true, false>", 100),
         8: ("acoustic3d_tiled<4, 4, 2, 1, false, true, false>", 200)}
    assert bench.traffic_of(t, 4, 4) == 100
    assert bench.traffic_of(t, 4, 0) is None        # counted for 64 x 24, launched 64 x 8
    assert bench.traffic_of(t, 8, 0) == 200
    assert bench.traffic_of(t, 8, 4) is None
    assert bench.traffic_of(t, 12, 0) is None       # not counted
    assert bench.traffic_of(None, 4, 4) is None
    assert bench.traffic_of(t, 4, 9) is None        # no such tile
