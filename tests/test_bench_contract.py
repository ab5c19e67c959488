"""The benchmark's command-line contract that needs no GPU: more than one GPU is
refused with a message and a non-zero exit before anything touches a device."""

import os
import subprocess
import sys

from conftest import ROOT


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _bench():
    import importlib

    sys.path.insert(0, ROOT)
    return importlib.import_module("bench")


def test_fp64_full_projection_counts_every_trajectory_per_launch():
    """A full update projects all T trajectories' H Psi in one launch: the orbitals
    are read once and each trajectory's H Psi once, and the flops grow with T."""
    b = _bench()
    N, ng = 240, 96 ** 3
    pairs = N * (N + 1) / 2
    by1, fl1, pk = b.roof("project_gemm", N, ng, False, 1, True)
    by3, fl3, _ = b.roof("project_gemm", N, ng, False, 3, True)
    assert pk == b.PEAK_FP64
    assert (by1, fl1) == (16.0 * N * ng, 2 * pairs * ng)
    assert (by3, fl3) == (32.0 * N * ng, 6 * pairs * ng)


def test_measured_traffic_needs_same_source_launch_bytes_and_tiling(tmp_path, monkeypatch):
    import hashlib
    import json

    b = _bench()
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source\n")
    rec = {"source": str(src), "source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "algorithmic_bytes_per_launch": 1000, "traffic_bytes_per_launch": 1234.0}
    table = {"kernels": {"plain": dict(rec), "stencil": dict(rec, tiling=[16, 1])}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(table))
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.measured_traffic("plain", 1000) == 1234.0
    assert b.measured_traffic("plain", 2000) is None  # another launch shape
    assert b.measured_traffic("missing", 1000) is None
    assert b.measured_traffic("stencil", 1000, (16, 1, 5)) == 1234.0  # look-ahead differs only
    assert b.measured_traffic("stencil", 1000, (16, 2, 3)) is None  # other z chunks
    assert b.measured_traffic("stencil", 1000, (0, 0, 0)) is None  # built-in tiling
    src.write_bytes(b"kernel source, changed\n")
    assert b.measured_traffic("plain", 1000) is None
