"""Host-side checks of bench.py's accounting (no GPU): the algorithmic
bytes it prices the roofline on, the per-pass bytes, the hash gate of the
stored counter traffic, and the single-GPU contract."""

import json
import os
import subprocess
import sys

import bench


class _P:
    def __init__(self, shape, nphases):
        self.shape = shape
        self.phases = [(1.0, 0.3, 1e-3)] * nphases


def test_algorithmic_bytes_per_voxel_apply():
    # input c+1, output c+1, tangent state c+3, one spectral round trip 2(c+1)
    # words: 22 in 2D (c = 3), 37 in 3D (c = 6); one phase byte when phases differ
    assert bench.alg_bytes_per_voxel(_P((128, 128, 128), 2), "mixed") == 37 * 4 + 1
    assert bench.alg_bytes_per_voxel(_P((64, 64, 64), 1), "fp64") == 37 * 8
    assert bench.alg_bytes_per_voxel(_P((1, 256, 256), 2), "fp64") == 22 * 8 + 1
    assert bench.alg_bytes_per_voxel(_P((1, 64, 64), 1), "mixed") == 22 * 4


def test_pass_bytes_of_the_128_cube():
    kb = bench.kernel_bytes((128, 128, 128), "mixed")
    nh = 65 * 128 * 128                       # half spectrum (nx/2 + 1) ny nz
    spec = 7 * nh * 8                         # seven complex FP32 fields
    assert kb[1] == kb[2] == kb[3] == 2 * spec
    N = 128 ** 3
    v = 7 * N * 4
    assert kb[0] == v + 4 + 10 * N * 4 + 2 * N + spec + N * 4
    assert kb[4] == spec + N * 4 + 2 * N + v
    # the fused variants read the vector of their inner product in the x-inverse pass
    assert bench.kernel_bytes((128, 128, 128), "mixed", 1)[4] == kb[4] + v


def test_stored_traffic_is_used_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    path = tmp_path / "profiles" / "traffic_w.json"
    path.write_text(json.dumps({"kernel_src_sha1": "0" * 40, "hbm_bytes_per_apply": 123}))
    assert bench.load_traffic("w") is None
    monkeypatch.setattr(bench, "src_hash", lambda: "0" * 40)
    assert bench.load_traffic("w") == 123
    assert bench.load_traffic("absent") is None


def test_committed_traffic_matches_the_committed_kernels():
    """profiles/traffic_particles3d_128.json was taken on the kernel sources in
    the tree (else the bench reports traffic as null)."""
    with open(os.path.join(bench.ROOT, "profiles", "traffic_particles3d_128.json")) as fh:
        d = json.load(fh)
    assert d["kernel_src_sha1"] == bench.src_hash()
    # each kernel's figure is rounded to the byte on its own
    assert abs(d["hbm_bytes_per_apply"] - sum(k["hbm_bytes_per_launch"] for k in d["kernels"].values())) \
        <= len(d["kernels"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
