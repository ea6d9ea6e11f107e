"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic byte
counts per voxel, the kernel each workload runs under AUTO, and the gating of
the committed traffic record on the kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench                                             # noqa: E402
import paper_1501_07844_amd as pf                        # noqa: E402
from paper_1501_07844_amd import synth                   # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("make,storage,expected", [
    (lambda: synth.potts3d_voronoi(shape=(4, 5, 6)), "fp32", 292),    # 2*4*(8+24) + 32 + 4
    (lambda: synth.potts3d_voronoi(shape=(4, 5, 6)), "bf16", 164),    # 2*2*(8+24) + 32 + 4
    (lambda: synth.hmf_ellipsoids(shape=(4, 5, 6)), "fp32", 360),     # 2*4*(8+33) + 32
    (lambda: synth.dagmf_blobs(shape=(4, 5, 6)), "fp32", 528),        # 2*4*(12+48) + 48
    (lambda: synth.dagmf_blobs(shape=(4, 5, 6)), "bf16", 288),
])
def test_algorithmic_bytes_per_voxel(make, storage, expected):
    assert bench.bytes_alg(make(), storage) == expected


@pytest.mark.skipif(not os.path.exists(pf.lib_path()), reason="library not built")
def test_kernel_choice_per_workload():
    p = synth.potts3d_voronoi(shape=(8, 8, 8))
    assert bench._kernel_choice(pf, p, "fp32", "auto") == "fused2"
    assert bench._kernel_choice(pf, p, "bf16", "auto") == "fused2"
    assert bench._kernel_choice(pf, p, "fp32", "fused") == "fused"
    # the HMF tree (8 leaves under 3 internal nodes) and the DAGMF graph (12
    # leaves under 4) fill a build with identity slots
    for st in ("fp32", "bf16", "fp16"):
        assert bench._kernel_choice(pf, synth.hmf_ellipsoids(shape=(4, 5, 6)), st, "auto") == "fused"
        assert bench._kernel_choice(pf, synth.dagmf_blobs(shape=(4, 5, 6)), st, "auto") == "fused"
    assert bench._kernel_name(synth.dagmf_blobs(shape=(4, 5, 6)), "fused") == "k_flow_label"
    q = synth.ishikawa_levels(shape=(4, 5, 6), n_levels=7)
    assert bench._kernel_choice(pf, q, "fp32", "auto") == "fused"        # chain build
    assert bench._kernel_choice(pf, q, "bf16", "auto") == "two_pass"
    assert bench._kernel_name(q, "fused") == "k_flow_label"
    assert bench._kernel_name(p, "fused") == "k_fused"
    # a small 2-D chain of one problem runs in LDS tiles with ghost zones
    c2 = synth.ishikawa_levels()
    assert bench._kernel_choice(pf, c2, "fp32", "auto") == "lds"
    assert bench._kernel_name(c2, "lds") == "k_tile2d"
    pb = synth.random_potts(1, (1, 20, 30), 2, 3, batch=8)
    assert bench._kernel_name(pb, "lds") == "k_lds2d"


@pytest.mark.parametrize("which", sorted(bench.TRAFFIC_FILES))
def test_traffic_record_is_gated_on_the_kernel_sources(which):
    path = os.path.join(ROOT, "profiles", bench.TRAFFIC_FILES[which])
    if not os.path.exists(path):
        pytest.skip(f"no traffic record for {which}")
    with open(path) as fh:
        rec = json.load(fh)
    assert bench._traffic(which, rec["kernel"], rec["source_hash"]) == rec["bytes_per_launch"]
    assert bench._traffic(which, rec["kernel"], "0" * 16) is None
    other = "k_label+k_flow" if rec["kernel"] != "k_label+k_flow" else "k_flow_label"
    assert bench._traffic(which, other, rec["source_hash"]) is None
    # the calibrated bytes are the counter values times the copy-kernel factors
    read = rec["fetch_kib_per_launch"] * 1024 * rec["fetch_factor"]
    write = rec["write_kib_per_launch"] * 1024 * rec["write_factor"]
    assert abs(read + write - rec["bytes_per_launch"]) <= 1e-4 * rec["bytes_per_launch"]
