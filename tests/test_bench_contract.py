"""bench.py: the one-GPU refusal, the algorithmic work behind its roofline
fractions (per-drop self-interaction flops and far-field interaction counts
against the per-degree table and the workload sizes), the traffic lookup,
and on a GPU the fields of its JSON line."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1811_10270_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "single-GPU" in msg["error"]


def test_count_shapes_argument_is_checked():
    for bad in ("2x", "2x15x1", "two"):
        with pytest.raises(SystemExit) as e:
            bench.main(["--count-shapes", bad])
        assert e.value.code == 2


@pytest.mark.parametrize("p, total", [(16, 1.35e9), (24, 9.27e9), (32, 3.72e10), (48, 2.68e11)])
def test_self_flops_match_the_per_degree_table(p, total):
    # q = 2p on the paper's grid: rotation + Legendre + longitude sums + kernel
    got = bench.self_flops_per_drop(p, 2 * p, 0)
    assert abs(got - total) / total < 6e-3, (p, got)


def test_self_flops_terms():
    # p = 1, q = 2 by hand: T = 2 * 4 = 8 targets, rotated grid 3 x 6
    T, nlq = 8, 6
    rot = 4 * 7 * T * (1 * 1 + 2 * 3)
    leg = 4 * 3 * 3 * 10 * T
    dft = 2 * nlq * 3 * 3 * 13 * T
    ker = bench.SELF_KERNEL_FLOPS_PER_NODE * T * 3 * nlq
    assert bench.self_flops_per_drop(1, 2, 0) == rot + leg + dft + ker
    # the 2p-longitude grid has 2p per latitude instead of 2p + 2
    T2, nlq2 = 2 * 2, 4
    rot2 = 4 * 7 * T2 * 7
    assert bench.self_flops_per_drop(1, 2, 1) == rot2 + 4 * 3 * 3 * 10 * T2 + 2 * nlq2 * 3 * 3 * 13 * T2 \
        + bench.SELF_KERNEL_FLOPS_PER_NODE * T2 * 3 * nlq2


def test_far_interactions_of_the_workloads():
    # every target against every other drop's upsampled nodes
    two = W.two_drops(32, seed=2)
    assert bench.far_interactions(two) == 2 * 2178 * (97 * 194)
    s = W.batched_suspension()
    assert abs(bench.far_interactions(s) - 7.54e10) / 7.54e10 < 1e-3
    assert bench.far_interactions(W.single_drop(16, seed=1)) == 0
    assert bench.FAR_FLOPS_PER_INTERACTION == 18 + 19 + 2 + 3 + 11


def test_self_exec_flops_by_hand():
    # p = 1, q = 2 on the paper's grid: T = 8 targets, rotated grid 3 x 6
    T, nlq = 8, 6
    rot = 7 * T * ((4 * 1 + 6 * 1) + (4 * 4 + 6 * 2))      # real-form rotation + phases, n = 0, 1
    leg = 4 * 3 * 3 * 10 * T
    dft = 13 * 3 * T * (nlq // 4 + 1) * (2 * 3 + 12)        # quarter-period rows 0..1, 2p+1 = 3 terms
    ker = bench.SELF_KERNEL_FLOPS_PER_NODE * T * 3 * nlq
    assert bench.self_exec_flops_per_drop(1, 2, 0) == rot + leg + dft + ker
    # the executed count is below the dense one: a quarter of the longitude
    # sums and about half of the rotation
    for p in (16, 32, 48):
        r = bench.self_exec_flops_per_drop(p, 2 * p, 0) / bench.self_flops_per_drop(p, 2 * p, 0)
        assert 0.3 < r < 0.45, (p, r)


def test_traffic_lookup_is_tied_to_source_workload_and_tile():
    assert bench.measured_traffic("k_far64 (x)", "no_such_workload", 0, "2x15") is None
    same = bench.kernel_source_sha256() == bench.TRAFFIC_SOURCE_SHA256
    for key, v in bench.TRAFFIC_BYTES.items():
        wl, prec, kern = key[:3]
        tile = key[3] if len(key) > 3 else "1x1"
        got = bench.measured_traffic(kern + " (x)", wl, 0 if prec == "fp64" else 1, tile)
        assert (got == v) if same else got is None
        if kern.startswith("k_far"):
            # another tile shape has no counted bytes
            assert bench.measured_traffic(kern + " (x)", wl, 0 if prec == "fp64" else 1, "1x1") is None
        else:
            assert len(key) == 3


@pytest.mark.gpu
def test_json_line_fields():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "single_drop_p16", "--steps",
                        "2", "--warmup", "1", "--no-autotune", "--cpu-sample", "8"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    b = json.loads(r.stdout.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in b, k
    assert b["n_gpus"] == 1 and b["steps"] == 2 and b["warmup"] == 1 and b["value"] > 0
    assert b["config"]["workload"] == "single_drop_p16" and b["vs_baseline"] is None
    assert b["dtype"] == "f64" and b["config"]["q_self"] == "2p" and "fp32_far" in b
    roof = b["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["unit"] == "TFLOP/s" and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    cb = b["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and "8 random targets" in cb["sample"]
    assert cb["one_core"]["cores"] == 1 and cb["one_core"]["value"] > 0 and cb["cpu_model"]


def test_kernel_hash_covers_the_device_code():
    """The traffic table is keyed to the device code only: the hash stops at
    the one host-side banner of the library source."""
    path = os.path.join(ROOT, "paper_1811_10270_amd", "csrc", "ehdbim.hip")
    text = open(path, "rb").read()
    assert text.count(b"\n// Host side\n") == 1
    import hashlib
    cut = text.find(b"\n// Host side\n")
    assert bench.kernel_source_sha256() == hashlib.sha256(text[:cut]).hexdigest()
