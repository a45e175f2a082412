"""Host-side pieces of bench.py: the algorithmic byte models behind the roofline fields, the
counter-based traffic lookup, the CPU description of the oracle baseline and the refusal of more
than one GPU.  No GPU is touched."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_step_bytes_follow_the_per_pixel_interval_model():
    npix, K, sel, ev = 921600, 119, 2_270_000, 4_911_194
    # sparse: both frame endpoints of every pixel-interval, flow and reference level (read and
    # written) of the selected ones, 8 B per event
    assert bench.step_bytes(npix, K, sel, ev, "sparse") == 2 * npix * K + 16 * sel + 8 * ev
    assert bench.step_bytes(npix, K, sel, ev, "sparse", memoryless=True) == \
        2 * npix * K + 8 * sel + 8 * ev
    assert bench.step_bytes(npix, K, 0, ev, "dense") == 18 * npix * K + 8 * ev
    assert bench.step_bytes(npix, K, 0, ev, "basic") == 10 * npix * K + 8 * ev
    assert bench.step_bytes(npix, K, 0, ev, "difference") == 11 * npix * K + 8 * ev


def test_chain_bytes_count_each_chain_once():
    npix, K, act, sel, ev = 1000, 10, 100, 300, 50
    assert bench.chain_bytes(npix, K, act, sel, ev, "sparse") == act * 28 + sel * 10 + 8 * ev
    assert bench.chain_bytes(npix, K, act, sel, ev, "dense") == npix * 8 + npix * K * 10 + 8 * ev


def test_counter_traffic_needs_the_same_kernels_and_variant(tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    block = {"workload": "w", "kernel": "k_chain", "variant": 2,
             "source_sha256": bench.kernel_source_hash(), "fetch_kib_per_dispatch": 10.0,
             "write_kib_per_dispatch": 3.0, "fetch_scale": 2.0, "write_scale": 1.0}
    (prof / "k_chain_w_counters.md").write_text("x\n```json\n" + json.dumps(block) + "\n```\n")
    f = str(prof)
    assert bench.counter_traffic("w", variant=2, folder=f) == (10.0 * 2.0 + 3.0) * 1024
    assert bench.counter_traffic("w", variant=1, folder=f) is None
    assert bench.counter_traffic("other", folder=f) is None
    block["source_sha256"] = "0" * 64
    (prof / "k_chain_w_counters.md").write_text("```json\n" + json.dumps(block) + "\n```\n")
    assert bench.counter_traffic("w", variant=2, folder=f) is None


@pytest.mark.parametrize("workload", ["sparse_1280x720", "difference_346x260",
                                      "memoryless_dense_346x260"])
def test_committed_counter_summary_is_readable(workload):
    """The committed summaries parse; their traffic applies only to the kernels they were taken
    on (then it is at least the chain pass's 74.96 MB or 86.7 MB of algorithmic bytes)."""
    t = bench.counter_traffic(workload, variant=2)
    assert t is None or t > 7e7


def test_host_cpu_names_the_logical_cpus():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and isinstance(h["model"], str)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert json.loads(r.stdout.strip().splitlines()[-1])["n_gpus"] == 2


@pytest.mark.parametrize("bad", ["--steps", "--warmup"])
def test_arguments_parse(bad):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), bad, "x"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
