"""The HIP sources on the CPU with deferred execution and shuffled block order (tests/cpu_emu).

Deferred execution queues kernels, memsets and copies of device or pinned memory per stream and
runs them only when a synchronisation needs them -- as late as HIP allows -- while the calls HIP
documents as synchronous (hipFree, hipHostFree, copies of pageable host memory) still wait.  A
host read of a result before its synchronisation, a host buffer rewritten while a queued copy
still reads it, or a device buffer freed or regrown under queued work then gives wrong results
or trips AddressSanitizer.  Blocks run in a seeded random order, so no kernel may depend on the
order of its blocks.  Test infrastructure only; the product never loads these builds.
"""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import test_cpu_emulated_batch as tb
from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import (HERE, _camera_videos, _server_worker_run,  # noqa: F401
                                       emu_build, emu_sim, monkeypatch_module, oracle_run)


@pytest.fixture
def deferred(emu_sim):
    lib = emu_sim.load()
    lib.emu_set_execution(1, 20261203)
    yield emu_sim
    lib.emu_set_execution(0, 0)
    lib.emu_host_memory_pinned(0)


@pytest.mark.parametrize("pinned", [False, True], ids=["copied-at-submit", "pulled-by-step"])
def test_deferred_server_worker(deferred, pinned):
    deferred.load().emu_host_memory_pinned(int(pinned))
    _server_worker_run(deferred)


def test_deferred_server_first_frame_only_step(deferred):
    """A step in which every camera sends only its first frame runs no batched window, so no
    host wait covers its ring fills: the next step must not rewrite the fill descriptors before
    those fills have run (with pinned inputs the fills are queued, and the descriptors are read
    when they run)."""
    deferred.load().emu_host_memory_pinned(1)
    cams = _camera_videos(deferred)
    srv = deferred.Server(hbm_budget_bytes=1 << 34, max_cameras=8, queue_depth=4)
    ids = [srv.admit(width=c["W"], height=c["H"], method=c["method"], c_pos=0.15, c_neg=0.15,
                     n_interp=4) for c in cams]
    for cid, c in zip(ids, cams):                  # first frames only
        srv.submit(cid, c["v"].frames[0], None, int(c["v"].t_us[0]))
    assert srv.step() == len(cams)
    for k in range(1, 9):
        for cid, c in zip(ids, cams):
            fl = None if c["method"] == "basic" else c["v"].flows[k - 1]
            srv.submit(cid, c["v"].frames[k], fl, int(c["v"].t_us[k]))
        if k % 3 == 0:
            srv.step()
    srv.sync()
    for cid, c in zip(ids, cams):
        np.testing.assert_array_equal(srv.drain_keys(cid), c["ok"], err_msg=c["method"])
    srv.close()


@pytest.mark.parametrize("splits", [[(0, 1), (1, 4), (4, 7)], [(0, 7)]])
def test_deferred_fused_batch_mixed_streams(deferred, splits):
    tb.test_emulated_fused_batch_mixed_streams(deferred, splits)


def test_deferred_batch_graph_replay(deferred):
    tb.test_emulated_batch_steps_replay_one_recorded_graph(deferred)


@pytest.mark.parametrize("mode", ["window", pytest.param("chunks", marks=pytest.mark.long)])
def test_deferred_dense_346x260_full_sequence(deferred, mode):
    """The dense 346x260 60-frame sequence with the initial event buffer: one window push grows
    the arena five times, re-running the chains that ran out of space each time."""
    v = synth.blob_video(synth.dense_346x260())
    cfg = dict(method=sim.DENSE, c_pos=0.15, c_neg=0.15, n_interp=10)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    s = deferred.Stream(346, 260, **cfg)
    if mode == "window":
        s.push_frames(v.frames, v.flows, v.t_us)
    else:
        for a in range(0, 60, 20):
            b = min(60, a + 20)
            s.push_frames(v.frames[a:b], v.flows[max(a - 1, 0):b - 1], v.t_us[a:b])
    np.testing.assert_array_equal(s.drain_keys(), ok)
    np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
    if mode == "window":
        assert s.stats()["retries"] >= 5
    s.close()


ASAN_DENSE = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim, synth
    sim.LIB_PATH = {lib!r}; sim._lib = None
    from test_cpu_emulated_kernels import oracle_run
    sim.load().emu_set_execution(1, 99)
    v = synth.blob_video(synth.dense_346x260(n_frames={frames}))
    cfg = dict(method=sim.DENSE, c_pos=0.15, c_neg=0.15, n_interp=10)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    s = sim.Stream(346, 260, **cfg)
    s.push_frames(v.frames, v.flows, v.t_us)
    assert np.array_equal(s.drain_keys(), ok)
    assert s.stats()["retries"] >= {retries}
    s.close()
    print("asan-clean")
""")


@pytest.mark.long
def test_deferred_dense_full_sequence_under_asan(tmp_path):
    """The full 60-frame dense window (five arena regrowths) under AddressSanitizer with deferred
    execution: no access outside a live allocation, events equal to the oracle's."""
    _asan_dense(tmp_path, 60, 5)


@pytest.mark.long
def test_deferred_dense_regrowth_under_asan(tmp_path):
    """A 12-frame prefix of the dense sequence, whose window also grows the arena while chains
    are queued, under AddressSanitizer with deferred execution."""
    _asan_dense(tmp_path, 12, 3)


def _asan_dense(tmp_path, frames, retries):
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_dense.py"
    script.write_text(ASAN_DENSE.format(root=os.path.dirname(HERE), tests=HERE, lib=lib,
                                        frames=frames, retries=retries))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=3000)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]
