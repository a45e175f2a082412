"""The fused batched push (one launch per phase over all streams of a sim_push_batch call),
executed on the CPU (tests/cpu_emu): every stream's events and state equal the oracle's for that
stream alone, whatever the mix.  Complements the GPU tests; the product never loads these builds."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from oracle.oracle import FLOW_LK
from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import (emu_build, emu_sim, monkeypatch_module,  # noqa: F401
                                       oracle_run, HERE)

# (width, height, stream options, oracle options)
MIX = [
    ((40, 24), dict(method="dense", c_pos=0.12, c_neg=0.12, n_interp=4, event_capacity=1),
     dict(method=sim.DENSE, c_pos=0.12, c_neg=0.12, n_interp=4)),
    ((33, 17), dict(method="sparse", c_pos=0.02, c_neg=0.02, n_interp=4,
                    thresh_mode="memoryless", event_capacity=8),
     dict(method=sim.SPARSE, c_pos=0.02, c_neg=0.02, n_interp=4, thresh_mode=1)),
    ((36, 20), dict(method="difference", c_pos=0.1, c_neg=0.1, n_interp=3),
     dict(method=sim.DIFFERENCE, c_pos=0.1, c_neg=0.1, n_interp=3)),
    ((29, 31), dict(method="basic", c_pos=0.15, c_neg=0.15, event_capacity=4),
     dict(method=sim.BASIC, c_pos=0.15, c_neg=0.15)),
    ((44, 28), dict(method="sparse", c_pos=0.12, c_neg=0.12, n_interp=3, flow_source="lk",
                    lk=dict(levels=2, radius=3)),
     dict(method=sim.SPARSE, c_pos=0.12, c_neg=0.12, n_interp=3, flow_source=FLOW_LK,
          lk_levels=2, lk_radius=3)),
    ((21, 19), dict(method="dense", c_pos=0.1, c_neg=0.1, n_interp=40, event_capacity=2),
     dict(method=sim.DENSE, c_pos=0.1, c_neg=0.1, n_interp=40)),
]


def _videos(n_frames, seed0=30):
    out = []
    for i, ((W, H), _, _) in enumerate(MIX):
        out.append(synth.blob_video(synth.BlobVideoSpec(W, H, n_frames, 30.0, 5, seed=seed0 + i,
                                                        motion="random", speed_max=5.0)))
    return out


def _flows_for(opts, v, a, b):
    if opts["method"] == "basic" or opts.get("flow_source") == "lk":
        return None
    return v.flows[max(a - 1, 0):b - 1]


@pytest.mark.parametrize("splits", [[(0, 1), (1, 4), (4, 7)], [(0, 7)], [(0, 2), (2, 3), (3, 7)]])
def test_emulated_fused_batch_mixed_streams(emu_sim, splits):
    """Six streams of every method, thresholding and flow source in each batch; capacities
    small enough that most windows re-run their chains; the same frames split differently
    over the batches (a first frame alone, single intervals, several)."""
    vids = _videos(7)
    streams = [emu_sim.Stream(W, H, **opts) for (W, H), opts, _ in MIX]
    for a, b in splits:
        emu_sim.push_batch([(st, v.frames[a:b], _flows_for(opts, v, a, b), v.t_us[a:b])
                            for st, v, (_, opts, _) in zip(streams, vids, MIX)])
    for st, v, (_, opts, ocfg) in zip(streams, vids, MIX):
        ok, oref = oracle_run(v.frames, v.flows if opts["method"] != "basic" else None, v.t_us,
                              **ocfg)
        np.testing.assert_array_equal(st.drain_keys(), ok, err_msg=str(opts))
        np.testing.assert_array_equal(st.reference().view(np.uint32), oref.view(np.uint32))
        assert st.stats()["intervals"] == 6
        st.close()


def test_emulated_fused_batch_uneven_windows(emu_sim):
    """One stream pushes 140 frames (two windows of the batch), the others 3 or only a first
    frame: later chunks carry fewer streams."""
    long = synth.blob_video(synth.BlobVideoSpec(20, 12, 140, 60.0, 3, seed=4, motion="random",
                                                speed_max=2.0))
    short = synth.blob_video(synth.BlobVideoSpec(26, 18, 3, 30.0, 4, seed=5, motion="random",
                                                 speed_max=4.0))
    first = synth.blob_video(synth.BlobVideoSpec(18, 10, 1, 30.0, 2, seed=6))
    a = emu_sim.Stream(20, 12, method="sparse", c_pos=0.1, c_neg=0.1, n_interp=3,
                       event_capacity=16)
    b = emu_sim.Stream(26, 18, method="difference", c_pos=0.1, c_neg=0.1, n_interp=3)
    c = emu_sim.Stream(18, 10, method="dense")
    counts = emu_sim.push_batch([(a, long.frames, long.flows, long.t_us),
                                 (b, short.frames, short.flows, short.t_us),
                                 (c, first.frames, None, first.t_us)])
    oa, _ = oracle_run(long.frames, long.flows, long.t_us, method=sim.SPARSE, c_pos=0.1,
                       c_neg=0.1, n_interp=3)
    ob, _ = oracle_run(short.frames, short.flows, short.t_us, method=sim.DIFFERENCE, c_pos=0.1,
                       c_neg=0.1, n_interp=3)
    np.testing.assert_array_equal(a.drain_keys(), oa)
    np.testing.assert_array_equal(b.drain_keys(), ob)
    assert c.pending() == 0 and counts == [len(oa), len(ob), 0]
    for s in (a, b, c):
        s.close()


def test_emulated_batch_steps_replay_one_recorded_graph(emu_sim):
    """Frame by frame, five streams without estimated flow (every other method and mode), one
    batch per frame step: the first step records the step's sequence as a graph, the later steps
    of the same shape replay it (the emulation records and replays kernels and copies like
    stream capture), and every stream equals the oracle; one stream overflows its tiny arena, so
    its windows take the re-run path after the replay."""
    mix = [m for m in MIX if m[1].get("flow_source") != "lk"]
    vids = [synth.blob_video(synth.BlobVideoSpec(W, H, 6, 30.0, 5, seed=90 + i,
                                                 motion="random", speed_max=5.0))
            for i, ((W, H), _, _) in enumerate(mix)]
    streams = [emu_sim.Stream(W, H, **opts) for (W, H), opts, _ in mix]
    before = emu_sim.batch_stats()
    emu_sim.push_batch([(st, v.frames[0:1], None, v.t_us[0:1]) for st, v in zip(streams, vids)])
    for k in range(1, 6):
        emu_sim.push_batch([(st, v.frames[k:k + 1], _flows_for(opts, v, k, k + 1),
                             v.t_us[k:k + 1]) for st, v, (_, opts, _) in zip(streams, vids, mix)])
    after = emu_sim.batch_stats()
    launches = after["graph_launches"] - before["graph_launches"]
    recorded = after["graphs_recorded"] - before["graphs_recorded"]
    assert launches == 5 and 1 <= recorded < launches     # later steps replay a recorded graph
    assert after["rerun_windows"] > before["rerun_windows"]
    for st, v, (_, opts, ocfg) in zip(streams, vids, mix):
        ok, oref = oracle_run(v.frames, v.flows if opts["method"] != "basic" else None, v.t_us,
                              **ocfg)
        np.testing.assert_array_equal(st.drain_keys(), ok, err_msg=str(opts))
        np.testing.assert_array_equal(st.reference().view(np.uint32), oref.view(np.uint32))
        st.close()


ASAN_SCRIPT = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim
    sim.LIB_PATH = {lib!r}; sim._lib = None
    import test_cpu_emulated_batch as t
    from test_cpu_emulated_kernels import oracle_run
    vids = t._videos(5, seed0=60)
    streams = [sim.Stream(W, H, **opts) for (W, H), opts, _ in t.MIX]
    for a, b in ((0, 2), (2, 5)):
        sim.push_batch([(st, v.frames[a:b], t._flows_for(opts, v, a, b), v.t_us[a:b])
                        for st, v, (_, opts, _) in zip(streams, vids, t.MIX)])
    for st, v, (_, opts, ocfg) in zip(streams, vids, t.MIX):
        ok, _ = oracle_run(v.frames, v.flows if opts["method"] != "basic" else None, v.t_us,
                           **ocfg)
        assert np.array_equal(st.drain_keys(), ok), opts
        st.close()
    print("asan-clean")
""")


@pytest.mark.long
def test_emulated_fused_batch_is_memory_safe_under_asan(tmp_path):
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_batch.py"
    script.write_text(ASAN_SCRIPT.format(root=os.path.dirname(HERE), tests=HERE, lib=lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]
