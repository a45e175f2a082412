"""The exact HIP kernel and runtime sources, executed on the CPU (tests/cpu_emu), against the oracle.

These tests do not replace the GPU parity tests (test_parity_gpu.py, marked gpu): they run the
same source files compiled for the host through a HIP emulation layer (one fiber per GPU thread,
lockstep wave64 intrinsics, block barriers), so index arithmetic, overflow re-runs, window splits
and every intrinsic use can be checked without a GPU -- and, in the AddressSanitizer build, every
memory access is bounds-checked.  The product never loads these builds.
"""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import golden_io
from oracle.oracle import OracleSim
from paper_2209_04634_amd import sim, synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "cpu_emu"))
import build as emu_build  # noqa: E402


@pytest.fixture(scope="module")
def emu_sim(monkeypatch_module):
    path = emu_build.build()
    monkeypatch_module.setattr(sim, "LIB_PATH", path)
    monkeypatch_module.setattr(sim, "_lib", None)
    yield sim
    sim._lib = None


@pytest.fixture(scope="module")
def monkeypatch_module():
    mp = pytest.MonkeyPatch()
    yield mp
    mp.undo()


def oracle_run(frames, flows, t, **cfg):
    T, H, W = frames.shape
    o = OracleSim(W, H, **cfg)
    out = []
    for k in range(T):
        ev = o.push(frames[k], None if (flows is None or k == 0) else flows[k - 1], int(t[k]))
        if k:
            out.append(ev)
    return (np.concatenate(out) if out else np.zeros(0, np.uint64)), o.lref()


def emu_run(s_mod, frames, flows, t, mode="window", **cfg):
    T, H, W = frames.shape
    s = s_mod.Stream(W, H, **cfg)
    if mode == "window":
        s.push_frames(frames, flows, t)
    else:
        for k in range(T):
            s.push(frames[k], None if (flows is None or k == 0) else flows[k - 1], int(t[k]))
    keys, ref, st = s.drain_keys(), s.reference(), s.stats()
    s.close()
    return keys, ref, st


def check(s_mod, frames, flows, t, modes=("window",), **cfg):
    ok, oref = oracle_run(frames, flows, t, **cfg)
    for mode in modes:
        keys, ref, st = emu_run(s_mod, frames, flows, t, mode=mode, **cfg)
        np.testing.assert_array_equal(keys, ok, err_msg=mode)
        np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32), err_msg=mode)
    return len(ok)


@pytest.mark.parametrize("path", golden_io.all_fixtures(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_emulated_hand_worked_fixtures(emu_sim, path):
    g = golden_io.load(path)
    for mode in ("window", "single"):
        keys, ref, _ = emu_run(emu_sim, g.frames, g.flows, g.t_us, mode=mode, **g.cfg)
        t, x, y, p = emu_sim.decode_keys(keys, g.t_us[0])
        assert list(zip(t.tolist(), x.tolist(), y.tolist(), p.tolist())) == \
            [e for iv in g.events for e in iv]
        np.testing.assert_array_equal(ref, g.lref)


@pytest.mark.parametrize("S", [1, 2, 11, 33])
@pytest.mark.parametrize("method", [sim.BASIC, sim.DENSE, sim.SPARSE])
def test_emulated_ragged_image(emu_sim, method, S):
    if method == sim.BASIC and S != 1:
        pytest.skip("basic has one sub-interval")
    rng = np.random.default_rng(100 * S + method)
    frames, flows = synth.random_frames(rng, 4, 23, 37, flow_scale=3.0)
    t = np.array([0, 33333, 50000, 83333])
    check(emu_sim, frames, flows, t, modes=("window", "single"), method=method, c_pos=0.2,
          c_neg=0.25, n_interp=S - 1)


def test_emulated_blob_video_dense_and_sparse(emu_sim):
    spec = synth.BlobVideoSpec(96, 64, 8, 30.0, 10, seed=5, motion="random", speed_max=8.0)
    v = synth.blob_video(spec)
    n1 = check(emu_sim, v.frames, v.flows, v.t_us, modes=("window", "single"),
               method=sim.DENSE, c_pos=0.15, c_neg=0.15)
    n2 = check(emu_sim, v.frames, v.flows, v.t_us, method=sim.SPARSE, c_pos=0.15, c_neg=0.15)
    assert n1 > n2 > 0


def test_emulated_overflow_reruns(emu_sim):
    spec = synth.BlobVideoSpec(64, 48, 6, 30.0, 8, seed=9, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, method=sim.DENSE, c_pos=0.15, c_neg=0.15)
    for cap in (1, 300, 5000):
        keys, ref, st = emu_run(emu_sim, v.frames, v.flows, v.t_us, method=sim.DENSE,
                                c_pos=0.15, c_neg=0.15, event_capacity=cap)
        np.testing.assert_array_equal(keys, ok)
        np.testing.assert_array_equal(ref, oref)
        assert st["retries"] > 0


def test_emulated_long_sparse_sequence_spans_windows(emu_sim):
    """140 frames: two windows (128 + 11 intervals) and all four selection mask words."""
    spec = synth.BlobVideoSpec(24, 16, 140, 60.0, 3, seed=4, motion="random", speed_max=2.0)
    v = synth.blob_video(spec)
    check(emu_sim, v.frames, v.flows, v.t_us, method=sim.SPARSE, c_pos=0.1, c_neg=0.1,
          n_interp=3)


@pytest.mark.parametrize("shape", [(1, 1), (1, 70), (70, 1), (3, 129)])
def test_emulated_degenerate_shapes(emu_sim, shape):
    H, W = shape
    rng = np.random.default_rng(H * 7 + W)
    frames, flows = synth.random_frames(rng, 3, H, W)
    for method in (sim.BASIC, sim.DENSE, sim.SPARSE):
        check(emu_sim, frames, flows, np.array([0, 900, 2100]), method=method, n_interp=4)


ASAN_SCRIPT = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim, synth
    sim.LIB_PATH = {lib!r}; sim._lib = None
    from test_cpu_emulated_kernels import oracle_run, emu_run
    cases = []
    spec = synth.BlobVideoSpec(64, 48, 6, 30.0, 8, seed=9, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    for method in (0, 1, 2):
        for cap in (1, 0):
            cases.append((v.frames, v.flows, v.t_us, dict(method=method, c_pos=0.15,
                          c_neg=0.15, event_capacity=cap)))
    spec = synth.BlobVideoSpec(20, 12, 140, 60.0, 3, seed=4, motion="random", speed_max=2.0)
    w = synth.blob_video(spec)
    cases.append((w.frames, w.flows, w.t_us, dict(method=2, c_pos=0.1, c_neg=0.1, n_interp=3,
                  event_capacity=1)))
    rng = np.random.default_rng(1)
    f, fl = synth.random_frames(rng, 3, 5, 7)
    cases.append((f, fl, np.array([0, 10, 20]), dict(method=1, n_interp=40, event_capacity=1)))
    for frames, flows, t, cfg in cases:
        ocfg = dict((k, v) for k, v in cfg.items() if k != "event_capacity")
        ok, oref = oracle_run(frames, flows, t, **ocfg)
        keys, ref, st = emu_run(sim, frames, flows, t, **cfg)
        assert np.array_equal(keys, ok) and np.array_equal(ref, oref), cfg
    print("asan-clean", len(cases))
""")


def test_emulated_kernels_are_memory_safe_under_asan(tmp_path):
    """Every device-memory access of the runtime and kernels, bounds-checked by AddressSanitizer
    (device buffers are host allocations in this build), on overflow re-runs, window splits and
    the recompute path beyond the LDS stash."""
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_case.py"
    script.write_text(ASAN_SCRIPT.format(root=os.path.dirname(HERE), tests=HERE, lib=lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]
