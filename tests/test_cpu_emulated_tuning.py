"""Chain-pass variants and their autotuner, executed on the CPU (tests/cpu_emu): every variant
(2, 5 or 10 interior samples' texel loads in flight per lane; 1, 2 or 4 for difference frames)
gives the oracle's events and levels bit for bit, and the autotuned stream picks one of them,
keeps it for later windows of the same shape and gives the same result.  The product never loads
these builds."""
import ctypes

import numpy as np
import pytest

from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import emu_sim, monkeypatch_module, oracle_run  # noqa: F401

CASES = [
    dict(method="sparse", c_pos=0.1, c_neg=0.1, n_interp=10),
    dict(method="dense", c_pos=0.12, c_neg=0.12, n_interp=7),
    dict(method="dense", c_pos=0.03, c_neg=0.03, n_interp=10, thresh_mode="memoryless"),
    dict(method="difference", c_pos=0.05, c_neg=0.05, n_interp=6),
]
ORACLE = {"sparse": sim.SPARSE, "dense": sim.DENSE, "difference": sim.DIFFERENCE}


@pytest.mark.parametrize("cfg", CASES, ids=lambda c: c["method"] + "-" + c.get("thresh_mode", ""))
def test_every_chain_variant_equals_the_oracle(emu_sim, cfg):
    v = synth.blob_video(synth.BlobVideoSpec(45, 29, 5, 30.0, 8, seed=12, motion="random",
                                             speed_max=5.0))
    ocfg = dict(cfg, method=ORACLE[cfg["method"]],
                thresh_mode=1 if cfg.get("thresh_mode") == "memoryless" else 0)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, **ocfg)
    assert len(ok) > 50
    for variant in (0, 1, 2, -1):
        s = emu_sim.Stream(45, 29, **cfg)
        s.set_chain_variant(variant)
        assert s.chain_variant() == -1
        s.push_frames(v.frames[:3], v.flows[:2], v.t_us[:3])
        chosen = s.chain_variant()
        s.push_frames(v.frames[3:], v.flows[2:], v.t_us[3:])
        assert s.chain_variant() == chosen     # the tuned choice stays with the shape
        assert chosen == variant if variant >= 0 else chosen in (0, 1, 2)
        np.testing.assert_array_equal(s.drain_keys(), ok, err_msg=str(variant))
        np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
        s.close()


def test_chain_variant_argument_is_validated(emu_sim):
    s = emu_sim.Stream(8, 8, method="dense")
    for bad in (-2, 3, 100):
        with pytest.raises(emu_sim.SimError) as e:
            s.set_chain_variant(bad)
        assert e.value.status == emu_sim.E_INVAL
    s.close()


def test_tuning_runs_are_not_cut_short_by_a_small_arena(emu_sim):
    """A fresh shape tuned on a window whose events overflow the stream's arena: the tuner's timed
    passes run on a scratch arena grown until no wave runs out of space (so each variant is timed
    on the whole window).  Against the same push with the variant forced (no tuning), the device
    allocation log of the tuned push holds a scratch arena of 4^k times the stream's capacity
    (k >= 1); both results equal the oracle's."""
    from collections import Counter
    lib = emu_sim.load()
    v = synth.blob_video(synth.BlobVideoSpec(43, 31, 6, 30.0, 8, seed=21, motion="random",
                                             speed_max=6.0))
    cfg = dict(method="dense", c_pos=0.02, c_neg=0.02, n_interp=9)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, method=sim.DENSE, c_pos=0.02, c_neg=0.02,
                          n_interp=9)
    logs, chosen = {}, None
    for forced in (-1, None):           # tuned, then the tuned choice forced (no tuning)
        s = emu_sim.Stream(43, 31, event_capacity=1, **cfg)   # the smallest arena
        cap0 = s.stats()["event_capacity"]
        assert len(ok) > 2 * cap0       # every timed pass on the stream's arena would overflow
        s.set_chain_variant(chosen if forced is None else forced)
        lib.emu_reset_alloc_log()
        s.push_frames(v.frames, v.flows, v.t_us)
        sizes = (ctypes.c_size_t * 4096)()
        n = lib.emu_alloc_log(sizes, 4096)
        logs[forced] = Counter(sizes[i] for i in range(min(n, 4096)))
        chosen = s.chain_variant()
        np.testing.assert_array_equal(s.drain_keys(), ok)
        np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
        s.close()
    extra = logs[-1] - logs[None]       # what the tuning allocated
    grown = {8 * cap0 * 4 ** k for k in range(1, 12)}   # scratch arenas the tuner grew
    assert grown & set(extra), sorted(extra)
