"""GPU: every chain-pass variant (2, 5 or 10 interior samples' texel loads in flight per lane;
1, 2 or 4 for difference frames) and the autotuner's choice give the oracle's events and
reference levels bit for bit, at the sparse 1280x720 workload's full size and on dense,
memoryless and difference-frame sequences."""
import numpy as np
import pytest

from paper_2209_04634_amd import sim, synth
from test_parity_gpu import oracle_keys

pytestmark = pytest.mark.gpu


def _run(v, variant, **cfg):
    T, H, W = v.frames.shape
    s = sim.Stream(W, H, **cfg)
    s.set_chain_variant(variant)
    s.push_frames(v.frames, v.flows, v.t_us)
    chosen = s.chain_variant()
    keys, ref = s.drain_keys(), s.reference()
    s.close()
    return keys, ref, chosen


def test_chain_variants_sparse_1280x720_full_sequence():
    v = synth.blob_video(synth.sparse_1280x720())
    cfg = dict(method=sim.SPARSE, c_pos=0.2, c_neg=0.2, n_interp=10)
    ok, oref = oracle_keys(v.frames, v.flows, v.t_us, **cfg)
    for variant in (0, 1, 2, -1):
        print(f"sparse 1280x720, chain variant {variant}", flush=True)
        keys, ref, chosen = _run(v, variant, **cfg)
        assert chosen in (0, 1, 2) and (variant < 0 or chosen == variant)
        np.testing.assert_array_equal(keys, ok, err_msg=str(variant))
        np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32))


@pytest.mark.parametrize("cfg", [
    dict(method=sim.DENSE, c_pos=0.15, c_neg=0.15, n_interp=10),
    dict(method=sim.DENSE, c_pos=0.03, c_neg=0.03, n_interp=10, thresh_mode=sim.MEMORYLESS),
    dict(method=sim.DIFFERENCE, c_pos=0.3, c_neg=0.3, n_interp=10),
], ids=["dense", "dense-memoryless", "difference"])
def test_chain_variants_346x260(cfg):
    v = synth.blob_video(synth.dense_346x260(n_frames=8))
    ok, oref = oracle_keys(v.frames, v.flows, v.t_us, **cfg)
    for variant in (0, 1, 2, -1):
        keys, ref, _ = _run(v, variant, **cfg)
        np.testing.assert_array_equal(keys, ok, err_msg=str(variant))
        np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32))
