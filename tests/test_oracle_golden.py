"""The oracle reproduces the hand-worked fixtures in tests/golden/ exactly."""
import numpy as np
import pytest

import golden_io
from oracle.oracle import OracleSim, decode


@pytest.mark.parametrize("path", golden_io.all_fixtures() + golden_io.next_fixtures(),
                         ids=lambda p: p.rsplit("/", 1)[-1])
def test_oracle_matches_hand_worked_fixture(oracle_mod, path):
    g = golden_io.load(path)
    T, H, W = g.frames.shape
    sim = OracleSim(W, H, **g.cfg)
    for k in range(T):
        keys = sim.push(g.frames[k], None if k == 0 else g.flows[k - 1], g.t_us[k])
        if k == 0:
            assert len(keys) == 0
            continue
        t, x, y, p = decode(keys, sim.epoch)
        got = list(zip(t.tolist(), x.tolist(), y.tolist(), p.tolist()))
        assert got == g.events[k - 1], f"interval {k}"
    np.testing.assert_array_equal(sim.lref(), g.lref)
