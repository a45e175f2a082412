"""Pins of the oracle's memoryless thresholding, difference-frame method, accumulated event frame
and events/(pixel s) statistic against facts fixed by the paper and by mathematics.

Each test targets a class of plausible mistakes: a non-strict comparison, a wrong sample pair,
a wrong time on the sub-frame grid, a swapped flow component or difference order, a state that
does not roll forward, a wrong polarity plane, an off-by-one window edge, a sample instead of a
population deviation.  None re-types the oracle's arithmetic.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import brute64
from oracle.oracle import (OracleSim, accumulate, decode, event_rate, BASIC, DENSE, SPARSE,
                           DIFFERENCE, LOG, LINEAR, REFERENCE, MEMORYLESS)
from paper_2209_04634_amd import synth

MCODE = {"basic": BASIC, "dense": DENSE, "sparse": SPARSE, "difference": DIFFERENCE}


def _run(frames, flows, t, **cfg):
    T, H, W = frames.shape
    sim = OracleSim(W, H, **cfg)
    out = []
    for k in range(T):
        ev = sim.push(frames[k], None if (flows is None or k == 0) else flows[k - 1], int(t[k]))
        if k:
            out.append(ev)
    return out, sim


def _per_pixel(keys, epoch=0):
    t, x, y, p = decode(keys, epoch)
    d = {}
    for ti, xi, yi, pi in zip(t.tolist(), x.tolist(), y.tolist(), p.tolist()):
        d.setdefault((xi, yi), []).append((ti, pi))
    return d


def _compare_memoryless(frames, flows, t, method, S, C=0.2, transform="log", mask=-1.0):
    evs, sim = _run(frames, flows, t, method=MCODE[method], c_pos=C, c_neg=C, n_interp=S - 1,
                    transform=LOG if transform == "log" else LINEAR, mask_threshold=mask,
                    thresh_mode=MEMORYLESS)
    ref, near = brute64.solve_memoryless_sequence(frames, flows, t, method, transform=transform,
                                                  c_pos=C, c_neg=C, n_interp=S - 1, mask=mask)
    compared = 0
    H, W = frames.shape[1:]
    for keys, bref in zip(evs, ref):
        got = _per_pixel(keys, sim.epoch)
        for y in range(H):
            for x in range(W):
                if near[y, x]:
                    continue
                a, b = sorted(got.get((x, y), [])), sorted(bref.get((x, y), []))
                assert len(a) == len(b), (method, S, x, y, a, b)
                assert [p for _, p in a] == [p for _, p, _ in b], (method, S, x, y, a, b)
                for (ta, _), (tb, _, exact) in zip(a, b):
                    assert abs(ta - tb) <= (0 if exact else 1), (method, S, x, y, a, b)
                compared += 1
    return compared


@pytest.mark.parametrize("method", ["basic", "dense", "sparse", "difference"])
@pytest.mark.parametrize("S", [1, 2, 11])
def test_memoryless_brute_force_8x8(oracle_mod, method, S):
    """Against the independent float64 solver: every pixel away from a threshold tie has the same
    events (count, polarity, time on the sub-frame grid)."""
    if method == "basic" and S != 1:
        pytest.skip("basic has one sub-interval")
    total = 0
    for seed in range(40):
        rng = np.random.default_rng(7000 + 100 * S + seed)
        frames, flows = synth.random_frames(rng, 4, 8, 8, flow_scale=2.5)
        t = np.cumsum(rng.integers(500, 40000, 4))
        C = 0.05 if method != "basic" else 0.3     # sub-frame steps are ~1/S of a frame step
        total += _compare_memoryless(frames, flows, t, method, S, C=C)
    intervals = 2 if method == "difference" else 3
    assert total > 0.8 * 40 * intervals * 64


@pytest.mark.parametrize("method", ["dense", "difference"])
def test_memoryless_brute_force_linear_table_i(oracle_mod, method):
    """Linear intensities with non-integer thresholds near Table I's scale."""
    total = 0
    for seed in range(30):
        rng = np.random.default_rng(seed)
        frames, flows = synth.random_frames(rng, 4, 8, 8, flow_scale=3.0)
        t = np.array([0, 33333, 66667, 100000])
        C = 2.3 if method == "dense" else 20.5
        total += _compare_memoryless(frames, flows, t, method, 11, C=C, transform="linear")
    assert total > 0.7 * 30 * 2 * 64


@pytest.mark.parametrize("method", [BASIC, DENSE, SPARSE, DIFFERENCE])
def test_memoryless_at_most_one_event_per_subframe_on_the_grid(oracle_mod, method):
    v = synth.blob_video(synth.BlobVideoSpec(40, 30, 4, 30.0, 6, seed=3, motion="random",
                                             speed_max=6.0))
    S = 1 if method == BASIC else 5
    evs, sim = _run(v.frames, v.flows, v.t_us, method=method, c_pos=0.02, c_neg=0.02,
                    n_interp=S - 1, thresh_mode=MEMORYLESS)
    n = 0
    for i, keys in enumerate(evs):
        t0, t1 = int(v.t_us[i]), int(v.t_us[i + 1])
        grid = {t0 + (j * (t1 - t0)) // S for j in range(1, S + 1)}
        grid |= {g - 1 for g in grid}                  # fp32 rounding of j/S * delta
        t, x, y, p = decode(keys, sim.epoch)
        assert set(t.tolist()) <= grid
        pix = list(zip(t.tolist(), x.tolist(), y.tolist()))
        assert len(pix) == len(set(pix))               # one event per pixel and sub-frame
        n += len(pix)
    assert n > 100
    np.testing.assert_array_equal(sim.lref(), oracle_lut_frame(v.frames[0]))


def oracle_lut_frame(frame):
    from oracle.oracle import lut
    return lut(LOG, 1e-3)[frame]


@pytest.mark.parametrize("method", [BASIC, DENSE, SPARSE, DIFFERENCE])
def test_memoryless_static_and_constant_inputs_emit_nothing(oracle_mod, method):
    rng = np.random.default_rng(2)
    f = rng.integers(0, 256, size=(12, 17), dtype=np.uint8)
    frames = np.stack([f, f, f, f])
    flows = (rng.standard_normal((3, 12, 17, 2)) * 0.0).astype(np.float32)
    evs, _ = _run(frames, flows, [0, 10, 20, 30], method=method, c_pos=0.01, c_neg=0.01,
                  n_interp=4, thresh_mode=MEMORYLESS)
    assert all(len(e) == 0 for e in evs)
    # spatially constant frames with arbitrary flow: bilinear samples are the constant itself
    frames = np.stack([np.full((12, 17), v, np.uint8) for v in (50, 50, 50, 50)])
    flows = (rng.standard_normal((3, 12, 17, 2)) * 4.0).astype(np.float32)
    evs, _ = _run(frames, flows, [0, 10, 20, 30], method=method, c_pos=0.01, c_neg=0.01,
                  n_interp=4, thresh_mode=MEMORYLESS)
    assert all(len(e) == 0 for e in evs)


def test_memoryless_dense_with_one_subinterval_is_basic(oracle_mod):
    rng = np.random.default_rng(11)
    frames, flows = synth.random_frames(rng, 5, 20, 24, flow_scale=3.0)
    t = [0, 1000, 2500, 2600, 9000]
    a, _ = _run(frames, None, t, method=BASIC, c_pos=0.3, c_neg=0.25, thresh_mode=MEMORYLESS)
    b, _ = _run(frames, flows, t, method=DENSE, n_interp=0, c_pos=0.3, c_neg=0.25,
                thresh_mode=MEMORYLESS)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_memoryless_and_reference_agree_below_two_thresholds(oracle_mod):
    """Basic method: where C < |dL| < 2C (away from both ends) both readings emit exactly one
    event of the same polarity; the memoryless one at the frame time, the reference one inside
    the interval; where |dL| < C neither fires."""
    rng = np.random.default_rng(4)
    f0 = rng.integers(30, 220, size=(16, 16), dtype=np.uint8)
    f1 = np.clip(f0.astype(int) + rng.integers(-60, 61, size=f0.shape), 0, 255).astype(np.uint8)
    C = 0.2
    frames = np.stack([f0, f1])
    mem, sm = _run(frames, None, [0, 40000], method=BASIC, c_pos=C, c_neg=C,
                   thresh_mode=MEMORYLESS)
    ref, sr = _run(frames, None, [0, 40000], method=BASIC, c_pos=C, c_neg=C)
    from oracle.oracle import lut
    L = lut(LOG, 1e-3).astype(np.float64)
    dl = L[f1] - L[f0]
    pm, pr = _per_pixel(mem[0]), _per_pixel(ref[0])
    checked = 0
    for y in range(16):
        for x in range(16):
            q = abs(dl[y, x]) / C
            if abs(q - 1) < 1e-4 or abs(q - 2) < 1e-4:
                continue
            if q < 1:
                assert (x, y) not in pm and (x, y) not in pr
            elif q < 2:
                (tm, sgn_m), = pm[(x, y)]
                (tr, sgn_r), = pr[(x, y)]
                assert sgn_m == sgn_r == (1 if dl[y, x] > 0 else -1)
                assert tm == 40000 and tr <= 40000
                checked += 1
            else:
                assert len(pm[(x, y)]) == 1 and len(pr[(x, y)]) == math.floor(q)
    assert checked > 20


def test_memoryless_time_reversal_flips_polarity(oracle_mod):
    rng = np.random.default_rng(8)
    frames, _ = synth.random_frames(rng, 2, 14, 18)
    fwd, _ = _run(frames, None, [0, 1000], method=BASIC, c_pos=0.3, c_neg=0.3,
                  thresh_mode=MEMORYLESS)
    bwd, _ = _run(frames[::-1].copy(), None, [0, 1000], method=BASIC, c_pos=0.3, c_neg=0.3,
                  thresh_mode=MEMORYLESS)
    a, b = _per_pixel(fwd[0]), _per_pixel(bwd[0])
    assert set(a) == set(b) and len(a) > 20
    for k in a:
        assert [p for _, p in a[k]] == [-p for _, p in b[k]]


@pytest.mark.parametrize("bright_left", [True, False])
@pytest.mark.parametrize("S,v", [(2, 2), (4, 4), (3, 6)])
def test_difference_translating_edge_closed_form(oracle_mod, bright_left, S, v):
    """A vertical edge moving v px per frame with exact flow (v, 0) between difference frames.
    The difference frame of interval i is a band of width v at columns [e_{i-1}, e_i) holding
    +-180 (LINEAR); interpolating at tau = k/S with k*v/S integral shifts that band by k*v/S
    exactly, so sub-frame k of interval i fires on columns [e_{i-2} + k v/S, e_{i-2} + k v/S + v)
    of every row, with the sign of the band, at t_{i-1} + floor(k/S * delta)."""
    H, W, e0, T = 3, 64, 10, 5
    cols = np.arange(W)
    frames = []
    for i in range(T):
        e = e0 + i * v
        row = np.where(cols < e, 200, 20) if bright_left else np.where(cols < e, 20, 200)
        frames.append(np.tile(row.astype(np.uint8), (H, 1)))
    frames = np.stack(frames)
    flows = np.zeros((T - 1, H, W, 2), np.float32)
    flows[..., 0] = v
    t = [0, 33333, 66667, 100000, 133333]
    evs, sim = _run(frames, flows, t, method=DIFFERENCE, transform=LINEAR, c_pos=20, c_neg=20,
                    n_interp=S - 1, thresh_mode=MEMORYLESS)
    assert len(evs[0]) == 0
    sign = 1 if bright_left else -1
    for i in range(2, T):
        expect = []
        t0, t1 = t[i - 1], t[i]
        for k in range(1, S + 1):
            start = e0 + (i - 2) * v + k * v // S
            tk = t0 + (k * (t1 - t0)) // S
            for y in range(H):
                for x in range(start, start + v):
                    expect.append((tk, x, y, sign))
        tt, xx, yy, pp = decode(evs[i - 1], sim.epoch)
        got = list(zip(tt.tolist(), xx.tolist(), yy.tolist(), pp.tolist()))
        assert sorted(got) == sorted(expect), (i, S, v)


def test_difference_vertical_motion_uses_the_y_component(oracle_mod):
    """The same closed form rotated: a horizontal edge moving down with flow (0, v)."""
    S, v, H, W, e0, T = 2, 2, 40, 3, 8, 4
    rows = np.arange(H)
    frames = np.stack([np.tile(np.where(rows < e0 + i * v, 200, 20).astype(np.uint8)[:, None],
                               (1, W)) for i in range(T)])
    flows = np.zeros((T - 1, H, W, 2), np.float32)
    flows[..., 1] = v
    t = [0, 1000, 2000, 3000]
    evs, sim = _run(frames, flows, t, method=DIFFERENCE, transform=LINEAR, c_pos=20, c_neg=20,
                    n_interp=S - 1, thresh_mode=MEMORYLESS)
    for i in range(2, T):
        tt, xx, yy, pp = decode(evs[i - 1], sim.epoch)
        for k in range(1, S + 1):
            start = e0 + (i - 2) * v + k * v // S
            sel = tt == t[i - 1] + (k * 1000) // S
            assert sorted(set(yy[sel].tolist())) == list(range(start, start + v))
            assert (pp[sel] == 1).all() and sel.sum() == v * W


def test_difference_first_interval_and_restart(oracle_mod):
    """Two frames give one difference frame: no events.  The third frame gives S sub-frames."""
    rng = np.random.default_rng(3)
    frames, flows = synth.random_frames(rng, 3, 10, 10, flow_scale=1.0)
    evs, _ = _run(frames, flows, [0, 100, 200], method=DIFFERENCE, c_pos=0.01, c_neg=0.01,
                  n_interp=3, thresh_mode=MEMORYLESS)
    assert len(evs[0]) == 0 and len(evs[1]) > 0
    # the thresholding mode field does not change the difference method
    evs2, _ = _run(frames, flows, [0, 100, 200], method=DIFFERENCE, c_pos=0.01, c_neg=0.01,
                   n_interp=3, thresh_mode=REFERENCE)
    np.testing.assert_array_equal(evs[1], evs2[1])


# ------------------------------------------------------------------------------------------
# Accumulated event frame and events/(pixel s)
# ------------------------------------------------------------------------------------------

def _key(t_rel, x, y, pos):
    return np.uint64((t_rel << 25) | (y << 13) | (x << 1) | (1 if pos else 0))


def test_accumulate_hand_example(oracle_mod):
    """3x2 sensor, epoch 1000, window [1010, 1030): events at t = 1005 (outside), 1010 (first
    inside), 1029 (last inside), 1030 (outside).  Worked by hand:
        (x=2, y=1, +) at 1010, (x=2, y=1, +) at 1015, (x=0, y=0, -) at 1029 are counted;
        (x=1, y=0, +) at 1005 and (x=1, y=1, -) at 1030 are not."""
    keys = np.array([_key(5, 1, 0, True), _key(10, 2, 1, True), _key(15, 2, 1, True),
                     _key(29, 0, 0, False), _key(30, 1, 1, False)], dtype=np.uint64)
    c = accumulate(keys, 1000, 1010, 1030, 3, 2)
    pos = np.array([[0, 0, 0], [0, 0, 2]], np.uint32)
    neg = np.array([[1, 0, 0], [0, 0, 0]], np.uint32)
    np.testing.assert_array_equal(c[0], pos)
    np.testing.assert_array_equal(c[1], neg)
    # accumulation adds to what the frame already holds
    c = accumulate(keys, 1000, 1000, 2000, 3, 2, counts=c)
    np.testing.assert_array_equal(c[0], [[0, 1, 0], [0, 0, 4]])
    np.testing.assert_array_equal(c[1], [[2, 0, 0], [0, 1, 0]])


def test_accumulate_matches_loop_and_windows_partition(oracle_mod):
    rng = np.random.default_rng(1)
    W, H, n = 23, 17, 5000
    t = np.sort(rng.integers(0, 10000, n))
    x = rng.integers(0, W, n)
    y = rng.integers(0, H, n)
    p = rng.integers(0, 2, n)
    keys = ((t.astype(np.uint64) << np.uint64(25)) | (y.astype(np.uint64) << np.uint64(13))
            | (x.astype(np.uint64) << np.uint64(1)) | p.astype(np.uint64))
    ref = np.zeros((2, H, W), np.uint32)
    for ti, xi, yi, pi in zip(t.tolist(), x.tolist(), y.tolist(), p.tolist()):
        if 2000 <= 5 + ti < 7000:
            ref[0 if pi else 1, yi, xi] += 1
    np.testing.assert_array_equal(accumulate(keys, 5, 2000, 7000, W, H), ref)
    a = accumulate(keys, 5, 0, 4321, W, H)
    b = accumulate(keys, 5, 4321, 20000, W, H)
    full = accumulate(keys, 5, 0, 20000, W, H)
    np.testing.assert_array_equal(a + b, full)
    assert int(full.sum()) == n


def test_event_rate_hand_example(oracle_mod):
    """2x2 sensor over 0.5 s with per-pixel counts (both polarities) 3, 1, 0, 0:
    S1 = 4, S2 = 10, mean count 1, mean square 2.5, variance 1.5 ->
    mean 2 events/(pixel s), standard deviation sqrt(1.5) / 0.5 = sqrt(6)."""
    counts = np.zeros((2, 2, 2), np.uint32)
    counts[0] = [[2, 1], [0, 0]]
    counts[1] = [[1, 0], [0, 0]]
    mean, std, sums = event_rate(counts, 0, 500000)
    assert sums == (4, 10)
    assert mean == 2.0
    assert abs(std - math.sqrt(6.0)) <= 4 * np.spacing(math.sqrt(6.0))


def test_event_rate_is_the_population_statistic(oracle_mod):
    rng = np.random.default_rng(9)
    counts = rng.integers(0, 50, size=(2, 31, 47)).astype(np.uint32)
    mean, std, (s1, s2) = event_rate(counts, 100, 1100100)
    c = (counts[0].astype(np.int64) + counts[1]).ravel()
    T = Fraction(1100000, 10 ** 6)
    assert s1 == int(c.sum()) and s2 == int((c * c).sum())
    exact_mean = Fraction(s1, c.size) / T
    exact_var = Fraction(s2, c.size) - Fraction(s1, c.size) ** 2
    assert abs(Fraction(mean) - exact_mean) <= Fraction(1, 10 ** 12) * exact_mean
    assert abs(std - math.sqrt(exact_var) / float(T)) <= 1e-12 * std
    assert abs(std - float(np.std(c / 1.1))) <= 1e-9 * std       # ddof = 0, not 1
