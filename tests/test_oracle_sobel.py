"""Pins of the oracle's Sobel edge detector (Sect. 4.2): a single-iteration
stencil whose output is the integer gradient magnitude, outside samples 0.

* closed forms: a constant image has magnitude 0 away from the border; a ramp
  u = j gives Gx = 8, Gy = 0, so magnitude 8, inside; a step of height 255 gives
  Gx = 4 * 255, clamped to 255, on both sides of the step;
* transposing the image transposes the output (Gx and Gy swap roles);
* brute force: an independent correlation with the two masks over a zero-padded
  image, then numpy's integer square root by floor(sqrt) with an exactness check;
* the reduce is the sum of the output, and later sweeps apply the same map again.
"""
import numpy as np

import oracle as O
from paper_1609_04567_amd import inputs as I

KX = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]])


def _brute(a):
    p = np.pad(a.astype(np.int64), 1)
    rows, cols = a.shape
    gx = np.zeros((rows, cols), np.int64)
    gy = np.zeros((rows, cols), np.int64)
    for di in range(3):
        for dj in range(3):
            win = p[di:di + rows, dj:dj + cols]
            gx += KX[di, dj] * win
            gy += KX.T[di, dj] * win
    m = gx * gx + gy * gy
    s = np.floor(np.sqrt(m.astype(np.float64))).astype(np.int64)
    assert np.all(s * s <= m) and np.all((s + 1) * (s + 1) > m)
    return np.minimum(s, 255).astype(np.uint8)


def test_closed_forms():
    c = np.full((9, 11), 77, np.uint8)
    o, r = O.sobel_run(c)
    assert np.all(o[1:-1, 1:-1] == 0) and r.n == 1
    ramp = np.tile(np.arange(20, dtype=np.uint8), (6, 1))
    o, _ = O.sobel_run(ramp)
    assert np.all(o[1:-1, 1:-1] == 8)
    step = np.zeros((5, 8), np.uint8)
    step[:, 4:] = 255
    o, _ = O.sobel_run(step)
    assert np.all(o[1:-1, 3:5] == 255) and np.all(o[1:-1, 1:3] == 0) and np.all(o[1:-1, 6] == 0)


def test_brute_force_and_transpose():
    rng = np.random.default_rng(3)
    for shape in ((8, 8), (17, 13), (1, 5), (4, 1)):
        a = rng.integers(0, 256, shape, dtype=np.uint8)
        o, r = O.sobel_run(a)
        assert np.array_equal(o, _brute(a))
        assert r.count == int(o.astype(np.uint64).sum())
        ot, _ = O.sobel_run(np.ascontiguousarray(a.T))
        assert np.array_equal(ot, o.T)


def test_sweeps_repeat_the_map_and_the_reduce_is_the_sum():
    a = I.restore_input(40, 30, seed=2).y
    o3, r3 = O.sobel_run(a, max_iter=3, trace_cap=3)
    x = a
    for k in range(3):
        x = _brute(x)
        assert r3.trace[k] == int(x.astype(np.uint64).sum())
    assert np.array_equal(o3, x) and r3.n == 3 and r3.checks == 3
