"""Pins of the oracle's radius-k box stencil (sigma_k with k > 1, Sect. 3.1) and
its 3D 7-point Jacobi.

Box (mean of the (2k+1)^2 neighbourhood, band of width k fixed):
* constant and affine fields are exact fixed points for every k (the box sum of
  an affine integer field is exactly (2k+1)^2 times its centre, and the division
  is exact), so the loop stops after one sweep with r = 0;
* integer-valued input: one sweep equals an independent numpy box sum divided by
  the count, bit for bit (all partial sums are exact integers);
* real-valued input: several sweeps agree with numpy to rounding;
* the maximum norm of the update never grows (an averaging operator), and all
  values stay within the initial range (maximum principle).

3D (b = (((W+E) + (N+S)) + (U+D)) / 6 inside, faces fixed):
* discrete harmonic polynomials (x^2 - y^2, xyz, x^2 + y^2 - 2 z^2) are exact
  fixed points;
* bit-exact against a numpy slice formulation with the same association;
* monotone growth from a zero interior under a non-negative boundary.
"""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_box_constant_and_affine_fixed_points(k):
    rows, cols = 4 * k + 7, 3 * k + 9
    i = np.arange(rows, dtype=np.float64)[:, None]
    j = np.arange(cols, dtype=np.float64)[None, :]
    for u in (np.full((rows, cols), 7.25), 3.0 * i - 2.0 * j + 5.0):
        o, r = O.box_run(np.ascontiguousarray(u + 0 * j), k, max_iter=10)
        assert r.n == 1 and r.r == 0.0 and np.array_equal(o, u + 0 * j)


def _box_numpy(a, k):
    rows, cols = a.shape
    b = a.copy()
    s = np.zeros((rows - 2 * k, cols - 2 * k))
    for di in range(2 * k + 1):
        for dj in range(2 * k + 1):
            s += a[di:di + rows - 2 * k, dj:dj + cols - 2 * k]
    b[k:rows - k, k:cols - k] = s / float((2 * k + 1) ** 2)
    return b


@pytest.mark.parametrize("k", [1, 2, 4])
def test_box_against_numpy(k):
    rng = np.random.default_rng(k)
    a = rng.integers(0, 1000, (23, 31)).astype(np.float64)
    o, _ = O.box_run(a, k, cond=O.COND_NEVER, max_iter=1)
    assert np.array_equal(o, _box_numpy(a, k))
    x = rng.uniform(0, 1, (29, 19))
    o, _ = O.box_run(x, k, cond=O.COND_NEVER, max_iter=5)
    y = x
    for _ in range(5):
        y = _box_numpy(y, k)
    assert np.max(np.abs(o - y)) < 1e-14


def test_box_update_norm_never_grows_and_range_is_kept():
    rng = np.random.default_rng(9)
    a = rng.uniform(-1, 2, (40, 40))
    _, r = O.box_run(a, 3, cond=O.COND_NEVER, max_iter=30, trace_cap=30)
    assert np.all(np.diff(r.trace) <= 1e-15)
    o, _ = O.box_run(a, 3, cond=O.COND_NEVER, max_iter=30)
    assert o.min() >= a.min() and o.max() <= a.max()


def test_jacobi3d_harmonic_fixed_points_and_numpy():
    nz, ny, nx = 7, 9, 11
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    for u in (x * x - y * y + 0 * z, x * y * z, x * x + y * y - 2 * z * z):
        o, r = O.jacobi3d_run(np.ascontiguousarray(u), max_iter=5)
        assert r.n == 1 and r.r == 0.0 and np.array_equal(o, u)
    rng = np.random.default_rng(4)
    a = rng.uniform(0, 1, (nz, ny, nx))
    o, _ = O.jacobi3d_run(a, cond=O.COND_NEVER, max_iter=3)
    b = a.copy()
    for _ in range(3):
        c = b.copy()
        c[1:-1, 1:-1, 1:-1] = (((b[1:-1, 1:-1, :-2] + b[1:-1, 1:-1, 2:]) +
                                (b[1:-1, :-2, 1:-1] + b[1:-1, 2:, 1:-1])) +
                               (b[:-2, 1:-1, 1:-1] + b[2:, 1:-1, 1:-1])) / 6.0
        b = c
    assert np.array_equal(o, b)


def test_jacobi3d_monotone_from_zero_interior():
    rng = np.random.default_rng(8)
    a = rng.uniform(0, 1, (6, 8, 10))
    a[1:-1, 1:-1, 1:-1] = 0.0
    prev = a
    for n in (1, 2, 5, 9):
        o, _ = O.jacobi3d_run(a, cond=O.COND_NEVER, max_iter=n)
        assert np.all(o >= prev) and o.max() < 1.0
        prev = o
