"""Pins of the oracle's -i form of the Helmholtz sweep (Sect. 3.1: the elemental
function also sees the cell's index), whose right-hand side is evaluated from the
indices as g(i, j) = c2 * (c1 * (p_i * q_j)) instead of being read from an array.

* It equals the array form bit for bit when the array holds the same products
  (an independent numpy evaluation), for asymmetric p and q, so a swapped or
  shifted index fails;
* with p = q = sin(pi x), c1 = 2 pi^2 + alpha and c2 = h^2 it is the manufactured
  solve, whose iterates follow the closed form c*(1 - mu^n) u*.
"""
import math

import numpy as np

import oracle as O
from paper_1609_04567_amd import inputs as I


def test_sep_equals_array_form_for_asymmetric_factors():
    rng = np.random.default_rng(11)
    rows, cols = 23, 17
    p = rng.uniform(-1, 1, rows)
    q = rng.uniform(0, 2, cols)
    c1, c2 = 3.7, 0.01
    a = rng.uniform(0, 1, (rows, cols))
    g = c2 * (c1 * np.outer(p, q))
    for red, every, mi in ((O.RED_L2_DELTA, 10, 300), (O.RED_MAX_ABS_DELTA, 1, 77)):
        o1, r1 = O.jacobi_run(a, helmholtz=True, g=g, alpha=2.0, h=0.1, reduce_op=red,
                              thr=1e-12, check_every=every, max_iter=mi)
        o2, r2 = O.jacobi_sep_run(a, p, q, c1, c2, alpha=2.0, h=0.1, reduce_op=red, thr=1e-12,
                                  check_every=every, max_iter=mi)
        assert np.array_equal(o1, o2) and r1.n == r2.n and r1.r == r2.r
    # the factors' roles are not interchangeable
    o3, _ = O.jacobi_sep_run(a, np.resize(q, rows), np.resize(p, cols), c1, c2, alpha=2.0, h=0.1,
                             max_iter=20)
    assert not np.array_equal(o3, O.jacobi_run(a, helmholtz=True, g=g, alpha=2.0, h=0.1,
                                               reduce_op=O.RED_L2_DELTA, max_iter=20)[0])


def test_sep_manufactured_solve_follows_the_closed_form():
    n, alpha, sweeps = 65, 1.0, 3000
    hin = I.helmholtz_input(n, alpha)
    s, h = I.helmholtz_factor(n)
    o, r = O.jacobi_sep_run(hin.u0, s, s, 2 * math.pi ** 2 + alpha, h * h, alpha=alpha, h=h,
                            thr=0.0, max_iter=sweeps)
    o_env, _ = O.jacobi_run(hin.u0, helmholtz=True, g=hin.g, alpha=alpha, h=h,
                            reduce_op=O.RED_L2_DELTA, thr=0.0, check_every=10, max_iter=sweeps)
    assert np.array_equal(o, o_env)
    s2 = math.sin(math.pi * h / 2) ** 2
    one_m_mu = (8 * s2 + alpha * h * h) / (4 + alpha * h * h)
    cstar = (2 * math.pi ** 2 + alpha) / (8 / (h * h) * s2 + alpha)
    coef = cstar * -math.expm1(sweeps * math.log1p(-one_m_mu))
    ref = coef * hin.ustar
    assert np.max(np.abs(o - ref)) / np.max(np.abs(ref)) < 1e-13
