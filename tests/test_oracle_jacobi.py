"""Pins for the oracle's 5-point Jacobi (Laplace and Helmholtz) loop.

Each pin is fixed by something other than the oracle: discrete harmonic
polynomials (exact fixed points), the discrete maximum principle and
monotonicity of the Jacobi operator, a matrix formulation of the same linear
map, the direct solve of the 5-point system, and the closed-form trajectory of
the manufactured Helmholtz solution (sin is an eigenvector of the 5-point
operator).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1609_04567_amd import inputs as I


@pytest.mark.parametrize("kind", ["x2-y2", "xy", "x3-3xy2"])
@pytest.mark.parametrize("shape", [(3, 3), (8, 8), (17, 13), (64, 48)])
def test_harmonic_fields_stop_after_one_sweep(kind, shape):
    """Loop form: at least one sweep; the condition sees the update of that sweep."""
    a = I.harmonic_input(*shape, kind)
    b, r = O.jacobi_run(a, thr=1e-6, max_iter=2000)
    assert r.n == 1 and r.r == 0.0 and r.converged and r.checks == 1
    assert np.array_equal(b, a)


def test_laplace_c1_recipe_hits_cap_and_obeys_max_principle():
    a = I.laplace_input(256, seed=1)
    b, r = O.jacobi_run(a, thr=1e-6, max_iter=2000, trace_cap=2000)
    assert r.n == 2000 and not r.converged and r.checks == 2000
    assert 5e-5 < r.r < 2e-4
    lo, hi = a[[0, -1], :].min(), a.max()
    assert b.min() >= 0.0 and b.max() <= hi and b.max() < 1.0 and lo >= 0.0
    assert np.array_equal(b[0], a[0]) and np.array_equal(b[:, -1], a[:, -1])
    # the residual decays (not necessarily monotonically, but overall)
    assert r.trace[-1] < r.trace[10]


def test_laplace_monotone_from_zero_interior():
    """Nonnegative boundary, zero start, monotone operator: u^{n+1} >= u^n pointwise."""
    a = I.laplace_input(40, 33, seed=11)
    prev = a
    for _ in range(25):
        nxt, r = O.jacobi_run(prev, thr=-1.0, max_iter=1)
        assert r.n == 1
        assert np.all(nxt >= prev)
        prev = nxt


def test_laplace_transpose_symmetry_bit_exact():
    a = I.laplace_input(31, 23, seed=5)
    b, _ = O.jacobi_run(a, thr=1e-6, max_iter=300)
    bt, _ = O.jacobi_run(np.ascontiguousarray(a.T), thr=1e-6, max_iter=300)
    assert np.array_equal(b.T, bt)


def _jacobi_matrix(rows, cols, alpha, h):
    """Dense matrix form x' = M x + c of the 5-point Jacobi map on interior unknowns."""
    idx = -np.ones((rows, cols), dtype=int)
    inner = [(i, j) for i in range(1, rows - 1) for j in range(1, cols - 1)]
    for k, (i, j) in enumerate(inner):
        idx[i, j] = k
    n = len(inner)
    diag = 4.0 + alpha * h * h
    M = np.zeros((n, n))
    B = np.zeros((n, rows * cols))  # contribution of boundary cells
    for k, (i, j) in enumerate(inner):
        for (ii, jj) in ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)):
            if idx[ii, jj] >= 0:
                M[k, idx[ii, jj]] = 1.0 / diag
            else:
                B[k, ii * cols + jj] = 1.0 / diag
    return inner, M, B, diag


@pytest.mark.parametrize("helm", [False, True])
def test_jacobi_matches_matrix_formulation(helm):
    rows, cols = 8, 9
    rng = np.random.default_rng(0)
    a = rng.random((rows, cols))
    alpha, h = (1.0, 1.0 / 7) if helm else (0.0, 1.0)
    g = rng.random((rows, cols)) if helm else None
    inner, M, B, diag = _jacobi_matrix(rows, cols, alpha, h)
    x = np.array([a[i, j] for (i, j) in inner])
    c = B @ a.reshape(-1)
    if helm:
        c = c + np.array([g[i, j] for (i, j) in inner]) / diag
    for _ in range(7):
        x = M @ x + c
    b, r = O.jacobi_run(a, helmholtz=helm, g=g, alpha=alpha, h=h, thr=-1.0, max_iter=7)
    assert r.n == 7
    got = np.array([b[i, j] for (i, j) in inner])
    assert np.max(np.abs(got - x)) <= 1e-14 * np.max(np.abs(x))


def test_helmholtz_converges_to_direct_solve():
    n = 9
    rng = np.random.default_rng(1)
    alpha, h = 1.0, 1.0 / (n - 1)
    f = rng.random((n, n))
    g = h * h * f
    a = np.zeros((n, n))
    a[0] = rng.random(n)
    a[:, -1] = rng.random(n)
    inner, M, B, diag = _jacobi_matrix(n, n, alpha, h)
    A = np.eye(len(inner)) - M
    rhs = B @ a.reshape(-1) + np.array([g[i, j] for (i, j) in inner]) / diag
    xs = np.linalg.solve(A, rhs)
    b, r = O.jacobi_run(a, helmholtz=True, g=g, alpha=alpha, h=h,
                        reduce_op=O.RED_L2_DELTA, thr=1e-15, max_iter=100000)
    assert r.converged
    got = np.array([b[i, j] for (i, j) in inner])
    assert np.max(np.abs(got - xs)) < 1e-13 * np.max(np.abs(xs)) * 100


def _closed_form(n, alpha, sweeps):
    """u^k = c*(1-mu^k) u*, ||Delta^k||_2 = c*(1-mu) mu^(k-1) (N-1)/2, with 1 - mu
    written without cancellation: (8 sin^2(pi h/2) + alpha h^2) / (4 + alpha h^2)."""
    h = 1.0 / (n - 1)
    s2 = math.sin(math.pi * h / 2) ** 2
    one_m_mu = (8.0 * s2 + alpha * h * h) / (4.0 + alpha * h * h)
    mu = 1.0 - one_m_mu
    lam = 8.0 / (h * h) * s2
    cstar = (2 * math.pi ** 2 + alpha) / (lam + alpha)
    lmu = math.log1p(-one_m_mu)
    coef = cstar * -math.expm1(sweeps * lmu)
    dnorm = cstar * one_m_mu * math.exp((sweeps - 1) * lmu) * (n - 1) / 2.0
    return coef, dnorm, mu, cstar


def test_closed_form_agrees_with_the_naive_expression_where_it_is_well_conditioned():
    n, alpha, k = 33, 1.0, 40
    h = 1.0 / (n - 1)
    mu = 4.0 * math.cos(math.pi * h) / (4.0 + alpha * h * h)
    lam = 8.0 / (h * h) * math.sin(math.pi * h / 2) ** 2
    cstar = (2 * math.pi ** 2 + alpha) / (lam + alpha)
    coef, dnorm, mu2, _ = _closed_form(n, alpha, k)
    assert abs(mu2 - mu) < 1e-15
    assert abs(coef - cstar * (1 - mu ** k)) / coef < 1e-12


@pytest.mark.parametrize("n,sweeps", [(65, 3000), (257, 1500)])
def test_helmholtz_closed_form_trajectory(n, sweeps):
    hin = I.helmholtz_input(n, alpha=1.0)
    b, r = O.jacobi_run(hin.u0, helmholtz=True, g=hin.g, alpha=hin.alpha, h=hin.h,
                        reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=sweeps,
                        trace_cap=sweeps // 10 + 1)
    coef, dnorm, _, _ = _closed_form(n, 1.0, sweeps)
    assert r.n == sweeps and not r.converged and r.checks == sweeps // 10
    err = np.max(np.abs(b - coef * hin.ustar)) / np.max(np.abs(coef * hin.ustar))
    assert err < 1e-12
    for k, rk in enumerate(r.trace):
        nk = 10 * (k + 1)
        _, dk, _, _ = _closed_form(n, 1.0, nk)
        assert abs(rk - dk) / dk < 1e-9, (nk, rk, dk)


def test_helmholtz_8192_closed_form_constants():
    """The full-size run is pinned by the closed form alone: it cannot stop before the cap."""
    coef, dnorm, mu, cstar = _closed_form(8192, 1.0, 5000)
    h = 1.0 / 8191
    one_m_mu = (8.0 * math.sin(math.pi * h / 2) ** 2 + h * h) / (4.0 + h * h)
    assert abs(one_m_mu - 7.727844e-8) / 7.727844e-8 < 1e-5
    assert dnorm > 1e-9 * 1e5  # ||Delta^5000|| ~ 3.16e-4, far above the threshold
    assert abs(dnorm - 3.1637e-4) / 3.1637e-4 < 1e-3
    assert abs(coef - 3.8632e-4) / 3.8632e-4 < 1e-3


def test_helmholtz_discrete_rhs_reading_has_unit_fixed_point():
    """With f = (lambda_h + alpha) u*, the discrete fixed point is u* itself."""
    n, alpha = 33, 1.0
    hin = I.helmholtz_input(n, alpha)
    h = hin.h
    lam = 8.0 / (h * h) * math.sin(math.pi * h / 2) ** 2
    g = (h * h) * (lam + alpha) * hin.ustar
    b, r = O.jacobi_run(hin.u0, helmholtz=True, g=g, alpha=alpha, h=h,
                        reduce_op=O.RED_L2_DELTA, thr=1e-14, max_iter=200000)
    assert r.converged
    assert np.max(np.abs(b - hin.ustar)) < 1e-11


def test_check_every_and_cap_semantics():
    a = I.laplace_input(20, seed=2)
    _, r = O.jacobi_run(a, thr=-1.0, check_every=10, max_iter=25, trace_cap=10)
    assert r.n == 25 and r.checks == 3          # checks at 10, 20 and the cap 25
    # the value checked at n = 10 is the update of sweep 10, not u^10 - u^0
    a9, _ = O.jacobi_run(a, thr=-1.0, max_iter=9)
    a10, _ = O.jacobi_run(a, thr=-1.0, max_iter=10)
    assert r.trace[0] == np.max(np.abs(a10 - a9))


def test_mean_and_l2_reduces():
    a = I.laplace_input(12, 10, seed=9)
    b1, _ = O.jacobi_run(a, thr=-1.0, max_iter=1)
    _, rm = O.jacobi_run(a, thr=-1.0, max_iter=1, reduce_op=O.RED_MEAN_ABS_DELTA)
    _, rl = O.jacobi_run(a, thr=-1.0, max_iter=1, reduce_op=O.RED_L2_DELTA)
    d = b1 - a
    assert abs(rm.r - np.abs(d).sum() / d.size) <= 1e-15 * np.abs(d).sum()
    assert abs(rl.r - math.sqrt((d * d).sum())) <= 1e-15 * math.sqrt((d * d).sum())


def test_nan_stops_with_numeric_error():
    a = I.laplace_input(16, seed=3)
    a[5, 5] = np.nan
    _, r = O.jacobi_run(a, thr=1e-6, max_iter=100, check_every=4)
    assert r.numeric_error and r.n == 4 and math.isnan(r.r) and not r.converged


def test_never_condition_runs_to_cap():
    a = I.harmonic_input(10, 10, "xy")
    _, r = O.jacobi_run(a, cond=O.COND_NEVER, max_iter=7, check_every=3)
    assert r.n == 7 and r.checks == 3 and not r.converged


def test_thread_count_does_not_change_results():
    hin = I.helmholtz_input(129)
    O.set_threads(1)
    b1, r1 = O.jacobi_run(hin.u0, helmholtz=True, g=hin.g, alpha=1.0, h=hin.h,
                          reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=200)
    O.set_threads(4)
    b4, r4 = O.jacobi_run(hin.u0, helmholtz=True, g=hin.g, alpha=1.0, h=hin.h,
                          reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=200)
    O.set_threads(0)
    assert np.array_equal(b1, b4) and r1.r == r4.r
