"""GPU parity of the temporally blocked Jacobi path (tb_depth > 1).

A fused launch computes every cell of every sweep from the same operands, in the
same expression order, as the unfused kernel, so the FP64 field must equal the
oracle bit for bit and the FP32 field must equal the unfused FP32 field bit for
bit (same stochastic-rounding keys). Stop sweeps are exact; the reduce value
matches to 1e-12 relative (only the partial-sum grouping differs).
"""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import closed_form_helmholtz, run_jacobi, say

pytestmark = pytest.mark.gpu


def _tuned(ctx, fn, **tune):
    ctx.tune(**tune)
    try:
        return fn()
    finally:
        ctx.tune()


@pytest.mark.parametrize("depth", [2, 4, 5, 8, 10])
@pytest.mark.parametrize("shape", [(3, 4), (8, 8), (130, 1030), (257, 260), (70, 250)])
def test_laplace_f64_fused_matches_oracle(ctx, depth, shape):
    say(f"tb laplace f64 depth={depth} shape={shape}")
    a = I.laplace_input(*shape, seed=11)
    ce, mi, thr = 40, 400, 2e-4
    o, ro = O.jacobi_run(a, thr=thr, check_every=ce, max_iter=mi)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, a, thr=thr, check_every=ce, max_iter=mi),
                  tb_depth=depth)
    assert r.iterations == ro.n and bool(r.converged) == ro.converged
    assert np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * abs(ro.r)


@pytest.mark.parametrize("depth", [2, 4, 5, 8, 10])
@pytest.mark.parametrize("tile_rows,waves", [(0, 0), (8, 1), (17, 2), (64, 4), (5, 1), (100, 2)])
def test_helmholtz_f64_fused_matches_oracle(ctx, depth, tile_rows, waves):
    say(f"tb helmholtz f64 depth={depth} tiles={tile_rows} waves={waves}")
    h = I.helmholtz_input(300)
    o, ro = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=1.0, h=h.h,
                         reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=40, max_iter=160)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, h.u0, helm=True, g=h.g, alpha=1.0, h=h.h,
                                          reduce_op=L.LSR_RED_L2_DELTA, thr=1e-9, check_every=40,
                                          max_iter=160),
                  tb_depth=depth, tile_rows=tile_rows, waves=waves)
    assert r.iterations == 160 and np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r


@pytest.mark.parametrize("depth", [2, 4])
@pytest.mark.parametrize("chunk,graph", [(0, 0), (8, -1), (40, 1)])
def test_fused_chunking_and_graphs(ctx, depth, chunk, graph):
    say(f"tb chunk={chunk} graph={graph} depth={depth}")
    a = I.laplace_input(200, 264, seed=12)
    o, ro = O.jacobi_run(a, thr=1e-4, check_every=4, max_iter=1000)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, a, thr=1e-4, check_every=4, max_iter=1000),
                  tb_depth=depth, chunk=chunk, use_graph=graph)
    assert r.iterations == ro.n and r.converged == ro.converged and np.array_equal(x, o)


@pytest.mark.parametrize("depth,view", [(4, {}), (5, dict(pitch=1031, offset=1)), (3, {})])
def test_other_depths_and_views(ctx, depth, view):
    """A depth that does not divide check_every (checks inside launches), an
    unaligned view (staged) and a depth that is not compiled (unfused) all give
    the oracle's result."""
    say(f"tb depth={depth} view={view}")
    a = I.laplace_input(70, 1030, seed=6)
    o, ro = O.jacobi_run(a, thr=1e-6, check_every=10, max_iter=150)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, a, thr=1e-6, check_every=10, max_iter=150, **view),
                  tb_depth=depth)
    assert r.iterations == ro.n and np.array_equal(x, o)


@pytest.mark.parametrize("depth", [10, 5, 4, 2])
@pytest.mark.parametrize("ce", [1, 3])
@pytest.mark.parametrize("thr", [3e-3, 2.44e-3, 1.98e-3])
def test_checks_inside_launches_stop_exactly(ctx, depth, ce, thr):
    """check_every smaller than (or not a multiple of) the depth: every check inside a
    launch is evaluated, and a stop inside a launch is replayed to the exact sweep
    (with check_every 1 these thresholds stop at sweeps 81, 97 and 117)."""
    say(f"tb multi-check depth={depth} ce={ce} thr={thr}")
    a = I.laplace_input(96, 100, seed=21)
    o, ro = O.jacobi_run(a, thr=thr, check_every=ce, max_iter=3000)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, a, thr=thr, check_every=ce, max_iter=3000),
                  tb_depth=depth)
    assert r.sweeps_per_launch == depth
    assert ro.converged and r.iterations == ro.n and bool(r.converged)
    assert np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r and r.checks == ro.n // ce


@pytest.mark.parametrize("depth", [10, 4])
def test_harmonic_start_stops_after_one_sweep_when_fused(ctx, depth):
    say(f"tb harmonic depth={depth}")
    a = I.harmonic_input(64, 66, "xy")
    o, ro = O.jacobi_run(a, thr=1e-9, max_iter=500)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, a, thr=1e-9, max_iter=500), tb_depth=depth)
    assert ro.n == 1 and r.iterations == 1 and r.converged and np.array_equal(x, o)


@pytest.mark.parametrize("cap", [123, 7, 1])
def test_cap_inside_a_launch(ctx, cap):
    say(f"tb cap {cap}")
    h = I.helmholtz_input(130)
    o, ro = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=1.0, h=h.h, reduce_op=O.RED_L2_DELTA,
                         thr=1e-12, check_every=10, max_iter=cap)
    x, r = _tuned(ctx, lambda: run_jacobi(ctx, h.u0, helm=True, g=h.g, alpha=1.0, h=h.h,
                                          reduce_op=L.LSR_RED_L2_DELTA, thr=1e-12, check_every=10,
                                          max_iter=cap), tb_depth=10)
    assert r.iterations == cap and np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r


@pytest.mark.parametrize("helm", [False, True])
def test_f32_multi_check_equals_unfused(ctx, helm):
    say(f"tb f32 multi-check helm={helm}")
    if helm:
        h = I.helmholtz_input(132)
        a, g, alpha, hh = h.u0, h.g, h.alpha, h.h
    else:
        a, g, alpha, hh = I.laplace_input(100, 132, seed=2), None, 0.0, 1.0
    kw = dict(helm=helm, g=g, alpha=alpha, h=hh, f32=True, reduce_op=L.LSR_RED_MAX_ABS_DELTA,
              thr=1e-4, check_every=1, max_iter=777)
    x1, r1 = _tuned(ctx, lambda: run_jacobi(ctx, a, **kw), tb_depth=1)
    xk, rk = _tuned(ctx, lambda: run_jacobi(ctx, a, **kw), tb_depth=0)
    assert rk.sweeps_per_launch > 1
    assert rk.iterations == r1.iterations and np.array_equal(xk, x1)
    assert rk.last_reduce == r1.last_reduce   # max is exact


@pytest.mark.parametrize("helm", [False, True])
@pytest.mark.parametrize("depth", [2, 5, 10])
def test_f32_fused_equals_unfused(ctx, helm, depth):
    say(f"tb f32 helm={helm} depth={depth}")
    if helm:
        h = I.helmholtz_input(260)
        a, g, alpha, hh = h.u0, h.g, h.alpha, h.h
    else:
        a, g, alpha, hh = I.laplace_input(256, 260, seed=1), None, 0.0, 1.0
    kw = dict(helm=helm, g=g, alpha=alpha, h=hh, f32=True, reduce_op=L.LSR_RED_L2_DELTA,
              thr=1e-9, check_every=10, max_iter=500)
    x1, r1 = _tuned(ctx, lambda: run_jacobi(ctx, a, **kw), tb_depth=1)
    xk, rk = _tuned(ctx, lambda: run_jacobi(ctx, a, **kw), tb_depth=depth)
    assert rk.iterations == r1.iterations and np.array_equal(xk, x1)
    assert abs(rk.last_reduce - r1.last_reduce) <= 1e-12 * abs(r1.last_reduce)


@pytest.mark.parametrize("depth", [2, 5, 10])
def test_helmholtz_8192_fused_closed_form(ctx, depth):
    """The benchmarked workload (8192^2 FP64, L2 every 10 sweeps, cap 5000) fused."""
    import torch
    say(f"tb helmholtz f64 8192^2 depth={depth}")
    n, sweeps = 8192, 5000
    h = I.helmholtz_input(n)
    t = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    g = torch.from_numpy(h.g).to("cuda:0")
    r = _tuned(ctx, lambda: ctx.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                                    L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), sweeps,
                                    L.LSR_BC_RING, env0=g, param=(1.0, h.h)),
               tb_depth=depth)
    assert r.status == L.LSR_OK and r.iterations == sweeps and r.checks == sweeps // 10
    coef, dn = closed_form_helmholtz(n, 1.0, sweeps)
    us = torch.from_numpy(h.ustar).to("cuda:0")
    err = float((t - coef * us).abs().max() / (coef * us).abs().max())
    say(f"  rel err {err:.3e}")
    assert err < 1e-11, err
    assert abs(r.last_reduce - dn) / dn < 1e-8
    assert float(t[0].abs().max()) == 0.0 and float(t[:, -1].abs().max()) == 0.0
