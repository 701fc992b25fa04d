"""GPU parity: 5-point Jacobi (Laplace / Helmholtz) through the C ABI against the oracle.

FP64: the field must match the oracle to 1e-12 relative (the kernels evaluate the
oracle's expression order without contraction, so it is in fact bit-identical and
that is asserted too); the reduce value to 1e-12 relative (only the summation
order differs); sweep counts exactly. FP32 storage: 1e-5 relative to the FP64
oracle, counts equal.
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import closed_form_helmholtz, rel_err, run_jacobi, say

pytestmark = pytest.mark.gpu

SHAPES = [(3, 3), (8, 8), (17, 13), (129, 257), (300, 1030)]


@pytest.mark.parametrize("shape", SHAPES)
def test_laplace_f64_matches_oracle(ctx, shape):
    say(f"laplace f64 {shape}")
    a = I.laplace_input(*shape, seed=1)
    o, ro = O.jacobi_run(a, thr=1e-6, max_iter=400)
    x, r = run_jacobi(ctx, a, thr=1e-6, max_iter=400)
    assert r.status == L.LSR_OK
    assert r.iterations == ro.n and bool(r.converged) == ro.converged and r.checks == ro.checks
    assert rel_err(x, o) <= 1e-12
    assert np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * max(abs(ro.r), 1e-300)


def test_laplace_c1_full_run(ctx):
    say("laplace f64 256x256 C1 full run")
    a = I.laplace_input(256, seed=1)
    o, ro = O.jacobi_run(a, thr=1e-6, max_iter=2000)
    x, r = run_jacobi(ctx, a, thr=1e-6, max_iter=2000)
    assert r.iterations == ro.n == 2000 and not r.converged
    assert np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r


@pytest.mark.parametrize("kind", ["x2-y2", "xy", "x3-3xy2"])
def test_harmonic_fields_stop_after_one_sweep(ctx, kind):
    say(f"harmonic {kind}")
    a = I.harmonic_input(64, 80, kind)
    x, r = run_jacobi(ctx, a, thr=1e-6, max_iter=2000)
    assert r.iterations == 1 and r.converged and r.last_reduce == 0.0 and r.checks == 1
    assert np.array_equal(x, a)


@pytest.mark.parametrize("red", [L.LSR_RED_L2_DELTA, L.LSR_RED_MEAN_ABS_DELTA])
def test_other_reduces(ctx, red):
    say(f"laplace reduce {red}")
    a = I.laplace_input(97, 130, seed=4)
    ored = {L.LSR_RED_L2_DELTA: O.RED_L2_DELTA, L.LSR_RED_MEAN_ABS_DELTA: O.RED_MEAN_ABS_DELTA}[red]
    o, ro = O.jacobi_run(a, reduce_op=ored, thr=1e-3, check_every=3, max_iter=500)
    x, r = run_jacobi(ctx, a, reduce_op=red, thr=1e-3, check_every=3, max_iter=500)
    assert r.iterations == ro.n and bool(r.converged) == ro.converged
    assert np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r


@pytest.mark.parametrize("n,sweeps", [(65, 1500), (257, 1000), (1030, 200)])
def test_helmholtz_f64_matches_oracle(ctx, n, sweeps):
    say(f"helmholtz f64 N={n} sweeps={sweeps}")
    h = I.helmholtz_input(n)
    o, ro = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                         reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=sweeps)
    x, r = run_jacobi(ctx, h.u0, helm=True, g=h.g, alpha=h.alpha, h=h.h,
                      reduce_op=L.LSR_RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=sweeps)
    assert r.iterations == ro.n == sweeps and r.checks == ro.checks
    assert np.array_equal(x, o)
    assert abs(r.last_reduce - ro.r) <= 1e-12 * ro.r
    # the closed form holds up to the rounding of the lattice sines (the discrete
    # eigen-relation is exact only in real arithmetic), ~1e-12 after few sweeps
    coef, dn = closed_form_helmholtz(n, 1.0, sweeps)
    assert rel_err(x, coef * h.ustar) < 1e-11
    assert abs(r.last_reduce - dn) / dn < 1e-9


def test_helmholtz_8192_full_run_closed_form(ctx):
    """The benchmarked workload at full size: 8192^2 FP64, L2 every 10 sweeps, cap 5000."""
    import torch
    say("helmholtz f64 8192^2 5000 sweeps (closed form)")
    n, sweeps = 8192, 5000
    h = I.helmholtz_input(n)
    t = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    g = torch.from_numpy(h.g).to("cuda:0")
    r = ctx.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
                L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), sweeps, L.LSR_BC_RING, env0=g,
                param=(1.0, h.h))
    assert r.status == L.LSR_OK and r.iterations == sweeps and not r.converged
    assert r.checks == sweeps // 10
    coef, dn = closed_form_helmholtz(n, 1.0, sweeps)
    us = torch.from_numpy(h.ustar).to("cuda:0")
    err = float((t - coef * us).abs().max() / (coef * us).abs().max())
    assert err < 1e-11, err
    assert abs(r.last_reduce - dn) / dn < 1e-8
    # sampled rows against the oracle's own sweep is impossible at this size; the
    # closed form holds at every cell, and the ring stays exactly zero
    assert float(t[0].abs().max()) == 0.0 and float(t[:, -1].abs().max()) == 0.0


@pytest.mark.parametrize("helm", [False, True])
def test_f32_storage_within_1e5_of_f64_oracle(ctx, helm):
    say(f"f32 storage helm={helm}")
    if helm:
        h = I.helmholtz_input(257)
        a, g, kw = h.u0, h.g, dict(helmholtz=True, alpha=h.alpha, h=h.h)
        red, ored, thr, ce, mi = L.LSR_RED_L2_DELTA, O.RED_L2_DELTA, 1e-9, 10, 1000
    else:
        a, g, kw = I.laplace_input(256, seed=1), None, {}
        red, ored, thr, ce, mi = L.LSR_RED_MAX_ABS_DELTA, O.RED_MAX_ABS_DELTA, 1e-6, 1, 2000
    o, ro = O.jacobi_run(a, g=g, reduce_op=ored, thr=thr, check_every=ce, max_iter=mi, **kw)
    x, r = run_jacobi(ctx, a, helm=helm, g=g, alpha=kw.get("alpha", 0.0), h=kw.get("h", 1.0),
                      f32=True, reduce_op=red, thr=thr, check_every=ce, max_iter=mi)
    assert r.iterations == ro.n
    err = rel_err(x, o)
    say(f"  f32 rel err {err:.3e}")
    assert err <= 1e-5
    # the update is a difference of nearby FP32 values, so r carries FP32 cancellation
    assert abs(r.last_reduce - ro.r) / ro.r < 5e-2


@pytest.mark.parametrize("n,sweeps", [(2049, 5000), (4096, 5000)])
@pytest.mark.parametrize("batched", [False, True])
def test_f32_helmholtz_large_within_1e5(ctx, n, sweeps, batched):
    """The FP32 form at the largest Helmholtz size of the served stream, against the
    closed form (which the FP64 oracle matches to ~1e-13 at every size tested)."""
    import torch
    say(f"f32 helmholtz N={n} sweeps={sweeps} batched={batched}")
    h = I.helmholtz_input(n)
    t = torch.zeros((n, n), dtype=torch.float32, device="cuda:0")
    g = torch.from_numpy(h.g.astype(np.float32)).to("cuda:0")
    c = L.Context(0, batched=True) if batched else ctx
    try:
        r = c.run(t, L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, L.make_cond(L.LSR_COND_BELOW, 1e-9, 10),
                  sweeps, L.LSR_BC_RING, env0=g, param=(h.alpha, h.h))
    finally:
        if batched:
            c.close()
    assert r.status == L.LSR_OK and r.iterations == sweeps
    coef, dn = closed_form_helmholtz(n, 1.0, sweeps)
    us = torch.from_numpy(h.ustar).to("cuda:0")
    err = float((t.double() - coef * us).abs().max() / (coef * us).abs().max())
    say(f"  rel err {err:.3e}")
    assert err <= 1e-5
    assert abs(r.last_reduce - dn) / dn < 5e-2


def test_check_every_and_cap(ctx):
    say("check_every 10, cap 25")
    a = I.laplace_input(40, seed=2)
    o, ro = O.jacobi_run(a, thr=-1.0, check_every=10, max_iter=25)
    x, r = run_jacobi(ctx, a, thr=-1.0, check_every=10, max_iter=25)
    assert r.iterations == 25 and r.checks == 3 and ro.checks == 3
    assert np.array_equal(x, o) and r.last_reduce == ro.r


def test_max_iter_one_and_odd_stop(ctx):
    say("max_iter 1 / odd stop")
    a = I.laplace_input(33, seed=3)
    for mi in (1, 3, 7):
        o, ro = O.jacobi_run(a, thr=-1.0, check_every=4, max_iter=mi)
        x, r = run_jacobi(ctx, a, thr=-1.0, check_every=4, max_iter=mi)
        assert r.iterations == mi and np.array_equal(x, o)


def test_nan_input_stops_with_numeric_status(ctx):
    say("nan input")
    a = I.laplace_input(50, seed=3)
    a[7, 9] = np.nan
    x, r = run_jacobi(ctx, a, thr=1e-6, check_every=4, max_iter=100)
    assert r.status == L.LSR_ENUMERIC and r.iterations == 4 and math.isnan(r.last_reduce)


@pytest.mark.parametrize("pitch,offset", [(1100, 0), (1031, 0), (1031, 1)])
def test_pitched_and_misaligned_views(ctx, pitch, offset):
    say(f"pitched view pitch={pitch} offset={offset}")
    a = I.laplace_input(70, 1029, seed=6)
    o, ro = O.jacobi_run(a, thr=1e-6, max_iter=150)
    x, r = run_jacobi(ctx, a, thr=1e-6, max_iter=150, pitch=pitch, offset=offset)
    assert r.iterations == ro.n and np.array_equal(x, o)


@pytest.mark.parametrize("tile_rows,chunk,graph", [(8, 0, 0), (64, 2, -1), (17, 6, 1), (256, 40, 0)])
def test_launch_shapes_give_identical_fields(ctx, tile_rows, chunk, graph):
    say(f"tiles {tile_rows} chunk {chunk} graph {graph}")
    h = I.helmholtz_input(300)
    ref, rr = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=1.0, h=h.h,
                           reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=2, max_iter=123)
    ctx.tune(tile_rows=tile_rows, chunk=chunk, use_graph=graph)
    try:
        x, r = run_jacobi(ctx, h.u0, helm=True, g=h.g, alpha=1.0, h=h.h,
                          reduce_op=L.LSR_RED_L2_DELTA, thr=1e-9, check_every=2, max_iter=123)
    finally:
        ctx.tune()
    assert r.iterations == 123 and np.array_equal(x, ref)
    assert abs(r.last_reduce - rr.r) <= 1e-12 * rr.r


def test_repeat_runs_are_bit_identical(ctx):
    say("determinism")
    h = I.helmholtz_input(513)
    outs = [run_jacobi(ctx, h.u0, helm=True, g=h.g, alpha=1.0, h=h.h, reduce_op=L.LSR_RED_L2_DELTA,
                       thr=1e-9, check_every=10, max_iter=200) for _ in range(3)]
    for x, r in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and r.last_reduce == outs[0][1].last_reduce


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("helm", [False, True])
def test_unaligned_rows_run_staged(ctx, f32, helm):
    """Rows that are not 16-byte aligned run on private aligned copies; the result
    lands in the caller's view and nothing around the view is touched."""
    import torch
    say(f"staged f32={f32} helm={helm}")
    if helm:
        h = I.helmholtz_input(129)
        a, g, alpha, hh = h.u0, h.g, h.alpha, h.h
        red, ored, thr, ce, mi = L.LSR_RED_L2_DELTA, O.RED_L2_DELTA, 1e-9, 10, 600
        kw = dict(helmholtz=True, g=g, alpha=alpha, h=hh)
    else:
        a, g = I.laplace_input(131, 129, seed=8), None
        red, ored, thr, ce, mi = L.LSR_RED_MAX_ABS_DELTA, O.RED_MAX_ABS_DELTA, 1e-6, 1, 700
        kw = {}
    o, ro = O.jacobi_run(a, reduce_op=ored, thr=thr, check_every=ce, max_iter=mi, **kw)
    dt = torch.float32 if f32 else torch.float64
    rows, cols = a.shape
    big = torch.full((rows, cols + 3), 7.0, dtype=dt, device="cuda:0")
    view = big[:, 1:1 + cols]
    view.copy_(torch.from_numpy(a).to(dt))
    env = None
    if helm:
        gbig = torch.zeros((rows, cols + 3), dtype=dt, device="cuda:0")
        env = gbig[:, 1:1 + cols]
        env.copy_(torch.from_numpy(g).to(dt))
    st = L.LSR_ST_HELMHOLTZ5 if helm else L.LSR_ST_LAPLACE5
    r = ctx.run(view, st, red, L.make_cond(L.LSR_COND_BELOW, thr, ce), mi, L.LSR_BC_RING,
                env0=env, param=(alpha, hh) if helm else ())
    torch.cuda.synchronize()
    x = view.cpu().numpy().astype(np.float64)
    assert r.status == L.LSR_OK and r.iterations == ro.n
    if f32:
        assert rel_err(x, o) <= 1e-5
    else:
        assert np.array_equal(x, o)
    b = big.cpu().numpy()
    assert (b[:, 0] == 7.0).all() and (b[:, 1 + cols:] == 7.0).all()
