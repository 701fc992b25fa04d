"""GPU test of lsr_run_noalloc, the entry point that allocates nothing: through
the C ABI, its fields, iteration counts and reduce values equal lsr_run's (the
same kernels on the same inputs) on consecutive calls whose second input is
smaller than the first, and FP64 / Life results equal the oracle. Sizes beyond
the fixed scratch and grids that would need staged copies are rejected."""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _both(ctx, make, run_kw):
    """(lsr_run field, result), (lsr_run_noalloc field, result) on equal inputs."""
    import torch
    out = []
    for mode in ("run", "noalloc"):
        t, env = make()
        kw = dict(run_kw)
        if mode == "run":
            r = ctx.run(t, env0=env, **kw)
        else:
            r = ctx.run_noalloc(t, env0=env, **kw)
        torch.cuda.synchronize()
        out.append((t.cpu().numpy(), r))
    return out


def _same(a, b):
    (xa, ra), (xb, rb) = a, b
    assert np.array_equal(xa, xb)
    assert ra.status == rb.status == L.LSR_OK
    assert ra.iterations == rb.iterations and ra.last_reduce == rb.last_reduce
    assert ra.last_count == rb.last_count and ra.converged == rb.converged
    assert ra.sweeps_per_launch == rb.sweeps_per_launch


def _helm(n, f32):
    import torch
    h = I.helmholtz_input(n)
    dt = torch.float32 if f32 else torch.float64

    def make():
        return (torch.from_numpy(h.u0).to("cuda:0", dt), torch.from_numpy(h.g).to("cuda:0", dt))
    kw = dict(stencil_id=L.LSR_ST_HELMHOLTZ5, reduce_op=L.LSR_RED_L2_DELTA,
              cond=L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), max_iter=437, bc=L.LSR_BC_RING,
              param=(h.alpha, h.h))
    return h, make, kw


def test_helmholtz_noalloc_equals_run_then_smaller(ctx):
    for n, f32 in ((1500, False), (514, False), (1024, True), (300, True)):
        say(f"noalloc helmholtz n={n} f32={f32}")
        h, make, kw = _helm(n, f32)
        a, b = _both(ctx, make, kw)
        _same(a, b)
        if not f32:
            o, ro = O.jacobi_run(h.u0, helmholtz=True, g=h.g, alpha=h.alpha, h=h.h,
                                 reduce_op=O.RED_L2_DELTA, thr=1e-9, check_every=10, max_iter=437)
            assert np.array_equal(b[0], o) and b[1].iterations == ro.n


def test_laplace_stop_inside_fused_launch_then_smaller(ctx):
    import torch
    # checks every sweep inside fused launches; the 333-sweep cap is not a
    # multiple of the depth, so the stop is replayed inside a launch
    for n in (700, 130):
        say(f"noalloc laplace n={n}")
        a0 = I.laplace_input(n, seed=n)
        kw = dict(stencil_id=L.LSR_ST_LAPLACE5, reduce_op=L.LSR_RED_MAX_ABS_DELTA,
                  cond=L.make_cond(L.LSR_COND_BELOW, 1e-6, 1), max_iter=333, bc=L.LSR_BC_RING)
        a, b = _both(ctx, lambda: (torch.from_numpy(a0).to("cuda:0"), None), kw)
        _same(a, b)
        o, ro = O.jacobi_run(a0, thr=1e-6, max_iter=333)
        assert np.array_equal(b[0], o) and b[1].iterations == ro.n == 333
    # a harmonic field stops at the first check
    hx = I.harmonic_input(96, 96, "x2-y2")
    kw["max_iter"] = 50
    a, b = _both(ctx, lambda: (torch.from_numpy(hx).to("cuda:0"), None), kw)
    _same(a, b)
    assert b[1].iterations == 1 and b[1].converged


def test_life_noalloc_equals_run_then_smaller(ctx):
    import torch
    for n, bc in ((1024, L.LSR_BC_TORUS), (256, L.LSR_BC_BOTTOM), (64, L.LSR_BC_TORUS)):
        say(f"noalloc life n={n} bc={bc}")
        s0 = I.life_input(n, seed=n)
        kw = dict(stencil_id=L.LSR_ST_LIFE, reduce_op=L.LSR_RED_SUM,
                  cond=L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10), max_iter=301, bc=bc)
        a, b = _both(ctx, lambda: (torch.from_numpy(s0).to("cuda:0"), None), kw)
        _same(a, b)
        o, ro = O.life_run(s0, bc=O.BC_TORUS if bc == L.LSR_BC_TORUS else O.BC_BOTTOM,
                           stable_window=10, max_iter=301)
        assert np.array_equal(b[0], o) and b[1].iterations == ro.n


def test_restore_noalloc_equals_run(ctx):
    import torch
    for n in (192, 80):
        say(f"noalloc restore n={n}")
        rin = I.restore_input(n, seed=4)
        m_o, u_o = O.amf_detect(rin.y, 19)
        kw = dict(stencil_id=L.LSR_ST_RESTORE, reduce_op=L.LSR_RED_MAX_ABS_DELTA,
                  cond=L.make_cond(L.LSR_COND_BELOW, 0.1, 1), max_iter=200, bc=L.LSR_BC_BOTTOM,
                  param=(100.0, 0.0))
        make = lambda: (torch.from_numpy(u_o.astype(np.float64)).to("cuda:0"),
                        torch.from_numpy(m_o).to("cuda:0"))
        a, b = _both(ctx, make, kw)
        _same(a, b)


def test_largest_grid_then_limits(ctx):
    import torch
    say("noalloc at the scratch limit")
    # a 4096 x 4096 FP32 partner (64 MiB) fits the 65 MiB scratch
    n = 4096
    h = I.helmholtz_input(n)
    kw = dict(stencil_id=L.LSR_ST_HELMHOLTZ5, reduce_op=L.LSR_RED_L2_DELTA,
              cond=L.make_cond(L.LSR_COND_BELOW, 1e-9, 10), max_iter=40, bc=L.LSR_BC_RING,
              param=(h.alpha, h.h))
    g = torch.from_numpy(h.g).to("cuda:0", torch.float32)
    a, b = _both(ctx, lambda: (torch.zeros((n, n), dtype=torch.float32, device="cuda:0"), g), kw)
    _same(a, b)
    # one row group more than the scratch holds
    big = torch.zeros((4096, 4200), dtype=torch.float32, device="cuda:0")
    gb = torch.zeros_like(big)
    with pytest.raises(L.LsrError) as ei:
        ctx.run_noalloc(big, env0=gb, **kw)
    assert ei.value.status == L.LSR_EINVAL and "scratch" in str(ei.value)
    # a Life grid whose rows are not a multiple of 16 cells would need staging
    s = torch.zeros((40, 100), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(L.LsrError) as ei:
        ctx.run_noalloc(s, L.LSR_ST_LIFE, L.LSR_RED_SUM,
                        L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10), 10, L.LSR_BC_TORUS)
    assert ei.value.status == L.LSR_EINVAL
    # after the rejected calls a small job still matches lsr_run
    _, make, kw2 = _helm(200, True)
    a, b = _both(ctx, make, kw2)
    _same(a, b)
