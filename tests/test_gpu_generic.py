"""GPU tests of the generic stencil forms: the radius-k box mean (sigma_k, k = 1..4)
and the 3D 7-point Jacobi. FP64 fields and iteration counts equal the oracle's bit
for bit (same summation order, one IEEE division); FP32 fields are within 1e-5 of
the FP64 oracle; pitched, misaligned and host grids give the same fields."""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from gpu_helpers import rel_err, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_box_matches_oracle(ctx, k):
    import torch
    rng = np.random.default_rng(k)
    for rows, cols, mi, red in ((2 * k + 1, 2 * k + 1, 5, L.LSR_RED_MAX_ABS_DELTA),
                                (37, 70, 60, L.LSR_RED_L2_DELTA), (300, 257, 25, L.LSR_RED_MAX_ABS_DELTA)):
        say(f"box k={k} {rows}x{cols}")
        a = rng.uniform(0, 1, (rows, cols))
        o, ro = O.box_run(a, k, reduce_op=red, thr=1e-9, max_iter=mi)
        for pitch, off in ((None, 0), (cols + 5, 3)):
            t = to_dev(a, pitch, off)
            r = ctx.run(t, L.LSR_ST_BOX, red, L.make_cond(L.LSR_COND_BELOW, 1e-9, 1), mi,
                        L.LSR_BC_RING, param=(float(k),))
            torch.cuda.synchronize()
            assert r.status == L.LSR_OK and r.iterations == ro.n
            assert np.array_equal(t.cpu().numpy(), o)
        t32 = to_dev(a.astype(np.float32))
        r = ctx.run(t32, L.LSR_ST_BOX, red, L.make_cond(L.LSR_COND_BELOW, 1e-9, 1), mi,
                    L.LSR_BC_RING, param=(float(k),))
        torch.cuda.synchronize()
        assert rel_err(t32.cpu().numpy().astype(np.float64), o) <= 1e-5


def test_box_affine_field_stops_at_once(ctx):
    import torch
    i = np.arange(40, dtype=np.float64)[:, None]
    j = np.arange(50, dtype=np.float64)[None, :]
    u = np.ascontiguousarray(3.0 * i - 2.0 * j + 5.0)
    t = to_dev(u)
    r = ctx.run(t, L.LSR_ST_BOX, L.LSR_RED_MAX_ABS_DELTA, L.make_cond(L.LSR_COND_BELOW, 1e-9, 1), 20,
                L.LSR_BC_RING, param=(3.0,))
    torch.cuda.synchronize()
    assert r.iterations == 1 and r.last_reduce == 0.0 and np.array_equal(t.cpu().numpy(), u)


@pytest.mark.parametrize("shape", [(3, 3, 3), (5, 7, 9), (34, 33, 130), (20, 64, 64)])
def test_laplace3d_matches_oracle(ctx, shape):
    import torch
    nz, ny, nx = shape
    say(f"3d {shape}")
    rng = np.random.default_rng(nz)
    a = rng.uniform(0, 1, shape)
    a[1:-1, 1:-1, 1:-1] = 0.0
    for red, every, mi in ((L.LSR_RED_MAX_ABS_DELTA, 1, 40), (L.LSR_RED_L2_DELTA, 7, 50)):
        o, ro = O.jacobi3d_run(a, reduce_op=red, thr=1e-7, check_every=every, max_iter=mi)
        flat = a.reshape(nz * ny, nx)
        for pitch, off in ((None, 0), (nx + 3, 1)):
            t = to_dev(flat, pitch, off)
            r = ctx.run(t, L.LSR_ST_LAPLACE7_3D, red, L.make_cond(L.LSR_COND_BELOW, 1e-7, every), mi,
                        L.LSR_BC_RING, param=(float(ny),))
            torch.cuda.synchronize()
            assert r.status == L.LSR_OK and r.iterations == ro.n
            assert np.array_equal(t.cpu().numpy().reshape(shape), o)
        t32 = to_dev(flat.astype(np.float32))
        r = ctx.run(t32, L.LSR_ST_LAPLACE7_3D, red, L.make_cond(L.LSR_COND_BELOW, 1e-7, every), mi,
                    L.LSR_BC_RING, param=(float(ny),))
        torch.cuda.synchronize()
        assert rel_err(t32.cpu().numpy().astype(np.float64).reshape(shape), o) <= 1e-5


def test_laplace3d_harmonic_and_host(ctx):
    import torch
    nz, ny, nx = 9, 10, 11
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    u = np.ascontiguousarray(x * y * z).reshape(nz * ny, nx)
    t = to_dev(u)
    r = ctx.run(t, L.LSR_ST_LAPLACE7_3D, L.LSR_RED_MAX_ABS_DELTA,
                L.make_cond(L.LSR_COND_BELOW, 1e-9, 1), 10, L.LSR_BC_RING, param=(float(ny),))
    torch.cuda.synchronize()
    assert r.iterations == 1 and r.last_reduce == 0.0 and np.array_equal(t.cpu().numpy(), u)
    # a host grid through lsr_run_host
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 1, (nz * ny, nx))
    o, ro = O.jacobi3d_run(a.reshape(nz, ny, nx), max_iter=30, thr=1e-7)
    h = torch.from_numpy(a.copy())
    r = ctx.result(ctx.submit_host(h, L.LSR_ST_LAPLACE7_3D, L.LSR_RED_MAX_ABS_DELTA,
                                   L.make_cond(L.LSR_COND_BELOW, 1e-7, 1), 30, L.LSR_BC_RING,
                                   param=(float(ny),)))
    assert r.iterations == ro.n and np.array_equal(h.numpy().reshape(nz, ny, nx), o)
