"""GPU tests of the Sobel edge detector (Sect. 4.2's single-iteration stencil):
every output pixel and the reduce (the sum of the new image) are bit-exact against
the oracle, on plain and batched contexts, for device and host images of odd
shapes, pitched and misaligned views, and several sweeps."""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (3, 7), (5, 300), (31, 257), (257, 513), (1000, 1000), (64, 4096)]


def _img(rows, cols, seed):
    # a smooth image with impulses: strong and weak edges, clamped magnitudes
    return I.restore_input(rows, cols, seed=seed, noise=0.2).y


def _cond():
    return L.make_cond(L.LSR_COND_NEVER, 0.0, 1, 1)


@pytest.mark.parametrize("shape", SHAPES)
def test_plain_sobel_matches_oracle(ctx, shape):
    import torch
    rows, cols = shape
    say(f"sobel plain {shape}")
    a = _img(rows, cols, rows + cols)
    o, ro = O.sobel_run(a, max_iter=1)
    for pitch, off in ((None, 0), (cols + 13, 3)):
        t = to_dev(a, pitch, off)
        r = ctx.run(t, L.LSR_ST_SOBEL, L.LSR_RED_SUM, _cond(), 1, L.LSR_BC_BOTTOM)
        torch.cuda.synchronize()
        assert r.status == L.LSR_OK and r.iterations == 1
        assert np.array_equal(t.cpu().numpy(), o) and r.last_count == ro.count


def test_sobel_several_sweeps_and_batched(ctx):
    import torch
    say("sobel sweeps and batched")
    a = _img(300, 333, 9)
    o3, r3 = O.sobel_run(a, max_iter=3)
    t = to_dev(a)
    r = ctx.run(t, L.LSR_ST_SOBEL, L.LSR_RED_SUM, _cond(), 3, L.LSR_BC_BOTTOM)
    torch.cuda.synchronize()
    assert r.iterations == 3 and np.array_equal(t.cpu().numpy(), o3) and r.last_count == r3.count
    with L.Context(0, batched=True) as b:
        jobs = []
        for k, (rows, cols) in enumerate(SHAPES):
            img = _img(rows, cols, 50 + k)
            if k % 2:
                g = torch.from_numpy(img.copy()).pin_memory()
                jid = b.submit_host(g, L.LSR_ST_SOBEL, L.LSR_RED_SUM, _cond(), 1, L.LSR_BC_BOTTOM)
            else:
                g = to_dev(img, cols + 5, 1)
                jid = b.submit(g, L.LSR_ST_SOBEL, L.LSR_RED_SUM, _cond(), 1, L.LSR_BC_BOTTOM)
            jobs.append((img, g, jid))
        for img, g, jid in jobs:
            rr = b.result(jid)
            torch.cuda.synchronize()
            o, ro = O.sobel_run(img, max_iter=1)
            assert rr.status == L.LSR_OK and rr.iterations == 1
            assert np.array_equal(g.cpu().numpy(), o) and rr.last_count == ro.count
