"""GPU parity: Game of Life through the C ABI against the oracle (bit-exact).

Small and ragged grids are compared whole; the full 16384^2 torus is checked on
sampled windows through the light cone: after k generations a cell depends only
on the (2k+1)^2 box around it, so the oracle run on a torus-wrapped crop with a
margin of k reproduces the centre of the crop exactly.
"""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import run_life, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(1, 1), (8, 8), (17, 13), (16, 16), (64, 48), (130, 1040),
                                   (257, 2048), (33, 4112)])
@pytest.mark.parametrize("torus", [True, False])
def test_life_matches_oracle(ctx, shape, torus):
    say(f"life {shape} torus={torus}")
    a = I.life_input(*shape, seed=3)
    bc = O.BC_TORUS if torus else O.BC_BOTTOM
    o, ro = O.life_run(a, bc=bc, stable_window=10, max_iter=300)
    x, r = run_life(ctx, a, torus=torus, window=10, max_iter=300)
    assert r.status == L.LSR_OK
    assert r.iterations == ro.n and bool(r.converged) == ro.converged
    assert r.last_count == ro.count and r.stable_run == ro.run
    assert np.array_equal(x, o)


@pytest.mark.parametrize("pitch,offset", [(80, 0), (72, 5), (64 + 16, 16)])
def test_life_pitched_views(ctx, pitch, offset):
    say(f"life pitched {pitch} {offset}")
    a = I.life_input(40, 64, seed=5)
    o, ro = O.life_run(a, cond=O.COND_NEVER, max_iter=37)
    x, r = run_life(ctx, a, cond=L.LSR_COND_NEVER, max_iter=37, pitch=pitch, offset=offset)
    assert r.iterations == 37 and r.last_count == ro.count and np.array_equal(x, o)


def test_blinker_stops_at_ten(ctx):
    say("blinker")
    g = I.life_pattern(16, 16, [(3, 2), (3, 3), (3, 4)])
    x, r = run_life(ctx, g, window=10)
    assert r.iterations == 10 and r.converged and r.last_count == 3 and np.array_equal(x, g)


def test_glider_returns_on_torus(ctx):
    say("glider")
    g = I.life_pattern(32, 32, [(0, 1), (1, 2), (2, 0), (2, 1), (2, 2)])
    x, r = run_life(ctx, g, cond=L.LSR_COND_NEVER, max_iter=128)
    assert r.iterations == 128 and np.array_equal(x, g)
    x, r = run_life(ctx, g, cond=L.LSR_COND_NEVER, max_iter=4)
    assert np.array_equal(x, np.roll(g, (1, 1), axis=(0, 1)))


def test_soups_with_data_dependent_stop(ctx):
    """Small soups settle; the stop generation must match exactly."""
    say("soups stop")
    stops = []
    for seed in range(4):
        a = I.life_input(128, seed=seed)
        o, ro = O.life_run(a, stable_window=10, max_iter=2000)
        x, r = run_life(ctx, a, window=10, max_iter=2000)
        assert r.iterations == ro.n and r.converged == ro.converged and np.array_equal(x, o)
        stops.append(ro.n)
    say(f"  stops {stops}")


def _torus_crop(a, r0, c0, size):
    n0, n1 = a.shape
    rr = (np.arange(r0, r0 + size) % n0)[:, None]
    cc = (np.arange(c0, c0 + size) % n1)[None, :]
    return a[rr, cc]


@pytest.mark.parametrize("gens", [64])
def test_full_16384_torus_light_cone(ctx, gens):
    import torch
    say(f"life 16384^2 {gens} generations, sampled windows")
    n = 16384
    a = I.life_input(n, seed=3)
    t = torch.from_numpy(a).to("cuda:0")
    r = ctx.run(t, L.LSR_ST_LIFE, L.LSR_RED_SUM, L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10),
                gens, L.LSR_BC_TORUS)
    assert r.status == L.LSR_OK and r.iterations == gens
    x = t.cpu().numpy()
    assert r.last_count == int(x.sum())
    w = 48
    for (r0, c0) in [(0, 0), (n - w // 2, n - w // 2), (5000, 123), (16000, 8000), (9999, 16380)]:
        crop = _torus_crop(a, r0 - gens, c0 - gens, w + 2 * gens)
        o, _ = O.life_run(crop, bc=O.BC_BOTTOM, cond=O.COND_NEVER, max_iter=gens)
        want = o[gens:gens + w, gens:gens + w]
        got = _torus_crop(x, r0, c0, w)
        assert np.array_equal(got, want), (r0, c0)


def test_full_16384_run_is_deterministic(ctx):
    import torch
    say("life 16384^2 300 generations twice")
    a = I.life_input(16384, seed=3)
    outs = []
    for _ in range(2):
        t = torch.from_numpy(a).to("cuda:0")
        r = ctx.run(t, L.LSR_ST_LIFE, L.LSR_RED_SUM, L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10),
                    300, L.LSR_BC_TORUS)
        outs.append((t.cpu().numpy(), r.last_count, r.iterations))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]


@pytest.mark.parametrize("shape", [(16, 16), (17, 13), (64, 1040)])
def test_nonzero_bytes_are_alive(ctx, shape):
    """Bytes other than 0/1 count as alive (the first pass normalises them in place)."""
    say(f"life non-0/1 bytes {shape}")
    rng = np.random.default_rng(9)
    a = I.life_input(*shape, seed=6) * rng.integers(1, 256, size=shape).astype(np.uint8)
    o, ro = O.life_run(a, bc=O.BC_TORUS, cond=O.COND_NEVER, max_iter=7)
    x, r = run_life(ctx, a, cond=L.LSR_COND_NEVER, max_iter=7)
    assert np.array_equal(x, o) and r.last_count == ro.count
