"""GPU parity of the temporally blocked Life path (several generations per launch).

A fused launch computes every stored cell of every generation from the cells a
chain of plain generations would read, so the grid, the live count of every
checked generation and the stop generation must equal the oracle exactly. Stops
and caps that fall inside a launch are replayed from the launch's source buffer.
"""
import numpy as np
import pytest

import oracle as O
import paper_1609_04567_amd as L
from paper_1609_04567_amd import inputs as I
from gpu_helpers import run_life, say

pytestmark = pytest.mark.gpu

DEPTHS = [2, 3, 4, 5, 6, 8]


def _tuned(ctx, fn, **tune):
    ctx.tune(**tune)
    try:
        return fn()
    finally:
        ctx.tune()


def _torus_crop(a, r0, c0, size):
    n0, n1 = a.shape
    rr = (np.arange(r0, r0 + size) % n0)[:, None]
    cc = (np.arange(c0, c0 + size) % n1)[None, :]
    return a[rr, cc]


@pytest.mark.parametrize("depth", [1] + DEPTHS)
@pytest.mark.parametrize("shape", [(1, 16), (2, 32), (3, 48), (16, 16), (65, 1008), (130, 2000),
                                   (257, 1024), (33, 4112)])
@pytest.mark.parametrize("torus", [True, False])
def test_life_fused_matches_oracle(ctx, depth, shape, torus):
    """29 generations: the cap falls inside a launch at every depth above 1."""
    say(f"life tb depth={depth} shape={shape} torus={torus}")
    a = I.life_input(*shape, seed=shape[0] * 31 + shape[1])
    bc = O.BC_TORUS if torus else O.BC_BOTTOM
    o, ro = O.life_run(a, bc=bc, cond=O.COND_NEVER, max_iter=29)
    x, r = _tuned(ctx, lambda: run_life(ctx, a, torus=torus, cond=L.LSR_COND_NEVER, max_iter=29),
                  tb_depth=depth)
    assert r.status == L.LSR_OK and r.sweeps_per_launch == depth
    assert r.iterations == 29 and r.last_count == ro.count
    assert np.array_equal(x, o)


@pytest.mark.parametrize("depth", DEPTHS)
def test_stable_stops_inside_fused_launches(ctx, depth):
    """Soups that settle at data-dependent generations, and a blinker that stops
    at 10: the stop generation, the run length and the field match the oracle."""
    say(f"life tb stops depth={depth}")
    inside = 0
    for seed in range(4):
        a = I.life_input(96, 128, seed=40 + seed)
        o, ro = O.life_run(a, stable_window=10, max_iter=2000)
        x, r = _tuned(ctx, lambda: run_life(ctx, a, window=10, max_iter=2000), tb_depth=depth)
        assert r.iterations == ro.n and bool(r.converged) == ro.converged
        assert r.last_count == ro.count and r.stable_run == ro.run
        assert np.array_equal(x, o), seed
        inside += ro.n % depth != 0
    g = I.life_pattern(16, 16, [(3, 2), (3, 3), (3, 4)])
    x, r = _tuned(ctx, lambda: run_life(ctx, g, window=10), tb_depth=depth)
    assert r.iterations == 10 and r.converged and r.last_count == 3 and np.array_equal(x, g)
    assert inside + (10 % depth != 0) > 0


@pytest.mark.parametrize("depth", [3, 4, 8])
@pytest.mark.parametrize("check_every,window", [(3, 2), (5, 1), (7, 3)])
def test_sparse_checks_fall_anywhere_in_a_launch(ctx, depth, check_every, window):
    say(f"life tb checks every {check_every} window {window} depth={depth}")
    a = I.life_input(48, 64, seed=7)
    o, ro = O.life_run(a, check_every=check_every, stable_window=window, max_iter=400)
    x, r = _tuned(ctx, lambda: run_life(ctx, a, window=window, check_every=check_every,
                                        max_iter=400), tb_depth=depth)
    assert r.iterations == ro.n and bool(r.converged) == ro.converged
    assert r.last_count == ro.count and np.array_equal(x, o)


@pytest.mark.parametrize("tile_rows", [1, 4, 5, 64, 200])
@pytest.mark.parametrize("chunk,graph", [(0, 0), (8, -1), (24, 1)])
def test_bands_chunks_and_graphs(ctx, tile_rows, chunk, graph):
    say(f"life tb tile_rows={tile_rows} chunk={chunk} graph={graph}")
    a = I.life_input(150, 2000, seed=8)
    o, ro = O.life_run(a, cond=O.COND_NEVER, max_iter=50)
    x, r = _tuned(ctx, lambda: run_life(ctx, a, cond=L.LSR_COND_NEVER, max_iter=50),
                  tb_depth=4, tile_rows=tile_rows, chunk=chunk, use_graph=graph)
    assert r.iterations == 50 and r.last_count == ro.count and np.array_equal(x, o)


@pytest.mark.parametrize("rows,cols", [(40, 50), (33, 1), (21, 17), (64, 1000), (30, 2001)])
@pytest.mark.parametrize("torus", [True, False])
def test_ragged_rows_fuse_on_padded_copies(ctx, rows, cols, torus):
    """Rows that are not a multiple of 16 cells run fused on the staged copy whose
    rows are padded to 16 cells (dead border: padding masked at every level; torus:
    edge lanes gathered from the wrapped columns), equal to the oracle; a stop
    inside a launch (cap 13 at depth 4) is replayed."""
    say(f"life tb ragged {rows}x{cols} torus={torus}")
    a = I.life_input(rows, cols, seed=9 + cols)
    bc = O.BC_TORUS if torus else O.BC_BOTTOM
    o, ro = O.life_run(a, bc=bc, cond=O.COND_NEVER, max_iter=13)
    x, r = _tuned(ctx, lambda: run_life(ctx, a, torus=torus, cond=L.LSR_COND_NEVER, max_iter=13),
                  tb_depth=4)
    assert r.sweeps_per_launch == 4 and r.iterations == 13
    assert np.array_equal(x, o) and r.last_count == ro.count


@pytest.mark.parametrize("depth", [2, 8])
def test_full_16384_fused_light_cone(ctx, depth):
    """The 16384^2 torus at 2 and 8 generations per launch, 64 generations, checked
    on sampled windows through the light cone (a cell after k generations depends
    only on the (2k+1)^2 box around it)."""
    import torch
    gens = 64
    say(f"life tb 16384^2 depth={depth}")
    n = 16384
    a = I.life_input(n, seed=3)
    t = torch.from_numpy(a).to("cuda:0")
    r = _tuned(ctx, lambda: ctx.run(t, L.LSR_ST_LIFE, L.LSR_RED_SUM,
                                    L.make_cond(L.LSR_COND_STABLE_FOR, 0.0, 1, 10), gens,
                                    L.LSR_BC_TORUS), tb_depth=depth)
    assert r.status == L.LSR_OK and r.iterations == gens and r.sweeps_per_launch == depth
    x = t.cpu().numpy()
    assert r.last_count == int(x.sum())
    w = 48
    for (r0, c0) in [(0, 0), (n - w // 2, n - w // 2), (5000, 123), (16000, 8000), (9999, 16380),
                     (64, 992 - 24), (8191, 992 * 7 - 5)]:
        crop = _torus_crop(a, r0 - gens, c0 - gens, w + 2 * gens)
        o, _ = O.life_run(crop, bc=O.BC_BOTTOM, cond=O.COND_NEVER, max_iter=gens)
        want = o[gens:gens + w, gens:gens + w]
        got = _torus_crop(x, r0, c0, w)
        assert np.array_equal(got, want), (r0, c0)
