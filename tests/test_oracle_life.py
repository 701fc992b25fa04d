"""Pins for the oracle's Game of Life loop (the rule of the paper's Fig. 1).

Pinned by the B3/S23 rule stated as birth/survival sets over all 512 3x3
neighbourhoods, by patterns with known periods and displacements (Gardner 1970),
by a wrap-around property of the torus, and by an independent roll-sum
formulation on small tori.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1609_04567_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _patterns():
    out = {}
    for line in open(os.path.join(GOLDEN, "life_patterns.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        head, cells = line.split(";")
        name, period, dr, dc = head.split()
        pts = [tuple(int(x) for x in c.split(",")) for c in cells.split()]
        out[name] = (int(period), int(dr), int(dc), pts)
    return out


PATTERNS = _patterns()


def _step(a, bc=O.BC_TORUS, k=1):
    b, r = O.life_run(a, bc=bc, cond=O.COND_NEVER, max_iter=k)
    assert r.n == k
    return b


def test_rule_table_all_512_neighbourhoods():
    birth, survive = {3}, {2, 3}
    for code in range(512):
        bits = [(code >> k) & 1 for k in range(9)]
        g = np.zeros((5, 5), dtype=np.uint8)
        g[1:4, 1:4] = np.array(bits, dtype=np.uint8).reshape(3, 3)
        b = _step(g, bc=O.BC_BOTTOM)
        centre = bits[4]
        nb = sum(bits) - centre
        expect = (nb in survive) if centre else (nb in birth)
        assert b[2, 2] == int(expect), code


@pytest.mark.parametrize("name", sorted(PATTERNS))
def test_known_patterns(name):
    period, dr, dc, pts = PATTERNS[name]
    g = I.life_pattern(12, 12, pts)
    after = _step(g, k=period)
    assert np.array_equal(after, np.roll(g, (dr, dc), axis=(0, 1)))
    if period > 1 and (dr, dc) == (0, 0):
        assert not np.array_equal(_step(g, k=1), g)


def test_glider_returns_after_4n_generations_on_torus():
    _, _, _, pts = PATTERNS["glider"]
    for n in (8, 10):
        g = I.life_pattern(n, n, pts)
        assert np.array_equal(_step(g, k=4 * n), g)
        assert not np.array_equal(_step(g, k=4 * n - 4), g)


def test_blinker_stops_at_ten_with_stable_count():
    _, _, _, pts = PATTERNS["blinker"]
    g = I.life_pattern(8, 8, pts)
    b, r = O.life_run(g, cond=O.COND_STABLE_FOR, stable_window=10, max_iter=2000, trace_cap=20)
    assert r.n == 10 and r.converged and r.count == 3 and r.run == 10
    assert list(r.trace) == [3] * 10
    assert np.array_equal(b, g)  # even number of generations


@pytest.mark.parametrize("cells", [[], PATTERNS["block"][3]])
def test_still_grids_stop_at_ten(cells):
    g = I.life_pattern(9, 9, cells)
    b, r = O.life_run(g, stable_window=10, max_iter=2000)
    assert r.n == 10 and r.converged and np.array_equal(b, g)


def test_stable_window_resets_on_change():
    # a glider keeps its count (5) every generation: stops at the window
    g = I.life_pattern(16, 16, PATTERNS["glider"][3])
    _, r = O.life_run(g, stable_window=7, max_iter=100, trace_cap=100)
    assert r.n == 7 and r.count == 5
    # a soup changes count early on: the run restarts, the stop comes later
    s = I.life_input(32, seed=8)
    _, r2 = O.life_run(s, stable_window=3, max_iter=500, trace_cap=500)
    tr = r2.trace.astype(np.int64)
    n0 = int(s.sum())
    seq = np.concatenate([[n0], tr])
    runs, run = [], 0
    for k in range(1, len(seq)):
        run = run + 1 if seq[k] == seq[k - 1] else 0
        runs.append(run)
    assert (r2.converged and runs[-1] >= 3 and all(x < 3 for x in runs[:-1])) or r2.n == 500


def _roll_life(a, k):
    a = a.astype(np.int32)
    for _ in range(k):
        nb = sum(np.roll(a, (di, dj), axis=(0, 1)) for di in (-1, 0, 1) for dj in (-1, 0, 1)
                 if (di, dj) != (0, 0))
        a = ((nb == 3) | ((a == 1) & (nb == 2))).astype(np.int32)
    return a.astype(np.uint8)


@pytest.mark.parametrize("shape,seed", [((8, 8), 1), ((17, 13), 2), ((33, 64), 3)])
def test_torus_against_roll_sum(shape, seed):
    g = I.life_input(*shape, seed=seed)
    assert np.array_equal(_step(g, k=9), _roll_life(g, 9))


def test_dead_border_differs_only_next_to_the_edge():
    g = I.life_input(20, 24, seed=4)
    t = _step(g, O.BC_TORUS)
    d = _step(g, O.BC_BOTTOM)
    diff = t != d
    assert not diff[1:-1, 1:-1].any()


def test_nonzero_bytes_count_as_alive():
    g = I.life_pattern(8, 8, PATTERNS["blinker"][3]) * 7
    assert np.array_equal(_step(g), _step((g != 0).astype(np.uint8)))


def test_soup_counts_and_cap():
    s = I.life_input(64, seed=3)
    b, r = O.life_run(s, stable_window=10, max_iter=50, trace_cap=50)
    assert r.n == 50 and r.count == int(b.sum()) and len(r.trace) == 50
