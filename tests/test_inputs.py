"""Generator pins: SplitMix64 known answers, counter-based slicing, recipe shapes."""
import os

import numpy as np

from paper_1609_04567_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for seed, idx, hexv in rows:
        assert int(I.splitmix64(int(seed), int(idx), 1)[0]) == int(hexv, 16)


def test_stream_slices_are_consistent():
    full = I.splitmix64(12345, 0, 5000)
    assert np.array_equal(full[1234:2345], I.splitmix64(12345, 1234, 2345 - 1234))
    u = I.uniform01(7, 0, 100000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01


def test_laplace_recipe():
    a = I.laplace_input(64, 40)
    assert a.shape == (64, 40) and a.dtype == np.float64
    assert np.all(a[1:-1, 1:-1] == 0.0)
    ring = np.concatenate([a[0], a[-1], a[:, 0], a[:, -1]])
    assert ring.min() >= 0.0 and ring.max() < 1.0 and ring.std() > 0.1
    # ring cell (i, j) is draw i*cols + j
    u = I.uniform01(1, 0, 64 * 40).reshape(64, 40)
    assert a[0, 5] == u[0, 5] and a[63, 39] == u[63, 39] and a[17, 0] == u[17, 0]


def test_helmholtz_recipe():
    h = I.helmholtz_input(65, alpha=1.0)
    assert h.s[0] == 0.0 and h.s[-1] == 0.0
    assert np.all(h.ustar[0] == 0.0) and np.all(h.ustar[:, -1] == 0.0)
    assert np.all(h.u0 == 0.0)
    assert abs(h.h - 1.0 / 64) < 1e-18
    assert np.allclose(h.g, h.h ** 2 * (2 * np.pi ** 2 + 1.0) * h.ustar, rtol=1e-15, atol=0)


def test_life_recipe_density():
    g = I.life_input(256, seed=3)
    assert set(np.unique(g)) <= {0, 1}
    assert abs(g.mean() - 0.3) < 0.01


def test_restore_recipe():
    r = I.restore_input(128, 96, seed=4, noise=0.4)
    assert r.clean.min() >= 16 and r.clean.max() <= 239
    assert r.clean.min() == 16 and r.clean.max() == 239
    assert abs(r.impulse.mean() - 0.4) < 0.02
    assert np.all((r.y[r.impulse] == 0) | (r.y[r.impulse] == 255))
    assert np.array_equal(r.y[~r.impulse], r.clean[~r.impulse])


def test_job_stream_mix():
    jobs = I.job_stream(2000)
    kinds = [j.kind for j in jobs]
    assert abs(kinds.count("laplace") / 2000 - 0.6) < 0.04
    assert abs(kinds.count("helmholtz") / 2000 - 0.25) < 0.04
    sides = np.array([j.side for j in jobs])
    assert sides.min() >= 128 and sides.max() <= 4096
    # log-uniform: the median side is near sqrt(128*4096) = 724
    assert 600 < np.median(sides) < 870
    assert I.job_stream(5)[3].seed == jobs[3].seed


def test_fill_forms_match_the_draw_definitions():
    """The buffer-filling generators (used to build jobs at their arrival) give the
    bytes of the draw-by-draw definitions: ring draw i*cols + j for Laplace, the
    double draw against the density for Life, the FP64 product for Helmholtz."""
    for rows, cols, seed in ((3, 3, 1), (5, 17, 2), (64, 40, 1), (257, 129, 99)):
        u = I.uniform01(seed, 0, rows * cols).reshape(rows, cols)
        ref = np.zeros((rows, cols))
        ref[0], ref[-1], ref[:, 0], ref[:, -1] = u[0], u[-1], u[:, 0], u[:, -1]
        assert np.array_equal(I.laplace_input(rows, cols, seed), ref)
        f32 = np.empty((rows, cols), np.float32)
        assert np.array_equal(I.laplace_fill(f32, seed), ref.astype(np.float32))
        for d in (0.3, 0.5, 0.01, 0.999, 1.0, 0.0):
            assert np.array_equal(I.life_input(rows, cols, seed, d), (u < d).astype(np.uint8)), d
    # the threshold test on the integer draw at the exact boundary of a draw
    x = I.splitmix64(4, 0, 1)[0]
    d = float((x >> np.uint64(11)) * 2.0 ** -53)
    assert I.life_input(1, 1, 4, d)[0, 0] == 0 and I.life_input(1, 1, 4, np.nextafter(d, 1))[0, 0] == 1
    for n in (3, 65, 300):
        h = I.helmholtz_input(n)
        u0, g = np.ones((n, n), np.float32), np.empty((n, n), np.float32)
        assert I.helmholtz_fill(u0, g) == h.h
        assert not u0.any() and np.array_equal(g, h.g.astype(np.float32))
        g64 = np.empty((n, n))
        I.helmholtz_fill(np.empty((n, n)), g64)
        assert np.array_equal(g64, (h.h * h.h) * ((2 * np.pi ** 2 + 1.0) * np.outer(h.s, h.s)))


def test_video_frame_recipe():
    """Draw layout and ranges of the video frames: impulses follow draws
    6*blobs + 2*(f*npx + p) and the next one, as doubles against the rates."""
    rows, cols, blobs = 37, 53, 8
    for f, noise in ((0, 0.3), (4, 0.7)):
        v = I.video_frame(rows, cols, f, seed=8, noise=noise)
        npx = rows * cols
        u = I.uniform01(8, 6 * blobs + 2 * f * npx, 2 * npx).reshape(-1, 2)
        hit = (u[:, 0] < noise).reshape(rows, cols)
        salt = (u[:, 1] < 0.5).reshape(rows, cols)
        assert np.array_equal(v.impulse, hit)
        assert np.all(v.y[hit & salt] == 255) and np.all(v.y[hit & ~salt] == 0)
        assert np.array_equal(v.y[~hit], v.clean[~hit])
        assert v.clean.min() == 16 and v.clean.max() == 239
    # the blobs move: consecutive frames differ, but only a little
    a, b = I.video_frame(64, 64, 0).clean, I.video_frame(64, 64, 1).clean
    assert 0 < np.abs(a.astype(int) - b.astype(int)).max() < 40
