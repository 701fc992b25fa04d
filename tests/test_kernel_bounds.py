"""Host-side bounds model of the sweep kernels' addressing.

For each launch geometry the library can choose, this replays the index
arithmetic of jacobi5_kernel and life_swar_kernel (which lanes load or store
which (row, column), including the wavefront halo elements) and asserts that
every access lies inside the rows x cols grid. It runs on the CPU, before any
GPU use, so an out-of-range address is caught here and not on the device.
"""
import itertools

import numpy as np
import pytest

JACOBI_SHAPES = [(1, 8), (2, 8), (4, 4), (4, 8), (4, 16)]


def _jacobi_accesses(rows, cols, vec, nw, unroll, tile_rows, tiles_subset=None):
    span = nw * 64 * vec
    strips = -(-cols // span)
    bands = -(-(rows - 2) // tile_rows)
    lanes = np.arange(64)
    bad = []
    tiles = range(strips * bands) if tiles_subset is None else tiles_subset(strips, bands)
    for t in tiles:
        band, strip = divmod(t, strips)
        r0 = 1 + band * tile_rows
        r1 = min(r0 + tile_rows, rows - 1)
        for w in range(nw):
            cw = strip * span + w * 64 * vec
            c = cw + lanes * vec
            ce = cw + 64 * vec
            has_w = cw >= 1 and cw < cols           # lane 0 only
            has_e = ce < cols                       # lane 63 only
            elem_cols = (c[:, None] + np.arange(vec)[None, :])
            in_cols = elem_cols[elem_cols < cols]   # guarded element loads / stores
            rows_read = list(range(r0 - 1, r1 + 1))  # up, mid, then r+1 for r < r1
            rows_written = list(range(r0, r1))
            for r in rows_read + rows_written:
                if not (0 <= r < rows):
                    bad.append(("row", t, w, r))
            if in_cols.size and (in_cols.min() < 0 or in_cols.max() >= cols):
                bad.append(("col", t, w))
            if has_w and not (0 <= cw - 1 < cols):
                bad.append(("west halo", t, w, cw - 1))
            if has_e and not (0 <= ce < cols):
                bad.append(("east halo", t, w, ce))
    return bad


@pytest.mark.parametrize("rows,cols", [(3, 3), (8, 8), (17, 13), (64, 64), (80, 80), (144, 144),
                                       (129, 257), (300, 1030), (70, 1029), (33, 4100), (5, 700)])
@pytest.mark.parametrize("nw,unroll", JACOBI_SHAPES)
@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("tile_rows", [8, 17, 32])
def test_jacobi_accesses_stay_in_grid(rows, cols, nw, unroll, vec, tile_rows):
    assert _jacobi_accesses(rows, cols, vec, nw, unroll, tile_rows) == []


def test_jacobi_edges_of_large_grids():
    def edge_tiles(strips, bands):
        pick = set()
        for b in (0, bands // 2, bands - 1):
            for s in range(strips):
                pick.add(b * strips + s)
        return sorted(pick)
    for (rows, cols), (nw, unroll), vec in itertools.product(
            [(8192, 8192), (4096, 4096), (8191, 8190), (2000, 3001)], JACOBI_SHAPES, [2, 4]):
        assert _jacobi_accesses(rows, cols, vec, nw, unroll, 8, edge_tiles) == []


def _life_pitch(cols):
    """Row pitch the runtime gives a Life grid: the caller's when cols is a multiple
    of 16 (the direct case), else a staged copy padded to 128 bytes."""
    return cols if cols % 16 == 0 else -(-cols // 128) * 128


def _life_geometry(cols, nw, lane_range=64):
    span = nw * 1024
    return span, -(-cols // span)


def _life_wave(cols, cw, torus):
    """(nact, last, wcol, has_w, ecol, has_e) as life_swar_tile computes them."""
    nact = min(64, -(-(cols - cw) // 16)) if cw < cols else 0
    last = nact - 1
    wcol, ecol = cw - 1, min(cw + nact * 16, cols)
    has_w = has_e = nact > 0
    if wcol < 0:
        if torus:
            wcol += cols
        else:
            has_w = False
    if ecol >= cols:
        if torus:
            ecol -= cols
        else:
            has_e = False
    return nact, last, wcol, has_w, ecol, has_e


def _life_accesses(rows, cols, nw, tile_rows, torus):
    pitch = _life_pitch(cols)
    span, strips = _life_geometry(cols, nw)
    bands = -(-rows // tile_rows)
    bad = []
    for t in range(strips * bands):
        band, strip = divmod(t, strips)
        r0 = band * tile_rows
        r1 = min(r0 + tile_rows, rows)
        for w in range(nw):
            cw = strip * span + w * 1024
            nact, last, wcol, has_w, ecol, has_e = _life_wave(cols, cw, torus)
            c = cw + np.arange(64) * 16
            active = c < cols
            # 16-byte words are loaded and stored whole: they must fit in the row pitch
            if active.any() and (c[active] + 15).max() >= pitch:
                bad.append(("word", t, w))
            if has_w and not (0 <= wcol < cols):
                bad.append(("west", t, w, wcol))
            if has_e and not (0 <= ecol < cols):
                bad.append(("east", t, w, ecol))
            for r in range(r0 - 1, r1 + 1):
                rr = r
                if r < 0 or r >= rows:
                    if not torus:
                        continue
                    rr = r + rows if r < 0 else r - rows  # the kernel wraps one step only
                if not (0 <= rr < rows):
                    bad.append(("row", t, w, r))
            for r in range(r0, r1):
                if not (0 <= r < rows):
                    bad.append(("store row", t, w, r))
    return bad


@pytest.mark.parametrize("rows,cols", [(1, 16), (16, 16), (64, 48), (130, 1040), (257, 2048),
                                       (33, 4112), (5, 5008), (1, 1), (17, 13), (9, 1027),
                                       (3, 4097)])
@pytest.mark.parametrize("nw", [1, 2, 4, 8])
@pytest.mark.parametrize("tile_rows", [16, 64])
@pytest.mark.parametrize("torus", [True, False])
def test_life_accesses_stay_in_grid(rows, cols, nw, tile_rows, torus):
    assert _life_accesses(rows, cols, nw, tile_rows, torus) == []


def _zero_bytes_hi(x):
    return ~(x + np.uint32(0x7F7F7F7F)) & np.uint32(0x80808080)


def _swar_generation(buf, rows, cols, torus, nw, tile_rows):
    """One generation of life_swar_tile, replayed word by word on the CPU (buf is
    the padded rows x pitch byte array; returns the new array and the count)."""
    pitch = buf.shape[1]
    out = np.zeros_like(buf)
    words = buf.view(np.uint32)             # rows x pitch/4
    span, strips = _life_geometry(cols, nw)
    bands = -(-rows // tile_rows)
    total = 0
    lanes = np.arange(64)
    for t in range(strips * bands):
        band, strip = divmod(t, strips)
        r0, r1 = band * tile_rows, min(band * tile_rows + tile_rows, rows)
        for w in range(nw):
            cw = strip * span + w * 1024
            nact, last, wcol, has_w, ecol, has_e = _life_wave(cols, cw, torus)
            c = cw + lanes * 16
            active = c < cols
            q = np.where(active, np.minimum(16, cols - c), 0)
            part = (q > 0) & (q < 16)

            def load(r):
                W = np.zeros((64, 4), np.uint32)
                hw = he = 0
                if r < 0 or r >= rows:
                    if not torus:
                        return W, 0, 0
                    r = r + rows if r < 0 else r - rows
                for ln in np.nonzero(active)[0]:
                    W[ln] = words[r, (c[ln] // 4):(c[ln] // 4) + 4]
                if has_w:
                    hw = int(buf[r, wcol])
                if has_e:
                    he = int(buf[r, ecol])
                return W, hw, he

            for r in range(r0, r1):
                up, uw, ue = load(r - 1)
                mid, mw, me = load(r)
                dn, dw, de = load(r + 1)
                V = (up + mid + dn).astype(np.uint32)
                vw_h, ve_h = uw + mw + dw, ue + me + de
                for ln in range(64):
                    if not active[ln]:
                        continue
                    Vl = V[ln].copy()
                    wv = int(V[ln - 1][3] >> np.uint32(24)) if ln > 0 else vw_h
                    ev = int(V[ln + 1][0] & np.uint32(0xFF)) if ln < 63 else int(V[ln][0] & 0xFF)
                    if ln == last:
                        ev = ve_h
                    if part[ln]:
                        m, sh = int(q[ln]) >> 2, (int(q[ln]) & 3) * 8
                        Vl[m] = (Vl[m] & np.uint32(~(0xFF << sh) & 0xFFFFFFFF)) | np.uint32(ve_h << sh)
                    o = np.zeros(4, np.uint32)
                    for m in range(4):
                        prev = int(Vl[m - 1] >> np.uint32(24)) if m > 0 else wv
                        nxt = int(Vl[m + 1] & np.uint32(0xFF)) if m < 3 else ev
                        T = (((Vl[m] << np.uint32(8)) | np.uint32(prev)) + Vl[m]
                             + ((Vl[m] >> np.uint32(8)) | np.uint32(nxt << 24))).astype(np.uint32)
                        alive = _zero_bytes_hi(((T - mid[ln][m]) | mid[ln][m]) ^ np.uint32(0x03030303))
                        o[m] = alive >> np.uint32(7)
                        k = int(q[ln]) - 4 * m
                        cm = 0x80808080 if k >= 4 else 0 if k <= 0 else 0x80808080 & ((1 << (8 * k)) - 1)
                        total += bin(int(alive) & cm).count("1")
                    out[r, c[ln]:c[ln] + 16] = o.view(np.uint8)
    return out, total


@pytest.mark.parametrize("rows,cols", [(1, 1), (3, 5), (17, 13), (20, 31), (9, 33), (12, 48),
                                       (6, 1027)])
@pytest.mark.parametrize("torus", [True, False])
def test_life_swar_model_matches_oracle_on_padded_rows(rows, cols, torus):
    """The word arithmetic of the SWAR tile, including the partial last lane of a
    padded row, against the oracle over three generations."""
    import oracle as O
    from paper_1609_04567_amd import inputs as I
    a = I.life_input(rows, cols, seed=rows * 100 + cols)
    pitch = _life_pitch(cols)
    buf = np.zeros((rows, pitch), np.uint8)
    buf[:, :cols] = a
    for gen in range(1, 4):
        buf, count = _swar_generation(buf, rows, cols, torus, 1, 8)
        o, ro = O.life_run(a, bc=O.BC_TORUS if torus else O.BC_BOTTOM, cond=O.COND_NEVER,
                           max_iter=gen)
        assert np.array_equal(buf[:, :cols], o), gen
        assert count == ro.count, gen
        assert buf.max() <= 1   # padding stays 0/1, so column sums never carry


def test_model_flags_the_unguarded_west_halo():
    """The model must catch a wavefront past the last column loading its halo."""
    rows, cols, vec, nw = 64, 64, 2, 4
    span = nw * 64 * vec
    cw = 3 * 64 * vec  # wave 3 of strip 0
    assert cw >= cols and cw < span
    # with the guard cw < cols removed, the halo column would be cw - 1 >= cols
    assert not (0 <= cw - 1 < cols)


# ---------------------------------------------------------------------------
# Temporally blocked Jacobi kernel (jacobi5_tb_kernel): a launch advances K
# sweeps. Each wavefront owns a window of 64 * vec columns starting at
# cw = window * ow, ow = (64 * vec - 2K) rounded down to a multiple of vec;
# it streams rows r0 - K .. r1 + K - 1 of the band through K levels and stores
# level K for rows [r0, r1), columns [olo, ohi). The model below replays that
# schedule on the CPU (zeros outside the grid and before the stream start, a
# zero west neighbour at lane 0 and east neighbour at lane 63, boundary cells
# carried unchanged) and checks that the stored cells cover the interior
# exactly once and equal K plain sweeps, and that the kernel's load guard only
# lets in-grid rows be read.
# ---------------------------------------------------------------------------

TB_CHUNK = 8                              # band groups per dispatch chunk (vertical tiles)


def _tb_geometry(rows, cols, vec, nw, k, tile_rows, vert=False):
    ow = (64 * vec - 2 * k) // vec * vec
    need = cols - 1 - k
    nwin = -(-need // ow) if need > 0 else 1
    bands = -(-(rows - 2) // tile_rows)
    if vert:                              # a workgroup: nw consecutive bands of one window
        return ow, nwin, -(-bands // nw)
    return ow, -(-nwin // nw), bands


def _tb_waves(rows, cols, vec, nw, k, tile_rows, vert):
    """(t, w, cw, r0, r1, up) of every wavefront of a launch, as the kernel derives them."""
    ow, strips, groups = _tb_geometry(rows, cols, vec, nw, k, tile_rows, vert)
    for t in range(strips * groups):
        if vert:                          # chunks of TB_CHUNK band groups, groups innermost
            ch, r = divmod(t, strips * TB_CHUNK)
            hb = min(TB_CHUNK, groups - ch * TB_CHUNK)
            strip, h = divmod(r, hb)
            tband = ch * TB_CHUNK + h
        else:
            tband, strip = divmod(t, strips)
        for w in range(nw):
            band = tband * nw + w if vert else tband
            cw = (strip if vert else strip * nw + w) * ow
            r0 = 1 + band * tile_rows
            r1 = min(r0 + tile_rows, rows - 1)
            yield t, w, cw, r0, r1, vert and w % 2 == 1


def _tb_stream(rows, cols, vec, k, cw, r0, r1, up):
    """Level-0 rows in stream order, the g row loaded with each, and the fast flag."""
    width = 64 * vec
    nstream = (r1 - r0 + 2 * k + 2) // 3 * 3
    d = -1 if up else 1
    first = r1 + k - 1 if up else r0 - k
    edge = cw == 0 or cw + width > cols - 1
    if up:
        fast = not edge and first - nstream + 1 >= 0 and r1 + 2 * k + 1 <= rows
    else:
        fast = not edge and r0 - 2 * k >= 1 and first + nstream <= rows
    return [(first + d * n, first + d * n - d) for n in range(nstream)], fast


def _tb_model(u, k, vec, nw, tile_rows, vert=False):
    rows, cols = u.shape
    ow = _tb_geometry(rows, cols, vec, nw, k, tile_rows, vert)[0]
    out = u.copy()                       # the partner buffer starts as a copy
    written = np.zeros(u.shape, dtype=np.int64)
    width = 64 * vec
    loads_ok = True
    for t, w, cw, r0, r1, up in _tb_waves(rows, cols, vec, nw, k, tile_rows, vert):
        if r0 >= r1:
            continue                     # a wavefront past the last band (vert)
        if True:   # (one wavefront)
            cidx = cw + np.arange(width)
            inside = cidx < cols
            olo = 1 if cw == 0 else cw + k
            ohi = min(cw + k + ow, cols - 1)
            if vec > 1 and cw % vec:
                loads_ok = False         # windows must start 16-byte aligned
            # rows stream in groups of three (level-0 row i and g row i -+ 1 at
            # step i); the kernel's load guard, as written: the fast path reads
            # unguarded, the other path only rows in [0, rows)
            stream, fast = _tb_stream(rows, cols, vec, k, cw, r0, r1, up)
            for pair in stream:
                for row in pair:
                    read = fast or 0 <= row < rows
                    if read and not 0 <= row < rows:
                        loads_ok = False
            if fast and cw + width > cols:
                loads_ok = False
            level = {}
            for i in range(r0 - k, r1 + k):
                row = np.zeros(width)
                if 0 <= i < rows:
                    row[inside] = u[i, cidx[inside]]
                level[i] = row
            col_inner = (cidx >= 1) & (cidx <= cols - 2)
            for j in range(1, k + 1):
                prev = level
                level = {}
                for i in range(r0 - k, r1 + k):
                    r = i + j if up else i - j     # level j's row at step i
                    zero = np.zeros(width)
                    n, c, s = prev.get(r - 1, zero), prev.get(r, zero), prev.get(r + 1, zero)
                    wv = np.concatenate([[0.0], c[:-1]])
                    ev = np.concatenate([c[1:], [0.0]])
                    upd = 0.25 * ((n + s) + (wv + ev))
                    inner = col_inner & (1 <= r <= rows - 2)
                    level[r] = np.where(inner, upd, c)
            for r in range(r0, r1):
                sel = (cidx >= olo) & (cidx < ohi)
                out[r, cidx[sel]] = level[r][sel]
                written[r, cidx[sel]] += 1
    return out, written, loads_ok


@pytest.mark.parametrize("rows,cols", [(3, 3), (4, 5), (9, 130), (40, 131), (37, 260), (20, 517),
                                       (70, 250)])
@pytest.mark.parametrize("vec", [2, 4])
@pytest.mark.parametrize("k", [2, 4, 5, 8, 10])
@pytest.mark.parametrize("nw,tile_rows,vert", [(1, 5, False), (2, 16, False), (4, 64, False),
                                                (2, 5, True), (2, 16, True), (4, 7, True)])
def test_tb_schedule_covers_interior_and_matches_k_sweeps(rows, cols, vec, k, nw, tile_rows, vert):
    rng = np.random.default_rng(rows * 1000 + cols)
    u = rng.standard_normal((rows, cols))
    out, written, loads_ok = _tb_model(u, k, vec, nw, tile_rows, vert)
    assert loads_ok
    want_written = np.zeros_like(written)
    want_written[1:-1, 1:-1] = 1
    assert np.array_equal(written, want_written)
    ref = u.copy()
    for _ in range(k):
        nxt = ref.copy()
        nxt[1:-1, 1:-1] = 0.25 * ((ref[:-2, 1:-1] + ref[2:, 1:-1]) + (ref[1:-1, :-2] + ref[1:-1, 2:]))
        ref = nxt
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("rows,cols", [(8192, 8192), (4096, 4096), (8191, 8190), (2049, 2049)])
@pytest.mark.parametrize("vec", [2, 4])
@pytest.mark.parametrize("k", [2, 4, 5, 8, 10])
def test_tb_stores_stay_in_interior_at_full_size(rows, cols, vec, k):
    """Window arithmetic at the benchmark sizes: stores inside [1, cols-1), loads aligned."""
    ow, strips, bands = _tb_geometry(rows, cols, vec, 1, k, 64)
    cws = np.arange(strips) * ow
    olo = np.where(cws == 0, 1, cws + k)
    ohi = np.minimum(cws + k + ow, cols - 1)
    assert (cws % vec == 0).all()
    assert olo.min() >= 1 and ohi.max() <= cols - 1
    live = olo < ohi
    # consecutive output ranges abut: no column is skipped or written twice
    assert (olo[live][1:] == ohi[live][:-1]).all() and ohi[live][-1] == cols - 1


@pytest.mark.parametrize("rows,cols", [(8192, 8192), (4096, 4096), (8191, 8190), (2049, 2049),
                                       (131, 8192), (4097, 257)])
@pytest.mark.parametrize("vec,k", [(2, 10), (2, 5), (4, 5), (4, 2), (2, 8)])
@pytest.mark.parametrize("nw,tile_rows", [(2, 40), (4, 40), (2, 32), (2, 7)])
def test_tb_vertical_groups_cover_rows_and_guard_loads_at_full_size(rows, cols, vec, k, nw,
                                                                   tile_rows):
    """Vertical band groups at the benchmark sizes: every interior row is stored by
    exactly one wavefront of each window, and a fast (unguarded) stream loads only
    rows in [0, rows) and computes only interior rows."""
    ow, strips, groups = _tb_geometry(rows, cols, vec, nw, k, tile_rows, vert=True)
    cover = {}
    for t, w, cw, r0, r1, up in _tb_waves(rows, cols, vec, nw, k, tile_rows, True):
        if cw // ow not in (0, 1, strips - 1):
            continue                     # windows are alike apart from the edge ones
        if r0 >= r1:
            continue
        cover.setdefault(cw, []).append((r0, r1))
        stream, fast = _tb_stream(rows, cols, vec, k, cw, r0, r1, up)
        lo = min(min(p) for p in stream)
        hi = max(max(p) for p in stream)
        if fast:
            assert 0 <= lo and hi < rows
            done_lo = lo + 1 if up else r0 - 2 * k      # rows the levels compute
            done_hi = r1 + 2 * k - 1 if up else hi - 1
            assert 1 <= done_lo and done_hi <= rows - 2
    for cw, spans in cover.items():
        spans.sort()
        assert spans[0][0] == 1 and spans[-1][1] == rows - 1
        assert all(a[1] == b[0] for a, b in zip(spans, spans[1:]))


# ---------------------------------------------------------------------------
# Temporally blocked Life kernel (life_tb_kernel): a launch advances K
# generations. Wavefront tile wt = t * NW + w covers band wt // strips and the
# 992-column window strip = wt % strips; lane l loads the 16 cells at column
# strip * 992 - 16 + 16 l (wrapped on a torus, zero outside a dead border) and
# lanes 1..62 store and count. Rows r0 - K .. r1 + K - 1 stream through K levels.
# The model replays that schedule word by word on the CPU (DPP lane shifts give
# zero at lanes 0 and 63) and checks every load and store address, that the
# stores cover the grid exactly once, and that the result and the per-level
# counts equal the oracle's K generations.
# ---------------------------------------------------------------------------
LIFE_TB_WIN = 992


def _c_rem(x, m):
    """C's % (truncating toward zero) followed by the kernel's wrap into [0, m)."""
    r = np.fmod(x, m)
    return np.where(r < 0, r + m, r)


def _life_tb_launch(buf, rows, cols, torus, k, tile_rows, nw, check_mask, lead=None, ragged=False):
    """ragged: rows (buf's width, a multiple of 16) end in padding past cols (zero at
    the start). On a torus, lanes inside the row load their word, the lane holding the
    row's end, the lane after it and the first window's left halo lane gather their
    cells from the wrapped columns, lanes further out load nothing."""
    lead = k if lead is None else lead   # rows streamed before and after the band
    words = buf.view(np.uint32)
    width = buf.shape[1]                  # bytes a row holds
    assert ragged or width == cols
    out = np.zeros_like(buf)
    writes = np.zeros((rows, width), np.int32)
    bad = []
    strips = -(-cols // LIFE_TB_WIN)
    bands = -(-rows // tile_rows)
    wave_tiles = strips * bands
    tiles = -(-wave_tiles // nw)
    counts = [0] * k
    lanes = np.arange(64)
    zero = np.zeros((64, 4), np.uint32)
    for t in range(tiles):
        for w in range(nw):
            wt = t * nw + w
            if wt >= wave_tiles:
                continue
            band, strip = divmod(wt, strips)
            col_raw = strip * LIFE_TB_WIN - 16 + lanes * 16
            in_cols = (col_raw >= 0) & (col_raw < cols)
            col = np.where(torus & ~in_cols, _c_rem(col_raw, cols), col_raw)
            loads = in_cols | bool(torus)
            rt = bool(torus) and ragged
            inside = (col_raw >= 0) & (col_raw + 16 <= cols)
            gather = rt & ~inside & (col_raw >= -16) & (col_raw < cols + 16)
            if rt:
                loads = inside
                col = col_raw
            own = (lanes >= 1) & (lanes <= 62) & (col_raw < cols)
            live = np.where(loads, np.uint32(0xFFFFFFFF), np.uint32(0))[:, None]
            inside = cols - col_raw[:, None] - 4 * np.arange(4)[None, :]   # cells of word m
            full = np.uint32(0xFFFFFFFF) if rt else live
            cmask = np.where(inside >= 4, full, np.where(
                inside <= 0, np.uint32(0),
                full >> (np.uint32(8) * (4 - np.clip(inside, 1, 3)).astype(np.uint32)))).astype(np.uint32)
            r0, r1 = band * tile_rows, min(band * tile_rows + tile_rows, rows)

            def load(r):
                if r < 0 or r >= rows:
                    if not torus:
                        return zero.copy()
                    r = int(_c_rem(r, rows))
                W = np.zeros((64, 4), np.uint32)
                if rt:
                    for ln in np.nonzero(gather)[0]:
                        cells = bytearray(16)
                        for q in range(16):
                            cc = int(col_raw[ln]) + q
                            assert -16 <= cc < cols + 32
                            cc %= cols
                            if not (0 <= r < rows and 0 <= cc < cols):
                                bad.append(("gather", t, w, ln, r, cc))
                                continue
                            cells[q] = buf[r, cc]
                        W[ln] = np.frombuffer(bytes(cells), np.uint32)
                for ln in np.nonzero(loads)[0]:
                    c = int(col[ln])
                    if not (0 <= r < rows and 0 <= c and c + 16 <= width and c % 16 == 0):
                        bad.append(("load", t, w, ln, r, c))
                        continue
                    W[ln] = words[r, c // 4:c // 4 + 4]
                return W

            up = [zero.copy() for _ in range(k)]
            mid = [zero.copy() for _ in range(k)]
            for i in range(r0 - lead, r1 + lead):
                cur = load(i)
                for lv in range(1, k + 1):
                    row = i - lv
                    V = (up[lv - 1] + mid[lv - 1] + cur).astype(np.uint32)
                    wv = np.concatenate([[0], V[:-1, 3]]).astype(np.uint32) >> np.uint32(24)
                    ev = np.concatenate([V[1:, 0], [0]]).astype(np.uint32) & np.uint32(0xFF)
                    o = np.zeros((64, 4), np.uint32)
                    for m in range(4):
                        prev = (V[:, m - 1] >> np.uint32(24)) if m > 0 else wv
                        nxt = (V[:, m + 1] & np.uint32(0xFF)) if m < 3 else ev
                        T = (((V[:, m] << np.uint32(8)) | prev) + V[:, m]
                             + ((V[:, m] >> np.uint32(8)) | (nxt << np.uint32(24)))).astype(np.uint32)
                        c = mid[lv - 1][:, m]
                        o[:, m] = _zero_bytes_hi(((T - c) | c) ^ np.uint32(0x03030303)) >> np.uint32(7)
                    in_rows = 0 <= row < rows
                    if ragged and not torus:
                        o &= cmask if in_rows else np.uint32(0)
                    elif not torus:
                        o &= live if in_rows else np.uint32(0)
                    if (check_mask >> (lv - 1)) & 1 and r0 <= row < r1:
                        oc = (o & cmask) if rt else o
                        counts[lv - 1] += int(np.unpackbits(oc[own].view(np.uint8)).sum())
                    up[lv - 1] = mid[lv - 1]
                    mid[lv - 1] = cur
                    cur = o
                row = i - k
                if r0 <= row < r1:
                    for ln in np.nonzero(own)[0]:
                        c = int(col_raw[ln])
                        if not (0 <= c and c + 16 <= width):
                            bad.append(("store", t, w, ln, row, c))
                            continue
                        out[row, c:c + 16] = cur[ln].view(np.uint8)
                        writes[row, c:c + 16] += 1
    return out, counts, writes, bad


@pytest.mark.parametrize("rows,cols,k,tile_rows", [
    (1, 16, 2, 64), (2, 32, 3, 8), (3, 48, 4, 4), (9, 64, 8, 4), (40, 1008, 4, 16),
    (37, 2000, 3, 8), (20, 992, 6, 64), (13, 1024, 2, 5), (29, 1040, 5, 7), (6, 16, 5, 2)])
@pytest.mark.parametrize("torus", [True, False])
def test_life_tb_model_matches_oracle(rows, cols, k, tile_rows, torus):
    import oracle as O
    from paper_1609_04567_amd import inputs as I
    a = I.life_input(rows, cols, seed=rows * 7 + cols + k)
    out, counts, writes, bad = _life_tb_launch(a.copy(), rows, cols, torus, k, tile_rows, 4,
                                               (1 << k) - 1)
    assert bad == []
    assert (writes == 1).all()
    bc = O.BC_TORUS if torus else O.BC_BOTTOM
    o, _ = O.life_run(a, bc=bc, cond=O.COND_NEVER, max_iter=k)
    assert np.array_equal(out, o)
    for lv in range(1, k + 1):
        _, ro = O.life_run(a, bc=bc, cond=O.COND_NEVER, max_iter=lv)
        assert counts[lv - 1] == ro.count, lv


@pytest.mark.parametrize("rows,cols,k,tile_rows", [
    (1, 5, 2, 64), (3, 17, 3, 2), (7, 31, 8, 4), (20, 1000, 4, 16), (13, 999, 8, 5),
    (9, 1009, 5, 3), (6, 2001, 6, 8)])
def test_life_tb_ragged_dead_border_model_matches_oracle(rows, cols, k, tile_rows):
    """Dead border, rows not a multiple of 16 cells (the batched fused family): the
    cells past cols stay dead at every level, are stored as zero and never counted;
    every access stays inside the padded rows."""
    import oracle as O
    from paper_1609_04567_amd import inputs as I
    a = I.life_input(rows, cols, seed=rows * 11 + cols + k)
    width = -(-cols // 16) * 16
    buf = np.zeros((rows, width), np.uint8)
    buf[:, :cols] = a
    out, counts, writes, bad = _life_tb_launch(buf, rows, cols, False, k, tile_rows, 4,
                                               (1 << k) - 1, ragged=True)
    assert bad == []
    assert (writes == 1).all()            # padding bytes are stored too, as zero
    assert not out[:, cols:].any()
    o, _ = O.life_run(a, bc=O.BC_BOTTOM, cond=O.COND_NEVER, max_iter=k)
    assert np.array_equal(out[:, :cols], o)
    for lv in range(1, k + 1):
        _, ro = O.life_run(a, bc=O.BC_BOTTOM, cond=O.COND_NEVER, max_iter=lv)
        assert counts[lv - 1] == ro.count, lv


@pytest.mark.parametrize("rows,cols,k,tile_rows", [
    (1, 5, 2, 64), (3, 17, 3, 2), (7, 31, 8, 4), (5, 1, 4, 2), (4, 2, 8, 3), (20, 1000, 4, 16),
    (13, 999, 8, 5), (9, 1009, 5, 3), (6, 2001, 6, 8), (11, 993, 8, 4), (8, 1983, 8, 8)])
def test_life_tb_ragged_torus_model_matches_oracle(rows, cols, k, tile_rows):
    """Torus, rows not a multiple of 16 cells (the batched fused family): the edge
    lanes' gathers read only cells of the grid, every cell is stored once, and the
    field and the counts of every level equal the oracle's."""
    import oracle as O
    from paper_1609_04567_amd import inputs as I
    a = I.life_input(rows, cols, seed=rows * 13 + cols + k)
    width = -(-cols // 16) * 16
    buf = np.zeros((rows, width), np.uint8)
    buf[:, :cols] = a
    out, counts, writes, bad = _life_tb_launch(buf, rows, cols, True, k, tile_rows, 4,
                                               (1 << k) - 1, ragged=True)
    assert bad == []
    assert (writes[:, :cols] == 1).all() and (writes[:, cols:] <= 1).all()
    o, _ = O.life_run(a, bc=O.BC_TORUS, cond=O.COND_NEVER, max_iter=k)
    assert np.array_equal(out[:, :cols], o)
    for lv in range(1, k + 1):
        _, ro = O.life_run(a, bc=O.BC_TORUS, cond=O.COND_NEVER, max_iter=lv)
        assert counts[lv - 1] == ro.count, lv


def test_life_tb_model_catches_a_short_halo():
    """A mistake planted in the model (one row less streamed before and after each
    band) must fail the comparison with the oracle, so the check is not vacuous."""
    import oracle as O
    from paper_1609_04567_amd import inputs as I
    rows, cols, k = 24, 48, 3
    a = I.life_input(rows, cols, seed=5)
    o, _ = O.life_run(a, bc=O.BC_TORUS, cond=O.COND_NEVER, max_iter=k)
    good, _, _, _ = _life_tb_launch(a.copy(), rows, cols, True, k, 8, 4, 0)
    assert np.array_equal(good, o)
    short, _, writes, _ = _life_tb_launch(a.copy(), rows, cols, True, k, 8, 4, 0, lead=k - 1)
    assert not np.array_equal(short, o)


@pytest.mark.parametrize("rows,cols,tile_rows", [(16384, 16384, 64), (4096, 4096, 64),
                                                 (1000, 160, 64), (8192, 992 * 3, 32)])
def test_life_tb_stores_tile_the_grid_at_full_size(rows, cols, tile_rows):
    """Owned windows x bands cover every cell exactly once; loaded columns stay in
    [0, cols - 16] after the wrap."""
    strips = -(-cols // LIFE_TB_WIN)
    bands = -(-rows // tile_rows)
    cover = np.zeros(cols, np.int32)
    lanes = np.arange(64)
    for strip in range(strips):
        col_raw = strip * LIFE_TB_WIN - 16 + lanes * 16
        own = (lanes >= 1) & (lanes <= 62) & (col_raw < cols)
        for c in col_raw[own]:
            cover[c:c + 16] += 1
        col = np.where((col_raw < 0) | (col_raw >= cols), _c_rem(col_raw, cols), col_raw)
        assert (col >= 0).all() and (col + 16 <= cols).all()
    assert (cover == 1).all()
    row_cover = np.zeros(rows, np.int32)
    for band in range(bands):
        row_cover[band * tile_rows:min(rows, band * tile_rows + tile_rows)] += 1
    assert (row_cover == 1).all()


# ---------------------------------------------------------------------------
# Small Life grids in LDS (batch_small_kernel, Life): rows of (cols + 3) // 4 + 2
# 32-bit words, byte 3 of word 0 and byte cols + 4 ghost copies of the row's last
# and first cells (torus; 0 on a dead border), cells at bytes 4 .. cols + 3. One
# thread per word 1 .. (cols + 3) // 4 of a row: column sums of three rows over
# words w-1 .. w+1, B3/S23 per byte, bytes past the last cell masked off. The
# model replays the word arithmetic with Python integers, checks every LDS index
# against the two buffers and compares generations with the oracle.
# ---------------------------------------------------------------------------

def _zero_bytes_hi(x):
    return ~(x + 0x7F7F7F7F) & 0x80808080 & 0xFFFFFFFF


def _small_life_model(a, torus, gens):
    rows, cols = a.shape
    wt = (cols + 3) // 4 + 2
    nw = (cols + 3) // 4
    lastb = cols + 3
    size = rows * wt * 4
    A = bytearray(size)
    for i in range(rows):
        A[i * wt * 4 + 4:i * wt * 4 + 4 + cols] = bytes(a[i])

    def ghosts(G):
        if torus:
            for i in range(rows):
                r = i * wt * 4
                assert r + cols + 4 < size
                first, last = G[r + 4], G[r + lastb]
                G[r + 3] = last
                G[r + cols + 4] = first

    def word(G, idx):
        assert 0 <= idx < rows * wt
        return int.from_bytes(G[4 * idx:4 * idx + 4], "little")

    ghosts(A)
    for _ in range(gens):
        B = bytearray(size)
        for i in range(rows):
            iu = i - 1 if i > 0 else (rows - 1 if torus else -1)
            idn = i + 1 if i + 1 < rows else (0 if torus else -1)
            for w in range(1, nw + 1):
                V = [word(A, i * wt + w + d) for d in (-1, 0, 1)]
                mid = V[1]
                for rr in (iu, idn):
                    if rr >= 0:
                        V = [v + word(A, rr * wt + w + d) for v, d in zip(V, (-1, 0, 1))]
                V0, V1, V2 = V
                T = ((((V1 << 8) & 0xFFFFFFFF) | (V0 >> 24)) + V1
                     + ((V1 >> 8) | ((V2 << 24) & 0xFFFFFFFF))) & 0xFFFFFFFF
                out = _zero_bytes_hi((((T - mid) & 0xFFFFFFFF) | mid) ^ 0x03030303) >> 7
                spare = 4 * w + 3 - lastb
                if spare > 0:
                    out &= 0xFFFFFFFF >> (8 * spare)
                B[4 * (i * wt + w):4 * (i * wt + w) + 4] = out.to_bytes(4, "little")
        ghosts(B)
        A = B
    return np.array([[A[i * wt * 4 + 4 + j] for j in range(cols)] for i in range(rows)],
                    dtype=np.uint8)


@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 6), (2, 2), (3, 5), (6, 1), (7, 13), (9, 16),
                                       (11, 22), (5, 31)])
@pytest.mark.parametrize("torus", [True, False])
def test_small_life_lds_model_matches_oracle(rows, cols, torus):
    import oracle as O
    from paper_1609_04567_amd import inputs as I
    a = I.life_input(rows, cols, seed=rows * 100 + cols, density=0.45)
    gens = 6
    got = _small_life_model(a, torus, gens)
    o, _ = O.life_run(a, bc=O.BC_TORUS if torus else O.BC_BOTTOM, cond=O.COND_NEVER,
                      max_iter=gens)
    assert np.array_equal(got, o)
