// Tile bodies of the Game of Life B3/S23 sweep (the elemental function of the
// paper's Fig. 1) with the live-cell count fused in. Shared by the single-job
// kernels (life.hip) and the batched kernel (batch.hip).
//
// SWAR tile (16-byte aligned rows of a multiple of 16 bytes, see below for other
// widths): each lane owns 16 consecutive cells held as four 32-bit words, one byte per
// cell. Per row it forms the byte-wise column sums V = up + mid + down (<= 3 per
// byte, no carries), shifts V by one byte left and right (the missing edge
// bytes come from the neighbouring lanes by cross-lane shuffles, or from a halo
// byte loaded by the wavefront's edge lanes), and adds the three to get the 3x3
// total T (<= 9). With the neighbour count being T - centre, the rule is
//   alive' = (T == 3) || (T == 4 && alive)
// evaluated on four bytes at once with a zero-byte test. The new word's
// popcount is the cell count. Wavefronts stream down `tile_rows` rows.
//
// The tile expects cells of 0 or 1: the job's initial live-count pass rewrites
// any other non-zero byte as 1 (a cell is alive iff its byte is non-zero).
// Boundaries: torus wraps rows and columns; bottom treats outside cells as dead.
#pragma once

#include "common.hpp"

namespace lsr {

__device__ __forceinline__ uint32_t zero_bytes_hi(uint32_t x) {
    // 0x80 in every byte equal to zero, for byte values below 0x80
    return ~(x + 0x7F7F7F7Fu) & 0x80808080u;
}

// Tile t (band-major over `strips` strips of NW*1024 columns); NW*64 threads.
// Cells must hold 0 or 1 (the job's first pass normalises the input in place).
// With count = T - centre, B3/S23 is exactly (count | centre) == 3: a dead cell
// is born on 3, a live one survives on 2 or 3.
// Rows must be 16-byte aligned and hold round_up(cols, 16) bytes, the bytes
// past cols starting at zero. When cols is not a multiple of 16 the last lane
// with cells owns q < 16 of them: the byte after its last cell takes the east
// neighbour's column sum, and the cells past cols are computed (0 or 1, so no
// byte sum carries into the next) and stored into the padding but neither
// counted nor read as anyone's neighbour.
// WT (wavefront tile): the calling wavefront alone owns tile t (NW must be 1)
// and reduces its count by itself; lane 0 writes the partial.
template <int NW, int U, bool NT, bool WT = false>
__device__ __forceinline__ void life_swar_tile(const uint8_t* __restrict__ a, uint8_t* __restrict__ b,
                                               int64_t rows, int64_t cols, int64_t pitch, int torus,
                                               bool check, int t, int strips, int tile_rows,
                                               unsigned long long* __restrict__ partials,
                                               unsigned long long* lds) {
    static_assert(!WT || NW == 1, "a wavefront tile has one wavefront");
    const int band = t / strips, strip = t - band * strips;
    const int lane = threadIdx.x & 63, wave = WT ? 0 : threadIdx.x >> 6;
    const int64_t cw = (int64_t)strip * (NW * 1024) + (int64_t)wave * 1024;
    const int64_t c = cw + (int64_t)lane * 16;
    const bool active = c < cols;
    int nact = 0;   // lanes of this wavefront that own cells
    if (cw < cols) nact = (int)min<int64_t>(64, (cols - cw + 15) / 16);
    const int last = nact - 1;
    const int q = active ? (int)min<int64_t>(16, cols - c) : 0;   // cells of this lane
    const bool part = q > 0 && q < 16;                            // only lane `last`
    int64_t wcol = cw - 1, ecol = min(cw + (int64_t)nact * 16, cols);
    bool has_w = (lane == 0) && nact > 0, has_e = (lane == last) && nact > 0;
    if (wcol < 0) { if (torus) wcol += cols; else has_w = false; }
    if (ecol >= cols) { if (torus) ecol -= cols; else has_e = false; }
    // count mask (0x80 per counted cell) of each word
    uint32_t cm[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int k = q - 4 * m;   // cells of this lane in word m
        cm[m] = k >= 4 ? 0x80808080u : k <= 0 ? 0u : (0x80808080u & ((1u << (8 * k)) - 1u));
    }

    const int64_t r0 = (int64_t)band * tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, rows);

    // rows r0-1 .. r1 are touched, so one step of wrap is enough on a torus;
    // outside rows of a bottom boundary are dead (all zero)
    auto load = [&](int64_t r, uint32_t (&w)[4], uint32_t& hw, uint32_t& he) {
        w[0] = w[1] = w[2] = w[3] = 0;
        hw = he = 0;
        if (r < 0) {
            if (!torus) return;
            r += rows;
        } else if (r >= rows) {
            if (!torus) return;
            r -= rows;
        }
        const uint8_t* p = a + r * pitch;
        if (active) {
            const uint4 x = *reinterpret_cast<const uint4*>(p + c);
            w[0] = x.x;
            w[1] = x.y;
            w[2] = x.z;
            w[3] = x.w;
        }
        if (has_w) hw = p[wcol];
        if (has_e) he = p[ecol];
    };

    uint32_t up[4], mid[4], up_w, up_e, mid_w, mid_e;
    load(r0 - 1, up, up_w, up_e);
    load(r0, mid, mid_w, mid_e);
    unsigned long long cnt = 0;

    for (int64_t r = r0; r < r1; r += U) {
        uint32_t dn[U][4], dn_w[U], dn_e[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (r + k < r1) load(r + k + 1, dn[k], dn_w[k], dn_e[k]);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (r + k < r1) {
                uint32_t V[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) V[m] = up[m] + mid[m] + dn[k][m];
                const uint32_t vw_h = up_w + mid_w + dn_w[k];
                const uint32_t ve_h = up_e + mid_e + dn_e[k];
                uint32_t wv = __shfl_up(V[3], 1, 64) >> 24;
                uint32_t ev = __shfl_down(V[0], 1, 64) & 0xFFu;
                if (lane == 0) wv = vw_h;
                if (lane == last) ev = ve_h;
                if (part) {
                    // the east neighbour of the last cell is byte q of this lane
                    const int sh = (q & 3) * 8;
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        if (m == (q >> 2)) V[m] = (V[m] & ~(0xFFu << sh)) | (ve_h << sh);
                }
                uint32_t out[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint32_t prev = (m > 0) ? (V[m - 1] >> 24) : wv;
                    const uint32_t next = (m < 3) ? (V[m + 1] & 0xFFu) : ev;
                    const uint32_t T = ((V[m] << 8) | prev) + V[m] + ((V[m] >> 8) | (next << 24));
                    const uint32_t alive = zero_bytes_hi(((T - mid[m]) | mid[m]) ^ 0x03030303u);
                    out[m] = alive >> 7;
                    cnt += (unsigned)__popc(alive & cm[m]);
                }
                if (active) {
                    typedef uint32_t W4 __attribute__((ext_vector_type(4)));
                    W4 o;
                    o[0] = out[0];
                    o[1] = out[1];
                    o[2] = out[2];
                    o[3] = out[3];
                    W4* dst = reinterpret_cast<W4*>(b + (r + k) * pitch + c);
                    if (NT) __builtin_nontemporal_store(o, dst);
                    else *dst = o;
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) { up[m] = mid[m]; mid[m] = dn[k][m]; }
                up_w = mid_w; up_e = mid_e;
                mid_w = dn_w[k]; mid_e = dn_e[k];
            }
        }
    }
    if (check) {
        if (WT) {
            const unsigned long long v = wave_sum_u64(cnt);
            if (lane == 0) partials[t] = v;
        } else {
            const unsigned long long v = block_reduce_u64<NW>(cnt, lds);
            if (threadIdx.x == 0) partials[t] = v;
        }
    }
}

}  // namespace lsr
