// Device side of the temporally blocked Game of Life (K generations per
// launch, Sect. 3.1's loop body applied K times between two reads of the grid):
// the per-wavefront band shared by the fused Life kernel and the batched
// engine's fused Life family.
//
// A wavefront owns a window of 992 columns (lanes 1..62, 16 cells per lane held
// as four 32-bit words, one byte per cell) and a band of rows. It loads 1024
// columns: lanes 0 and 63 are halo lanes whose cells are computed but never
// stored or counted. A lane's edge bytes take the neighbouring lane's column sum
// by a DPP lane shift; at lanes 0 and 63 that shift brings in zero, so their
// outer cells go wrong, but the error moves inward by one cell per generation
// and does not leave the 16 cells of a halo lane for K <= 16.
// Rows stream through a register pipeline of K levels: level l holds its input
// rows (the output of level l - 1) i - l - 1 and i - l, and computes row i - l of
// generation n + l from them and the row level l - 1 produced in the same step.
// Neighbouring bands overlap by K rows, so every stored cell of generation n + K
// is computed from exactly the cells of generation n a plain sweep chain would
// read. A torus wraps rows and columns (any size, also below one window);
// outside cells of a dead border are zero at every level.
//
// Requirements: 16-byte aligned rows holding a multiple of 16 cells, no
// padding; the cells hold 0 or 1.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "tile_life.hpp"   // zero_bytes_hi

namespace lsr {

constexpr int kLifeTbWinLanes = 62;               // lanes of a window that are stored
constexpr int kLifeTbWinCols = kLifeTbWinLanes * 16;    // 992 columns per wavefront

namespace life_tb_detail {

constexpr int kDppShr1 = 0x138;   // wave_shr:1, lane l receives lane l-1 (lane 0 gets 0)
constexpr int kDppShl1 = 0x130;   // wave_shl:1, lane l receives lane l+1 (lane 63 gets 0)

template <int CTRL>
__device__ __forceinline__ uint32_t lane_shift_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, true);
}

// One generation of 16 cells from the byte-wise column sums V of the lane's
// rows i-1, i, i+1 and its centre row c (bytes 0/1). With T the 3x3 total,
// B3/S23 is (T - c | c) == 3.
__device__ __forceinline__ void life_rule16(const uint32_t (&V)[4], const uint32_t (&c)[4],
                                            uint32_t (&out)[4]) {
    const uint32_t wv = lane_shift_u32<kDppShr1>(V[3]) >> 24;
    const uint32_t ev = lane_shift_u32<kDppShl1>(V[0]) & 0xFFu;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint32_t prev = (m > 0) ? (V[m - 1] >> 24) : wv;
        const uint32_t next = (m < 3) ? (V[m + 1] & 0xFFu) : ev;
        const uint32_t T = ((V[m] << 8) | prev) + V[m] + ((V[m] >> 8) | (next << 24));
        out[m] = zero_bytes_hi(((T - c[m]) | c[m]) ^ 0x03030303u) >> 7;
    }
}

}  // namespace life_tb_detail

// One wavefront of a K-generation launch: window `strip` (992 stored columns)
// and band `band` (tile_rows rows, the last one shorter). Loads generation n,
// stores generation n + K, and adds the live cells it owns of every checked
// generation n + l (check_mask bit l - 1) to the lane's cnt[l - 1].
// RAGGED: rows hold round_up(cols, 16) bytes and cols need not be a multiple of
// 16. On a dead border the bytes past cols start at zero and the lane holding the
// last cell masks them at every level, so they stay dead, are never counted and
// are stored as zero. On a torus, lanes whose 16 cells lie inside the row load
// them as a word; the lane holding the row's end, the lane after it and the left
// halo lane of the first window gather their cells byte by byte from the wrapped
// columns (a row read as its periodic extension); lanes further out load nothing,
// as no cell they feed lies within K of a stored one. The bytes past cols of the
// last lane are counted out, and stored into the padding (0 or 1, never read).
template <int K, int U, bool TORUS, bool RAGGED = false>
__device__ __forceinline__ void life_tb_band(const uint8_t* a, uint8_t* b,
                                             int64_t rows, int64_t cols, int64_t pitch, uint32_t mask,
                                             int band, int strip, int tile_rows, uint32_t (&cnt)[K]) {
    static_assert(K >= 2 && K <= 16, "halo lanes cover at most 16 generations");
    using namespace life_tb_detail;
    const int lane = threadIdx.x & 63;
    const int64_t col_raw = (int64_t)strip * kLifeTbWinCols - 16 + (int64_t)lane * 16;
    const bool in_cols = col_raw >= 0 && col_raw < cols;
    int64_t col = col_raw;
    if (TORUS && !RAGGED && !in_cols) {
        col %= cols;
        if (col < 0) col += cols;
    }
    constexpr bool RT = TORUS && RAGGED;
    const bool inside = col_raw >= 0 && col_raw + 16 <= cols;
    const bool gather = RT && !inside && col_raw >= -16 && col_raw < cols + 16;
    const bool loads = RT ? inside : TORUS || in_cols;
    const uint32_t own = (lane >= 1 && lane <= kLifeTbWinLanes && col_raw < cols) ? 0xFFFFFFFFu : 0u;
    const uint32_t live = loads ? 0xFFFFFFFFu : 0u;   // dead columns of a dead border
    uint32_t cmask[4];   // RAGGED: bytes of the lane's word m that hold cells
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int64_t in = cols - col_raw - 4 * m;   // cells of word m inside the grid
        const uint32_t full = RT ? 0xFFFFFFFFu : live;
        cmask[m] = !RAGGED || in >= 4 ? full : in <= 0 ? 0u : full >> (8 * (4 - (int)in));
    }
    const int64_t r0 = (int64_t)band * tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, rows);
    const int64_t i_beg = r0 - K, i_end = r1 + K;

    // rows i0 .. i0 + U - 1 of generation n (those below i_end), zero outside a dead border
    auto load_group = [&](int64_t i0, uint32_t (&w)[U][4]) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            w[k][0] = w[k][1] = w[k][2] = w[k][3] = 0;
            int64_t r = i0 + k;
            if (r >= i_end) continue;
            if (r < 0 || r >= rows) {
                if (!TORUS) continue;
                r %= rows;
                if (r < 0) r += rows;
            }
            if (RT && gather) {
                const uint8_t* row = a + r * pitch;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    int64_t cc = col_raw + q;   // in [-16, cols + 31)
                    while (cc < 0) cc += cols;
                    while (cc >= cols) cc -= cols;
                    w[k][q >> 2] |= (uint32_t)row[cc] << (8 * (q & 3));
                }
                continue;
            }
            if (!loads) continue;
            const uint4 x = *reinterpret_cast<const uint4*>(a + r * pitch + col);
            w[k][0] = x.x;
            w[k][1] = x.y;
            w[k][2] = x.z;
            w[k][3] = x.w;
        }
    };

    // R[l][s]: the last three rows of level l (l = 0: the loaded rows of generation
    // n), in slots by row phase: at step i (phase P = (i - i_beg) mod 3) level l
    // writes its row into slot P and level l + 1 reads rows i-l-2, i-l-1, i-l
    // from slots P+1, P+2, P (mod 3). Steps go in groups of three, so slot
    // numbers are compile-time constants and rows never move between registers.
    uint32_t R[K][3][4];
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int m = 0; m < 4; ++m) R[l][q][m] = 0;

    // the K levels of step i (input row i of generation n), then the store of row i - K
    auto step = [&](auto phase, int64_t i, const uint32_t (&row_in)[4]) {
        constexpr int P = decltype(phase)::value, PU = (P + 1) % 3, PM = (P + 2) % 3;
#pragma unroll
        for (int m = 0; m < 4; ++m) R[0][P][m] = row_in[m];
        uint32_t out[4];
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const int64_t row = i - l;   // row of generation n + l computed here
            const uint32_t(&src)[3][4] = R[l - 1];
            uint32_t V[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) V[m] = src[PU][m] + src[PM][m] + src[P][m];
            life_rule16(V, src[PM], out);
            if (RAGGED && !TORUS) {
                const bool in_rows = row >= 0 && row < rows;
#pragma unroll
                for (int m = 0; m < 4; ++m) out[m] &= in_rows ? cmask[m] : 0u;
            } else if (!TORUS) {
                const uint32_t lv = (row >= 0 && row < rows) ? live : 0u;
#pragma unroll
                for (int m = 0; m < 4; ++m) out[m] &= lv;
            }
            if (((mask >> (l - 1)) & 1u) && row >= r0 && row < r1)
                cnt[l - 1] += (uint32_t)(__popc(RT ? out[0] & cmask[0] : out[0]) +
                                         __popc(RT ? out[1] & cmask[1] : out[1]) +
                                         __popc(RT ? out[2] & cmask[2] : out[2]) +
                                         __popc(RT ? out[3] & cmask[3] : out[3])) & own;
            if (l < K) {
#pragma unroll
                for (int m = 0; m < 4; ++m) R[l][P][m] = out[m];
            }
        }
        const int64_t row = i - K;
        if (row >= r0 && row < r1 && own) {
            typedef uint32_t W4 __attribute__((ext_vector_type(4)));
            W4 o;
            o[0] = out[0];
            o[1] = out[1];
            o[2] = out[2];
            o[3] = out[3];
            __builtin_nontemporal_store(o, reinterpret_cast<W4*>(b + row * pitch + col_raw));
        }
    };
    static_assert(U == 3, "a load group is one rotation of the row slots");
    auto process_group = [&](int64_t i0, const uint32_t (&w)[U][4]) {
        step(std::integral_constant<int, 0>{}, i0, w[0]);
        if (i0 + 1 >= i_end) return;
        step(std::integral_constant<int, 1>{}, i0 + 1, w[1]);
        if (i0 + 2 >= i_end) return;
        step(std::integral_constant<int, 2>{}, i0 + 2, w[2]);
    };

    uint32_t ga[U][4], gb[U][4];
    load_group(i_beg, ga);
    for (int64_t i0 = i_beg; i0 < i_end; i0 += 2 * U) {
        load_group(i0 + U, gb);
        process_group(i0, ga);
        if (i0 + U >= i_end) break;
        load_group(i0 + 2 * U, ga);
        process_group(i0 + U, gb);
    }
}

}  // namespace lsr
