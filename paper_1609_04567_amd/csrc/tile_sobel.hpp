// Sobel edge detector (Sect. 4.2): the per-wavefront tile shared by the plain
// sweep kernel and the batched engine. Each output pixel is the integer gradient
// magnitude floor(sqrt(Gx^2 + Gy^2)) clamped to 255, Gx and Gy the 3x3 Sobel
// derivative masks, samples outside the image 0 (the bottom value, as in Fig. 1).
#pragma once

#include "common.hpp"

namespace lsr {

constexpr int kSobelRows = 8;                     // output rows of a wavefront tile
constexpr int kSobelCols = 256;                   // output columns (4 per lane)
constexpr int kSobelLdsRow = kSobelCols + 8;      // bytes per staged row: 4 halo columns a side
constexpr int kSobelLdsBytes = (kSobelRows + 2) * kSobelLdsRow;

// floor(sqrt(m)) exactly for 0 <= m < 2^24: the float conversion is exact and the
// hardware square root is within one unit of the integer answer, which the two
// corrections settle.
__device__ __forceinline__ int isqrt_small(int m) {
    int s = (int)__builtin_sqrtf((float)m);
    s -= (s * s > m);
    s += ((s + 1) * (s + 1) <= m);
    return s;
}

// One wavefront: output rows row0 .. row0+7 (those below rows), columns col0 ..
// col0+255 (those below cols). The input rows row0-1 .. row0+8 and columns col0-4
// .. col0+259 are staged in `lds` (kSobelLdsBytes, this wavefront's own), zero
// outside the image. Returns the lane's sum of the values it wrote.
__device__ __forceinline__ unsigned long long sobel_wave(const uint8_t* __restrict__ a,
                                                         uint8_t* __restrict__ b, int64_t rows,
                                                         int64_t cols, int64_t pitch, int64_t row0,
                                                         int64_t col0, uint8_t* lds) {
    const int lane = threadIdx.x & 63;
    const bool words = ((reinterpret_cast<uintptr_t>(a) | (uintptr_t)pitch | (uintptr_t)col0) & 3) == 0;
    constexpr int kChunks = kSobelLdsRow / 4;   // 4-byte chunks per staged row
    for (int k = lane; k < (kSobelRows + 2) * kChunks; k += 64) {
        const int r = k / kChunks, q = k - r * kChunks;
        const int64_t i = row0 - 1 + r, j = col0 - 4 + 4 * q;
        uint32_t v = 0;
        if (i >= 0 && i < rows) {
            const uint8_t* p = a + i * pitch;
            if (words && j >= 0 && j + 3 < cols) {
                v = *reinterpret_cast<const uint32_t*>(p + j);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (j + e >= 0 && j + e < cols) v |= (uint32_t)p[j + e] << (8 * e);
            }
        }
        *reinterpret_cast<uint32_t*>(lds + r * kSobelLdsRow + 4 * q) = v;
    }
    // the staged rows are this wavefront's own: its own ordering suffices
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    unsigned long long acc = 0;
    const int c0 = 4 + 4 * lane;   // staged column of the lane's first pixel
    const int64_t j0 = col0 + 4 * lane;
    for (int rr = 0; rr < kSobelRows; ++rr) {
        const int64_t i = row0 + rr;
        if (i >= rows) break;
        int px[3][6];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint8_t* L = lds + (rr + d) * kSobelLdsRow + c0 - 1;
#pragma unroll
            for (int e = 0; e < 6; ++e) px[d][e] = L[e];
        }
        uint32_t packed = 0;
        int out[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int nw = px[0][e], n = px[0][e + 1], ne = px[0][e + 2];
            const int w = px[1][e], ea = px[1][e + 2];
            const int sw = px[2][e], s = px[2][e + 1], se = px[2][e + 2];
            const int gx = (ne + 2 * ea + se) - (nw + 2 * w + sw);
            const int gy = (sw + 2 * s + se) - (nw + 2 * n + ne);
            const int m = isqrt_small(gx * gx + gy * gy);
            out[e] = m > 255 ? 255 : m;
            packed |= (uint32_t)out[e] << (8 * e);
        }
        uint8_t* q = b + i * pitch;
        const bool wstore = ((reinterpret_cast<uintptr_t>(b) | (uintptr_t)pitch) & 3) == 0;
        if (wstore && j0 + 3 < cols) {
            *reinterpret_cast<uint32_t*>(q + j0) = packed;
            acc += (unsigned long long)(out[0] + out[1] + out[2] + out[3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (j0 + e < cols) {
                    q[j0 + e] = (uint8_t)out[e];
                    acc += (unsigned long long)out[e];
                }
        }
    }
    return acc;
}

}  // namespace lsr
