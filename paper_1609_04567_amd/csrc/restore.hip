// Two-phase impulse-noise restoration (Sect. 4.3).
//
// Phase 1, adaptive-median detection (integer, one shot). A 16x16 workgroup
// stages its pixels plus a halo of w_max/2 in LDS. Each thread grows its window
// w = 3, 5, ..., w_max over the in-range pixels only. A full 3x3, 5x5 or 7x7
// window goes through a comparator network (select_networks.hpp) that leaves its min,
// lower median (rank (count-1)/2) and max in known registers; any other window
// finds min and max in one pass and the lower median by a radix select: the
// largest v with #{x < v} <= rank, decided two bits at a time from the top (four
// passes over the window). The first window with min < med < max decides the flag
// !(min < y < max); otherwise the w_max window decides (y == min || y == max).
// Output: mask (0/1) and the initial iterate (med where flagged, y elsewhere).
//
// Phase 2, restoration sweep. Each flagged pixel takes the minimiser of
// sum_m phi(t - u_m) over its in-range 8-neighbourhood, phi(t) = sqrt(beta+t^2)
// (or t^2), reading only the previous iterate. The minimiser is the root of the
// strictly increasing g(t) = sum (t - v)/sqrt(beta + (t - v)^2) inside
// [min v, max v]; it is found by Newton steps kept inside a shrinking bracket
// (a step that leaves the bracket is replaced by its midpoint). Unflagged pixels
// are never written: both ping-pong buffers hold them from the start.
#include "kernels.hpp"
#include "select_networks.hpp"
#include "tile_restore.hpp"

namespace lsr {
namespace {

constexpr int kAmfTile = 16;

__global__ __launch_bounds__(kAmfTile * kAmfTile) void amf_detect_kernel(
    const uint8_t* __restrict__ y, int64_t rows, int64_t cols, int64_t pitch, int w_max,
    uint8_t* __restrict__ mask, void* __restrict__ u_init, int u_dtype) {
    extern __shared__ uint8_t tile[];
    const int K = w_max / 2;
    const int TW = kAmfTile + 2 * K;
    const int64_t gi0 = (int64_t)blockIdx.y * kAmfTile - K;
    const int64_t gj0 = (int64_t)blockIdx.x * kAmfTile - K;
    for (int idx = threadIdx.y * kAmfTile + threadIdx.x; idx < TW * TW; idx += kAmfTile * kAmfTile) {
        const int ti = idx / TW, tj = idx - ti * TW;
        const int64_t gi = gi0 + ti, gj = gj0 + tj;
        tile[idx] = (gi >= 0 && gi < rows && gj >= 0 && gj < cols) ? y[gi * pitch + gj] : 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.y * kAmfTile + threadIdx.y;
    const int64_t jx = (int64_t)blockIdx.x * kAmfTile + threadIdx.x;
    if (i >= rows || jx >= cols) return;
    const int ci = threadIdx.y + K, cj = threadIdx.x + K;
    const int yv = tile[ci * TW + cj];
    int lo = 0, hi = 0, med = 0, flag = 0;
    bool decided = false;
    // full 3x3, 5x5 and 7x7 windows (most pixels decide in one of them): minimum,
    // lower median and maximum by comparator networks on registers; windows
    // clipped by the border and larger ones by the radix select below
    int w0 = 3;
    if (i >= 1 && i + 1 < rows && jx >= 1 && jx + 1 < cols) {
        int v[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) v[a * 3 + b] = tile[(ci - 1 + a) * TW + cj - 1 + b];
        select9(v);
        lo = v[kSel9Min];
        med = v[kSel9Med];
        hi = v[kSel9Max];
        if (lo < med && med < hi) {
            flag = !(lo < yv && yv < hi);
            decided = true;
        }
        w0 = 5;
        if (!decided && w_max >= 5 && i >= 2 && i + 2 < rows && jx >= 2 && jx + 2 < cols) {
            int u[25];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b) u[a * 5 + b] = tile[(ci - 2 + a) * TW + cj - 2 + b];
            select25(u);
            lo = u[kSel25Min];
            med = u[kSel25Med];
            hi = u[kSel25Max];
            if (lo < med && med < hi) {
                flag = !(lo < yv && yv < hi);
                decided = true;
            }
            w0 = 7;
            if (!decided && w_max >= 7 && i >= 3 && i + 3 < rows && jx >= 3 && jx + 3 < cols) {
                int x[49];
#pragma unroll
                for (int a = 0; a < 7; ++a)
#pragma unroll
                    for (int b = 0; b < 7; ++b) x[a * 7 + b] = tile[(ci - 3 + a) * TW + cj - 3 + b];
                select49(x);
                lo = x[kSel49Min];
                med = x[kSel49Med];
                hi = x[kSel49Max];
                if (lo < med && med < hi) {
                    flag = !(lo < yv && yv < hi);
                    decided = true;
                }
                w0 = 9;
            }
        }
    }
    for (int w = w0; w <= w_max && !decided; w += 2) {
        const int k = w / 2;
        // in-range part of the w x w box, in tile coordinates
        const int ia = ci - (int)min<int64_t>(k, i), ib = ci + (int)min<int64_t>(k, rows - 1 - i);
        const int ja = cj - (int)min<int64_t>(k, jx), jb = cj + (int)min<int64_t>(k, cols - 1 - jx);
        const int cnt = (ib - ia + 1) * (jb - ja + 1);
        lo = 255;
        hi = 0;
        for (int a = ia; a <= ib; ++a)
            for (int b = ja; b <= jb; ++b) {
                const int v = tile[a * TW + b];
                lo = min(lo, v);
                hi = max(hi, v);
            }
        const int rank = (cnt - 1) / 2;
        // two bits per pass: of the candidates med | d << bit (d = 1, 2, 3), whose
        // counts below grow with d, keep the largest with at most `rank` below
        // (the same choice as two one-bit steps, with half the window reads)
        med = 0;
        for (int bit = 6; bit >= 0; bit -= 2) {
            const int c1 = med | (1 << bit), c2 = med | (2 << bit), c3 = med | (3 << bit);
            int b1 = 0, b2 = 0, b3 = 0;
            for (int a = ia; a <= ib; ++a)
                for (int b = ja; b <= jb; ++b) {
                    const int v = tile[a * TW + b];
                    b1 += v < c1;
                    b2 += v < c2;
                    b3 += v < c3;
                }
            med = b3 <= rank ? c3 : b2 <= rank ? c2 : b1 <= rank ? c1 : med;
        }
        if (lo < med && med < hi) {
            flag = !(lo < yv && yv < hi);
            decided = true;
        }
    }
    if (!decided) flag = (yv == lo || yv == hi);
    const int64_t p = i * pitch + jx;
    mask[p] = (uint8_t)flag;
    const int u = flag ? med : yv;
    if (u_dtype == 1) static_cast<uint8_t*>(u_init)[p] = (uint8_t)u;
    else if (u_dtype == 4) static_cast<float*>(u_init)[p] = (float)u;
    else static_cast<double*>(u_init)[p] = (double)u;
}

template <typename T, int TR>
__global__ __launch_bounds__(256) void restore_kernel(
    const T* __restrict__ a, T* __restrict__ b, const uint8_t* __restrict__ mask, int64_t rows,
    int64_t cols, int64_t pitch, T beta, int quadratic, JobState* __restrict__ st,
    double* __restrict__ partials, LoopCtl ctl, int j, int strips, int tiles) {
    __shared__ double lds[4];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    const int band = t / strips, strip = t - band * strips;
    const int ly = threadIdx.x >> 6;
    const bool is_max = ctl.reduce == RED_MAX_ABS;
    // wavefront ly owns rows ly, ly + 4, ... of the band
    __shared__ uint16_t list[4][TR / 4 * 64];
    const double acc = restore_wave<T, true>(a, b, mask, rows, cols, pitch, beta, quadratic != 0,
                                             (int64_t)band * TR, ly, 4, TR, (int64_t)strip * 64,
                                             list[ly], check, is_max);
    if (check) {
        const double s = block_reduce<4>(acc, is_max, lds);
        if (threadIdx.x == 0) partials[t] = s;
    }
}

constexpr int kRestoreRows = 16;

}  // namespace

SweepGeom restore_geom(const RestoreArgs& a, int tile_rows) {
    (void)tile_rows;
    SweepGeom g;
    g.vec = 1;
    g.waves = 4;
    g.tile_rows = kRestoreRows;
    g.strips = (int)((a.cols + 63) / 64);
    g.bands = (int)((a.rows + kRestoreRows - 1) / kRestoreRows);
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_restore(const RestoreArgs& a, const SweepGeom& g, JobState* st, void* partials,
                          const LoopCtl& c, int j, hipStream_t s) {
    double* parts = static_cast<double*>(partials);
    if (a.f32) {
        hipLaunchKernelGGL((restore_kernel<float, kRestoreRows>), dim3(g.blocks), dim3(256), 0, s,
                           static_cast<const float*>(a.a), static_cast<float*>(a.b), a.mask, a.rows,
                           a.cols, a.pitch, (float)a.beta, a.quadratic, st, parts, c, j, g.strips,
                           g.tiles);
    } else {
        hipLaunchKernelGGL((restore_kernel<double, kRestoreRows>), dim3(g.blocks), dim3(256), 0, s,
                           static_cast<const double*>(a.a), static_cast<double*>(a.b), a.mask,
                           a.rows, a.cols, a.pitch, a.beta, a.quadratic, st, parts, c, j, g.strips,
                           g.tiles);
    }
    return hipGetLastError();
}

hipError_t launch_amf_detect(const uint8_t* y, int64_t rows, int64_t cols, int64_t pitch,
                             int w_max, uint8_t* mask, void* u_init, int u_dtype, hipStream_t s) {
    const int K = w_max / 2;
    const int TW = kAmfTile + 2 * K;
    dim3 grid((unsigned)((cols + kAmfTile - 1) / kAmfTile), (unsigned)((rows + kAmfTile - 1) / kAmfTile));
    hipLaunchKernelGGL(amf_detect_kernel, grid, dim3(kAmfTile, kAmfTile), TW * TW, s, y, rows, cols,
                       pitch, w_max, mask, u_init, u_dtype);
    return hipGetLastError();
}

}  // namespace lsr
