// The generic forms of the pattern beyond the 5-point neighbourhood (Sect. 3.1):
//  * radius-k box stencil (sigma_k, k = 1..4): each cell at least k from the edge
//    takes the mean of its (2k+1) x (2k+1) neighbourhood; the band of width k at
//    the edge is fixed. A workgroup stages a 32 x 64 output tile plus its k-wide
//    halo in LDS; each thread sums its boxes in the fixed order (each box row left
//    to right, the row sums top to bottom) and divides once by (2k+1)^2.
//  * 3D 7-point Jacobi (Laplace) on nz planes of ny rows stored plane after plane:
//    b = (((W+E) + (N+S)) + (U+D)) / 6 inside, faces fixed. A thread owns one (y, x)
//    column of a 64 x 4 tile and walks 16 planes keeping the planes below, at and
//    above in registers; N/S/W/E come from neighbouring threads' loads through the
//    caches.
// Both fuse the delta reduce (max, sum of squares or sum of |b - a|) on a check
// sweep into one partial per workgroup.
#include "kernels.hpp"
#include "tile_jacobi.hpp"

namespace lsr {
namespace {

constexpr int kBoxRows = 32, kBoxCols = 64;

template <typename T, int K>
__global__ __launch_bounds__(256) void box_kernel(const T* __restrict__ a, T* __restrict__ b,
                                                  int64_t rows, int64_t cols, int64_t pitch,
                                                  JobState* __restrict__ st,
                                                  double* __restrict__ partials, LoopCtl ctl, int j,
                                                  int strips, int tiles) {
    constexpr int TW = kBoxCols + 2 * K, TH = kBoxRows + 2 * K;
    __shared__ T tile[TH * TW];
    __shared__ double lds[4];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    const int band = t / strips, strip = t - band * strips;
    const int64_t r0 = (int64_t)band * kBoxRows, c0 = (int64_t)strip * kBoxCols;
    for (int idx = threadIdx.x; idx < TH * TW; idx += 256) {
        const int ti = idx / TW, tj = idx - ti * TW;
        const int64_t gi = r0 - K + ti, gj = c0 - K + tj;
        tile[idx] = (gi >= 0 && gi < rows && gj >= 0 && gj < cols) ? a[gi * pitch + gj] : T(0);
    }
    __syncthreads();
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const T cnt = T((2 * K + 1) * (2 * K + 1));
    double acc = 0.0;
    for (int rr = ty * (kBoxRows / 4); rr < (ty + 1) * (kBoxRows / 4); ++rr) {
        const int64_t i = r0 + rr, jx = c0 + tx;
        if (i >= rows || jx >= cols) continue;
        const T old = tile[(rr + K) * TW + tx + K];
        T nv = old;
        if (i >= K && i < rows - K && jx >= K && jx < cols - K) {
            T total = T(0);
#pragma unroll
            for (int di = -K; di <= K; ++di) {
                T row = T(0);
#pragma unroll
                for (int dj = -K; dj <= K; ++dj) row = row + tile[(rr + K + di) * TW + tx + K + dj];
                total = total + row;
            }
            nv = total / cnt;
            if (check) acc = jacobi_accum(ctl.reduce, acc, (double)nv - (double)old);
        }
        b[i * pitch + jx] = nv;
    }
    if (check) {
        const double s = block_reduce<4>(acc, ctl.reduce == RED_MAX_ABS, lds);
        if (threadIdx.x == 0) partials[t] = s;
    }
}

constexpr int kLapX = 64, kLapY = 4, kLapZ = 16;

template <typename T>
__global__ __launch_bounds__(256) void laplace3d_kernel(const T* __restrict__ a, T* __restrict__ b,
                                                        int64_t nz, int64_t ny, int64_t nx,
                                                        int64_t pitch, JobState* __restrict__ st,
                                                        double* __restrict__ partials, LoopCtl ctl,
                                                        int j, int sx, int sy, int tiles) {
    __shared__ double lds[4];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    // tiles enumerate x fastest, then y, then z bands
    const int tz = t / (sx * sy), rem = t - tz * (sx * sy), tyi = rem / sx, txi = rem - tyi * sx;
    const int64_t x = (int64_t)txi * kLapX + (threadIdx.x & 63);
    const int64_t y = (int64_t)tyi * kLapY + (threadIdx.x >> 6);
    const int64_t z0 = 1 + (int64_t)tz * kLapZ;
    const int64_t z1 = min(z0 + (int64_t)kLapZ, nz - 1);
    double acc = 0.0;
    const bool inside = x >= 1 && x < nx - 1 && y >= 1 && y < ny - 1;
    if (inside) {
        const int64_t plane = ny * pitch;   // the row pitch applies to every row of every plane
        const T* p = a + y * pitch + x;
        T dn = p[(z0 - 1) * plane], cur = p[z0 * plane];
        for (int64_t z = z0; z < z1; ++z) {
            const T up = p[(z + 1) * plane];
            const T* c = p + z * plane;
            const T nv = (((c[-1] + c[1]) + (c[-pitch] + c[pitch])) + (dn + up)) / T(6);
            b[z * plane + y * pitch + x] = nv;
            if (check) acc = jacobi_accum(ctl.reduce, acc, (double)nv - (double)cur);
            dn = cur;
            cur = up;
        }
    }
    if (check) {
        const double s = block_reduce<4>(acc, ctl.reduce == RED_MAX_ABS, lds);
        if (threadIdx.x == 0) partials[t] = s;
    }
}

template <typename T>
hipError_t launch_box_t(const void* a, void* b, int64_t rows, int64_t cols, int64_t pitch, int k,
                        const SweepGeom& g, JobState* st, double* parts, const LoopCtl& c, int j,
                        hipStream_t s) {
    const T* pa = static_cast<const T*>(a);
    T* pb = static_cast<T*>(b);
    switch (k) {
        case 1: hipLaunchKernelGGL((box_kernel<T, 1>), dim3(g.blocks), dim3(256), 0, s, pa, pb, rows, cols, pitch, st, parts, c, j, g.strips, g.tiles); break;
        case 2: hipLaunchKernelGGL((box_kernel<T, 2>), dim3(g.blocks), dim3(256), 0, s, pa, pb, rows, cols, pitch, st, parts, c, j, g.strips, g.tiles); break;
        case 3: hipLaunchKernelGGL((box_kernel<T, 3>), dim3(g.blocks), dim3(256), 0, s, pa, pb, rows, cols, pitch, st, parts, c, j, g.strips, g.tiles); break;
        case 4: hipLaunchKernelGGL((box_kernel<T, 4>), dim3(g.blocks), dim3(256), 0, s, pa, pb, rows, cols, pitch, st, parts, c, j, g.strips, g.tiles); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

SweepGeom box_geom(int64_t rows, int64_t cols) {
    SweepGeom g;
    g.waves = 4;
    g.tile_rows = kBoxRows;
    g.strips = (int)((cols + kBoxCols - 1) / kBoxCols);
    g.bands = (int)((rows + kBoxRows - 1) / kBoxRows);
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_box(const void* a, void* b, int64_t rows, int64_t cols, int64_t pitch, int k,
                      int f32, const SweepGeom& g, JobState* st, void* partials, const LoopCtl& c,
                      int j, hipStream_t s) {
    double* parts = static_cast<double*>(partials);
    return f32 ? launch_box_t<float>(a, b, rows, cols, pitch, k, g, st, parts, c, j, s)
               : launch_box_t<double>(a, b, rows, cols, pitch, k, g, st, parts, c, j, s);
}

SweepGeom laplace3d_geom(int64_t nz, int64_t ny, int64_t nx) {
    SweepGeom g;
    g.waves = 4;
    g.tile_rows = kLapZ;
    g.strips = (int)((nx + kLapX - 1) / kLapX);                 // x tiles
    const int sy = (int)((ny + kLapY - 1) / kLapY);             // y tiles
    g.bands = sy * (int)((nz - 2 + kLapZ - 1) / kLapZ);         // y tiles x z bands
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_laplace3d(const void* a, void* b, int64_t nz, int64_t ny, int64_t nx,
                            int64_t pitch, int f32, const SweepGeom& g, JobState* st,
                            void* partials, const LoopCtl& c, int j, hipStream_t s) {
    const int sy = (int)((ny + kLapY - 1) / kLapY);
    double* parts = static_cast<double*>(partials);
    if (f32)
        hipLaunchKernelGGL(laplace3d_kernel<float>, dim3(g.blocks), dim3(256), 0, s,
                           static_cast<const float*>(a), static_cast<float*>(b), nz, ny, nx, pitch,
                           st, parts, c, j, g.strips, sy, g.tiles);
    else
        hipLaunchKernelGGL(laplace3d_kernel<double>, dim3(g.blocks), dim3(256), 0, s,
                           static_cast<const double*>(a), static_cast<double*>(b), nz, ny, nx,
                           pitch, st, parts, c, j, g.strips, sy, g.tiles);
    return hipGetLastError();
}

}  // namespace lsr
