// Sobel sweep kernel (Sect. 4.2, the single-iteration stencil of the streaming
// edge detector): a workgroup of four wavefronts covers 32 rows x 256 columns,
// each wavefront an 8-row tile (tile_sobel.hpp); the sum of the new image is
// reduced per workgroup on a check sweep.
#include "kernels.hpp"
#include "tile_sobel.hpp"

namespace lsr {
namespace {

constexpr int kSobelWaves = 4;

__global__ __launch_bounds__(kSobelWaves * 64) void sobel_kernel(
    const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t rows, int64_t cols,
    int64_t pitch, JobState* __restrict__ st, unsigned long long* __restrict__ partials,
    LoopCtl ctl, int j, int strips, int tiles) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kSobelWaves][kSobelLdsBytes];
    __shared__ unsigned long long red[kSobelWaves];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    const int band = t / strips, strip = t - band * strips;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned long long acc =
        sobel_wave(a, b, rows, cols, pitch, ((int64_t)band * kSobelWaves + wave) * kSobelRows,
                   (int64_t)strip * kSobelCols, lds[wave]);
    if (check) {
        const unsigned long long s = block_reduce_u64<kSobelWaves>(acc, red);
        if (threadIdx.x == 0) partials[t] = s;
    }
}

}  // namespace

SweepGeom sobel_geom(int64_t rows, int64_t cols) {
    SweepGeom g;
    g.vec = 4;
    g.waves = kSobelWaves;
    g.tile_rows = kSobelWaves * kSobelRows;
    g.strips = (int)((cols + kSobelCols - 1) / kSobelCols);
    g.bands = (int)((rows + g.tile_rows - 1) / g.tile_rows);
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_sobel(const uint8_t* a, uint8_t* b, int64_t rows, int64_t cols, int64_t pitch,
                        const SweepGeom& g, JobState* st, void* partials, const LoopCtl& c, int j,
                        hipStream_t s) {
    hipLaunchKernelGGL(sobel_kernel, dim3(g.blocks), dim3(kSobelWaves * 64), 0, s, a, b, rows, cols,
                       pitch, st, static_cast<unsigned long long*>(partials), c, j, g.strips, g.tiles);
    return hipGetLastError();
}

}  // namespace lsr
