// Single-job Game of Life sweep kernel: loop control at entry, then one SWAR
// tile of tile_life.hpp per workgroup. Rows must be 16-byte aligned and either
// a multiple of 16 cells or padded (the runtime stages any other grid into
// padded rows).
#include "kernels.hpp"
#include "tile_life.hpp"

namespace lsr {
namespace {

template <int NW, int U, bool NT = false>
__global__ __launch_bounds__(NW * 64) void life_swar_kernel(
    const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t rows, int64_t cols,
    int64_t pitch, int torus, JobState* __restrict__ st, unsigned long long* __restrict__ partials,
    LoopCtl ctl, int j, int strips, int tiles, int tile_rows) {
    __shared__ unsigned long long lds[NW];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    life_swar_tile<NW, U, NT>(a, b, rows, cols, pitch, torus, check, t, strips, tile_rows, partials,
                              lds);
}

// Launch shape measured on a 16384^2 torus (4 waves, 8-row load groups,
// non-temporal stores, 32-row tiles: 65% of 8 TB/s for the sweep alone).
constexpr int kWaves = 4;
constexpr int kUnroll = 8;
constexpr int kTileRows = 32;

}  // namespace

bool life_rows_ok(const LifeArgs& a) {
    const bool al = ((reinterpret_cast<uintptr_t>(a.a) | reinterpret_cast<uintptr_t>(a.b)) & 15) == 0;
    return al && a.pitch % 16 == 0 && (a.cols % 16 == 0 || a.padded);
}

SweepGeom life_geom(const LifeArgs& a, int tile_rows) {
    SweepGeom g;
    g.vec = 16;
    g.waves = kWaves;
    g.unroll = kUnroll;
    g.tile_rows = tile_rows > 0 ? tile_rows : kTileRows;
    const int64_t span = (int64_t)kWaves * 1024;
    g.strips = (int)((a.cols + span - 1) / span);
    g.bands = (int)((a.rows + g.tile_rows - 1) / g.tile_rows);
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_life(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                       const LoopCtl& c, int j, hipStream_t s) {
    if (g.tb > 1) return launch_life_tb(a, g, st, partials, c, j, s);
    if (!life_rows_ok(a)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((life_swar_kernel<kWaves, kUnroll, true>), dim3(g.blocks), dim3(kWaves * 64),
                       0, s, a.a, a.b, a.rows, a.cols, a.pitch, a.torus, st,
                       static_cast<unsigned long long*>(partials), c, j, g.strips, g.tiles,
                       g.tile_rows);
    return hipGetLastError();
}

}  // namespace lsr
