// Temporally blocked Game of Life: one launch advances the grid by K
// generations (the loop body of Sect. 3.1 applied K times between two reads of
// the grid), with the live-cell count of every checked generation fused in.
// Each wavefront runs one band of one 992-column window (tile_life_tb.hpp);
// a workgroup of NW wavefronts folds their counts into one partial per checked
// generation.
//
// Requirements (life_tb_ok): 16-byte aligned rows holding a multiple of 16
// cells, or (staged copies) round_up(cols, 16) bytes with the padding zero at the
// start, taken by the RAGGED band. The cells hold 0 or 1 (the job's initial
// count pass normalises them).
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "kernels.hpp"
#include "tile_life_tb.hpp"

namespace lsr {
namespace {

// NW wavefronts per workgroup, each its own window (wave tile wt = t * NW + w,
// strip-major within a band); K generations; U = 3 rows per load group (one
// rotation of the row slots; two groups alternate, so the next group's loads are
// in flight while the current one is computed).
// check_mask bit l-1: generation n1 + l - 1 is checked; its count over the
// workgroup's windows goes to partials[(l - 1) * tiles + t].
template <int NW, int K, int U, bool TORUS, bool RAGGED = false>
__global__ __launch_bounds__(NW * 64) void life_tb_kernel(
    const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t rows, int64_t cols, int64_t pitch,
    JobState* __restrict__ st, unsigned long long* __restrict__ partials, LoopCtl ctl, int j,
    int strips, int wave_tiles, int tiles, int tile_rows) {
    static_assert(K >= 2 && K <= 16, "halo lanes cover at most 16 generations");
    __shared__ unsigned long long lds[K * NW];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    // generations n1 .. n1 + K - 1 (those past the cap are computed and never kept:
    // the driver replays up to a stop inside the launch)
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    uint32_t mask = 0;
#pragma unroll
    for (int lev = 1; lev <= K; ++lev) {
        const int64_t n = n1 + lev - 1;
        if (n <= ctl.max_iter && is_check_sweep(n, ctl)) mask |= 1u << (lev - 1);
    }
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    // the wavefront index is uniform across a wavefront: readfirstlane tells the
    // compiler, so band and row bounds live in scalar registers and the per-row
    // tests below are scalar branches
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wt = t * NW + wave;
    uint32_t cnt[K];
#pragma unroll
    for (int l = 0; l < K; ++l) cnt[l] = 0;

    if (wt < wave_tiles) {
        const int band = wt / strips, strip = wt - band * strips;
        life_tb_band<K, U, TORUS, RAGGED>(a, b, rows, cols, pitch, mask, band, strip, tile_rows, cnt);
    }
    if (mask == 0) return;
#pragma unroll
    for (int l = 0; l < K; ++l) {
        if ((mask >> l) & 1u) {
            const unsigned long long v = wave_sum_u64(cnt[l]);
            if (lane == 0) lds[l * NW + wave] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < K && ((mask >> threadIdx.x) & 1u)) {
        unsigned long long s = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += lds[threadIdx.x * NW + w];
        partials[(size_t)threadIdx.x * (size_t)tiles + t] = s;
    }
}

constexpr int kWaves = 4;
constexpr int kUnroll = 3;
constexpr int kDepths[] = {2, 3, 4, 5, 6, 8};
constexpr int kDefaultDepth = 8;   // 16384^2 torus: 2: 3.8, 4: 7.2, 6: 8.4, 8: 8.5 TLUP/s

constexpr int64_t kMaxAutoRows = 256;

// Workgroups of the depth-K kernel the whole device holds at once (occupancy
// times compute units), measured once per depth and boundary on the current
// device (the library's devices are all of one kind).
template <int K, bool TORUS>
int64_t resident_k() {
    static std::atomic<int64_t> cached{0};
    if (cached.load() > 0) return cached.load();
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, life_tb_kernel<kWaves, K, kUnroll, TORUS>,
                                                     kWaves * 64, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    cached.store((int64_t)per_cu * cus);
    return cached.load();
}

int64_t resident_workgroups(int depth, bool torus) {
    switch (depth) {
        case 2: return torus ? resident_k<2, true>() : resident_k<2, false>();
        case 3: return torus ? resident_k<3, true>() : resident_k<3, false>();
        case 4: return torus ? resident_k<4, true>() : resident_k<4, false>();
        case 5: return torus ? resident_k<5, true>() : resident_k<5, false>();
        case 6: return torus ? resident_k<6, true>() : resident_k<6, false>();
        case 8: return torus ? resident_k<8, true>() : resident_k<8, false>();
    }
    return 1024;
}

template <int K>
hipError_t launch_k(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                    const LoopCtl& c, int j, hipStream_t s) {
    auto* p = static_cast<unsigned long long*>(partials);
    const dim3 grid(g.blocks), block(kWaves * 64);
    const int wt = g.strips * g.bands;
    if (a.cols % 16 == 0) {
        if (a.torus)
            hipLaunchKernelGGL((life_tb_kernel<kWaves, K, kUnroll, true>), grid, block, 0, s, a.a, a.b,
                               a.rows, a.cols, a.pitch, st, p, c, j, g.strips, wt, g.tiles, g.tile_rows);
        else
            hipLaunchKernelGGL((life_tb_kernel<kWaves, K, kUnroll, false>), grid, block, 0, s, a.a, a.b,
                               a.rows, a.cols, a.pitch, st, p, c, j, g.strips, wt, g.tiles, g.tile_rows);
    } else {   // padded rows
        if (a.torus)
            hipLaunchKernelGGL((life_tb_kernel<kWaves, K, kUnroll, true, true>), grid, block, 0, s, a.a,
                               a.b, a.rows, a.cols, a.pitch, st, p, c, j, g.strips, wt, g.tiles,
                               g.tile_rows);
        else
            hipLaunchKernelGGL((life_tb_kernel<kWaves, K, kUnroll, false, true>), grid, block, 0, s, a.a,
                               a.b, a.rows, a.cols, a.pitch, st, p, c, j, g.strips, wt, g.tiles,
                               g.tile_rows);
    }
    return hipGetLastError();
}

}  // namespace

bool life_tb_ok(const LifeArgs& a) {
    const bool al = ((reinterpret_cast<uintptr_t>(a.a) | reinterpret_cast<uintptr_t>(a.b)) & 15) == 0;
    // rows of a multiple of 16 cells, or padded rows (staged: round_up(cols, 16)
    // bytes, the padding zero at the start) for the RAGGED band
    return al && a.pitch % 16 == 0 && (a.cols % 16 == 0 || a.padded);
}

bool life_tb_depth_ok(int depth) {
    for (int k : kDepths)
        if (k == depth) return true;
    return false;
}

int life_tb_choose(const LifeArgs& a, int requested) {
    if (requested == 1 || !life_tb_ok(a)) return 1;
    if (requested > 1) {
        for (int k : kDepths)
            if (k == requested) return k;
        return 1;
    }
    return kDefaultDepth;
}

SweepGeom life_tb_geom(const LifeArgs& a, int depth, int tile_rows) {
    SweepGeom g;
    g.vec = 16;
    g.waves = kWaves;
    g.unroll = kUnroll;
    g.tb = depth;
    g.mc = 1;   // every generation of a launch may be checked
    g.strips = (int)((a.cols + kLifeTbWinCols - 1) / kLifeTbWinCols);
    if (tile_rows > 0) {
        g.tile_rows = tile_rows;
    } else {
        // The launch is ALU-bound and its workgroups take equal time, so the
        // last partial wave of workgroups costs as much as a full one. Take the
        // most bands whose workgroups all fit on the device at once (one round;
        // more rounds only when a band would exceed kMaxAutoRows rows), and no
        // band below 2K rows, where the K-row overlaps would double the work.
        const int64_t slots = resident_workgroups(depth, a.torus != 0);
        int64_t t = 0;
        for (int64_t m = 1;; ++m) {
            const int64_t bands = std::max<int64_t>(1, m * slots * kWaves / g.strips);
            t = (a.rows + bands - 1) / bands;
            if (t <= kMaxAutoRows) break;
        }
        g.tile_rows = (int)std::max<int64_t>(t, 2 * depth);
    }
    g.bands = (int)((a.rows + g.tile_rows - 1) / g.tile_rows);
    g.tiles = (g.strips * g.bands + kWaves - 1) / kWaves;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_life_tb(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                          const LoopCtl& c, int j, hipStream_t s) {
    if (!life_tb_ok(a) || g.waves != kWaves) return hipErrorInvalidValue;
    switch (g.tb) {
        case 2: return launch_k<2>(a, g, st, partials, c, j, s);
        case 3: return launch_k<3>(a, g, st, partials, c, j, s);
        case 4: return launch_k<4>(a, g, st, partials, c, j, s);
        case 5: return launch_k<5>(a, g, st, partials, c, j, s);
        case 6: return launch_k<6>(a, g, st, partials, c, j, s);
        case 8: return launch_k<8>(a, g, st, partials, c, j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lsr
