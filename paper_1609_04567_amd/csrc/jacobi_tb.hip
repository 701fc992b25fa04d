// Temporally blocked 5-point Jacobi kernel: one launch advances the field by K
// sweeps (Sect. 3.1's loop body applied K times between two condition tests).
// Every workgroup streams a band of rows through a register pipeline of K
// levels (tile_jacobi.hpp, jacobi5_tb_tile); neighbouring windows overlap by K
// columns and neighbouring bands by K rows, so tiles never exchange data and
// each cell of every level is computed from exactly the operands a plain sweep
// would read. Per K sweeps a cell is read once (plus the g term) and written
// once, instead of K times each.
//
// Used only where K divides both the check period and the sweep cap, so every
// condition test falls on a launch's last level and the stop sweep is exact.
#include "kernels.hpp"
#include "tile_jacobi.hpp"

namespace lsr {
namespace {

// FP64: at least three wavefronts per SIMD (168 VGPRs). At depth 10 the register
// pipeline needs about 174, and the compiler fits it in 168 with a few values
// spilled, which the third wavefront repays (8192^2 Helmholtz +10 %).
template <typename T, bool HELM, int VEC, int NW, int K, bool MC, bool SEP = false,
          bool VERT = false, int RED = -1>
__global__ __launch_bounds__(NW * 64, sizeof(T) == 8 ? 3 : 1) void jacobi5_tb_kernel(
    const T* __restrict__ a, T* __restrict__ b, const T* __restrict__ g, int64_t rows,
    int64_t cols, int64_t pitch, T rd, T rd_lo, JobState* __restrict__ st,
    double* __restrict__ partials, LoopCtl ctl, int j, int strips, int tiles, int tile_rows,
    SepSource sep) {
    __shared__ double lds[NW];
    __shared__ __attribute__((aligned(16))) T gring[HELM && !SEP ? tb_gring_elems<VEC, NW, K>() : 1];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    // sweeps n1 .. n1 + K - 1 (sweeps past the cap are computed and never kept:
    // the stop lands inside the launch and the driver replays up to it)
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    uint32_t mask = 0;
#pragma unroll
    for (int lev = 1; lev <= K; ++lev) {
        const int64_t n = n1 + lev - 1;
        if (n <= ctl.max_iter && is_check_sweep(n, ctl)) mask |= 1u << (lev - 1);
    }
    if (!MC) mask &= 1u << (K - 1);   // K divides the check period and the cap
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    // FP64: g rows read two levels ahead (8192^2 Helmholtz, depth 10: +1.5 %)
    jacobi5_tb_tile<T, HELM, VEC, NW, K, true, HELM && !SEP, false, MC, SEP, VERT,
                    sizeof(T) == 8 ? 2 : 0, RED>(
        a, b, g, rows, cols, pitch, rd, rd_lo, (uint32_t)n1, mask, ctl.reduce, t, strips, tiles,
        tile_rows, partials, lds, gring, sep);
}

// Fused depths and wavefronts per workgroup compiled for the vector (16-byte
// aligned) path; rows stream three at a time (one load group per iteration).
constexpr int kDepths[] = {2, 4, 5, 8, 10};

bool waves_ok(int waves) { return waves == 1 || waves == 2 || waves == 4; }

// Fewest tiles a default fused launch aims for (bands are halved down to 2 rows
// until it has them; 1024^2 measured best at 4-row bands, 1280 tiles).
constexpr int64_t kMinTiles = 1024;


// Workgroups of several wavefronts take consecutive bands of one window, odd
// bands streamed upwards (8192^2 FP64 Helmholtz: depth 10 +1-2 %, depth 5 +3 %).
constexpr bool kVertical = true;

template <typename T, bool HELM, int VEC, int NW, int K, bool MC, bool SEP, bool VERT, int RED = -1>
hipError_t launch_v(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                    const LoopCtl& c, int j, hipStream_t s) {
    // the L2 reduce (the Helmholtz checks) of two-wavefront vertical launches at
    // depths 5 and 10 has its own kernels: 60 of the ~620 vector instructions of a
    // depth-10 loop iteration were selects between the reduce kinds
    constexpr bool kL2Own = RED < 0 && NW == 2 && VERT && !MC && !SEP && (K == 5 || K == 10);
    if constexpr (kL2Own) {
        if (c.reduce == RED_L2)
            return launch_v<T, HELM, VEC, NW, K, MC, SEP, VERT, RED_L2>(a, g, st, partials, c, j, s);
    }
    hipLaunchKernelGGL((jacobi5_tb_kernel<T, HELM, VEC, NW, K, MC, SEP, VERT, RED>), dim3(g.blocks),
                       dim3(NW * 64), 0, s, static_cast<const T*>(a.a), static_cast<T*>(a.b),
                       static_cast<const T*>(a.g), a.rows, a.cols, a.pitch, T(a.rd),
                       T(0.25 - a.rd), st, static_cast<double*>(partials), c, j, g.strips,
                       g.tiles, g.tile_rows, SepSource{a.sp, a.sq, a.c1, a.c2});
    return hipGetLastError();
}

// several wavefronts per workgroup: vertical band groups (the geometry sets
// g.vert the same way); one wavefront has no vertical layout
template <typename T, bool HELM, int VEC, int NW, int K, bool MC = false, bool SEP = false>
hipError_t launch_t(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                    const LoopCtl& c, int j, hipStream_t s) {
    constexpr bool kVert = NW > 1 && kVertical;
    if (g.vert != (int)kVert) return hipErrorInvalidValue;
    return launch_v<T, HELM, VEC, NW, K, MC, SEP, kVert>(a, g, st, partials, c, j, s);
}

// The -i form: compiled for two wavefronts per workgroup at depths 10 and 5.
template <typename T, int VEC>
hipError_t launch_sep(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                      const LoopCtl& c, int j, hipStream_t s) {
    if (g.waves != 2) return hipErrorInvalidValue;
    if (g.tb == 10 && !g.mc) return launch_t<T, true, VEC, 2, 10, false, true>(a, g, st, partials, c, j, s);
    if (g.tb == 5)
        return g.mc ? launch_t<T, true, VEC, 2, 5, true, true>(a, g, st, partials, c, j, s)
                    : launch_t<T, true, VEC, 2, 5, false, true>(a, g, st, partials, c, j, s);
    return hipErrorInvalidValue;
}

template <typename T, bool HELM, int VEC, int K>
hipError_t launch_shape(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                        const LoopCtl& c, int j, hipStream_t s) {
    if (g.mc) return g.waves == 2 ? launch_t<T, HELM, VEC, 2, K, true>(a, g, st, partials, c, j, s)
                                  : hipErrorInvalidValue;
    switch (g.waves) {
        case 1: return launch_t<T, HELM, VEC, 1, K>(a, g, st, partials, c, j, s);
        case 2: return launch_t<T, HELM, VEC, 2, K>(a, g, st, partials, c, j, s);
        case 4: return launch_t<T, HELM, VEC, 4, K>(a, g, st, partials, c, j, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, bool HELM, int VEC>
hipError_t launch_depth(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                        const LoopCtl& c, int j, hipStream_t s) {
    switch (g.tb) {
        case 2: return launch_shape<T, HELM, VEC, 2>(a, g, st, partials, c, j, s);
        case 4: return launch_shape<T, HELM, VEC, 4>(a, g, st, partials, c, j, s);
        case 5: return launch_shape<T, HELM, VEC, 5>(a, g, st, partials, c, j, s);
        case 8: return launch_shape<T, HELM, VEC, 8>(a, g, st, partials, c, j, s);
        case 10: return launch_shape<T, HELM, VEC, 10>(a, g, st, partials, c, j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool jacobi_tb_depth_ok(int depth) {
    for (int k : kDepths)
        if (k == depth) return true;
    return false;
}

// Depth preference measured on the MI355X at 8192^2 (GLUP/s of the whole job,
// 1000 sweeps, L2 check every 10): FP64 K=10 1160, K=5 887 (HBM-bound), unfused
// 254; FP32 (compensated, stochastically rounded update, ALU-heavy) K=5 685,
// K=10 628, unfused 435. A depth that divides both the check period and the cap
// puts every check on a launch's last level; otherwise the launches carry
// per-level checks (MC) and a stop inside a launch is replayed by the driver.
void jacobi_tb_choose(const JacobiArgs& a, int check_every, int64_t max_iter, int requested,
                      int* depth, int* mc) {
    static constexpr int kPrefF64[] = {10, 8, 5, 4, 2};
    static constexpr int kPrefF32[] = {5, 4, 10, 8, 2};
    if (a.sep) {   // the -i form's compiled depths: FP64 10 (checks on the last level) or 5
        int k = requested == 1 ? 1 : 5;
        if (!a.f32 && requested != 1 && requested != 5 && check_every % 10 == 0 && max_iter % 10 == 0)
            k = 10;
        *depth = k;
        *mc = k > 1 && !(check_every % k == 0 && max_iter % k == 0);
        return;
    }
    int k = 1;
    if (requested > 1) {
        k = jacobi_tb_depth_ok(requested) ? requested : 1;
    } else if (requested == 0) {
        for (int cand : (a.f32 ? kPrefF32 : kPrefF64))
            if (check_every % cand == 0 && max_iter % cand == 0) { k = cand; break; }
        if (k == 1) k = 5;   // checks inside launches: 5 measured best at 256^2 and 1024^2
    }
    *depth = k;
    *mc = k > 1 && !(check_every % k == 0 && max_iter % k == 0);
}

void jacobi_tb_geom(const JacobiArgs& a, int depth, int mc, int tile_rows, int waves, int unroll,
                    SweepGeom& g) {
    (void)unroll;   // rows always stream in groups of three
    if (!waves_ok(waves) || mc || a.sep) waves = 2;   // per-level checks, -i form: 2 waves
    g.tb = depth;
    g.mc = mc;
    g.waves = waves;
    g.unroll = 3;
    g.vert = waves > 1 && kVertical;
    // deeper blocks want taller bands (the 2K halo rows are re-read per band),
    // small grids want more, shorter bands: a band is a serial stream of rows
    // through K levels, so a launch lasts as long as its tallest band (256^2
    // Laplace, checks every sweep: 2-row bands 11.5 ms per job, 32-row 30.4 ms)
    g.tile_rows = tile_rows > 0 ? tile_rows : (depth >= 8 ? 40 : 32);
    // windows of 64 * vec columns step by ow (a multiple of vec) and output the
    // ow columns after their first `depth`; the first window outputs from column 1
    const int64_t ow = (64 * g.vec - 2 * depth) / g.vec * g.vec;
    const int64_t need = a.cols - 1 - depth;
    const int64_t nwin = need > 0 ? (need + ow - 1) / ow : 1;
    // a workgroup: `waves` windows of one band, or (vert) `waves` bands of one window
    g.strips = (int)(g.vert ? nwin : (nwin + waves - 1) / waves);
    auto bands_of = [&](int tr) { return (int)((a.rows - 2 + tr - 1) / tr); };
    auto groups_of = [&](int tr) { return g.vert ? (bands_of(tr) + waves - 1) / waves : bands_of(tr); };
    if (tile_rows <= 0)
        while (g.tile_rows > 2 && (int64_t)g.strips * groups_of(g.tile_rows) < kMinTiles)
            g.tile_rows = g.tile_rows > 4 ? g.tile_rows / 2 : 2;
    g.bands = groups_of(g.tile_rows);
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
}

hipError_t launch_jacobi_tb(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                            const LoopCtl& c, int j, hipStream_t s) {
    if (a.sep) {
        if (g.vec != (a.f32 ? 4 : 2)) return hipErrorInvalidValue;
        return a.f32 ? launch_sep<float, 4>(a, g, st, partials, c, j, s)
                     : launch_sep<double, 2>(a, g, st, partials, c, j, s);
    }
    if (a.f32) {
        if (g.vec != 4) return hipErrorInvalidValue;
        return a.helm ? launch_depth<float, true, 4>(a, g, st, partials, c, j, s)
                      : launch_depth<float, false, 4>(a, g, st, partials, c, j, s);
    }
    if (g.vec != 2) return hipErrorInvalidValue;
    return a.helm ? launch_depth<double, true, 2>(a, g, st, partials, c, j, s)
                  : launch_depth<double, false, 2>(a, g, st, partials, c, j, s);
}

}  // namespace lsr
