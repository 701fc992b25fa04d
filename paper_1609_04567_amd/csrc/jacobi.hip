// Single-job 5-point Jacobi sweep kernel (Laplace / Helmholtz, FP64 or FP32
// storage): loop control at entry, then one tile of tile_jacobi.hpp per
// workgroup, tiles dealt to the XCDs in contiguous runs.
#include "kernels.hpp"
#include "tile_jacobi.hpp"

namespace lsr {
namespace {

template <typename T, bool HELM, int VEC, int NW, int U, bool NT = false, bool NTG = false,
          bool NTU = false, bool SEP = false>
__global__ __launch_bounds__(NW * 64) void jacobi5_kernel(
    const T* __restrict__ a, T* __restrict__ b, const T* __restrict__ g, int64_t rows,
    int64_t cols, int64_t pitch, T rd, T rd_lo, JobState* __restrict__ st,
    double* __restrict__ partials, LoopCtl ctl, int j, int strips, int tiles, int tile_rows,
    SepSource sep) {
    __shared__ double lds[NW];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    jacobi5_tile<T, HELM, VEC, NW, U, NT, NTG, NTU, false, SEP>(a, b, g, rows, cols, pitch, rd,
                                                                rd_lo, (uint32_t)n1, check,
                                                                ctl.reduce, t, strips, tile_rows,
                                                                partials, lds, sep);
}

int pick_vec(const JacobiArgs& a) {
    const int esz = a.f32 ? 4 : 8;
    const int want = a.f32 ? 4 : 2;
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if ((a.pitch * esz) % 16 == 0 && al(a.a) && al(a.b) && (!a.helm || a.sep || al(a.g))) return want;
    return 1;
}

// Launch shapes measured on the MI355X at 8192^2 (sweep kernel alone, % of 8 TB/s):
//   FP64 Helmholtz  1 wave x 8-row unroll, 8-row tiles        79 %
//   FP64 Laplace    4 waves x 8                               75 %
//   FP32 Helmholtz  4 waves x 8                               76 %
//   FP32 Laplace    4 waves x 16                              73 %
// Vector paths store the next iterate non-temporally and read g non-temporally
// (both are touched once per sweep); the unaligned scalar path uses 4 x 4.
struct Shape {
    int waves, unroll;
};
constexpr Shape kShapes[] = {{1, 8}, {2, 8}, {4, 4}, {4, 8}, {4, 16}};

bool shape_ok(int waves, int unroll) {
    for (const Shape& s : kShapes)
        if (s.waves == waves && s.unroll == unroll) return true;
    return false;
}

template <typename T, bool HELM, int VEC, int NW, int U, bool SEP = false>
hipError_t launch_t(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                    const LoopCtl& c, int j, hipStream_t s) {
    hipLaunchKernelGGL((jacobi5_kernel<T, HELM, VEC, NW, U, true, HELM && !SEP, false, SEP>),
                       dim3(g.blocks), dim3(NW * 64), 0, s, static_cast<const T*>(a.a),
                       static_cast<T*>(a.b), static_cast<const T*>(a.g), a.rows, a.cols, a.pitch,
                       T(a.rd), T(0.25 - a.rd), st, static_cast<double*>(partials), c, j, g.strips,
                       g.tiles, g.tile_rows, SepSource{a.sp, a.sq, a.c1, a.c2});
    return hipGetLastError();
}

template <typename T, bool HELM, int VEC>
hipError_t launch_shape(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                        const LoopCtl& c, int j, hipStream_t s) {
    if (VEC == 1) return launch_t<T, HELM, VEC, 4, 4>(a, g, st, partials, c, j, s);
    switch (g.waves * 100 + g.unroll) {
        case 108: return launch_t<T, HELM, VEC, 1, 8>(a, g, st, partials, c, j, s);
        case 208: return launch_t<T, HELM, VEC, 2, 8>(a, g, st, partials, c, j, s);
        case 404: return launch_t<T, HELM, VEC, 4, 4>(a, g, st, partials, c, j, s);
        case 408: return launch_t<T, HELM, VEC, 4, 8>(a, g, st, partials, c, j, s);
        case 416: return launch_t<T, HELM, VEC, 4, 16>(a, g, st, partials, c, j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

SweepGeom jacobi_geom(const JacobiArgs& a, int tile_rows, int waves, int unroll, int depth,
                      int mc) {
    SweepGeom g;
    g.vec = pick_vec(a);
    if (depth > 1 && g.vec > 1 && jacobi_tb_depth_ok(depth)) {
        jacobi_tb_geom(a, depth, mc, tile_rows, waves, unroll, g);
        return g;
    }
    if (g.vec == 1) {
        waves = 4;
        unroll = 4;
    } else if (a.sep) {   // the -i form is compiled for the measured Helmholtz shapes only
        waves = a.f32 ? 4 : 1;
        unroll = 8;
    } else if (!shape_ok(waves, unroll)) {
        if (a.f32) { waves = 4; unroll = a.helm ? 8 : 16; }
        else { waves = a.helm ? 1 : 4; unroll = 8; }
    }
    g.waves = waves;
    g.unroll = unroll;
    g.tile_rows = tile_rows > 0 ? tile_rows : 8;
    const int64_t span = (int64_t)waves * 64 * g.vec;
    g.strips = (int)((a.cols + span - 1) / span);
    g.bands = (int)((a.rows - 2 + g.tile_rows - 1) / g.tile_rows);
    g.tiles = g.strips * g.bands;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_jacobi(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                         const LoopCtl& c, int j, hipStream_t s) {
    if (g.tb > 1) return launch_jacobi_tb(a, g, st, partials, c, j, s);
    if (a.sep) {   // vector path only: unaligned grids are staged by the runtime
        if (a.f32) return g.vec == 4 ? launch_t<float, true, 4, 4, 8, true>(a, g, st, partials, c, j, s)
                                     : hipErrorInvalidValue;
        return g.vec == 2 ? launch_t<double, true, 2, 1, 8, true>(a, g, st, partials, c, j, s)
                          : hipErrorInvalidValue;
    }
    if (a.f32) {
        if (a.helm) return g.vec == 4 ? launch_shape<float, true, 4>(a, g, st, partials, c, j, s)
                                      : launch_shape<float, true, 1>(a, g, st, partials, c, j, s);
        return g.vec == 4 ? launch_shape<float, false, 4>(a, g, st, partials, c, j, s)
                          : launch_shape<float, false, 1>(a, g, st, partials, c, j, s);
    }
    if (a.helm) return g.vec == 2 ? launch_shape<double, true, 2>(a, g, st, partials, c, j, s)
                                  : launch_shape<double, true, 1>(a, g, st, partials, c, j, s);
    return g.vec == 2 ? launch_shape<double, false, 2>(a, g, st, partials, c, j, s)
                      : launch_shape<double, false, 1>(a, g, st, partials, c, j, s);
}

}  // namespace lsr
