// 5-point Jacobi sweep with the fused residual reduce (Laplace and the
// Helmholtz solver of Sect. 4.1), FP64 storage or FP32 storage.
//
// One workgroup = NW wavefronts side by side; each wavefront owns 64*VEC
// consecutive columns and streams down `tile_rows` rows of the grid, keeping
// the rows above/at/below the current one in registers (each row of the iterate
// is read from HBM once per tile, plus the two halo rows). Horizontal
// neighbours come from the adjacent lanes through cross-lane shuffles; only the
// first and last lane of a wavefront load one extra halo element per row. Loads
// of U rows are issued before any of them is used, so each wavefront keeps
// 2*U row segments in flight. The update never runs in place (the paper notes a
// stencil cannot): it reads `a` and writes `b`.
//
// Expression order is fixed (the build uses -ffp-contract=off):
//   Laplace   b = 0.25 * ((N + S) + (W + E))
//   Helmholtz b = (((N + S) + (W + E)) + g) * rd
// On a check sweep each lane accumulates delta = b - a in FP64 over its cells
// (max |delta|, sum delta^2 or sum |delta|); the workgroup folds the lanes in a
// fixed order and writes one partial per tile.
#include "kernels.hpp"

namespace lsr {
namespace {

// NTL = non-temporal load (for data read exactly once per sweep, such as g).
template <typename T, int VEC, bool NTL = false>
__device__ __forceinline__ void load_row(const T* __restrict__ p, int64_t c, int64_t cols,
                                         T (&v)[VEC]) {
    if (VEC > 1 && c + VEC <= cols) {
        typedef T V __attribute__((ext_vector_type(VEC)));
        V x = NTL ? __builtin_nontemporal_load(reinterpret_cast<const V*>(p + c))
                  : *reinterpret_cast<const V*>(p + c);
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = x[e];
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = (c + e < cols) ? p[c + e] : T(0);
    }
}

// NT = non-temporal: the next iterate is not read again before the whole grid has
// streamed through, so keeping it out of L2/MALL leaves room for the halo rows.
template <typename T, int VEC, bool NT>
__device__ __forceinline__ void store_row(T* __restrict__ p, int64_t c, int64_t cols,
                                          const T (&v)[VEC]) {
    if (VEC > 1 && c + VEC <= cols) {
        typedef T V __attribute__((ext_vector_type(VEC)));
        V x;
#pragma unroll
        for (int e = 0; e < VEC; ++e) x[e] = v[e];
        if (NT) __builtin_nontemporal_store(x, reinterpret_cast<V*>(p + c));
        else *reinterpret_cast<V*>(p + c) = x;
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (c + e < cols) p[c + e] = v[e];
    }
}

__device__ __forceinline__ double accum(int red, double acc, double d) {
    if (red == RED_MAX_ABS) return max_nan(acc, fabs(d));
    if (red == RED_L2) return acc + d * d;
    return acc + fabs(d);
}

template <typename T, bool HELM, int VEC, int NW, int U, bool NT = false, bool NTG = false,
          bool NTU = false>
__global__ __launch_bounds__(NW * 64) void jacobi5_kernel(
    const T* __restrict__ a, T* __restrict__ b, const T* __restrict__ g, int64_t rows,
    int64_t cols, int64_t pitch, T rd, JobState* __restrict__ st, double* __restrict__ partials,
    LoopCtl ctl, int j, int strips, int tiles, int tile_rows) {
    __shared__ double lds[NW];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;

    const int band = t / strips, strip = t - band * strips;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cw = (int64_t)strip * (NW * 64 * VEC) + (int64_t)wave * (64 * VEC);
    const int64_t c = cw + (int64_t)lane * VEC;
    const int64_t r0 = 1 + (int64_t)band * tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, rows - 1);
    const int64_t ce = cw + 64 * VEC;           // first column after this wavefront
    // Halo elements exist only for wavefronts that own columns of the grid
    // (cw < cols); a wavefront past the last column loads nothing at all.
    const bool has_w = (lane == 0) && cw >= 1 && cw < cols;
    const bool has_e = (lane == 63) && ce < cols;
    const int red = ctl.reduce;

    T up[VEC], mid[VEC];
    T mid_w = T(0), mid_e = T(0);
    load_row<T, VEC>(a + (r0 - 1) * pitch, c, cols, up);
    load_row<T, VEC>(a + r0 * pitch, c, cols, mid);
    if (has_w) mid_w = a[r0 * pitch + cw - 1];
    if (has_e) mid_e = a[r0 * pitch + ce];

    double acc = 0.0;
    for (int64_t r = r0; r < r1; r += U) {
        T dn[U][VEC], dn_w[U], dn_e[U], gr[U][VEC];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (r + k < r1) {
                const T* prow = a + (r + k + 1) * pitch;
                load_row<T, VEC, NTU>(prow, c, cols, dn[k]);
                dn_w[k] = has_w ? prow[cw - 1] : T(0);
                dn_e[k] = has_e ? prow[ce] : T(0);
                if (HELM) load_row<T, VEC, NTG>(g + (r + k) * pitch, c, cols, gr[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (r + k < r1) {
                T wl = __shfl_up(mid[VEC - 1], 1, 64);
                T er = __shfl_down(mid[0], 1, 64);
                if (lane == 0) wl = mid_w;
                if (lane == 63) er = mid_e;
                T out[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T W = (e > 0) ? mid[e - 1] : wl;
                    const T E = (e < VEC - 1) ? mid[e + 1] : er;
                    const T N = up[e], S = dn[k][e];
                    T nv;
                    if (HELM) nv = (((N + S) + (W + E)) + gr[k][e]) * rd;
                    else nv = T(0.25) * ((N + S) + (W + E));
                    const int64_t col = c + e;
                    const bool inner = col >= 1 && col <= cols - 2;
                    out[e] = inner ? nv : mid[e];
                    if (check && inner) acc = accum(red, acc, (double)nv - (double)mid[e]);
                }
                store_row<T, VEC, NT>(b + (r + k) * pitch, c, cols, out);
#pragma unroll
                for (int e = 0; e < VEC; ++e) { up[e] = mid[e]; mid[e] = dn[k][e]; }
                mid_w = dn_w[k];
                mid_e = dn_e[k];
            }
        }
    }
    if (check) {
        const double v = block_reduce<NW>(acc, red == RED_MAX_ABS, lds);
        if (threadIdx.x == 0) partials[t] = v;
    }
}

int pick_vec(const JacobiArgs& a) {
    const int esz = a.f32 ? 4 : 8;
    const int want = a.f32 ? 4 : 2;
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if ((a.pitch * esz) % 16 == 0 && al(a.a) && al(a.b) && (!a.helm || al(a.g))) return want;
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

template <typename T, bool HELM, int VEC, int NW, int U>
hipError_t launch_t(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                    const LoopCtl& c, int j, hipStream_t s) {
    hipLaunchKernelGGL((jacobi5_kernel<T, HELM, VEC, NW, U, true, HELM, false>), dim3(g.blocks),
                       dim3(NW * 64), 0, s, static_cast<const T*>(a.a), static_cast<T*>(a.b),
                       static_cast<const T*>(a.g), a.rows, a.cols, a.pitch, T(a.rd), st,
                       static_cast<double*>(partials), c, j, g.strips, g.tiles, g.tile_rows);
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

SweepGeom jacobi_geom(const JacobiArgs& a, int tile_rows, int waves, int unroll) {
    SweepGeom g;
    g.vec = pick_vec(a);
    if (g.vec == 1) {
        waves = 4;
        unroll = 4;
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
