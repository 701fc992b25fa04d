// Tile body of the 5-point Jacobi sweep with the fused residual reduce (Laplace
// and the Helmholtz solver of Sect. 4.1), FP64 or FP32 storage. Shared by the
// single-job kernel (jacobi.hip) and the batched kernel (batch.hip).
//
// One workgroup = NW wavefronts side by side; each wavefront owns 64*VEC
// consecutive columns and streams down `tile_rows` rows of the grid, keeping
// the rows above/at/below the current one in registers (each row of the iterate
// is read from HBM once per tile, plus the two halo rows). Horizontal
// neighbours come from the adjacent lanes through cross-lane shuffles; only the
// first and last lane of a wavefront load one extra halo element per row. Loads
// of U rows are issued before any of them is used. The update never runs in
// place (a stencil cannot, Sect. 3.1): it reads `a` and writes `b`.
//
// Expression order is fixed (the build uses -ffp-contract=off):
//   Laplace   b = 0.25 * ((N + S) + (W + E))
//   Helmholtz b = (((N + S) + (W + E)) + g) * rd
// FP32 Helmholtz is compensated (still only FP32 operations): late in a slow
// solve g is ~1/n of the neighbour sum s, so a plain fl(s + g) quantises each
// sweep's increment to ulp(s) with a bias that is coherent over the smooth field,
// and fl(rd) misplaces the alpha h^2 part of 1/(4 + alpha h^2) by up to 10 %;
// both errors then accumulate over thousands of sweeps. So t = fl(s + g) keeps
// its exact rounding error e (TwoSum), rd is applied as 0.25 - rd_lo, and
//   x = 0.25 t + (0.25 e - rd_lo t)
// is rounded to FP32 stochastically: with p = |x - fl(x)| / ulp, the stored value
// moves one ulp from fl(x) towards x with probability p, drawn from a 32-bit hash
// of (row, column, sweep). Round-to-nearest errors of a smooth field are
// correlated between neighbours and feed the slowly decaying smooth mode;
// unbiased, decorrelated rounding does not (max error vs the FP64 solution at
// 1025^2 x 5000 sweeps: 3.3e-6 with round-to-nearest, 7.7e-7 stochastic). The
// draw depends only on the cell and the sweep, so results are reproducible.
// On a check sweep each lane accumulates delta = b - a in FP64 over its cells
// (max |delta|, sum delta^2 or sum |delta|); the workgroup folds the lanes in a
// fixed order and writes one partial per tile.
#pragma once

#include "common.hpp"

namespace lsr {

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

// 32-bit integer hash ("lowbias32", C. Wellons, 2018: xorshift-multiply
// rounds with constants found by search for low bias).
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// fl(p + c) rounded stochastically by the exact remainder (TwoSum): one ulp
// towards p + c with probability |remainder| / ulp, using 24 bits of `bits`.
__device__ __forceinline__ float add_round_stochastic(float p, float c, uint32_t bits) {
    const float hi = p + c;
    const float bb = hi - p;
    const float rem = (p - (hi - bb)) + (c - bb);
    const float ulp = __uint_as_float(__float_as_uint(hi) & 0x7f800000u) * 1.1920928955078125e-7f;
    const float u = (float)(bits >> 8) * 5.9604644775390625e-8f;  // [0, 1)
    return (fabsf(rem) > u * ulp) ? hi + copysignf(ulp, rem) : hi;
}

__device__ __forceinline__ double jacobi_accum(int red, double acc, double d) {
    if (red == RED_MAX_ABS) return max_nan(acc, fabs(d));
    if (red == RED_L2) return acc + d * d;
    return acc + fabs(d);
}

// Tile t of a grid split into `strips` column strips and bands of `tile_rows`
// rows (band-major). The workgroup must have NW*64 threads; lds holds NW doubles.
template <typename T, bool HELM, int VEC, int NW, int U, bool NT, bool NTG, bool NTU = false>
__device__ __forceinline__ void jacobi5_tile(const T* __restrict__ a, T* __restrict__ b,
                                             const T* __restrict__ g, int64_t rows, int64_t cols,
                                             int64_t pitch, T rd, T rd_lo, uint32_t sweep,
                                             bool check, int red, int t,
                                             int strips, int tile_rows,
                                             double* __restrict__ partials, double* lds) {
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
                    if constexpr (HELM && sizeof(T) == 8) {
                        nv = (((N + S) + (W + E)) + gr[k][e]) * rd;
                    } else if constexpr (HELM) {
                        const T sn = (N + S) + (W + E), gv = gr[k][e];
                        const T tt = sn + gv, bb = tt - sn;
                        const T te = (sn - (tt - bb)) + (gv - bb);  // exact: sn + gv = tt + te
                        const uint32_t key = (uint32_t)(r + k) * 0x9e3779b1u ^
                                             (uint32_t)(c + e) * 0x85ebca77u ^ sweep * 0xc2b2ae3du;
                        nv = add_round_stochastic(T(0.25) * tt, T(0.25) * te - rd_lo * tt,
                                                  hash32(key));
                    } else {
                        nv = T(0.25) * ((N + S) + (W + E));
                    }
                    const int64_t col = c + e;
                    const bool inner = col >= 1 && col <= cols - 2;
                    out[e] = inner ? nv : mid[e];
                    if (check && inner) acc = jacobi_accum(red, acc, (double)nv - (double)mid[e]);
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

}  // namespace lsr
