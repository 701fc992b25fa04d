// Restoration update of the two-phase impulse-noise filter (Sect. 4.3), shared by
// the plain sweep kernel and the batched engine: the per-pixel minimiser and the
// wavefront routine that solves the flagged pixels of a set of rows.
#pragma once

#include "common.hpp"

namespace lsr {

// ---------------------------------------------------------------------------
// 1/sqrt(x) for the x = beta + d^2 >= beta > 0 of the update: the hardware
// estimate refined by Newton's iteration for 1/s^2 = x, s <- s + s (1 - x s^2) / 2,
// which doubles the correct bits per step (twice for FP64, once for FP32). The
// correctly rounded sqrt followed by a correctly rounded division cost about
// three times as many instructions.
template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) {
    double s = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) s = fma(0.5 * s, fma(-x * s, s, 1.0), s);
    return s;
}
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) {
    const float s = __builtin_amdgcn_rsqf(x);
    return fmaf(0.5f * s, fmaf(-x * s, s, 1.0f), s);
}

// Root of g(t) = sum phi'(t - v_m) on [lo, hi] by bracketed Newton. The eight
// neighbour slots are fixed (register resident); `valid` marks the in-range ones.
template <typename T>
__device__ T restore_argmin(const T (&v)[8], unsigned valid, T beta, bool quadratic, T start) {
    T lo = T(0), hi = T(0);
    bool first = true;
    int cnt = 0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        if (valid & (1u << m)) {
            lo = (first || v[m] < lo) ? v[m] : lo;
            hi = (first || v[m] > hi) ? v[m] : hi;
            first = false;
            ++cnt;
        }
    }
    if (!(lo < hi)) return lo;
    if (quadratic) {
        T s = T(0);
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (valid & (1u << m)) s = s + v[m];
        return s / T(cnt);
    }
    T t = (start > lo && start < hi) ? start : lo + T(0.5) * (hi - lo);
    const int max_steps = sizeof(T) == 8 ? 64 : 40;
    for (int it = 0; it < max_steps; ++it) {
        T gs = T(0), dg = T(0);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            if (valid & (1u << m)) {
                const T d = t - v[m];
                const T q = beta + d * d;
                const T s = rsqrt_t<T>(q);
                gs = gs + d * s;
                dg = dg + beta * (s * s * s);
            }
        }
        if (gs == T(0)) return t;
        if (gs < T(0)) lo = t; else hi = t;
        const T dt = gs / dg;
        T tn = t - dt;
        // a Newton step below the tolerance: t is the root to working accuracy
        // (its step may round back onto t, a bracket end, which must not turn into
        // a bisection that walks back to the same root)
        if (fabs(dt) <= (sizeof(T) == 8 ? T(4e-16) : T(2e-7)) * (fabs(t) > T(1) ? fabs(t) : T(1)))
            return (tn > lo && tn < hi) ? tn : t;
        if (!(tn > lo && tn < hi)) tn = lo + T(0.5) * (hi - lo);
        const T step = tn - t;
        t = tn;
        if (!(hi > lo) || step == T(0)) break;
        const T tol = (sizeof(T) == 8 ? T(4e-16) : T(2e-7)) * (fabs(t) > T(1) ? fabs(t) : T(1));
        if (fabs(step) <= tol) break;
    }
    return t;
}

// One wavefront updates the flagged pixels of rows row0 + rfirst, row0 + rfirst +
// rstep, ... (below row0 + TR) in the 64 columns from col0. About 40 % of pixels
// are flagged, so the wavefront first lists its flagged pixels (row-in-band << 6 |
// lane) in `list` (LDS, at least ceil(TR / rstep) * 64 entries, this wavefront's
// own) and then solves them 64 at a time with every lane busy, instead of running
// each row's Newton loop with the unflagged lanes idle. Returns the lane's share
// of the delta reduce (max or sum of |new - old|) when check is set. BLOCK: the
// whole workgroup calls this together (a workgroup barrier orders the list);
// otherwise only this wavefront's own ordering is needed (a wavefront fence).
template <typename T, bool BLOCK>
__device__ __forceinline__ double restore_wave(const T* __restrict__ a, T* __restrict__ b,
                                               const uint8_t* __restrict__ mask, int64_t rows,
                                               int64_t cols, int64_t pitch, T beta, bool quadratic,
                                               int64_t row0, int rfirst, int rstep, int TR,
                                               int64_t col0, uint16_t* list, bool check,
                                               bool is_max) {
    const int lx = threadIdx.x & 63;
    int n = 0;
    for (int rr = rfirst; rr < TR; rr += rstep) {
        const int64_t i = row0 + rr;
        const int64_t jx = col0 + lx;
        const bool flagged = i < rows && jx < cols && mask[i * pitch + jx];
        const uint64_t ballot = __ballot(flagged);
        const int pos = n + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
        if (flagged) list[pos] = (uint16_t)((rr << 6) | lx);
        n += __popcll(ballot);
    }
    if (BLOCK) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    double acc = 0.0;
    for (int e = lx; e < n; e += 64) {
        const int code = list[e];
        const int64_t i = row0 + (code >> 6);
        const int64_t jx = col0 + (code & 63);
        const int64_t p = i * pitch + jx;
        T v[8];
        unsigned valid = 0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int o = m < 4 ? m : m + 1;  // 3x3 box in row order, centre skipped
            const int64_t ii = i + o / 3 - 1, jj = jx + o % 3 - 1;
            const bool in = ii >= 0 && jj >= 0 && ii < rows && jj < cols;
            v[m] = in ? a[ii * pitch + jj] : T(0);
            valid |= in ? (1u << m) : 0u;
        }
        if (valid == 0) continue;
        const T old = a[p];
        const T nv = restore_argmin<T>(v, valid, beta, quadratic, old);
        b[p] = nv;
        if (check) {
            const double d = fabs((double)nv - (double)old);
            acc = is_max ? max_nan(acc, d) : acc + d;
        }
    }
    return acc;
}

}  // namespace lsr
