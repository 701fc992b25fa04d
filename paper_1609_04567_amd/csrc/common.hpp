// Shared device/host definitions of the gfx950 loop-of-stencil-reduce library.
//
// The loop of Sect. 3.1 (repeat a = stencil(sigma_1, f):a until c(/(+):...)) is
// executed as a stream of sweep kernels with the reduce fused into the sweep and
// a one-workgroup finalize kernel that folds the per-workgroup partials in a
// fixed order and evaluates the condition on the device. The job state below is
// the -s variant's global state s plus the loop's control flags.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsr {

enum Reduce : int { RED_MAX_ABS = 1, RED_L2 = 2, RED_SUM = 3, RED_MEAN_ABS = 4 };
enum Cond : int { COND_BELOW = 1, COND_STABLE_FOR = 2, COND_NEVER = 3 };
enum Status : int { ST_OK = 0, ST_NUMERIC = 5, ST_CANCELED = 6 };

// Device-resident per-job state (64 bytes). Written only by the finalize kernel
// (and the init/cancel kernels); read by every sweep kernel at entry.
struct alignas(64) JobState {
    int64_t n_base;      // sweeps completed before the current chunk
    int64_t n;           // sweep count at the last check (the final n once done)
    double r;            // reduce value at the last check
    uint64_t count;      // live cells at the last check (Life)
    uint64_t prev;       // reference count for the stable-window test
    int64_t checks;      // number of checks evaluated
    int32_t run;         // consecutive checks with an unchanged count
    int32_t done;        // 1: the loop has stopped; later sweeps are no-ops
    int32_t converged;   // the condition held at the stop
    int32_t status;      // ST_OK, ST_NUMERIC, ST_CANCELED
};
static_assert(sizeof(JobState) == 64, "JobState is 64 bytes");

// Loop-control constants of a job, passed by value to sweep and finalize kernels.
struct LoopCtl {
    int64_t max_iter;
    int32_t check_every;
    int32_t chunk;        // sweeps per enqueued chunk (multiple of check_every, even)
    int32_t reduce;       // Reduce
    int32_t cond;         // Cond
    int32_t stable_window;
    int32_t nparts;       // partials written per check sweep
    double threshold;
    double mean_div;      // rows*cols, the divisor of RED_MEAN_ABS
};

__host__ __device__ inline bool is_check_sweep(int64_t n, const LoopCtl& c) {
    return (n % c.check_every) == 0 || n == c.max_iter;
}

// Max that keeps a NaN once one is seen, whatever the operand order.
__device__ __forceinline__ double max_nan(double acc, double d) {
    return (d > acc || d != d) ? d : acc;
}

// ---------------------------------------------------------------------------
// Deterministic reductions: a butterfly over the 64 lanes of a wavefront, then
// the waves of a workgroup combined in wave order by lane 0 of wave 0. For a
// fixed launch shape the association order is fixed, so results repeat bit for
// bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max_nan(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup reduce of a double; the result is valid in thread 0.
template <int NWAVES>
__device__ __forceinline__ double block_reduce(double v, bool is_max, double* lds) {
    v = is_max ? wave_max(v) : wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (NWAVES == 1) return v;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double acc = 0.0;
    if (threadIdx.x == 0) {
        acc = lds[0];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) acc = is_max ? max_nan(acc, lds[w]) : acc + lds[w];
    }
    return acc;
}

template <int NWAVES>
__device__ __forceinline__ unsigned long long block_reduce_u64(unsigned long long v,
                                                              unsigned long long* lds) {
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (NWAVES == 1) return v;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    unsigned long long acc = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NWAVES; ++w) acc += lds[w];
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Final fold of per-tile partials (the reduce's last level): thread t folds the
// contiguous run [t*per, (t+1)*per) in index order with eight loads in flight,
// then the fixed workgroup tree. The order depends only on the partial count.
// The result is valid in thread 0.
// ---------------------------------------------------------------------------
template <int NTHREADS>
__device__ inline double fold_partials(const double* __restrict__ p, int n, bool is_max,
                                       double* lds) {
    const int per = (n + NTHREADS - 1) / NTHREADS;
    const int lo = min((int)threadIdx.x * per, n), hi = min(lo + per, n);
    double acc = 0.0;
    int i = lo;
    for (; i + 8 <= hi; i += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[i + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc = is_max ? max_nan(acc, v[k]) : acc + v[k];
    }
    for (; i < hi; ++i) acc = is_max ? max_nan(acc, p[i]) : acc + p[i];
    return block_reduce<NTHREADS / 64>(acc, is_max, lds);
}

template <int NTHREADS>
__device__ inline unsigned long long fold_partials_u64(const unsigned long long* __restrict__ p, int n,
                                                       unsigned long long* lds) {
    const int per = (n + NTHREADS - 1) / NTHREADS;
    const int lo = min((int)threadIdx.x * per, n), hi = min(lo + per, n);
    unsigned long long acc = 0;
    int i = lo;
    for (; i + 8 <= hi; i += 8) {
        unsigned long long v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[i + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    for (; i < hi; ++i) acc += p[i];
    return block_reduce_u64<NTHREADS / 64>(acc, lds);
}

// One evaluation of the condition at check sweep n1 (the -s variant's update and
// test): r = max | sqrt(sum) | sum/(rows*cols) | count;
//   BELOW:      stop when r < threshold
//   STABLE_FOR: run = (count == prev) ? run + 1 : 0; prev = count; stop when run >= window
//   an FP reduce that is NaN or Inf stops the loop with a numeric status;
//   n1 == max_iter always stops.
__device__ inline void apply_check(JobState& s, const LoopCtl& c, int64_t n1, double rsum,
                                   unsigned long long rcount) {
    s.checks += 1;
    s.n = n1;
    bool stop = false;
    if (c.reduce == RED_SUM) {
        s.count = rcount;
        s.r = (double)rcount;
        s.run = (rcount == s.prev) ? s.run + 1 : 0;
        s.prev = rcount;
        if (c.cond == COND_STABLE_FOR && s.run >= c.stable_window) stop = true;
    } else {
        double r = rsum;
        if (c.reduce == RED_L2) r = sqrt(r);
        else if (c.reduce == RED_MEAN_ABS) r = r / c.mean_div;
        s.r = r;
        if (isnan(r) || isinf(r)) {
            s.status = ST_NUMERIC;
            s.done = 1;
        } else if (c.cond == COND_BELOW && r < c.threshold) {
            stop = true;
        }
    }
    if (stop) {
        s.converged = 1;
        s.done = 1;
    }
    if (n1 == c.max_iter) s.done = 1;
}

// Writes the state, and mirrors it into pinned host memory once the loop has
// stopped (the only transition a host driver waits for; the mirror starts
// zeroed, so no host write is needed on the other checks).
__device__ inline void publish_state(JobState* st, JobState* mirror, const JobState& s) {
    *st = s;
    if (mirror && s.done) {
        volatile int64_t* m = reinterpret_cast<volatile int64_t*>(mirror);
        const int64_t* v = reinterpret_cast<const int64_t*>(&s);
#pragma unroll
        for (int i = 0; i < 8; ++i) m[i] = v[i];
    }
}

// ---------------------------------------------------------------------------
// XCD-aware tile order. Workgroups are dealt to the 8 XCDs of the MI355X round
// robin by workgroup id; remapping id -> logical tile so that each XCD gets one
// contiguous run of logical tiles keeps neighbouring tiles (and their shared
// halo rows and columns) in the same 4 MiB L2. The grid is padded to a multiple
// of 8; logical ids >= ntiles are idle.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_logical_tile(int bid, int nblocks_padded) {
    const int per = nblocks_padded / kXcds;
    return (bid % kXcds) * per + bid / kXcds;
}

inline int pad_to_xcds(int n) { return (n + kXcds - 1) / kXcds * kXcds; }

}  // namespace lsr
