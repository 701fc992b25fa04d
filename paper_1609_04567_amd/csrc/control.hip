// Loop control on the device: job-state initialisation, the final reduce of
// the per-tile partials with the condition test (the part the paper's runtime
// runs on the host after every iteration, Fig. 2), and cancellation.
//
// The finalize kernel is one workgroup. It walks the partials in index order
// (thread t takes t, t+1024, ... in that order), folds the 1024 lanes with the
// fixed wave/workgroup tree, then thread 0 updates the state:
//   r = max | sqrt(sum) | sum/(rows*cols) | count
//   BELOW:      stop when r < threshold
//   STABLE_FOR: run = (count == prev) ? run + 1 : 0; prev = count; stop when run >= window
//   any FP reduce that is NaN or Inf stops the loop with a numeric status
//   n == max_iter always stops.
// The state is mirrored into pinned host memory so the host driver can see the
// stop without a copy on the stream.
#include "kernels.hpp"

namespace lsr {
namespace {

constexpr int kFinThreads = 1024;

// The host mirror starts zeroed (done == 0) and is written only once the loop
// has stopped: that is the only transition the host driver waits for, and it
// keeps a write to host memory off every other check.
__device__ void publish(JobState* st, JobState* mirror, const JobState& s) {
    *st = s;
    if (mirror && s.done) {
        volatile int64_t* m = reinterpret_cast<volatile int64_t*>(mirror);
        const int64_t* v = reinterpret_cast<const int64_t*>(&s);
#pragma unroll
        for (int i = 0; i < 8; ++i) m[i] = v[i];
    }
}

__global__ __launch_bounds__(kFinThreads) void finalize_kernel(JobState* st, const void* partials,
                                                               LoopCtl c, int j, JobState* mirror) {
    __shared__ double lds_d[kFinThreads / 64];
    __shared__ unsigned long long lds_u[kFinThreads / 64];
    if (st->done) return;
    const int64_t n1 = st->n_base + j + 1;
    if (n1 > c.max_iter) return;
    const bool check = is_check_sweep(n1, c);
    double rd = 0.0;
    unsigned long long ru = 0;
    if (check) {
        // thread t folds the contiguous run [t*per, (t+1)*per) in index order,
        // eight loads in flight at a time; then the fixed workgroup tree
        const int per = (c.nparts + kFinThreads - 1) / kFinThreads;
        const int lo = min((int)threadIdx.x * per, c.nparts), hi = min(lo + per, c.nparts);
        if (c.reduce == RED_SUM) {
            const unsigned long long* p = static_cast<const unsigned long long*>(partials);
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
            ru = block_reduce_u64<kFinThreads / 64>(acc, lds_u);
        } else {
            const double* p = static_cast<const double*>(partials);
            const bool is_max = c.reduce == RED_MAX_ABS;
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
            rd = block_reduce<kFinThreads / 64>(acc, is_max, lds_d);
        }
    }
    if (threadIdx.x != 0) return;
    JobState s = *st;
    if (check) {
        s.checks += 1;
        s.n = n1;
        bool stop = false;
        if (c.reduce == RED_SUM) {
            s.count = ru;
            s.r = (double)ru;
            s.run = (ru == s.prev) ? s.run + 1 : 0;
            s.prev = ru;
            if (c.cond == COND_STABLE_FOR && s.run >= c.stable_window) stop = true;
        } else {
            double r = rd;
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
    if (!s.done && j == c.chunk - 1) s.n_base += c.chunk;
    publish(st, mirror, s);
}

__global__ __launch_bounds__(256) void init_state_kernel(JobState* st, const unsigned long long* parts,
                                                         int nparts) {
    __shared__ unsigned long long lds[4];
    unsigned long long acc = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += parts[i];
    acc = block_reduce_u64<4>(acc, lds);
    if (threadIdx.x == 0) {
        JobState s;
        s.n_base = 0;
        s.n = 0;
        s.r = __builtin_nan("");
        s.count = acc;
        s.prev = acc;
        s.checks = 0;
        s.run = 0;
        s.done = 0;
        s.converged = 0;
        s.status = ST_OK;
        *st = s;
    }
}

__global__ void cancel_kernel(JobState* st, JobState* mirror) {
    if (threadIdx.x != 0) return;
    JobState s = *st;
    if (!s.done) {
        s.done = 1;
        s.status = ST_CANCELED;
    }
    publish(st, mirror, s);
}

// Live-cell count of a u8 grid: one partial per workgroup of 256 threads, each
// thread summing non-zero bytes of whole rows it strides over.
constexpr int kCountBlocks = 512;

__global__ __launch_bounds__(256) void count_u8_kernel(const uint8_t* __restrict__ a, int64_t rows,
                                                       int64_t cols, int64_t pitch,
                                                       unsigned long long* __restrict__ parts) {
    __shared__ unsigned long long lds[4];
    unsigned long long acc = 0;
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / cols, c = i - r * cols;
        acc += a[r * pitch + c] != 0;
    }
    acc = block_reduce_u64<4>(acc, lds);
    if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

}  // namespace

int count_u8_parts(int64_t rows, int64_t cols) {
    const int64_t need = (rows * cols + 255) / 256;
    return (int)(need < kCountBlocks ? need : kCountBlocks);
}

hipError_t launch_count_u8(const uint8_t* a, int64_t rows, int64_t cols, int64_t pitch,
                           void* partials, int* nparts_out, hipStream_t s) {
    const int nb = count_u8_parts(rows, cols);
    hipLaunchKernelGGL(count_u8_kernel, dim3(nb), dim3(256), 0, s, a, rows, cols, pitch,
                       static_cast<unsigned long long*>(partials));
    *nparts_out = nb;
    return hipGetLastError();
}

hipError_t launch_init_state(JobState* st, const void* count_parts, int nparts, hipStream_t s) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st,
                       static_cast<const unsigned long long*>(count_parts), nparts);
    return hipGetLastError();
}

hipError_t launch_finalize(JobState* st, const void* partials, const LoopCtl& c, int j,
                           JobState* mirror, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, s, st, partials, c, j,
                       mirror);
    return hipGetLastError();
}

hipError_t launch_cancel(JobState* st, JobState* mirror, hipStream_t s) {
    hipLaunchKernelGGL(cancel_kernel, dim3(1), dim3(64), 0, s, st, mirror);
    return hipGetLastError();
}

}  // namespace lsr
