// Loop control on the device: job-state initialisation, the final reduce of
// the per-tile partials with the condition test (the part the paper's runtime
// runs on the host after every iteration, Fig. 2), and cancellation.
//
// The finalize kernel is one 1024-thread workgroup: fold_partials walks the
// partials in index order (contiguous runs per thread, then the fixed tree),
// apply_check evaluates the condition and updates the -s state, and
// publish_state mirrors the state into pinned host memory once the loop stops,
// so the host driver sees the stop without a copy on the stream. The job state
// here counts sweeps per enqueued chunk: n_base advances by `chunk` at the
// chunk's last check, and a sweep's number is n_base + offset + 1.
#include "kernels.hpp"

namespace lsr {
namespace {

constexpr int kFinThreads = 1024;

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
        if (c.reduce == RED_SUM)
            ru = fold_partials_u64<kFinThreads>(static_cast<const unsigned long long*>(partials),
                                                c.nparts, lds_u);
        else
            rd = fold_partials<kFinThreads>(static_cast<const double*>(partials), c.nparts,
                                            c.reduce == RED_MAX_ABS, lds_d);
    }
    if (threadIdx.x != 0) return;
    JobState s = *st;
    if (check) apply_check(s, c, n1, rd, ru);
    // the chunk's last sweep is always a check sweep (chunk % check_every == 0)
    if (!s.done && j == c.chunk - 1) s.n_base += c.chunk;
    publish_state(st, mirror, s);
}

// Finalize of a fused launch that may hold several checks (sweeps
// n_base + j0 + 1 .. n_base + j0 + K): wavefront l - 1 folds level l's slice of
// tiles partials (lane-strided, then the fixed butterfly), all checked levels at
// once; thread 0 then evaluates the checks in sweep order and stops at the first
// that ends the loop.
__global__ __launch_bounds__(kFinThreads) void finalize_levels_kernel(JobState* st,
                                                                      const void* partials,
                                                                      LoopCtl c, int j0, int K,
                                                                      int tiles, JobState* mirror) {
    __shared__ double rd_l[kFinThreads / 64];
    __shared__ unsigned long long ru_l[kFinThreads / 64];
    if (st->done) return;
    const int64_t nb = st->n_base;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave < K) {
        const int64_t n = nb + j0 + wave + 1;
        if (n <= c.max_iter && is_check_sweep(n, c)) {
            const size_t off = (size_t)wave * (size_t)tiles;
            if (c.reduce == RED_SUM) {
                const unsigned long long* p = static_cast<const unsigned long long*>(partials) + off;
                unsigned long long acc = 0;
                for (int i = lane; i < c.nparts; i += 64) acc += p[i];
                acc = wave_sum_u64(acc);
                if (lane == 0) ru_l[wave] = acc;
            } else {
                const double* p = static_cast<const double*>(partials) + off;
                const bool is_max = c.reduce == RED_MAX_ABS;
                double acc = 0.0;
                for (int i = lane; i < c.nparts; i += 64) acc = is_max ? max_nan(acc, p[i]) : acc + p[i];
                acc = is_max ? wave_max(acc) : wave_sum(acc);
                if (lane == 0) rd_l[wave] = acc;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    JobState s = *st;
    for (int lev = 1; lev <= K; ++lev) {
        const int64_t n = nb + j0 + lev;
        if (n > c.max_iter) break;
        if (!is_check_sweep(n, c)) continue;
        apply_check(s, c, n, rd_l[lev - 1], ru_l[lev - 1]);
        if (s.done) break;
    }
    if (!s.done && j0 + K == c.chunk) s.n_base += c.chunk;
    publish_state(st, mirror, s);
}

__global__ __launch_bounds__(256) void init_state_kernel(JobState* st, const unsigned long long* parts,
                                                         int nparts, int64_t n_base) {
    __shared__ unsigned long long lds[4];
    unsigned long long acc = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += parts[i];
    acc = block_reduce_u64<4>(acc, lds);
    if (threadIdx.x == 0) {
        JobState s;
        s.n_base = n_base;
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
    publish_state(st, mirror, s);
}

// Live-cell count of a u8 grid before the first sweep (one partial per
// 256-thread workgroup). A cell is alive iff its byte is non-zero; the pass also
// rewrites every byte above 1 as 1 (in place, only those bytes), so the sweep
// kernels can treat cells as 0/1 words.
constexpr int kCountBlocks = 512;

__global__ __launch_bounds__(256) void count_u8_kernel(uint8_t* __restrict__ a, int64_t rows,
                                                       int64_t cols, int64_t pitch,
                                                       unsigned long long* __restrict__ parts) {
    __shared__ unsigned long long lds[4];
    unsigned long long acc = 0;
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / cols, c = i - r * cols;
        const uint8_t v = a[r * pitch + c];
        if (v > 1) a[r * pitch + c] = 1;
        acc += v != 0;
    }
    acc = block_reduce_u64<4>(acc, lds);
    if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

}  // namespace

int count_u8_parts(int64_t rows, int64_t cols) {
    const int64_t need = (rows * cols + 255) / 256;
    return (int)(need < kCountBlocks ? need : kCountBlocks);
}

hipError_t launch_count_u8(uint8_t* a, int64_t rows, int64_t cols, int64_t pitch,
                           void* partials, int* nparts_out, hipStream_t s) {
    const int nb = count_u8_parts(rows, cols);
    hipLaunchKernelGGL(count_u8_kernel, dim3(nb), dim3(256), 0, s, a, rows, cols, pitch,
                       static_cast<unsigned long long*>(partials));
    *nparts_out = nb;
    return hipGetLastError();
}

hipError_t launch_init_state(JobState* st, const void* count_parts, int nparts, hipStream_t s,
                             int64_t n_base) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st,
                       static_cast<const unsigned long long*>(count_parts), nparts, n_base);
    return hipGetLastError();
}

hipError_t launch_finalize_levels(JobState* st, const void* partials, const LoopCtl& c, int j0,
                                  int K, int tiles, JobState* mirror, hipStream_t s) {
    hipLaunchKernelGGL(finalize_levels_kernel, dim3(1), dim3(kFinThreads), 0, s, st, partials, c,
                       j0, K, tiles, mirror);
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
