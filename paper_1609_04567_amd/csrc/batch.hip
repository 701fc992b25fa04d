// Batched execution of many grids of uneven size: one launch sweeps every tile
// of every active job, one launch then folds each job's partials and evaluates
// its condition. A "round" is these two launches; every active job advances by
// one sweep per round, finished jobs' tiles exit at entry, and the host engine
// rebuilds the work list between windows of rounds (continuous batching).
//
// Each job keeps its own state (completed sweeps n, reduce value, stop flags),
// its own partials and its own ping-pong parity (sweep n+1 reads buf[n % 2]).
// A job's tile geometry depends only on its shape, dtype and alignment (see
// batch_geometry), never on the batch it shares, so the fold order of its reduce
// and hence every result is the same alone and in a mix.
#include "kernels.hpp"
#include "tile_jacobi.hpp"
#include "tile_life.hpp"

namespace lsr {
namespace {

constexpr int kBatchThreads = 256;
constexpr int kJacTileRows = 8;
constexpr int kLifeTileRows = 32;
constexpr int kLifeGenericMax = 2048;

template <typename T, int VEC, int U, bool NT>
__device__ __forceinline__ void jac_tile(const BatchJob& J, const void* src, void* dst, bool check,
                                         uint32_t sweep, int t, double* lds) {
    const T* a = static_cast<const T*>(src);
    T* b = static_cast<T*>(dst);
    const T* g = static_cast<const T*>(J.env);
    double* parts = static_cast<double*>(J.partials);
    if (J.helm)
        jacobi5_tile<T, true, VEC, 4, U, NT, NT>(a, b, g, J.rows, J.cols, J.pitch, (T)J.rd,
                                                 (T)(0.25 - J.rd), sweep, check,
                                                 J.ctl.reduce, t, J.strips, J.tile_rows, parts, lds);
    else
        jacobi5_tile<T, false, VEC, 4, U, NT, false>(a, b, g, J.rows, J.cols, J.pitch, (T)J.rd,
                                                     (T)0, sweep, check, J.ctl.reduce, t, J.strips, J.tile_rows,
                                                     parts, lds);
}

// Tiles of one kernel family; the work list segment of this launch holds only
// jobs of that family (one launch per family keeps each its own register budget).
template <int KIND>
__global__ __launch_bounds__(kBatchThreads) void batch_sweep_kernel(const BatchJob* __restrict__ jobs,
                                                                    const WorkItem* __restrict__ work) {
    __shared__ double lds_d[kBatchThreads / 64];
    __shared__ unsigned long long lds_u[kBatchThreads / 64];
    const WorkItem w = work[xcd_logical_tile(blockIdx.x, gridDim.x)];
    if (w.job < 0) return;
    const BatchJob& J = jobs[w.job];
    if (__hip_atomic_load(&J.st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n = __hip_atomic_load(&J.st->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n >= J.ctl.max_iter) return;
    const bool check = is_check_sweep(n + 1, J.ctl);
    const void* src = J.buf[n & 1];
    void* dst = const_cast<void*>(J.buf[(n + 1) & 1]);
    const uint32_t sw = (uint32_t)(n + 1);
    if (KIND == BK_JAC_F64_V2) jac_tile<double, 2, 8, true>(J, src, dst, check, sw, w.tile, lds_d);
    if (KIND == BK_JAC_F64_V1) jac_tile<double, 1, 4, false>(J, src, dst, check, sw, w.tile, lds_d);
    if (KIND == BK_JAC_F32_V4) jac_tile<float, 4, 8, true>(J, src, dst, check, sw, w.tile, lds_d);
    if (KIND == BK_JAC_F32_V1) jac_tile<float, 1, 4, false>(J, src, dst, check, sw, w.tile, lds_d);
    if (KIND == BK_LIFE_SWAR)
        life_swar_tile<4, 2, true>(static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst),
                                   J.rows, J.cols, J.pitch, J.torus, check, w.tile, J.strips,
                                   J.tile_rows, static_cast<unsigned long long*>(J.partials), lds_u);
    if (KIND == BK_LIFE_GEN)
        life_generic_tile(static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst), J.rows,
                          J.cols, J.pitch, J.torus, check, w.tile, J.tiles,
                          static_cast<unsigned long long*>(J.partials), lds_u);
}

// One workgroup per job: count the sweep, and on a check sweep fold the job's
// partials in index order and evaluate its condition.
__global__ __launch_bounds__(kBatchThreads) void batch_finalize_kernel(const BatchJob* __restrict__ jobs) {
    __shared__ double lds_d[kBatchThreads / 64];
    __shared__ unsigned long long lds_u[kBatchThreads / 64];
    const BatchJob& J = jobs[blockIdx.x];
    JobState* st = J.st;
    if (st->done) return;
    const int64_t n1 = st->n + 1;
    if (n1 > J.ctl.max_iter) return;
    const bool check = is_check_sweep(n1, J.ctl);
    double rd = 0.0;
    unsigned long long ru = 0;
    if (check) {
        if (J.ctl.reduce == RED_SUM)
            ru = fold_partials_u64<kBatchThreads>(static_cast<const unsigned long long*>(J.partials),
                                                  J.ctl.nparts, lds_u);
        else
            rd = fold_partials<kBatchThreads>(static_cast<const double*>(J.partials), J.ctl.nparts,
                                              J.ctl.reduce == RED_MAX_ABS, lds_d);
    }
    if (threadIdx.x != 0) return;
    JobState s = *st;
    s.n = n1;
    if (check) apply_check(s, J.ctl, n1, rd, ru);
    publish_state(st, J.mirror, s);
}

}  // namespace

void batch_geometry(BatchJob& j, int is_life, int f32, uintptr_t align_bits) {
    const bool aligned16 = (align_bits & 15) == 0;
    if (is_life) {
        if (j.cols % 16 == 0 && j.pitch % 16 == 0 && aligned16) {
            j.kind = BK_LIFE_SWAR;
            j.tile_rows = kLifeTileRows;
            const int64_t span = 4 * 1024;
            j.strips = (int)((j.cols + span - 1) / span);
            j.tiles = j.strips * (int)((j.rows + kLifeTileRows - 1) / kLifeTileRows);
        } else {
            j.kind = BK_LIFE_GEN;
            j.tile_rows = 0;
            j.strips = 0;
            const int64_t need = (j.rows * j.cols + 255) / 256;
            j.tiles = (int)(need < kLifeGenericMax ? need : kLifeGenericMax);
        }
        return;
    }
    const int esz = f32 ? 4 : 8;
    const int want = f32 ? 4 : 2;
    const int vec = ((j.pitch * esz) % 16 == 0 && aligned16) ? want : 1;
    j.kind = f32 ? (vec > 1 ? BK_JAC_F32_V4 : BK_JAC_F32_V1) : (vec > 1 ? BK_JAC_F64_V2 : BK_JAC_F64_V1);
    j.tile_rows = kJacTileRows;
    const int64_t span = (int64_t)4 * 64 * vec;
    j.strips = (int)((j.cols + span - 1) / span);
    j.tiles = j.strips * (int)((j.rows - 2 + kJacTileRows - 1) / kJacTileRows);
}

hipError_t launch_batch_sweep(const BatchJob* jobs, const WorkItem* work, int kind,
                              int nwork_padded, hipStream_t s) {
    if (nwork_padded <= 0) return hipSuccess;
    const dim3 g(nwork_padded), b(kBatchThreads);
    switch (kind) {
        case BK_JAC_F64_V2: hipLaunchKernelGGL(batch_sweep_kernel<BK_JAC_F64_V2>, g, b, 0, s, jobs, work); break;
        case BK_JAC_F64_V1: hipLaunchKernelGGL(batch_sweep_kernel<BK_JAC_F64_V1>, g, b, 0, s, jobs, work); break;
        case BK_JAC_F32_V4: hipLaunchKernelGGL(batch_sweep_kernel<BK_JAC_F32_V4>, g, b, 0, s, jobs, work); break;
        case BK_JAC_F32_V1: hipLaunchKernelGGL(batch_sweep_kernel<BK_JAC_F32_V1>, g, b, 0, s, jobs, work); break;
        case BK_LIFE_SWAR: hipLaunchKernelGGL(batch_sweep_kernel<BK_LIFE_SWAR>, g, b, 0, s, jobs, work); break;
        case BK_LIFE_GEN: hipLaunchKernelGGL(batch_sweep_kernel<BK_LIFE_GEN>, g, b, 0, s, jobs, work); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchJob* jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(njobs), dim3(kBatchThreads), 0, s, jobs);
    return hipGetLastError();
}

}  // namespace lsr
