// Batched execution of many grids of uneven size: one launch sweeps every tile
// of every active job, one launch then folds each job's partials and evaluates
// its condition. A "round" is these two launches; every active job advances by
// its step (1 sweep, or K sweeps for a job on a fused-depth family), finished
// jobs' tiles exit at entry, and the host engine rebuilds the work list between
// windows of rounds (continuous batching).
//
// A tile belongs to one wavefront: a workgroup of four wavefronts runs four work
// items, possibly of four different jobs, so a narrow grid occupies only the
// wavefronts its columns need. Each job keeps its own state (completed sweeps n,
// reduce value, stop flags), its own partials and its own ping-pong parity
// (its launch number n / step selects the source buffer). A job's tile geometry
// and family depend only on its shape, dtype and condition (see
// batch_geometry), never on the batch it shares, so the fold order of its
// reduce and hence every result is the same alone and in a mix.
#include <type_traits>

#include "kernels.hpp"
#include "tile_jacobi.hpp"
#include "tile_life.hpp"
#include "tile_life_tb.hpp"
#include "tile_restore.hpp"
#include "tile_sobel.hpp"

namespace lsr {
namespace {

constexpr int kBatchThreads = 256;
constexpr int kWavesPerGroup = kBatchThreads / 64;
constexpr int kLifeTileRows = 32;
constexpr int kLifeTbRows = 64;   // band of a fused Life tile (8 generations: 16 halo rows)
constexpr int kRestoreTileRows = 16;

template <typename T, int VEC, int K, bool MC>
__device__ __forceinline__ void jac_tb_tile(const BatchJob& J, const void* src, void* dst,
                                            uint32_t mask, uint32_t sweep0, int t, T* gring) {
    const T* a = static_cast<const T*>(src);
    T* b = static_cast<T*>(dst);
    const T* g = static_cast<const T*>(J.env);
    double* parts = static_cast<double*>(J.partials);
    // each stencil's usual reduce (Helmholtz L2, Laplace max |delta|) compiled in,
    // so the per-level delta sums carry no selects between the reduce kinds
    if (J.helm) {
        if (J.ctl.reduce == RED_L2)
            jacobi5_tb_tile<T, true, VEC, 1, K, true, true, true, MC, false, false, 0, RED_L2>(
                a, b, g, J.rows, J.cols, J.pitch, (T)J.rd, (T)(0.25 - J.rd), sweep0, mask,
                J.ctl.reduce, t, J.strips, J.tiles, J.tile_rows, parts, nullptr, gring);
        else
            jacobi5_tb_tile<T, true, VEC, 1, K, true, true, true, MC>(
                a, b, g, J.rows, J.cols, J.pitch, (T)J.rd, (T)(0.25 - J.rd), sweep0, mask,
                J.ctl.reduce, t, J.strips, J.tiles, J.tile_rows, parts, nullptr, gring);
    } else {
        if (J.ctl.reduce == RED_MAX_ABS)
            jacobi5_tb_tile<T, false, VEC, 1, K, true, false, true, MC, false, false, 0, RED_MAX_ABS>(
                a, b, g, J.rows, J.cols, J.pitch, (T)J.rd, (T)0, sweep0, mask, J.ctl.reduce, t,
                J.strips, J.tiles, J.tile_rows, parts, nullptr, gring);
        else
            jacobi5_tb_tile<T, false, VEC, 1, K, true, false, true, MC>(
                a, b, g, J.rows, J.cols, J.pitch, (T)J.rd, (T)0, sweep0, mask, J.ctl.reduce, t,
                J.strips, J.tiles, J.tile_rows, parts, nullptr, gring);
    }
}

// Per family: sweeps per round, element type width (0 = Life), and whether a
// round may hold several checks.
template <int KIND> struct KindInfo { static constexpr int step = 1, vec = 0; static constexpr bool mc = false; };
template <> struct KindInfo<BK_JAC_F64_TB10> { static constexpr int step = 10, vec = 2; static constexpr bool mc = false; };
template <> struct KindInfo<BK_JAC_F64_TB5> { static constexpr int step = 5, vec = 2; static constexpr bool mc = false; };
template <> struct KindInfo<BK_JAC_F64_TB2> { static constexpr int step = 2, vec = 2; static constexpr bool mc = false; };
template <> struct KindInfo<BK_JAC_F32_TB5> { static constexpr int step = 5, vec = 4; static constexpr bool mc = false; };
template <> struct KindInfo<BK_JAC_F32_TB2> { static constexpr int step = 2, vec = 4; static constexpr bool mc = false; };
template <> struct KindInfo<BK_JAC_F64_TB5_MC> { static constexpr int step = 5, vec = 2; static constexpr bool mc = true; };
template <> struct KindInfo<BK_JAC_F32_TB5_MC> { static constexpr int step = 5, vec = 4; static constexpr bool mc = true; };
template <> struct KindInfo<BK_LIFE_TB8> { static constexpr int step = 8, vec = 0; static constexpr bool mc = true; };

// Work items of one kernel family; the work list segment of this launch holds only
// jobs of that family (one launch per family keeps each its own register budget).
template <int KIND>
__global__ __launch_bounds__(kBatchThreads) void batch_sweep_kernel(const BatchJob* __restrict__ jobs,
                                                                    const WorkItem* __restrict__ work) {
    constexpr int STEP = KindInfo<KIND>::step, VEC = KindInfo<KIND>::vec;
    constexpr bool MC = KindInfo<KIND>::mc;
    __shared__ __attribute__((aligned(16))) double ring_d[VEC == 2 ? tb_gring_elems<2, kWavesPerGroup, STEP>() : 1];
    __shared__ __attribute__((aligned(16))) float ring_f[VEC == 4 ? tb_gring_elems<4, kWavesPerGroup, STEP>() : 1];
    // the wavefront index is wave-uniform: the work item and its job load as scalars
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const WorkItem w = work[xcd_logical_tile(blockIdx.x, gridDim.x) * kWavesPerGroup + wave];
    if (w.job < 0) return;
    const BatchJob& J = jobs[w.job];
    if (__hip_atomic_load(&J.st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n = __hip_atomic_load(&J.st->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n >= J.ctl.max_iter) return;
    // sweeps n+1 .. n+STEP; without MC, STEP divides the check period and the cap
    uint32_t mask = 0;
#pragma unroll
    for (int lev = 1; lev <= STEP; ++lev)
        if (n + lev <= J.ctl.max_iter && is_check_sweep(n + lev, J.ctl)) mask |= 1u << (lev - 1);
    if (!MC) mask &= 1u << (STEP - 1);
    const int64_t launch = n / STEP;
    const void* src = J.buf[launch & 1];
    void* dst = const_cast<void*>(J.buf[(launch + 1) & 1]);
    const uint32_t sw = (uint32_t)(n + 1);
    if constexpr (VEC == 2) jac_tb_tile<double, 2, STEP, MC>(J, src, dst, mask, sw, w.tile, ring_d);
    if constexpr (VEC == 4) jac_tb_tile<float, 4, STEP, MC>(J, src, dst, mask, sw, w.tile, ring_f);
    const bool check = mask != 0;
    if constexpr (KIND == BK_LIFE_SWAR)
        life_swar_tile<1, 8, true, true>(static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst),
                                         J.rows, J.cols, J.pitch, J.torus, check, w.tile, J.strips,
                                         J.tile_rows, static_cast<unsigned long long*>(J.partials),
                                         nullptr);
    if constexpr (KIND == BK_LIFE_TB8) {
        // generations n+1 .. n+8 of one band of one window; generation n+l's count
        // goes to partials[(l - 1) * tiles + tile]
        const int band = w.tile / J.strips, strip = w.tile - band * J.strips;
        uint32_t cnt[STEP];
#pragma unroll
        for (int l = 0; l < STEP; ++l) cnt[l] = 0;
        const uint8_t* a = static_cast<const uint8_t*>(src);
        uint8_t* b = static_cast<uint8_t*>(dst);
        if (J.torus && J.cols % 16 == 0)
            life_tb_band<STEP, 3, true>(a, b, J.rows, J.cols, J.pitch, mask, band, strip, J.tile_rows, cnt);
        else if (J.torus)
            life_tb_band<STEP, 3, true, true>(a, b, J.rows, J.cols, J.pitch, mask, band, strip,
                                              J.tile_rows, cnt);
        else if (J.cols % 16 == 0)
            life_tb_band<STEP, 3, false>(a, b, J.rows, J.cols, J.pitch, mask, band, strip, J.tile_rows, cnt);
        else
            life_tb_band<STEP, 3, false, true>(a, b, J.rows, J.cols, J.pitch, mask, band, strip,
                                               J.tile_rows, cnt);
        auto* parts = static_cast<unsigned long long*>(J.partials);
#pragma unroll
        for (int l = 0; l < STEP; ++l) {
            if ((mask >> l) & 1u) {
                const unsigned long long v = wave_sum_u64(cnt[l]);
                if ((threadIdx.x & 63) == 0) parts[(size_t)l * (size_t)J.tiles + w.tile] = v;
            }
        }
    }
    if constexpr (KIND == BK_RESTORE_F64 || KIND == BK_RESTORE_F32) {
        typedef typename std::conditional<KIND == BK_RESTORE_F64, double, float>::type T;
        __shared__ uint16_t rlist[kWavesPerGroup][kRestoreTileRows * 64];
        const int band = w.tile / J.strips, strip = w.tile - band * J.strips;
        const bool is_max = J.ctl.reduce == RED_MAX_ABS;
        double acc = restore_wave<T, false>(
            static_cast<const T*>(src), static_cast<T*>(dst), static_cast<const uint8_t*>(J.env),
            J.rows, J.cols, J.pitch, (T)J.beta, J.quadratic != 0, (int64_t)band * kRestoreTileRows,
            0, 1, kRestoreTileRows, (int64_t)strip * 64, rlist[wave], check, is_max);
        if (check) {
            acc = is_max ? wave_max(acc) : wave_sum(acc);
            if ((threadIdx.x & 63) == 0) static_cast<double*>(J.partials)[w.tile] = acc;
        }
    }
    if constexpr (KIND == BK_SOBEL) {
        __shared__ __attribute__((aligned(16))) uint8_t slds[kWavesPerGroup][kSobelLdsBytes];
        const int band = w.tile / J.strips, strip = w.tile - band * J.strips;
        unsigned long long acc =
            sobel_wave(static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst), J.rows, J.cols,
                       J.pitch, (int64_t)band * kSobelRows, (int64_t)strip * kSobelCols, slds[wave]);
        if (check) {
            acc = wave_sum_u64(acc);
            if ((threadIdx.x & 63) == 0) static_cast<unsigned long long*>(J.partials)[w.tile] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Whole-grid-in-LDS execution of a small job (both buffers fit in the 160 KiB of
// one CU's LDS): one 1024-thread workgroup loads the grid once, runs the whole
// loop in LDS (sweep, reduce, condition, as in the -d/-s procedures of
// Sect. 3.1, with the same per-cell update and stopping rule as the tiled
// path), then writes the stop iterate to buf[n % 2] and publishes the state.
// Cells are dealt to threads in row-major order; the reduce is the fixed
// workgroup tree. A small job therefore finishes within one round; a cancel
// posted while it runs takes effect only if it arrives before that round.
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / 64;

template <typename T, bool HELM>
__device__ void small_jacobi(const BatchJob& J, T* A, T* B, double* red_lds, int* flag) {
    const int tid = threadIdx.x;
    const int64_t rows = J.rows, cols = J.cols, cells = rows * cols;
    JobState s = *J.st;
    const T* src = static_cast<const T*>(J.buf[s.n & 1]);
    for (int64_t k = tid; k < cells; k += kSmallThreads) {
        const int64_t i = k / cols, jj = k - i * cols;
        A[k] = B[k] = src[i * J.pitch + jj];   // B keeps the fixed ring too
    }
    __syncthreads();
    const T* g = static_cast<const T*>(J.env);
    const T rd = (T)J.rd, rd_lo = (T)(0.25 - J.rd);
    // the grid fits in LDS, so cell indices fit in 32 bits. Wavefront w takes
    // interior rows 1 + w, 1 + w + 16, ..., its lanes consecutive columns (no
    // division per cell; a narrow grid's rows still spread over the wavefronts).
    const int cols32 = (int)cols, rows32 = (int)rows;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    int64_t n = s.n;
    while (n < J.ctl.max_iter) {
        const int64_t n1 = n + 1;
        const bool check = is_check_sweep(n1, J.ctl);
        double acc = 0.0;
        for (int i = 1 + wave; i < rows32 - 1; i += kSmallWaves) {
            const T* grow = HELM ? g + (int64_t)i * J.pitch : nullptr;
            for (int jj = 1 + lane; jj < cols32 - 1; jj += 64) {
                const int c = i * cols32 + jj;
                const T v = jacobi_update<T, HELM>(A[c - cols32], A[c + cols32], A[c - 1], A[c + 1],
                                                   HELM ? grow[jj] : T(0), rd, rd_lo, (int64_t)i,
                                                   (int64_t)jj, (uint32_t)n1);
                if (check) acc = jacobi_accum(J.ctl.reduce, acc, (double)v - (double)A[c]);
                B[c] = v;
            }
        }
        __syncthreads();
        T* t = A;
        A = B;
        B = t;
        n = n1;
        if (check) {
            const double r = block_reduce<kSmallWaves>(acc, J.ctl.reduce == RED_MAX_ABS, red_lds);
            if (tid == 0) {
                apply_check(s, J.ctl, n1, r, 0);
                *flag = s.done;
            }
            __syncthreads();
            if (*flag) break;
        }
    }
    T* dst = static_cast<T*>(const_cast<void*>(J.buf[n & 1]));
    for (int64_t k = tid; k < cells; k += kSmallThreads) {
        const int64_t i = k / cols, jj = k - i * cols;
        dst[i * J.pitch + jj] = A[k];
    }
    if (tid == 0) publish_state(J.st, J.mirror, s);
}

__device__ void small_life(const BatchJob& J, uint8_t* A, uint8_t* B, unsigned long long* red_lds,
                           int* flag) {
    // LDS rows of small_life_words(cols) 32-bit words, one byte per cell: byte 3 of
    // word 0 is a ghost copy of the row's last cell, bytes 4 .. cols + 3 are the
    // cells, byte cols + 4 is a ghost copy of the first cell (torus; both ghosts 0
    // on a dead border), every other byte 0. A thread takes one word (4 cells) of
    // one row: column sums of the three rows, the two outer neighbours from the
    // next words' edge bytes, and B3/S23 as (T - c | c) == 3 per byte, T the 3x3
    // total. Bytes past the last cell are masked to 0 and the ghosts refreshed
    // after every generation.
    const int tid = threadIdx.x;
    const int rows = (int)J.rows, cols = (int)J.cols;
    const int wt = small_life_words(cols);   // words per LDS row
    const int nw = (cols + 3) / 4;           // words holding cells: 1 .. nw
    const int lastb = cols + 3;              // byte index of the last cell in a row
    const bool torus = J.torus != 0;
    uint32_t* A32 = reinterpret_cast<uint32_t*>(A);
    uint32_t* B32 = reinterpret_cast<uint32_t*>(B);
    JobState s = *J.st;
    const uint8_t* src = static_cast<const uint8_t*>(J.buf[s.n & 1]);
    for (int k = tid; k < 2 * rows * wt; k += kSmallThreads) A32[k] = 0;   // both buffers
    __syncthreads();
    for (int64_t k = tid; k < (int64_t)rows * cols; k += kSmallThreads) {
        const int i = (int)(k / cols), jj = (int)(k - (int64_t)i * cols);
        A[i * wt * 4 + 4 + jj] = src[i * J.pitch + jj];   // 0/1 after the job's initial count pass
    }
    __syncthreads();
    auto ghosts = [&](uint8_t* G) {
        if (!torus) return;
        for (int i = tid; i < rows; i += kSmallThreads) {
            uint8_t* r = G + i * wt * 4;
            const uint8_t first = r[4], last = r[lastb];
            r[3] = last;
            r[cols + 4] = first;
        }
    };
    ghosts(A);
    __syncthreads();
    int64_t n = s.n;
    while (n < J.ctl.max_iter) {
        const int64_t n1 = n + 1;
        const bool check = is_check_sweep(n1, J.ctl);
        uint32_t cnt = 0;
        for (int k = tid; k < rows * nw; k += kSmallThreads) {
            const int i = k / nw, w = k - i * nw + 1;
            const int iu = i > 0 ? i - 1 : (torus ? rows - 1 : -1);
            const int id = i + 1 < rows ? i + 1 : (torus ? 0 : -1);
            const uint32_t* c = A32 + i * wt + w;
            uint32_t V0 = c[-1], V1 = c[0], V2 = c[1];
            const uint32_t mid = V1;
            if (iu >= 0) {
                const uint32_t* u = A32 + iu * wt + w;
                V0 += u[-1];
                V1 += u[0];
                V2 += u[1];
            }
            if (id >= 0) {
                const uint32_t* d = A32 + id * wt + w;
                V0 += d[-1];
                V1 += d[0];
                V2 += d[1];
            }
            // bytes hold column sums <= 3; the 3x3 totals <= 9 stay inside their bytes
            const uint32_t T = ((V1 << 8) | (V0 >> 24)) + V1 + ((V1 >> 8) | (V2 << 24));
            uint32_t out = zero_bytes_hi(((T - mid) | mid) ^ 0x03030303u) >> 7;
            const int spare = 4 * w + 3 - lastb;   // bytes of this word past the last cell
            if (spare > 0) out &= 0xFFFFFFFFu >> (8 * spare);
            B32[i * wt + w] = out;
            cnt += (uint32_t)__popc(out);
        }
        __syncthreads();
        ghosts(B);
        __syncthreads();
        uint8_t* t = A;
        A = B;
        B = t;
        A32 = reinterpret_cast<uint32_t*>(A);
        B32 = reinterpret_cast<uint32_t*>(B);
        n = n1;
        if (check) {
            const unsigned long long total = block_reduce_u64<kSmallWaves>(cnt, red_lds);
            if (tid == 0) {
                apply_check(s, J.ctl, n1, 0.0, total);
                *flag = s.done;
            }
            __syncthreads();
            if (*flag) break;
        }
    }
    uint8_t* dst = static_cast<uint8_t*>(const_cast<void*>(J.buf[n & 1]));
    for (int64_t k = tid; k < (int64_t)rows * cols; k += kSmallThreads) {
        const int i = (int)(k / cols), jj = (int)(k - (int64_t)i * cols);
        dst[i * J.pitch + jj] = A[i * wt * 4 + 4 + jj];
    }
    if (tid == 0) publish_state(J.st, J.mirror, s);
}

// The job's descriptor travels by value: the engine rebuilds its device job table
// while a small job may still be running on its own stream.
template <int KIND>
__global__ __launch_bounds__(kSmallThreads) void batch_small_kernel(const BatchJob J) {
    __shared__ __attribute__((aligned(16))) unsigned char grid_lds[kSmallLdsBytes];
    __shared__ double red_d[kSmallWaves];
    __shared__ unsigned long long red_u[kSmallWaves];
    __shared__ int flag;
    if (J.st->done || J.st->n >= J.ctl.max_iter) return;
    const int64_t cells = J.rows * J.cols;
    if (KIND == BK_SMALL_F64) {
        double* A = reinterpret_cast<double*>(grid_lds);
        if (J.helm) small_jacobi<double, true>(J, A, A + cells, red_d, &flag);
        else small_jacobi<double, false>(J, A, A + cells, red_d, &flag);
    } else if (KIND == BK_SMALL_F32) {
        float* A = reinterpret_cast<float*>(grid_lds);
        if (J.helm) small_jacobi<float, true>(J, A, A + cells, red_d, &flag);
        else small_jacobi<float, false>(J, A, A + cells, red_d, &flag);
    } else {
        small_life(J, grid_lds, grid_lds + J.rows * small_life_words(J.cols) * 4, red_u, &flag);
    }
}

// One workgroup per job: count the job's round, and fold and evaluate each check
// the round holds, in sweep order (the last level's only, without mc), stopping
// at the first that ends the loop.
__global__ __launch_bounds__(kBatchThreads) void batch_finalize_kernel(const BatchJob* __restrict__ jobs) {
    __shared__ double lds_d[kBatchThreads / 64];
    __shared__ unsigned long long lds_u[kBatchThreads / 64];
    __shared__ int stop;
    const BatchJob& J = jobs[blockIdx.x];
    JobState* st = J.st;
    if (st->done) return;
    const int64_t n0 = st->n;
    if (n0 + 1 > J.ctl.max_iter) return;
    JobState s = *st;   // only thread 0's copy is updated
    for (int lev = J.mc ? 1 : J.step; lev <= J.step; ++lev) {
        const int64_t n = n0 + lev;
        if (n > J.ctl.max_iter) break;
        if (!is_check_sweep(n, J.ctl)) continue;
        const size_t off = J.mc ? (size_t)(lev - 1) * (size_t)J.tiles : 0;
        double rd = 0.0;
        unsigned long long ru = 0;
        if (J.ctl.reduce == RED_SUM)
            ru = fold_partials_u64<kBatchThreads>(
                static_cast<const unsigned long long*>(J.partials) + off, J.ctl.nparts, lds_u);
        else
            rd = fold_partials<kBatchThreads>(static_cast<const double*>(J.partials) + off,
                                              J.ctl.nparts, J.ctl.reduce == RED_MAX_ABS, lds_d);
        if (threadIdx.x == 0) {
            apply_check(s, J.ctl, n, rd, ru);
            stop = s.done;
        }
        __syncthreads();   // thread 0 is done with lds before the next fold
        if (stop) break;
    }
    if (threadIdx.x != 0) return;
    if (!s.done) s.n = n0 + J.step;
    publish_state(st, J.mirror, s);
}

template <int KIND>
void launch_kind(const BatchJob* jobs, const WorkItem* work, int groups, hipStream_t s) {
    hipLaunchKernelGGL(batch_sweep_kernel<KIND>, dim3(groups), dim3(kBatchThreads), 0, s, jobs, work);
}

}  // namespace

void batch_geometry(BatchJob& j, int is_life, int f32, int want_depth, int want_tile_rows) {
    j.step = 1;
    j.mc = 0;
    if (batch_small_fits(j.rows, j.cols, is_life ? 1 : f32 ? 4 : 8)) {
        j.kind = is_life ? BK_SMALL_LIFE : f32 ? BK_SMALL_F32 : BK_SMALL_F64;
        j.tile_rows = (int)j.rows;
        j.strips = 1;
        j.tiles = 1;   // one work item = the whole job; no partials
        return;
    }
    if (is_life && want_depth != 1) {
        // rows are 16-byte aligned and may end in padding (zeroed at the start)
        j.kind = BK_LIFE_TB8;
        j.step = KindInfo<BK_LIFE_TB8>::step;
        j.mc = 1;
        j.tile_rows = want_tile_rows > 0 ? want_tile_rows : kLifeTbRows;
        j.strips = (int)((j.cols + kLifeTbWinCols - 1) / kLifeTbWinCols);
        j.tiles = j.strips * (int)((j.rows + j.tile_rows - 1) / j.tile_rows);
        return;
    }
    if (is_life) {
        // rows are 16-byte aligned with zeroed padding to a multiple of 16 cells
        j.kind = BK_LIFE_SWAR;
        j.tile_rows = want_tile_rows > 0 ? want_tile_rows : kLifeTileRows;
        j.strips = (int)((j.cols + 1023) / 1024);
        j.tiles = j.strips * (int)((j.rows + j.tile_rows - 1) / j.tile_rows);
        return;
    }
    // rows are 16-byte aligned (the engine stages any other grid)
    const int vec = f32 ? 4 : 2;
    int depth = 0;
    const auto depths = f32 ? std::initializer_list<int>{5, 2} : std::initializer_list<int>{10, 5, 2};
    for (int k : depths)   // a requested depth the families hold, if it divides both
        if (k == want_depth && j.ctl.check_every % k == 0 && j.ctl.max_iter % k == 0) depth = k;
    if (depth == 0 && want_depth != 5)
        for (int k : depths)
            if (j.ctl.check_every % k == 0 && j.ctl.max_iter % k == 0) { depth = k; break; }
    if (depth == 0) {
        depth = 5;
        j.mc = 1;
        j.kind = f32 ? BK_JAC_F32_TB5_MC : BK_JAC_F64_TB5_MC;
    } else {
        j.kind = f32 ? (depth == 5 ? BK_JAC_F32_TB5 : BK_JAC_F32_TB2)
                     : (depth == 10 ? BK_JAC_F64_TB10 : depth == 5 ? BK_JAC_F64_TB5 : BK_JAC_F64_TB2);
    }
    j.step = depth;
    j.tile_rows = want_tile_rows > 0 ? want_tile_rows : depth >= 8 ? 48 : 32;
    const int64_t ow = (64 * vec - 2 * depth) / vec * vec;
    const int64_t need = j.cols - 1 - depth;
    j.strips = (int)(need > 0 ? (need + ow - 1) / ow : 1);
    j.tiles = j.strips * (int)((j.rows - 2 + j.tile_rows - 1) / j.tile_rows);
}

void batch_geometry_restore(BatchJob& j, int f32) {
    j.step = 1;
    j.mc = 0;
    j.kind = f32 ? BK_RESTORE_F32 : BK_RESTORE_F64;
    j.tile_rows = kRestoreTileRows;
    j.strips = (int)((j.cols + 63) / 64);
    j.tiles = j.strips * (int)((j.rows + kRestoreTileRows - 1) / kRestoreTileRows);
}

void batch_geometry_sobel(BatchJob& j) {
    j.step = 1;
    j.mc = 0;
    j.kind = BK_SOBEL;
    j.tile_rows = kSobelRows;
    j.strips = (int)((j.cols + kSobelCols - 1) / kSobelCols);
    j.tiles = j.strips * (int)((j.rows + kSobelRows - 1) / kSobelRows);
}

hipError_t launch_batch_sweep(const BatchJob* jobs, const WorkItem* work, int kind,
                              int nwork_padded, hipStream_t s) {
    if (nwork_padded <= 0) return hipSuccess;
    if (nwork_padded % (kWavesPerGroup * kXcds)) return hipErrorInvalidValue;
    const int groups = nwork_padded / kWavesPerGroup;
    switch (kind) {
        case BK_JAC_F64_TB10: launch_kind<BK_JAC_F64_TB10>(jobs, work, groups, s); break;
        case BK_JAC_F64_TB5: launch_kind<BK_JAC_F64_TB5>(jobs, work, groups, s); break;
        case BK_JAC_F64_TB2: launch_kind<BK_JAC_F64_TB2>(jobs, work, groups, s); break;
        case BK_JAC_F32_TB5: launch_kind<BK_JAC_F32_TB5>(jobs, work, groups, s); break;
        case BK_JAC_F32_TB2: launch_kind<BK_JAC_F32_TB2>(jobs, work, groups, s); break;
        case BK_JAC_F64_TB5_MC: launch_kind<BK_JAC_F64_TB5_MC>(jobs, work, groups, s); break;
        case BK_JAC_F32_TB5_MC: launch_kind<BK_JAC_F32_TB5_MC>(jobs, work, groups, s); break;
        case BK_LIFE_SWAR: launch_kind<BK_LIFE_SWAR>(jobs, work, groups, s); break;
        case BK_RESTORE_F64: launch_kind<BK_RESTORE_F64>(jobs, work, groups, s); break;
        case BK_RESTORE_F32: launch_kind<BK_RESTORE_F32>(jobs, work, groups, s); break;
        case BK_SOBEL: launch_kind<BK_SOBEL>(jobs, work, groups, s); break;
        case BK_LIFE_TB8: launch_kind<BK_LIFE_TB8>(jobs, work, groups, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_small(const BatchJob& j, hipStream_t s) {
    const dim3 g(1), b(kSmallThreads);
    switch (j.kind) {
        case BK_SMALL_F64: hipLaunchKernelGGL(batch_small_kernel<BK_SMALL_F64>, g, b, 0, s, j); break;
        case BK_SMALL_F32: hipLaunchKernelGGL(batch_small_kernel<BK_SMALL_F32>, g, b, 0, s, j); break;
        case BK_SMALL_LIFE: hipLaunchKernelGGL(batch_small_kernel<BK_SMALL_LIFE>, g, b, 0, s, j); break;
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
