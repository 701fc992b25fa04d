// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace lsr {

// Geometry of one sweep launch: tiles of `tile_rows` rows x the columns covered
// by one workgroup, enumerated band-major, padded to a multiple of 8 workgroups.
struct SweepGeom {
    int vec = 1;         // elements per lane (1, 2 or 4)
    int waves = 4;       // waves per workgroup
    int unroll = 4;      // rows whose loads are issued together
    int tile_rows = 32;  // rows streamed per workgroup
    int strips = 0;      // column strips
    int bands = 0;       // row bands
    int tiles = 0;       // strips * bands (= partials per check sweep)
    int blocks = 0;      // tiles padded to a multiple of 8
    int tb = 1;          // sweeps advanced per launch (temporal blocking depth)
    int mc = 0;          // fused launches may hold several checks (partials per level)
    int vert = 0;        // fused Jacobi: a workgroup's waves take consecutive bands of one window
};

// Jacobi 5-point (Laplace / Helmholtz) -------------------------------------
struct JacobiArgs {
    const void* a;       // current iterate
    void* b;             // next iterate
    const void* g;       // Helmholtz env (same dtype), or nullptr
    int64_t rows, cols, pitch;
    double rd;           // 1 / (4 + alpha h^2) (Helmholtz)
    int helm;            // 0 Laplace, 1 Helmholtz
    int f32;             // 0 FP64 storage, 1 FP32 storage
    // the -i form (helm must be set): g(i, j) = c2 * (c1 * (sp[i] * sq[j])) from the
    // cell's indices instead of the env array g
    int sep = 0;
    const double* sp = nullptr;
    const double* sq = nullptr;
    double c1 = 0.0, c2 = 0.0;
};
// tile_rows / waves / unroll of 0 (or an unsupported pair) select the measured default.
// depth > 1 selects the temporally blocked kernel (one launch = `depth` sweeps)
// when it is a compiled depth and the grid takes the vector path; the caller
// checks g.tb for what was chosen. With g.tb = K, launch_jacobi's j is the
// offset of the launch's first sweep (a multiple of K) and the result lands in b.
// mc: launches may hold several checks (see jacobi_tb_choose).
SweepGeom jacobi_geom(const JacobiArgs& a, int tile_rows, int waves = 0, int unroll = 0,
                      int depth = 1, int mc = 0);
hipError_t launch_jacobi(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                         const LoopCtl& c, int j, hipStream_t s);
bool jacobi_tb_depth_ok(int depth);
// Fused depth for a job: `requested` (0 = automatic, 1 = unfused, else that depth
// if compiled); *mc = 1 when some check falls inside a launch (the check period
// or the cap is not a multiple of the depth).
void jacobi_tb_choose(const JacobiArgs& a, int check_every, int64_t max_iter, int requested,
                      int* depth, int* mc);
void jacobi_tb_geom(const JacobiArgs& a, int depth, int mc, int tile_rows, int waves, int unroll,
                    SweepGeom& g);
hipError_t launch_jacobi_tb(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                            const LoopCtl& c, int j, hipStream_t s);

// Game of Life B3/S23 --------------------------------------------------------
struct LifeArgs {
    const uint8_t* a;
    uint8_t* b;
    int64_t rows, cols, pitch;
    int torus;
    int padded;          // rows hold round_up(cols, 16) bytes, the padding zero at start
};
// Rows the SWAR kernel can sweep: 16-byte aligned, and a multiple of 16 cells
// or padded. launch_life rejects anything else.
bool life_rows_ok(const LifeArgs& a);
SweepGeom life_geom(const LifeArgs& a, int tile_rows);
hipError_t launch_life(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                       const LoopCtl& c, int j, hipStream_t s);
// Temporally blocked Life (life_tb.hip): g.tb generations per launch, the count of
// each checked generation in its own slice of partials (g.mc). Rows must be
// 16-byte aligned and hold a multiple of 16 cells, or be padded (life_tb_ok).
bool life_tb_ok(const LifeArgs& a);
// True for a compiled fused Life depth (2, 3, 4, 5, 6, 8).
bool life_tb_depth_ok(int depth);
// Generations per launch for a job: `requested` (0 = automatic, 1 = unfused, or
// a compiled depth), 1 when the rows do not qualify.
int life_tb_choose(const LifeArgs& a, int requested);
SweepGeom life_tb_geom(const LifeArgs& a, int depth, int tile_rows);
hipError_t launch_life_tb(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                          const LoopCtl& c, int j, hipStream_t s);
// Live-cell count of a u8 grid into partials (one per block), normalising bytes
// above 1 to 1 in place; returns the partial count.
hipError_t launch_count_u8(uint8_t* a, int64_t rows, int64_t cols, int64_t pitch,
                           void* partials, int* nparts_out, hipStream_t s);
int count_u8_parts(int64_t rows, int64_t cols);

// Restoration (phase 2) and detection (phase 1) ----------------------------
struct RestoreArgs {
    const void* a;
    void* b;
    const uint8_t* mask;
    int64_t rows, cols, pitch;
    double beta;
    int quadratic;
    int f32;
};
SweepGeom restore_geom(const RestoreArgs& a, int tile_rows);
hipError_t launch_restore(const RestoreArgs& a, const SweepGeom& g, JobState* st, void* partials,
                          const LoopCtl& c, int j, hipStream_t s);
hipError_t launch_amf_detect(const uint8_t* y, int64_t rows, int64_t cols, int64_t pitch,
                             int w_max, uint8_t* mask, void* u_init, int u_dtype, hipStream_t s);

// Radius-k box stencil and 3D 7-point Jacobi (generic.hip) -------------------------
SweepGeom box_geom(int64_t rows, int64_t cols);
hipError_t launch_box(const void* a, void* b, int64_t rows, int64_t cols, int64_t pitch, int k,
                      int f32, const SweepGeom& g, JobState* st, void* partials, const LoopCtl& c,
                      int j, hipStream_t s);
// the grid holds nz planes of ny rows (rows = nz * ny), each row `pitch` elements
SweepGeom laplace3d_geom(int64_t nz, int64_t ny, int64_t nx);
hipError_t launch_laplace3d(const void* a, void* b, int64_t nz, int64_t ny, int64_t nx,
                            int64_t pitch, int f32, const SweepGeom& g, JobState* st,
                            void* partials, const LoopCtl& c, int j, hipStream_t s);

// Sobel edge detector (u8 in, u8 out; partials are u64 sums of the new image) ----
SweepGeom sobel_geom(int64_t rows, int64_t cols);
hipError_t launch_sobel(const uint8_t* a, uint8_t* b, int64_t rows, int64_t cols, int64_t pitch,
                        const SweepGeom& g, JobState* st, void* partials, const LoopCtl& c, int j,
                        hipStream_t s);

// Batched execution ----------------------------------------------------------
// Kernel family of one job inside a batch; every batch kernel uses 256-thread
// workgroups (4 wavefronts).
enum BatchKind : int32_t {
    BK_JAC_F64_TB10 = 1,   // FP64 Jacobi, 10 fused sweeps per round, check on the last
    BK_JAC_F64_TB5 = 2,
    BK_JAC_F64_TB2 = 3,
    BK_JAC_F32_TB5 = 4,    // FP32 Jacobi, 5 fused sweeps per round, check on the last
    BK_JAC_F32_TB2 = 5,
    BK_JAC_F64_TB5_MC = 6, // FP64 Jacobi, 5 fused sweeps per round, any checks inside
    BK_JAC_F32_TB5_MC = 7,
    BK_LIFE_SWAR = 8,      // Life, 16 cells per lane, one generation per round
    BK_SMALL_F64 = 9,      // whole job in LDS, one launch on the engine's second stream: FP64 Jacobi
    BK_SMALL_F32 = 10,     //   FP32 Jacobi
    BK_SMALL_LIFE = 11,    //   Life
    BK_RESTORE_F64 = 12,   // restoration sweep (phase 2 of Sect. 4.3), FP64, 16 x 64 pixels per tile
    BK_RESTORE_F32 = 13,   //   FP32 storage
    BK_SOBEL = 14,         // Sobel edge detector, 8 rows x 256 columns per tile
    BK_LIFE_TB8 = 15       // Life, 8 fused generations per round, any checks inside
};
constexpr int kBatchKinds = 15;
// A grid runs whole-grid-in-LDS when both of its buffers fit in this many bytes
// (rows * cols * element size * 2; one 1024-thread workgroup per job).
constexpr int64_t kSmallLdsBytes = 160 * 1024 - 1024;
// 32-bit words of one LDS row of a small Life grid: the cells from byte 4 on, a
// ghost byte on either side, whole words up to one past the last cell's word.
__host__ __device__ inline int64_t small_life_words(int64_t cols) { return (cols + 3) / 4 + 2; }
// esz 1 is a Life grid (rows of small_life_words words).
inline bool batch_small_fits(int64_t rows, int64_t cols, int esz) {
    if (esz == 1) return rows * small_life_words(cols) * 4 * 2 <= kSmallLdsBytes;
    return rows * cols * (int64_t)esz * 2 <= kSmallLdsBytes;
}

// Device descriptor of one job of a batch. The job's completed-sweep count n
// lives in its JobState; a round advances it by `step` sweeps, reading
// buf[(n / step) % 2] and writing the other buffer (a stop inside a round leaves
// n at the stop sweep, and the engine replays that round up to it). Rows of both
// buffers (and env) are 16-byte aligned; Life rows hold round_up(cols, 16) bytes
// with the padding starting at zero. With mc, a round may hold several checks:
// level l's partials are at partials[(l - 1) * tiles + tile].
struct BatchJob {
    const void* buf[2];
    const void* env;       // Helmholtz g, the restoration mask (u8, grid pitch), or null
    JobState* st;
    void* partials;        // one 8-byte partial per tile
    JobState* mirror;      // device pointer of the pinned host mirror
    int64_t rows, cols, pitch;
    double rd;
    LoopCtl ctl;
    int32_t kind, helm, torus, strips, tiles, tile_rows, step, mc;
    double beta;           // restoration: phi(t) = sqrt(beta + t^2)
    int32_t quadratic;     // restoration: phi(t) = t^2 instead
    int32_t pad_;
};

struct WorkItem {
    int32_t job;   // index into the batch's job table, -1 = idle padding
    int32_t tile;  // tile of that job (one wavefront's work)
};

// Family, step and tile geometry a job gets inside a batch: a function of its
// shape, dtype and loop control only (j.ctl must be set), so its reduce order is
// the same alone and in any mix. Small grids (batch_small_fits) run their whole
// loop in LDS in one round; other Jacobi jobs take want_depth when a family holds
// it (FP64 10, 5, 2; FP32 5, 2) and it divides both the check period and the
// cap, else the deepest such depth, else depth 5 with checks inside (also
// chosen by want_depth = 5); want_tile_rows > 0 sets the band height. The
// wanted values come from the context's tuning table, so the geometry is still
// a function of the job's own key. A Life job runs 8 generations per round (one
// band of one 992-column window per wavefront, tile_life_tb.hpp) unless
// want_depth is 1 (one generation per round). j.torus must be set.
void batch_geometry(BatchJob& j, int is_life, int f32, int want_depth = 0, int want_tile_rows = 0);
// The same for a restoration job: one tile = 16 rows x 64 columns (one wavefront),
// one sweep per round; never whole-grid-in-LDS.
void batch_geometry_restore(BatchJob& j, int f32);
// The same for a Sobel job: one tile = 8 rows x 256 columns (one wavefront).
void batch_geometry_sobel(BatchJob& j);
// One launch per kernel family: `work` points at that family's segment of the
// work list (nwork_padded entries, a multiple of 32; idle entries have job -1).
// A workgroup runs four consecutive entries, one per wavefront.
constexpr int kBatchWorkQuantum = 32;
hipError_t launch_batch_sweep(const BatchJob* jobs, const WorkItem* work, int kind,
                              int nwork_padded, hipStream_t s);
hipError_t launch_batch_finalize(const BatchJob* jobs, int njobs, hipStream_t s);
inline bool batch_is_small(const BatchJob& j) {
    return j.kind == BK_SMALL_F64 || j.kind == BK_SMALL_F32 || j.kind == BK_SMALL_LIFE;
}
// Runs a small job's whole loop in one workgroup (its state must be initialised).
hipError_t launch_batch_small(const BatchJob& j, hipStream_t s);

// HBM copy probe: bytes must be a multiple of 16, buffers 16-byte aligned.
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s);

// Loop control ---------------------------------------------------------------
// A fresh state (count from the count partials, if any) with n_base sweeps done.
hipError_t launch_init_state(JobState* st, const void* count_parts, int nparts, hipStream_t s,
                             int64_t n_base = 0);
// After the launch whose last sweep is chunk offset j (one check, partials[tile]).
hipError_t launch_finalize(JobState* st, const void* partials, const LoopCtl& c, int j,
                           JobState* mirror, hipStream_t s);
// After a fused launch of K sweeps from chunk offset j0 that may hold several
// checks (level l's partials at partials[(l - 1) * tiles + tile]).
hipError_t launch_finalize_levels(JobState* st, const void* partials, const LoopCtl& c, int j0,
                                  int K, int tiles, JobState* mirror, hipStream_t s);
hipError_t launch_cancel(JobState* st, JobState* mirror, hipStream_t s);

}  // namespace lsr
