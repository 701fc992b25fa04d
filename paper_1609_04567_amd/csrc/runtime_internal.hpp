// Internal host-side definitions shared by the runtime (C ABI, plain driver)
// and the batched engine.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "lsr.h"

namespace lsr_rt {

// Thread-local text of the last error (lsr_last_error).
extern thread_local std::string g_last_error;

// Records a formatted message as the last error and returns the status.
lsr_status fail(lsr_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(LSR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kDepth = 3;          // chunks in flight per job
constexpr int kMirrorSlots = 4096; // pinned state mirrors per context
constexpr double kChunkTargetUs = 1500.0;
constexpr int kMaxChunk = 512;

// ---------------------------------------------------------------------------
// Caching pool. Sizes are rounded to a class (powers of two below 2 MiB,
// multiples of 2 MiB above) and freed blocks are kept for reuse; live plus
// cached bytes never exceed the budget (cached blocks are released first).
// ---------------------------------------------------------------------------
class Pool {
  public:
    void init(uint64_t budget) { budget_ = budget; }
    static size_t size_class(size_t n) {
        if (n < 4096) n = 4096;
        if (n <= (2u << 20)) {
            size_t p = 4096;
            while (p < n) p <<= 1;
            return p;
        }
        const size_t g = 2u << 20;
        return (n + g - 1) / g * g;
    }
    lsr_status alloc(size_t n, void** out) {
        std::lock_guard<std::mutex> lk(mu_);
        const size_t sz = size_class(n);
        auto it = free_.find(sz);
        if (it != free_.end()) {
            *out = it->second;
            free_.erase(it);
            cached_ -= sz;
            live_[*out] = sz;
            live_bytes_ += sz;
            return LSR_OK;
        }
        if (live_bytes_ + cached_ + sz > budget_) trim_locked();
        if (live_bytes_ + sz > budget_)
            return fail(LSR_EBUSY, "scratch of %zu bytes exceeds the HBM budget (%llu live of %llu)",
                        sz, (unsigned long long)live_bytes_, (unsigned long long)budget_);
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim_locked();
            e = hipMalloc(&p, sz);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(LSR_ENOMEM, "hipMalloc(%zu): %s", sz, hipGetErrorString(e));
            }
        }
        live_[p] = sz;
        live_bytes_ += sz;
        *out = p;
        return LSR_OK;
    }
    void release(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        auto it = live_.find(p);
        if (it == live_.end()) return;
        const size_t sz = it->second;
        live_.erase(it);
        live_bytes_ -= sz;
        free_.emplace(sz, p);
        cached_ += sz;
    }
    void trim() {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked();
    }
    void destroy() {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked();
        for (auto& kv : live_) (void)hipFree(kv.first);
        live_.clear();
        live_bytes_ = 0;
    }
    uint64_t budget() const { return budget_; }
    void usage(uint64_t* live, uint64_t* cached) {
        std::lock_guard<std::mutex> lk(mu_);
        *live = live_bytes_;
        *cached = cached_;
    }

  private:
    void trim_locked() {
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        cached_ = 0;
    }
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> live_;
    uint64_t budget_ = 0, live_bytes_ = 0, cached_ = 0;
};

inline size_t dtype_size(int dt) { return dt == LSR_U8 ? 1 : dt == LSR_F32 ? 4 : 8; }

// True when every row of a Jacobi grid (and its env) starts 16-byte aligned,
// the condition of the vector sweep kernels.
inline bool jacobi_rows_aligned(const lsr_grid& g, int stencil) {
    const size_t esz = dtype_size(g.dtype);
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    bool ok = (g.pitch * esz) % 16 == 0 && al(g.data);
    if (stencil == LSR_ST_HELMHOLTZ5) ok = ok && al(g.env0);
    return ok;
}

// True when the SWAR Life kernel can sweep the caller's grid in place: 16-byte
// aligned rows of a multiple of 16 cells (no padding to keep at zero).
inline bool life_rows_direct(const lsr_grid& g) {
    return g.cols % 16 == 0 && g.pitch % 16 == 0 && (reinterpret_cast<uintptr_t>(g.data) & 15) == 0;
}

// True when a job runs on staged copies (see Job::staged).
inline bool needs_staging(const lsr_grid& g, int stencil) {
    if (stencil == LSR_ST_LAPLACE5 || stencil == LSR_ST_HELMHOLTZ5 || stencil == LSR_ST_HELMHOLTZ5_SEP)
        return !jacobi_rows_aligned(g, stencil);
    if (stencil == LSR_ST_LIFE) return !life_rows_direct(g);
    return false;
}

// Row pitch (elements) of a staged copy: rows padded to 128 bytes.
inline int64_t stage_pitch(const lsr_grid& g) {
    const int64_t esz = (int64_t)dtype_size(g.dtype);
    return (g.cols * esz + 127) / 128 * 128 / esz;
}

enum class Phase { Queued, Running, Finished };

struct Job {
    lsr_job id = 0;
    lsr_grid grid{};
    int stencil = 0;
    lsr_cond cond{};
    int64_t max_iter = 0;
    lsr::LoopCtl ctl{};
    lsr::SweepGeom geom{};
    lsr::SweepGeom replay_geom{};       // unfused Jacobi geometry (replay after a mid-launch stop)
    lsr_grid xgrid{};                   // the grid the kernels sweep (staged copy or the caller's)
    void* buf[2] = {nullptr, nullptr};  // buf[0] = exec grid, buf[1] = partner
    // A Jacobi grid whose rows are not 16-byte aligned (pitch or base), or a Life
    // grid whose rows are not aligned runs of 16 cells, runs on private copies
    // with a 128-byte row pitch (both buffers and env; Life padding zeroed), so
    // it takes the vector / SWAR kernels; the result is copied back into the
    // caller's grid.
    bool staged = false;
    // A host-resident job (lsr_run_host): grid and env are host memory. It always
    // runs staged: the device copies come from the pool (under the HBM budget),
    // are filled by H2D copies when the job is admitted and the last iterate goes
    // back by a D2H copy when it retires.
    bool host = false;
    hipEvent_t ev_in = nullptr;         // batched engine: end of a host job's H2D copies
    // A two-phase restoration job (lsr_run_restore_host): the host frame y is
    // copied into stage_y, detection writes the mask (stage_env) and the initial
    // iterate (buf[0]) on the device, and the restored frame goes back to out_host.
    bool two_phase = false;
    int w_max = 0;
    void* stage_y = nullptr;
    const void* in_host = nullptr;      // the frame (u8, pitch host_pitch)
    void* out_host = nullptr;           // the result (grid dtype, pitch host_pitch)
    int64_t host_pitch = 0;
    void* stage_env = nullptr;
    void* partials = nullptr;
    lsr::JobState* st = nullptr;
    int slot = -1;
    lsr::JobState* mirror_host = nullptr;
    lsr::JobState* mirror_dev = nullptr;
    hipEvent_t ev_user = nullptr, ev_begin = nullptr, ev_end = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = true;
    std::atomic<bool> cancel{false};
    Phase phase = Phase::Queued;
    lsr_job_result result{};
    lsr_status status = LSR_OK;
    std::string error;
    // batched engine
    lsr::BatchJob desc{};               // device descriptor (valid once admitted)
    size_t bytes = 0;                   // grid bytes (partner size)
    int nparts_alloc = 0;               // partials allocated (tiles, or the initial count's)
    double est_us = 0.0;                // estimated device time of one sweep
    bool cancel_posted = false;         // a cancel kernel has been enqueued
    hipEvent_t ev_small = nullptr;      // end of a small job's launch on the second stream
    std::chrono::steady_clock::time_point t_submit, t_admit, t_done;

    // True when a finalize launch follows the sweep at chunk offset off: a check
    // offset (a multiple of the check period), the offset of the cap sweep, and the
    // chunk's last sweep (where the state's chunk base advances).
    bool fin_at(int off) const {
        const int jmax = (int)((max_iter - 1) % ctl.chunk);
        return ((off + 1) % ctl.check_every) == 0 || off == jmax || off == ctl.chunk - 1;
    }

    // Returns the job's scratch (partner, staged copies, partials, state) to the pool.
    void release_scratch(Pool& pool) {
        pool.release(buf[1]);
        pool.release(partials);
        pool.release(st);
        if (staged) {
            pool.release(buf[0]);
            pool.release(stage_env);
            pool.release(stage_y);
            buf[0] = stage_env = stage_y = nullptr;
        }
        buf[1] = partials = nullptr;
        st = nullptr;
    }
};

using Clock = std::chrono::steady_clock;
inline double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Argument validation shared by lsr_run and lsr_check_args.
lsr_status validate(const lsr_grid* g, int stencil, int reduce, const lsr_cond* c, int64_t max_iter);

// Kernel arguments of a Jacobi job's sweep from src to dst (its exec grid).
lsr::JacobiArgs jacobi_args(const Job* j, const void* src, void* dst);
// The same for a Life job.
lsr::LifeArgs life_args(const Job* j, const void* src, void* dst);

// Key of the autotuner's table: a job's stencil, dtype, boundary, size class
// (bit lengths of rows and cols) and check period. A choice is a pure function of
// this key.
struct TuneKey {
    int stencil, dtype, bc, rows_log2, cols_log2, check_every;
    bool operator<(const TuneKey& o) const {
        if (stencil != o.stencil) return stencil < o.stencil;
        if (dtype != o.dtype) return dtype < o.dtype;
        if (bc != o.bc) return bc < o.bc;
        if (rows_log2 != o.rows_log2) return rows_log2 < o.rows_log2;
        if (cols_log2 != o.cols_log2) return cols_log2 < o.cols_log2;
        return check_every < o.check_every;
    }
};
TuneKey tune_key(int stencil, int dtype, int bc, int64_t rows, int64_t cols, int check_every);
struct TuneEntry {
    lsr_tuning tuning;
    double us_per_sweep;   // measured device time per sweep of the winner
};

}  // namespace lsr_rt


struct lsr_ctx {
    int device = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;    // internal execution stream
    hipStream_t small_stream = nullptr;  // batched engine: whole-grid-in-LDS jobs
    hipStream_t copy_stream = nullptr;       // batched engine: H2D copies of host jobs
    hipStream_t copy_out_stream = nullptr;   // batched engine: D2H copies at retirement (the two
                                             // directions of the link run at the same time)
    hipStream_t detect_stream = nullptr;     // batched engine: detection of two-phase frames
    hipStream_t capture = nullptr;   // stream used only for graph capture
    lsr_rt::Pool pool;
    lsr_tuning tuning{};
    std::map<lsr_rt::TuneKey, lsr_rt::TuneEntry> tune_table;   // autotuner's choices (under mu)
    // Launch settings for a job: the context's overrides, or, when those leave the
    // launch shape automatic, the autotuner's entry for the job's key (caller holds mu).
    lsr_tuning tuned_for(const lsr_grid& g, int stencil, int check_every) const;
    lsr::JobState* mirrors_host = nullptr;
    lsr::JobState* mirrors_dev = nullptr;
    std::vector<int> free_slots;
    std::vector<hipEvent_t> event_pool;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<lsr_rt::Job*> queue;
    std::unordered_map<lsr_job, std::unique_ptr<lsr_rt::Job>> jobs;
    lsr_job next_id = 1;
    std::deque<lsr_job> done_q;         // finished jobs in completion order (lsr_wait_any)
    int64_t unfinished = 0;             // jobs submitted and not finished yet (under mu)
    bool stopping = false;
    std::thread driver;

    void drive();
    lsr_status run_job(lsr_rt::Job* j);
    hipEvent_t get_event();
    void put_event(hipEvent_t e) { event_pool.push_back(e); }

    // Batched engine (LSR_FLAG_BATCHED), see engine.cpp.
    bool batched = false;
    std::deque<lsr_rt::Job*> pending;   // submitted, waiting for admission (arrival order)
    std::vector<lsr_rt::Job*> ingesting; // host jobs admitted, H2D copies in flight
    std::vector<lsr_rt::Job*> active;   // admitted, in the device tables
    std::vector<lsr_rt::Job*> retiring; // stopped, waiting for their end event
    lsr::BatchJob* d_jobs = nullptr;
    lsr::WorkItem* d_work = nullptr;
    lsr::BatchJob* h_jobs[2] = {nullptr, nullptr};
    lsr::WorkItem* h_work[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage = 0;
    int seg_off[lsr::kBatchKinds + 1] = {};
    int seg_len[lsr::kBatchKinds + 1] = {};
    int64_t work_items = 0;
    int n_table = 0;                    // jobs in the device table (small jobs are not)
    // engine-thread counts published for lsr_get_stats (read from other threads)
    std::atomic<int64_t> pub_ingesting{0}, pub_active{0}, pub_retiring{0};
    bool tables_dirty = false;
    void serve();
    lsr_status engine_submit(lsr_rt::Job* j);
    lsr_status engine_admit();
    lsr_status engine_activate(lsr_rt::Job* j);
    lsr_status engine_poll_ingest(bool block);
    lsr_status engine_upload();
    lsr_status engine_window();
    void engine_scan();
    void engine_poll_retiring(bool block);
    void engine_finish(lsr_rt::Job* j, lsr_status st);
    lsr_status engine_setup();
    void engine_teardown();
};

namespace lsr_rt {
// Plans a plain-path job whose exec grid (xgrid) and buffer roles are set:
// sweep geometry (fused depth from the tuning), the unfused replay geometry, the
// loop control with its chunk, and the partial count to allocate. EINVAL when the
// check period makes a chunk too long to capture.
lsr_status plan_plain(Job* j, int reduce_op, const lsr_tuning& tun, int* nparts_out);
// Enqueues the sweep launch that starts at chunk offset off (and the finalize
// that follows it, if any) on stream s.
lsr_status launch_sweep(Job* j, int off, hipStream_t s);
// Enqueues one whole chunk of sweep and finalize launches on s.
lsr_status enqueue_chunk(Job* j, hipStream_t s);
// After a stop: replays a stop inside a fused launch with unfused sweeps (on s)
// and returns in *last the buffer that holds sweep fin.n.
lsr_status finish_fused(Job* j, const lsr::JobState& fin, int K, const lsr::LoopCtl& ctl,
                        int* last, hipStream_t s);
lsr_status submit_plain(lsr_ctx* ctx, std::unique_ptr<Job> j, const lsr_grid* grid,
                        int32_t stencil_id, int32_t reduce_op, const lsr_cond* cond,
                        int64_t max_iter, const lsr_tuning& tun, lsr_job* job_out);
// Records the device address of lsr_run_noalloc's scratch array on `device`
// (current); called once per context creation.
lsr_status noalloc_setup(int device);
// Queues a job on a batched context: engine descriptor, events, the pending queue.
lsr_status submit_batched(lsr_ctx* ctx, std::unique_ptr<Job> j, lsr_job* job_out);
// lsr_run and lsr_run_host: validation, then the plain or the batched submission.
lsr_status submit(lsr_ctx* ctx, const lsr_grid* grid, int32_t stencil_id, int32_t reduce_op,
                  const lsr_cond* cond, int64_t max_iter, bool host, lsr_job* job_out);
// Element size of a job's env array: the restoration mask is u8, Helmholtz g has
// the grid's dtype.
inline size_t env_esz(const Job* j) {
    return j->stencil == LSR_ST_RESTORE ? 1 : dtype_size(j->grid.dtype);
}
// Copy direction of a staged job's copy into (in = true) or out of its device grid.
inline hipMemcpyKind stage_kind(const Job* j, bool in) {
    if (!j->host) return hipMemcpyDeviceToDevice;
    return in ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
}
}  // namespace lsr_rt

