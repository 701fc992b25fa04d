// Batched engine (LSR_FLAG_BATCHED): continuous batching of many
// loop-of-stencil-reduce jobs on one GPU, the single-device form of the paper's
// stream of tasks (Sect. 3.2; the streaming experiments of Sect. 4 reuse device
// memory across items).
//
// One engine thread per context owns the device tables and the context stream:
//   admit  - queued jobs, in arrival order, get their scratch (ping-pong
//            partner, partials, 64 B state) from the pool while the HBM budget
//            allows; their initialisation (partner copy, initial live count,
//            state) is enqueued on the stream after the caller's prior work.
//   upload - when the active set changed, the job descriptors and the work list
//            (one entry per tile, grouped by kernel family, band-major per job so
//            that neighbouring tiles land on one XCD) are copied to the device
//            through double-buffered pinned staging.
//   window - R rounds are enqueued; a round is one sweep launch per kernel
//            family present plus one finalize launch for all jobs. R is chosen
//            so a window is ~1.5 ms of device time; two windows stay in flight.
//   scan   - after a window completes, jobs whose pinned mirror shows `done`
//            are retired: an odd final sweep count costs one D2D copy back into
//            the caller's grid, their scratch returns to the pool (every later
//            use of a block is ordered after the copy on the same stream), and
//            the next arrivals can be admitted into the freed memory.
// Nothing here blocks on the device except the window and retirement events.
#include "runtime_internal.hpp"

using namespace lsr_rt;

namespace {

constexpr int kMaxBatch = 4096;          // active jobs (the pinned mirror slots)
constexpr int64_t kMaxWork = 1 << 21;    // tiles of all active jobs
constexpr int kPad = lsr::kBatchWorkQuantum * (lsr::kBatchKinds + 1);
constexpr double kWindowUs = 1500.0;     // device time per window of rounds
constexpr double kRoundOverheadUs = 12.0;
constexpr int kMaxRounds = 64;
constexpr int kWindowsInFlight = 2;

}  // namespace

lsr_status lsr_ctx::engine_setup() {
    HIP_TRY(hipStreamCreateWithFlags(&small_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&copy_out_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&detect_stream, hipStreamNonBlocking));
    HIP_TRY(hipMalloc(&d_jobs, sizeof(lsr::BatchJob) * kMaxBatch));
    HIP_TRY(hipMalloc(&d_work, sizeof(lsr::WorkItem) * (kMaxWork + kPad)));
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipHostMalloc((void**)&h_jobs[i], sizeof(lsr::BatchJob) * kMaxBatch, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&h_work[i], sizeof(lsr::WorkItem) * (kMaxWork + kPad),
                              hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&stage_ev[i], hipEventDisableTiming));
        HIP_TRY(hipEventRecord(stage_ev[i], stream));
    }
    return LSR_OK;
}

void lsr_ctx::engine_teardown() {
    (void)hipStreamSynchronize(stream);
    if (small_stream) {
        (void)hipStreamSynchronize(small_stream);
        (void)hipStreamDestroy(small_stream);
        small_stream = nullptr;
    }
    for (hipStream_t* cs : {&copy_stream, &copy_out_stream, &detect_stream}) {
        if (*cs) {
            (void)hipStreamSynchronize(*cs);
            (void)hipStreamDestroy(*cs);
            *cs = nullptr;
        }
    }
    for (int i = 0; i < 2; ++i) {
        if (stage_ev[i]) (void)hipEventDestroy(stage_ev[i]);
        if (h_jobs[i]) (void)hipHostFree(h_jobs[i]);
        if (h_work[i]) (void)hipHostFree(h_work[i]);
    }
    if (d_jobs) (void)hipFree(d_jobs);
    if (d_work) (void)hipFree(d_work);
}

// Called by lsr_run (caller thread): fills the job's descriptor from its shape
// and queues it.
lsr_status lsr_ctx::engine_submit(Job* j) {
    const lsr_grid& g = j->grid;
    const bool life = j->stencil == LSR_ST_LIFE;
    const bool restore = j->stencil == LSR_ST_RESTORE;
    const bool sobel = j->stencil == LSR_ST_SOBEL;
    const bool f32 = g.dtype == LSR_F32;
    j->xgrid = g;
    // small grids are swept in LDS from any pitch or alignment, restoration at any
    // pitch: staged only when they live in host memory
    j->staged = j->host || (!restore && !sobel &&
                            !lsr::batch_small_fits(g.rows, g.cols, (int)dtype_size(g.dtype)) &&
                            needs_staging(g, j->stencil));
    if (j->staged) j->xgrid.pitch = stage_pitch(g);   // buffers assigned at admission
    lsr::BatchJob& d = j->desc;
    d = lsr::BatchJob{};
    d.buf[0] = j->staged ? nullptr : g.data;
    d.env = j->staged ? nullptr : g.env0;
    d.rows = g.rows;
    d.cols = g.cols;
    d.pitch = j->xgrid.pitch;
    d.helm = j->stencil == LSR_ST_HELMHOLTZ5;
    d.torus = g.bc == LSR_BC_TORUS;
    d.rd = 1.0 / (4.0 + g.param[0] * (g.param[1] * g.param[1]));
    d.beta = g.param[0];
    d.quadratic = g.param[1] != 0.0;
    lsr::LoopCtl& c = d.ctl;
    c.max_iter = j->max_iter;
    // a check period of at least max_iter leaves only the check at the cap
    c.check_every = (int32_t)std::min<int64_t>(j->cond.check_every, j->max_iter);
    c.chunk = 1;
    c.reduce = j->ctl.reduce;
    c.cond = j->cond.kind;
    c.stable_window = j->cond.stable_window;
    c.threshold = j->cond.threshold;
    c.mean_div = (double)g.rows * (double)g.cols;
    // rows are aligned (or staged into aligned copies, 256-byte aligned pool blocks);
    // fused depth and band height from the tuning table or overrides, as on the
    // plain path
    lsr_tuning tu;
    {
        std::lock_guard<std::mutex> lk(mu);
        tu = tuned_for(g, j->stencil, j->cond.check_every);
    }
    if (restore) lsr::batch_geometry_restore(d, f32);
    else if (sobel) lsr::batch_geometry_sobel(d);
    else lsr::batch_geometry(d, life, f32, tu.tb_depth, tu.tile_rows);
    c.nparts = d.tiles;
    const size_t esz = dtype_size(g.dtype);
    j->bytes = (size_t)g.rows * (size_t)j->xgrid.pitch * esz;
    int nparts = d.mc ? d.tiles * d.step : d.tiles;
    if (life) {
        nparts = std::max(nparts, lsr::count_u8_parts(g.rows, g.cols));
        if (d.step > 1) {
            // single generations that replay a stop inside a fused round
            j->replay_geom = lsr::life_geom(life_args(j, nullptr, nullptr), 0);
            nparts = std::max(nparts, j->replay_geom.tiles);
        }
    } else if (!restore && !sobel) {
        // unfused geometry that replays a stop inside a round (rows are aligned:
        // null pointers stand for the buffers, which are not allocated yet)
        lsr::JacobiArgs ra = jacobi_args(j, nullptr, nullptr);
        ra.g = nullptr;
        j->replay_geom = lsr::jacobi_geom(ra, 0);
        nparts = std::max(nparts, j->replay_geom.tiles);
    }
    j->nparts_alloc = nparts;
    // device time of a round per cell, in bytes at 5 TB/s (restoration: its
    // measured ALU time per pixel; a fused Life round of 8 generations: 2.1
    // single ones)
    const double per_cell = life ? (d.step > 1 ? 4.3 : 2.0)
                            : sobel ? 2.0 : restore ? (f32 ? 28.0 : 58.0)
                                      : (double)esz * (d.helm ? 3.0 : 2.0);
    j->est_us = (double)g.rows * (double)g.cols * per_cell / 5.0e6;
    if (d.tiles > kMaxWork) return fail(LSR_EINVAL, "grid too large for the batched engine");
    return LSR_OK;
}

void lsr_ctx::engine_finish(Job* j, lsr_status st) {
    std::lock_guard<std::mutex> lk(mu);
    j->result.status = st;
    j->status = st;
    j->result.queue_ms = ms_between(j->t_submit, j->t_admit);
    j->result.latency_ms = ms_between(j->t_submit, j->t_done);
    j->phase = Phase::Finished;
    done_q.push_back(j->id);
    --unfinished;
    cv_done.notify_all();
}

// Admission in arrival order while the pool can hold a job's device memory: the
// partner, partials and state, plus the staged copies of its grid and env (a
// host job's grids therefore count against the budget like its scratch). A device
// job is activated at once; a host job first has its H2D copies enqueued on the
// copy stream, behind everything already enqueued on the execution stream (its
// blocks may have been released by jobs retired while earlier windows still ran),
// and is activated by engine_poll_ingest once they have completed.
lsr_status lsr_ctx::engine_admit() {
    while (true) {
        Job* j = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (pending.empty() || (int)(active.size() + ingesting.size()) >= kMaxBatch ||
                free_slots.empty())
                return LSR_OK;
            j = pending.front();
        }
        if (j->cancel.load()) {
            {
                std::lock_guard<std::mutex> lk(mu);
                pending.pop_front();
            }
            j->t_admit = j->t_done = Clock::now();
            engine_finish(j, LSR_ECANCELED);
            continue;
        }
        if (work_items + j->desc.tiles > kMaxWork) return LSR_OK;
        void* partner = nullptr;
        void* parts = nullptr;
        void* st = nullptr;
        void* s0 = nullptr;
        void* senv = nullptr;
        lsr_status s = pool.alloc(j->bytes, &partner);
        if (s == LSR_OK) s = pool.alloc((size_t)j->nparts_alloc * 8, &parts);
        if (s == LSR_OK) s = pool.alloc(sizeof(lsr::JobState), &st);
        if (s == LSR_OK && j->staged) s = pool.alloc(j->bytes, &s0);
        void* sy = nullptr;
        const size_t env_bytes = (size_t)j->xgrid.rows * (size_t)j->xgrid.pitch * env_esz(j);
        if (s == LSR_OK && j->staged && (j->desc.helm || j->stencil == LSR_ST_RESTORE))
            s = pool.alloc(env_bytes, &senv);
        if (s == LSR_OK && j->two_phase) s = pool.alloc(env_bytes, &sy);
        if (s != LSR_OK) {
            pool.release(partner);
            pool.release(parts);
            pool.release(st);
            pool.release(s0);
            pool.release(senv);
            pool.release(sy);
            if (!active.empty() || !retiring.empty() || !ingesting.empty())
                return LSR_OK;  // wait for memory
            {
                std::lock_guard<std::mutex> lk(mu);
                pending.pop_front();
            }
            j->error = g_last_error;
            j->t_admit = j->t_done = Clock::now();
            engine_finish(j, s);  // cannot fit even on an idle device
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            pending.pop_front();
            j->slot = free_slots.back();
            free_slots.pop_back();
            j->phase = Phase::Running;
        }
        work_items += j->desc.tiles;
        j->buf[1] = partner;
        j->partials = parts;
        j->st = static_cast<lsr::JobState*>(st);
        if (j->staged) {
            j->buf[0] = s0;
            j->stage_env = senv;
            j->stage_y = sy;
            j->xgrid.data = s0;
            j->xgrid.env0 = senv;
            j->desc.buf[0] = s0;
            j->desc.env = senv;
        } else {
            j->buf[0] = j->grid.data;
        }
        j->mirror_host = mirrors_host + j->slot;
        j->mirror_dev = mirrors_dev + j->slot;
        std::memset((void*)j->mirror_host, 0, sizeof(lsr::JobState));
        lsr::BatchJob& d = j->desc;
        d.buf[1] = partner;
        d.st = j->st;
        d.partials = parts;
        d.mirror = j->mirror_dev;
        if (!j->host) {
            active.push_back(j);  // from here on a device failure also finishes this job
            HIP_TRY(hipStreamWaitEvent(stream, j->ev_user, 0));
            HIP_TRY(hipEventRecord(j->ev_begin, stream));
            lsr_status a = engine_activate(j);
            if (a != LSR_OK) return a;
            continue;
        }
        ingesting.push_back(j);
        const lsr_grid& g = j->xgrid;
        const lsr_grid& ug = j->grid;
        const size_t esz = dtype_size(g.dtype);
        hipEvent_t behind = get_event();
        if (!behind) return fail(LSR_EDEVICE, "event pool");
        HIP_TRY(hipEventRecord(behind, stream));
        HIP_TRY(hipStreamWaitEvent(copy_stream, behind, 0));
        put_event(behind);
        HIP_TRY(hipStreamWaitEvent(copy_stream, j->ev_user, 0));
        HIP_TRY(hipEventRecord(j->ev_begin, copy_stream));
        if (j->stencil == LSR_ST_LIFE) {   // padding cells start (and stay) 0
            HIP_TRY(hipMemsetAsync(s0, 0, (size_t)g.rows * g.pitch * esz, copy_stream));
            HIP_TRY(hipMemsetAsync(partner, 0, (size_t)g.rows * g.pitch * esz, copy_stream));
        }
        if (j->two_phase) {
            // the frame only; detection (the mask and the initial iterate) follows
            // on a stream of its own after the copy, so it overlaps the sweep rounds
            // of the frames already in the tables and the next frames' copies
            HIP_TRY(hipMemcpy2DAsync(sy, g.pitch, j->in_host, j->host_pitch, g.cols, g.rows,
                                     hipMemcpyHostToDevice, copy_stream));
            hipEvent_t copied = get_event();
            if (!copied) return fail(LSR_EDEVICE, "event pool");
            HIP_TRY(hipEventRecord(copied, copy_stream));
            HIP_TRY(hipStreamWaitEvent(detect_stream, copied, 0));
            put_event(copied);
            HIP_TRY(lsr::launch_amf_detect(static_cast<const uint8_t*>(sy), g.rows, g.cols, g.pitch,
                                           j->w_max, static_cast<uint8_t*>(senv), s0, g.dtype,
                                           detect_stream));
        } else {
            const size_t ee = env_esz(j);
            HIP_TRY(hipMemcpy2DAsync(s0, g.pitch * esz, ug.data, ug.pitch * esz, g.cols * esz,
                                     g.rows, hipMemcpyHostToDevice, copy_stream));
            if (senv)
                HIP_TRY(hipMemcpy2DAsync(senv, g.pitch * ee, ug.env0, ug.pitch * ee, g.cols * ee,
                                         g.rows, hipMemcpyHostToDevice, copy_stream));
        }
        j->ev_in = get_event();
        if (!j->ev_in) return fail(LSR_EDEVICE, "event pool");
        HIP_TRY(hipEventRecord(j->ev_in, j->two_phase ? detect_stream : copy_stream));
        j->t_admit = Clock::now();
    }
}

// Host jobs whose H2D copies have completed join the device tables. With block,
// waits for the oldest one when none is ready (nothing else to do).
lsr_status lsr_ctx::engine_poll_ingest(bool block) {
    if (ingesting.empty()) return LSR_OK;
    std::vector<Job*> keep;
    keep.reserve(ingesting.size());
    for (size_t k = 0; k < ingesting.size(); ++k) {
        Job* j = ingesting[k];
        hipError_t e = (block && k == 0) ? hipEventSynchronize(j->ev_in) : hipEventQuery(j->ev_in);
        if (e == hipErrorNotReady) {
            keep.push_back(j);
            continue;
        }
        if (e != hipSuccess) {
            // the failure path finishes this job (now active) and the rest
            for (size_t r = k + 1; r < ingesting.size(); ++r) keep.push_back(ingesting[r]);
            ingesting.swap(keep);
            active.push_back(j);
            return fail(LSR_EDEVICE, "H2D copy: %s", hipGetErrorString(e));
        }
        active.push_back(j);
        HIP_TRY(hipStreamWaitEvent(stream, j->ev_in, 0));
        put_event(j->ev_in);
        j->ev_in = nullptr;
        lsr_status a = engine_activate(j);
        if (a != LSR_OK) {
            for (size_t r = k + 1; r < ingesting.size(); ++r) keep.push_back(ingesting[r]);
            ingesting.swap(keep);
            return a;
        }
    }
    ingesting.swap(keep);
    return LSR_OK;
}

// Enqueues an admitted job's initialisation on the execution stream (a device
// job's staging copies, the partner copy or the initial live count, the state),
// and launches a small job's whole loop on the second stream.
lsr_status lsr_ctx::engine_activate(Job* j) {
    const lsr_grid& g = j->xgrid;
    const lsr_grid& ug = j->grid;
    const size_t esz = dtype_size(g.dtype);
    void* partner = j->buf[1];
    if (j->staged && !j->host) {
        if (j->stencil == LSR_ST_LIFE) {   // padding cells start (and stay) 0/1
            HIP_TRY(hipMemsetAsync(j->buf[0], 0, (size_t)g.rows * g.pitch * esz, stream));
            HIP_TRY(hipMemsetAsync(partner, 0, (size_t)g.rows * g.pitch * esz, stream));
        }
        HIP_TRY(hipMemcpy2DAsync(j->buf[0], g.pitch * esz, ug.data, ug.pitch * esz, g.cols * esz,
                                 g.rows, hipMemcpyDeviceToDevice, stream));
        if (j->stage_env) {
            const size_t ee = env_esz(j);
            HIP_TRY(hipMemcpy2DAsync(j->stage_env, g.pitch * ee, ug.env0, ug.pitch * ee,
                                     g.cols * ee, g.rows, hipMemcpyDeviceToDevice, stream));
        }
    }
    // (a two-phase frame's detection ran on the copy stream after its H2D copy)
    if (j->stencil == LSR_ST_LIFE) {
        int np = 0;
        HIP_TRY(lsr::launch_count_u8(static_cast<uint8_t*>(g.data), g.rows, g.cols, g.pitch,
                                     j->partials, &np, stream));
        HIP_TRY(lsr::launch_init_state(j->st, j->partials, np, stream));
    } else {
        HIP_TRY(hipMemcpy2DAsync(partner, g.pitch * esz, g.data, g.pitch * esz, g.cols * esz,
                                 g.rows, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(lsr::launch_init_state(j->st, nullptr, 0, stream));
    }
    if (lsr::batch_is_small(j->desc)) {
        // the whole loop in one workgroup on the second stream, after the init
        hipEvent_t ready = get_event();
        if (!ready) return fail(LSR_EDEVICE, "event pool");
        HIP_TRY(hipEventRecord(ready, stream));
        HIP_TRY(hipStreamWaitEvent(small_stream, ready, 0));
        put_event(ready);
        HIP_TRY(lsr::launch_batch_small(j->desc, small_stream));
        j->ev_small = get_event();
        if (!j->ev_small) return fail(LSR_EDEVICE, "event pool");
        HIP_TRY(hipEventRecord(j->ev_small, small_stream));
    }
    if (!j->host) j->t_admit = Clock::now();
    tables_dirty = true;
    return LSR_OK;
}

lsr_status lsr_ctx::engine_upload() {
    const int s = stage;
    HIP_TRY(hipEventSynchronize(stage_ev[s]));
    lsr::BatchJob* hj = h_jobs[s];
    lsr::WorkItem* hw = h_work[s];
    int n = 0;
    for (Job* j : active)
        if (!lsr::batch_is_small(j->desc)) hj[n++] = j->desc;
    n_table = n;
    int64_t pos = 0;
    for (int k = 1; k <= lsr::kBatchKinds; ++k) {
        seg_off[k] = (int)pos;
        for (int i = 0; i < n; ++i) {
            if (hj[i].kind != k) continue;
            for (int t = 0; t < hj[i].tiles; ++t) hw[pos++] = lsr::WorkItem{i, t};
        }
        while ((pos - seg_off[k]) % lsr::kBatchWorkQuantum) hw[pos++] = lsr::WorkItem{-1, 0};
        seg_len[k] = (int)(pos - seg_off[k]);
    }
    if (n > 0) HIP_TRY(hipMemcpyAsync(d_jobs, hj, sizeof(lsr::BatchJob) * n, hipMemcpyHostToDevice, stream));
    if (pos > 0) HIP_TRY(hipMemcpyAsync(d_work, hw, sizeof(lsr::WorkItem) * pos, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(stage_ev[s], stream));
    stage ^= 1;
    tables_dirty = false;
    return LSR_OK;
}

lsr_status lsr_ctx::engine_window() {
    if (n_table == 0) return LSR_OK;   // only small jobs, each on the second stream
    double round_us = kRoundOverheadUs;
    for (Job* j : active)
        if (!lsr::batch_is_small(j->desc)) round_us += j->est_us;
    const int rounds = (int)std::min<double>(kMaxRounds, std::max(1.0, std::floor(kWindowUs / round_us)));
    const int n = n_table;
    for (int r = 0; r < rounds; ++r) {
        for (int k = 1; k <= lsr::kBatchKinds; ++k) {
            if (seg_len[k] == 0) continue;
            HIP_TRY(lsr::launch_batch_sweep(d_jobs, d_work + seg_off[k], k, seg_len[k], stream));
        }
        HIP_TRY(lsr::launch_batch_finalize(d_jobs, n, stream));
    }
    return LSR_OK;
}

void lsr_ctx::engine_scan() {
    std::vector<Job*> keep;
    keep.reserve(active.size());
    for (Job* j : active) {
        volatile lsr::JobState* m = j->mirror_host;
        const bool small = lsr::batch_is_small(j->desc);
        // a small job is over when its launch is (its writes are then all visible)
        const bool over = small ? hipEventQuery(j->ev_small) == hipSuccess : (bool)m->done;
        if (!over) {
            keep.push_back(j);
            continue;
        }
        if (small) {
            (void)hipStreamWaitEvent(stream, j->ev_small, 0);
            put_event(j->ev_small);
            j->ev_small = nullptr;
        }
        lsr::JobState fin;
        std::memcpy(&fin, (const void*)m, sizeof fin);
        const lsr_grid& g = j->xgrid;
        const lsr_grid& ug = j->grid;
        const size_t esz = dtype_size(g.dtype);
        // a stop inside a fused round is replayed first; then the buffer holding
        // sweep n goes back to the caller's grid (a host job's by a D2H copy on
        // the copy-out stream, after the execution stream's work so far)
        int last = 0;
        hipError_t e = finish_fused(j, fin, j->desc.step, j->desc.ctl, &last, stream) == LSR_OK
                           ? hipSuccess : hipErrorLaunchFailure;
        if (e == hipSuccess && j->host) {
            hipEvent_t done_ev = get_event();
            if (!done_ev) e = hipErrorOutOfMemory;
            if (e == hipSuccess) e = hipEventRecord(done_ev, stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(copy_out_stream, done_ev, 0);
            if (done_ev) put_event(done_ev);
            void* dst = j->two_phase ? j->out_host : ug.data;
            const size_t dpitch = (size_t)(j->two_phase ? j->host_pitch : ug.pitch) * esz;
            if (e == hipSuccess)
                e = hipMemcpy2DAsync(dst, dpitch, j->buf[last], g.pitch * esz, g.cols * esz,
                                     g.rows, hipMemcpyDeviceToHost, copy_out_stream);
            if (e == hipSuccess) e = hipEventRecord(j->ev_end, copy_out_stream);
        } else {
            if (e == hipSuccess && j->staged)
                e = hipMemcpy2DAsync(ug.data, ug.pitch * esz, j->buf[last], g.pitch * esz,
                                     g.cols * esz, g.rows, hipMemcpyDeviceToDevice, stream);
            else if (e == hipSuccess && last)
                e = hipMemcpy2DAsync(j->buf[0], g.pitch * esz, j->buf[1], g.pitch * esz,
                                     g.cols * esz, g.rows, hipMemcpyDeviceToDevice, stream);
            if (e == hipSuccess) e = hipEventRecord(j->ev_end, stream);
        }
        lsr_job_result& r = j->result;
        r.iterations = fin.n;
        r.last_reduce = fin.r;
        r.last_count = fin.count;
        r.converged = fin.converged;
        r.stable_run = fin.run;
        r.sweeps_per_launch = j->desc.step;
        r.checks = fin.checks;
        r.status = fin.status == lsr::ST_NUMERIC ? LSR_ENUMERIC
                 : fin.status == lsr::ST_CANCELED ? LSR_ECANCELED : LSR_OK;
        if (e != hipSuccess) {
            j->error = hipGetErrorString(e);
            r.status = LSR_EDEVICE;
        }
        // a host job's blocks are read by its D2H copy: released once that is done
        if (!j->host) j->release_scratch(pool);
        {
            std::lock_guard<std::mutex> lk(mu);
            free_slots.push_back(j->slot);
            j->slot = -1;
        }
        work_items -= j->desc.tiles;
        retiring.push_back(j);
        tables_dirty = true;
    }
    active.swap(keep);
}

void lsr_ctx::engine_poll_retiring(bool block) {
    std::vector<Job*> keep;
    for (Job* j : retiring) {
        hipError_t e = block ? hipEventSynchronize(j->ev_end) : hipEventQuery(j->ev_end);
        if (e == hipErrorNotReady) {
            keep.push_back(j);
            continue;
        }
        j->t_done = Clock::now();
        if (j->host) j->release_scratch(pool);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, j->ev_begin, j->ev_end);
        j->result.device_ms = ms;
        lsr_status st = (lsr_status)j->result.status;
        if (e != hipSuccess) {
            j->error = hipGetErrorString(e);
            st = LSR_EDEVICE;
        }
        engine_finish(j, st);
        block = false;  // one blocking wait per call is enough to make progress
    }
    retiring.swap(keep);
}

void lsr_ctx::serve() {
    (void)hipSetDevice(device);
    std::deque<hipEvent_t> inflight;
    std::string fatal;
    while (true) {
        {
            std::unique_lock<std::mutex> lk(mu);
            const bool idle = pending.empty() && active.empty() && retiring.empty() &&
                              inflight.empty() && ingesting.empty();
            if (idle) {
                if (stopping) break;
                cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
                if (pending.empty()) continue;
            }
        }
        lsr_status s = engine_admit();
        // host jobs whose copies are in: wait for one only when nothing else can run
        if (s == LSR_OK)
            s = engine_poll_ingest(active.empty() && inflight.empty() && retiring.empty());
        for (Job* j : active) {
            if (j->cancel.load() && !j->cancel_posted) {
                j->cancel_posted = true;
                if (lsr::launch_cancel(j->st, j->mirror_dev, stream) != hipSuccess)
                    s = fail(LSR_EDEVICE, "cancel launch failed");
            }
        }
        if (s == LSR_OK && tables_dirty) s = engine_upload();
        if (s == LSR_OK && n_table > 0) {
            s = engine_window();
            if (s == LSR_OK) {
                hipEvent_t ev = get_event();
                if (!ev || hipEventRecord(ev, stream) != hipSuccess) s = fail(LSR_EDEVICE, "event record failed");
                else inflight.push_back(ev);
            }
        } else if (s == LSR_OK && !active.empty() && inflight.empty()) {
            // only small jobs (each a single launch on the second stream): poll them
            const size_t before = active.size();
            engine_scan();
            bool waiting;
            {
                std::lock_guard<std::mutex> lk(mu);
                waiting = pending.empty();
            }
            if (active.size() == before && waiting)
                std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        // drain the oldest window when two are queued, or when no further window
        // will be enqueued (no table jobs left: only small jobs, or none, remain)
        if (s == LSR_OK && (inflight.size() >= (size_t)kWindowsInFlight || (n_table == 0 && !inflight.empty()))) {
            hipEvent_t ev = inflight.front();
            inflight.pop_front();
            hipError_t e = hipEventSynchronize(ev);
            put_event(ev);
            if (e != hipSuccess) s = fail(LSR_EDEVICE, "window: %s", hipGetErrorString(e));
            else engine_scan();
        }
        if (s == LSR_OK) {
            const bool nothing_else = active.empty() && inflight.empty();
            engine_poll_retiring(nothing_else && !retiring.empty());
        }
        pub_ingesting.store((int64_t)ingesting.size());
        pub_active.store((int64_t)active.size());
        pub_retiring.store((int64_t)retiring.size());
        if (s != LSR_OK && s != LSR_EBUSY) {
            // a device failure ends every job of the context
            fatal = g_last_error;
            (void)hipStreamSynchronize(stream);
            (void)hipStreamSynchronize(copy_stream);
            (void)hipStreamSynchronize(copy_out_stream);
            (void)hipStreamSynchronize(detect_stream);
            std::vector<Job*> all(active.begin(), active.end());
            all.insert(all.end(), retiring.begin(), retiring.end());
            all.insert(all.end(), ingesting.begin(), ingesting.end());
            ingesting.clear();
            {
                std::lock_guard<std::mutex> lk(mu);
                all.insert(all.end(), pending.begin(), pending.end());
                pending.clear();
            }
            active.clear();
            retiring.clear();
            for (Job* j : all) {
                j->error = fatal;
                j->t_done = Clock::now();
                engine_finish(j, LSR_EDEVICE);
            }
        }
    }
    for (hipEvent_t ev : inflight) {
        (void)hipEventSynchronize(ev);
        put_event(ev);
    }
}
