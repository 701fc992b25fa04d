// Host runtime of the loop-of-stencil-reduce library: the C ABI of lsr.h, a
// caching device-memory pool bounded by an HBM budget, the job table and the
// loop driver.
//
// Execution model (the paper's Fig. 2 loop, restructured for one MI355X):
//  * The grid stays resident in HBM for the whole job; a ping-pong partner of
//    the same shape is drawn from the pool and the two only swap roles (device
//    memory persistence by buffer swap, Sect. 3.3). The job's sweep kernels
//    read buffer j%2 and write (j+1)%2.
//  * The final reduce and the condition run on the device (finalize kernel),
//    so no value crosses to the host per iteration. The host driver thread
//    enqueues chunks of `chunk` sweeps (a multiple of check_every, even) as HIP
//    graph replays, stays at most kDepth chunks ahead of the device, and stops
//    enqueueing as soon as the device-written done flag (mirrored into pinned
//    host memory) is seen. Sweeps enqueued past the stop exit at entry.
//  * Each context owns one internal stream (default priority). A job starts
//    after the work the caller had enqueued on its stream when lsr_run was
//    called; lsr_result orders the caller's stream after the job's end.
#include "runtime_internal.hpp"

namespace lsr_rt {

thread_local std::string g_last_error = "";

lsr_status fail(lsr_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

}  // namespace lsr_rt

using namespace lsr_rt;

lsr_status lsr_rt::validate(const lsr_grid* g, int stencil, int reduce, const lsr_cond* c,
                            int64_t max_iter) {
    if (!g || !c) return fail(LSR_EINVAL, "grid and cond must not be NULL");
    if (!g->data) return fail(LSR_EINVAL, "grid->data is NULL");
    if (g->pitch < g->cols) return fail(LSR_EINVAL, "pitch (%lld) < cols (%lld)", (long long)g->pitch, (long long)g->cols);
    if (c->check_every < 1) return fail(LSR_EINVAL, "check_every must be >= 1");
    if (max_iter < 1) return fail(LSR_EINVAL, "max_iter must be >= 1");
    if (g->env1 && stencil != LSR_ST_HELMHOLTZ5_SEP)
        return fail(LSR_EINVAL, "env1 is reserved and must be NULL");
    const bool fp = g->dtype == LSR_F64 || g->dtype == LSR_F32;
    switch (stencil) {
        case LSR_ST_HELMHOLTZ5_SEP:
            if (!g->env0 || !g->env1)
                return fail(LSR_EINVAL, "the -i Helmholtz form needs env0 = p (rows) and env1 = q (cols)");
            if (!std::isfinite(g->param[2]) || !std::isfinite(g->param[3]))
                return fail(LSR_EINVAL, "c1 and c2 must be finite");
            [[fallthrough]];
        case LSR_ST_LAPLACE5:
        case LSR_ST_HELMHOLTZ5:
            if (g->rows < 3 || g->cols < 3) return fail(LSR_EINVAL, "Jacobi grids need rows, cols >= 3");
            if (!fp) return fail(LSR_EINVAL, "Jacobi grids are F64 or F32");
            if (g->bc != LSR_BC_RING) return fail(LSR_EINVAL, "Jacobi stencils use the RING boundary");
            if (stencil == LSR_ST_HELMHOLTZ5 && !g->env0) return fail(LSR_EINVAL, "Helmholtz needs env0 = h^2 f");
            if (stencil == LSR_ST_LAPLACE5 && g->env0) return fail(LSR_EINVAL, "Laplace takes no env0");
            if (stencil != LSR_ST_LAPLACE5) {
                const double rd = 1.0 / (4.0 + g->param[0] * (g->param[1] * g->param[1]));
                if (!std::isfinite(rd)) return fail(LSR_EINVAL, "1/(4 + alpha h^2) is not finite");
                // the FP32 update rounds 0.25 t + (0.25 e - (0.25 - rd) t) with an add
                // that needs |0.25 - rd| <= 1/8
                if (g->dtype == LSR_F32 && !(rd >= 0.125 && rd <= 0.375))
                    return fail(LSR_EINVAL, "FP32 Helmholtz needs 1/(4 + alpha h^2) in [1/8, 3/8] "
                                            "(alpha h^2 in [-4/3, 4])");
            }
            if (reduce != LSR_RED_MAX_ABS_DELTA && reduce != LSR_RED_L2_DELTA && reduce != LSR_RED_MEAN_ABS_DELTA)
                return fail(LSR_EINVAL, "Jacobi reduces are MAX_ABS_DELTA, L2_DELTA, MEAN_ABS_DELTA");
            if (c->kind != LSR_COND_BELOW && c->kind != LSR_COND_NEVER)
                return fail(LSR_EINVAL, "Jacobi conditions are BELOW or NEVER");
            break;
        case LSR_ST_LIFE:
            if (g->rows < 1 || g->cols < 1) return fail(LSR_EINVAL, "empty grid");
            if (g->dtype != LSR_U8) return fail(LSR_EINVAL, "Life grids are U8");
            if (g->bc != LSR_BC_TORUS && g->bc != LSR_BC_BOTTOM) return fail(LSR_EINVAL, "Life uses TORUS or BOTTOM");
            if (g->env0) return fail(LSR_EINVAL, "Life takes no env0");
            if (reduce != LSR_RED_SUM) return fail(LSR_EINVAL, "Life reduces with SUM");
            if (c->kind != LSR_COND_STABLE_FOR && c->kind != LSR_COND_NEVER)
                return fail(LSR_EINVAL, "Life conditions are STABLE_FOR or NEVER");
            if (c->kind == LSR_COND_STABLE_FOR && c->stable_window < 1)
                return fail(LSR_EINVAL, "stable_window must be >= 1");
            break;
        case LSR_ST_RESTORE:
            if (g->rows < 1 || g->cols < 1) return fail(LSR_EINVAL, "empty grid");
            if (!fp) return fail(LSR_EINVAL, "restoration grids are F64 or F32");
            if (g->bc != LSR_BC_BOTTOM) return fail(LSR_EINVAL, "restoration uses the BOTTOM boundary");
            if (!g->env0) return fail(LSR_EINVAL, "restoration needs env0 = mask");
            if (g->param[1] == 0.0 && !(g->param[0] > 0.0)) return fail(LSR_EINVAL, "beta must be > 0");
            if (reduce != LSR_RED_MAX_ABS_DELTA && reduce != LSR_RED_MEAN_ABS_DELTA)
                return fail(LSR_EINVAL, "restoration reduces are MAX_ABS_DELTA or MEAN_ABS_DELTA");
            if (c->kind != LSR_COND_BELOW && c->kind != LSR_COND_NEVER)
                return fail(LSR_EINVAL, "restoration conditions are BELOW or NEVER");
            break;
        case LSR_ST_BOX:
        case LSR_ST_LAPLACE7_3D: {
            if (!fp) return fail(LSR_EINVAL, "box and 3D grids are F64 or F32");
            if (g->bc != LSR_BC_RING) return fail(LSR_EINVAL, "box and 3D stencils use the RING boundary");
            if (g->env0) return fail(LSR_EINVAL, "box and 3D stencils take no env0");
            if (stencil == LSR_ST_BOX) {
                const double k = g->param[0];
                if (!(k == 1.0 || k == 2.0 || k == 3.0 || k == 4.0))
                    return fail(LSR_EINVAL, "box radius param[0] must be 1, 2, 3 or 4");
                if (g->rows < 2 * (int64_t)k + 1 || g->cols < 2 * (int64_t)k + 1)
                    return fail(LSR_EINVAL, "the grid must be at least 2k+1 wide");
            } else {
                const double ny = g->param[0];
                if (!(ny >= 3.0 && ny == std::floor(ny)) || ny > (double)g->rows ||
                    g->rows % (int64_t)ny != 0 || g->rows / (int64_t)ny < 3 || g->cols < 3)
                    return fail(LSR_EINVAL, "3D grids: param[0] = ny >= 3 dividing rows, nz = rows/ny "
                                            ">= 3, cols = nx >= 3");
            }
            if (reduce != LSR_RED_MAX_ABS_DELTA && reduce != LSR_RED_L2_DELTA && reduce != LSR_RED_MEAN_ABS_DELTA)
                return fail(LSR_EINVAL, "box and 3D reduces are MAX_ABS_DELTA, L2_DELTA, MEAN_ABS_DELTA");
            if (c->kind != LSR_COND_BELOW && c->kind != LSR_COND_NEVER)
                return fail(LSR_EINVAL, "box and 3D conditions are BELOW or NEVER");
            break;
        }
        case LSR_ST_SOBEL:
            if (g->rows < 1 || g->cols < 1) return fail(LSR_EINVAL, "empty grid");
            if (g->dtype != LSR_U8) return fail(LSR_EINVAL, "Sobel images are U8");
            if (g->bc != LSR_BC_BOTTOM) return fail(LSR_EINVAL, "Sobel uses the BOTTOM boundary");
            if (g->env0) return fail(LSR_EINVAL, "Sobel takes no env0");
            if (reduce != LSR_RED_SUM) return fail(LSR_EINVAL, "Sobel reduces with SUM");
            if (c->kind != LSR_COND_NEVER) return fail(LSR_EINVAL, "Sobel runs to max_iter (NEVER)");
            break;
        default:
            return fail(LSR_EINVAL, "unknown stencil_id %d", stencil);
    }
    if (c->kind == LSR_COND_BELOW && !std::isfinite(c->threshold))
        return fail(LSR_EINVAL, "threshold must be finite");
    return LSR_OK;
}

namespace {

// Longest chunk base (sweeps) the driver captures into one graph.
constexpr int64_t kMaxChunkBase = 65536;

// Sweeps per chunk: a multiple of lcm(check_every, 2 * tb) that keeps a chunk
// near kChunkTargetUs of device time at HBM speed, so the enqueue-ahead window
// stays a few milliseconds and the overshoot after a stop stays bounded. A
// chunk then holds an even number of launches, so every chunk (and every replay
// of a captured one) starts from buffer 0, and every chunk has its check sweeps
// at the same offsets. A check period of at least max_iter leaves only the check
// at the cap, which falls at one fixed offset of the last chunk: the base is then
// 2 * tb. Computed in 64 bits; 0 when the base exceeds kMaxChunkBase. The
// restoration sweep is bound by its per-pixel solve rather than by HBM: its
// estimate is the measured time per pixel (4096^2 at 40 % impulses: 196 us per
// FP64 sweep, 94 us FP32), which keeps its chunks short; such jobs usually stop
// after a few sweeps, and every launch enqueued past the stop still costs its
// early exit.
int pick_chunk(const lsr_grid* g, int stencil_id, int check_every, int64_t max_iter,
               int override_chunk, int tb) {
    const int64_t base = (int64_t)check_every >= max_iter ? 2 * (int64_t)tb
                                                           : std::lcm((int64_t)check_every, 2 * (int64_t)tb);
    if (base > kMaxChunkBase) return 0;
    int64_t chunk;
    if (override_chunk > 0) {
        chunk = ((int64_t)override_chunk + base - 1) / base * base;
    } else {
        const double cells = (double)g->rows * (double)g->cols;
        const double bytes = cells * (double)dtype_size(g->dtype) * 3.0;
        double est_us = std::max(4.0, bytes / 5.0e6);
        if (stencil_id == LSR_ST_RESTORE)
            est_us = std::max(est_us, cells * (g->dtype == LSR_F32 ? 5.6e-6 : 1.17e-5));
        const int64_t m = (int64_t)std::max(1.0, std::floor(kChunkTargetUs / (est_us * (double)base)));
        chunk = base * m;
        if (chunk > kMaxChunk) chunk = std::max(base, kMaxChunk / base * base);
    }
    const int64_t cap = (max_iter + base - 1) / base * base;
    if (chunk > cap) chunk = cap;
    if (chunk > kMaxChunkBase) chunk = base;
    return (int)chunk;
}

}  // namespace

hipEvent_t lsr_ctx::get_event() {
    if (!event_pool.empty()) {
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

lsr::JacobiArgs lsr_rt::jacobi_args(const Job* j, const void* src, void* dst) {
    const lsr_grid& g = j->xgrid;
    lsr::JacobiArgs a;
    a.a = src;
    a.b = dst;
    a.g = g.env0;
    a.rows = g.rows;
    a.cols = g.cols;
    a.pitch = g.pitch;
    a.rd = 1.0 / (4.0 + g.param[0] * (g.param[1] * g.param[1]));
    a.helm = j->stencil == LSR_ST_HELMHOLTZ5 || j->stencil == LSR_ST_HELMHOLTZ5_SEP;
    a.f32 = g.dtype == LSR_F32;
    if (j->stencil == LSR_ST_HELMHOLTZ5_SEP) {
        a.g = nullptr;
        a.sep = 1;
        a.sp = static_cast<const double*>(g.env0);
        a.sq = static_cast<const double*>(g.env1);
        a.c1 = g.param[2];
        a.c2 = g.param[3];
    }
    return a;
}

lsr::LifeArgs lsr_rt::life_args(const Job* j, const void* src, void* dst) {
    const lsr_grid& g = j->xgrid;
    lsr::LifeArgs a;
    a.a = static_cast<const uint8_t*>(src);
    a.b = static_cast<uint8_t*>(dst);
    a.rows = g.rows;
    a.cols = g.cols;
    a.pitch = g.pitch;
    a.torus = g.bc == LSR_BC_TORUS;
    a.padded = j->staged;
    return a;
}

lsr_status lsr_rt::launch_sweep(Job* j, int off, hipStream_t s) {
    // one launch advances tb sweeps (off .. off + tb - 1 of the chunk)
    const int tb = j->geom.tb;
    const int launch = off / tb;
    void* src = j->buf[launch & 1];
    void* dst = j->buf[(launch + 1) & 1];
    hipError_t e = hipSuccess;
    const lsr_grid& g = j->xgrid;
    switch (j->stencil) {
        case LSR_ST_LAPLACE5:
        case LSR_ST_HELMHOLTZ5:
        case LSR_ST_HELMHOLTZ5_SEP:
            e = lsr::launch_jacobi(jacobi_args(j, src, dst), j->geom, j->st, j->partials, j->ctl,
                                   off, s);
            break;
        case LSR_ST_LIFE:
            e = lsr::launch_life(life_args(j, src, dst), j->geom, j->st, j->partials, j->ctl, off, s);
            break;
        case LSR_ST_BOX:
            e = lsr::launch_box(src, dst, g.rows, g.cols, g.pitch, (int)g.param[0],
                                g.dtype == LSR_F32, j->geom, j->st, j->partials, j->ctl, off, s);
            break;
        case LSR_ST_LAPLACE7_3D: {
            const int64_t ny = (int64_t)g.param[0];
            e = lsr::launch_laplace3d(src, dst, g.rows / ny, ny, g.cols, g.pitch, g.dtype == LSR_F32,
                                      j->geom, j->st, j->partials, j->ctl, off, s);
            break;
        }
        case LSR_ST_SOBEL:
            e = lsr::launch_sobel(static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst), g.rows,
                                  g.cols, g.pitch, j->geom, j->st, j->partials, j->ctl, off, s);
            break;
        case LSR_ST_RESTORE: {
            lsr::RestoreArgs a;
            a.a = src;
            a.b = dst;
            a.mask = static_cast<const uint8_t*>(g.env0);
            a.rows = g.rows;
            a.cols = g.cols;
            a.pitch = g.pitch;
            a.beta = g.param[0];
            a.quadratic = g.param[1] != 0.0;
            a.f32 = g.dtype == LSR_F32;
            e = lsr::launch_restore(a, j->geom, j->st, j->partials, j->ctl, off, s);
            break;
        }
    }
    if (e != hipSuccess) return fail(LSR_EDEVICE, "sweep launch: %s", hipGetErrorString(e));
    const int last = off + tb - 1;
    if (j->geom.mc) {
        bool any = false;
        for (int k = off; k <= last; ++k) any = any || j->fin_at(k);
        if (any)
            e = lsr::launch_finalize_levels(j->st, j->partials, j->ctl, off, tb, j->geom.tiles,
                                            j->mirror_dev, s);
    } else if (j->fin_at(last)) {
        e = lsr::launch_finalize(j->st, j->partials, j->ctl, last, j->mirror_dev, s);
    }
    if (e != hipSuccess) return fail(LSR_EDEVICE, "finalize launch: %s", hipGetErrorString(e));
    return LSR_OK;
}

// A stop inside a fused launch (possible when the launches carry several
// checks, or at a cap that is not a multiple of the depth) leaves that launch's
// last level in its destination. Its source still holds the state before it, so
// the sweeps up to the stop are replayed there with the unfused kernel, under a
// scratch loop state (the job's real final state is already in the host mirror).
// Returns the buffer holding sweep n in *last.
lsr_status lsr_rt::finish_fused(Job* j, const lsr::JobState& fin, int K, const lsr::LoopCtl& ctl,
                                int* last, hipStream_t s) {
    if (K == 1 || fin.n % K == 0) {
        *last = (int)((fin.n / K) & 1);
        return LSR_OK;
    }
    const int64_t L = (fin.n - 1) / K;          // the launch holding the stop
    const int m = (int)(fin.n - L * K);         // its sweeps to keep (1 .. K-1)
    HIP_TRY(lsr::launch_init_state(j->st, nullptr, 0, s, L * K));
    lsr::LoopCtl rc = ctl;
    rc.max_iter = fin.n;
    rc.check_every = 0x7fffffff;                // only sweep n is a "check" (its partials are unused)
    rc.chunk = 0x7fffffff;
    for (int k = 0; k < m; ++k) {
        void* src = j->buf[(L + k) & 1];
        void* dst = j->buf[(L + k + 1) & 1];
        if (j->stencil == LSR_ST_LIFE) {
            lsr::LifeArgs a = life_args(j, src, dst);
            HIP_TRY(lsr::launch_life(a, j->replay_geom, j->st, j->partials, rc, k, s));
        } else {
            HIP_TRY(lsr::launch_jacobi(jacobi_args(j, src, dst), j->replay_geom, j->st, j->partials,
                                       rc, k, s));
        }
    }
    *last = (int)((L + m) & 1);
    return LSR_OK;
}

lsr_status lsr_rt::enqueue_chunk(Job* j, hipStream_t s) {
    for (int off = 0; off < j->ctl.chunk; off += j->geom.tb) {
        lsr_status st = launch_sweep(j, off, s);
        if (st != LSR_OK) return st;
    }
    return LSR_OK;
}

lsr_status lsr_ctx::run_job(Job* j) {
    HIP_TRY(hipStreamWaitEvent(stream, j->ev_user, 0));
    HIP_TRY(hipEventRecord(j->ev_begin, stream));
    const lsr_grid& g = j->xgrid;
    const lsr_grid& ug = j->grid;   // the caller's grid
    const size_t esz = dtype_size(g.dtype);
    if (j->staged) {
        if (j->stencil == LSR_ST_LIFE) {   // padding cells start (and stay) 0/1
            HIP_TRY(hipMemsetAsync(j->buf[0], 0, (size_t)g.rows * g.pitch * esz, stream));
            HIP_TRY(hipMemsetAsync(j->buf[1], 0, (size_t)g.rows * g.pitch * esz, stream));
        }
        HIP_TRY(hipMemcpy2DAsync(j->buf[0], g.pitch * esz, ug.data, ug.pitch * esz, g.cols * esz,
                                 g.rows, stage_kind(j, true), stream));
        if (j->stage_env) {
            const size_t ee = env_esz(j);
            HIP_TRY(hipMemcpy2DAsync(j->stage_env, g.pitch * ee, ug.env0, ug.pitch * ee,
                                     g.cols * ee, g.rows, stage_kind(j, true), stream));
        }
    }
    // Partner buffer starts as a copy: boundary ring (Jacobi) and unflagged
    // pixels (restoration) are never rewritten, so both buffers must hold them.
    if (j->stencil != LSR_ST_LIFE)
        HIP_TRY(hipMemcpy2DAsync(j->buf[1], g.pitch * esz, j->buf[0], g.pitch * esz, g.cols * esz,
                                 g.rows, hipMemcpyDeviceToDevice, stream));
    if (j->stencil == LSR_ST_LIFE) {
        int np = 0;
        HIP_TRY(lsr::launch_count_u8(static_cast<uint8_t*>(j->buf[0]), g.rows, g.cols, g.pitch,
                                     j->partials, &np, stream));
        HIP_TRY(lsr::launch_init_state(j->st, j->partials, np, stream));
    } else {
        HIP_TRY(lsr::launch_init_state(j->st, nullptr, 0, stream));
    }
    if (j->use_graph) {
        HIP_TRY(hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal));
        lsr_status st = enqueue_chunk(j, capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(capture, &graph);
        if (st != LSR_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(LSR_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        j->graph = graph;
        HIP_TRY(hipGraphInstantiate(&j->exec, graph, nullptr, nullptr, 0));
    }
    const int64_t max_chunks = (j->max_iter + j->ctl.chunk - 1) / j->ctl.chunk;
    std::deque<hipEvent_t> inflight;
    int64_t issued = 0;
    bool stop_seen = false, cancel_sent = false;
    volatile lsr::JobState* mir = j->mirror_host;
    lsr_status status = LSR_OK;
    while (true) {
        while ((int)inflight.size() < kDepth && issued < max_chunks && !stop_seen && !cancel_sent) {
            if (j->cancel.load()) {
                hipError_t e = lsr::launch_cancel(j->st, j->mirror_dev, stream);
                if (e != hipSuccess) { status = fail(LSR_EDEVICE, "cancel: %s", hipGetErrorString(e)); break; }
                cancel_sent = true;
                break;
            }
            if (j->use_graph) {
                hipError_t e = hipGraphLaunch(j->exec, stream);
                if (e != hipSuccess) { status = fail(LSR_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e)); break; }
            } else {
                status = enqueue_chunk(j, stream);
                if (status != LSR_OK) break;
            }
            hipEvent_t ev = get_event();
            if (!ev || hipEventRecord(ev, stream) != hipSuccess) {
                status = fail(LSR_EDEVICE, "event record failed");
                break;
            }
            inflight.push_back(ev);
            ++issued;
        }
        if (status != LSR_OK) break;
        if (inflight.empty()) {
            if (cancel_sent) {
                hipError_t e = hipStreamSynchronize(stream);
                if (e != hipSuccess) status = fail(LSR_EDEVICE, "sync: %s", hipGetErrorString(e));
            }
            break;
        }
        hipEvent_t ev = inflight.front();
        inflight.pop_front();
        hipError_t e = hipEventSynchronize(ev);
        put_event(ev);
        if (e != hipSuccess) { status = fail(LSR_EDEVICE, "hipEventSynchronize: %s", hipGetErrorString(e)); break; }
        if (mir->done) stop_seen = true;
        if (j->cancel.load() && !stop_seen && !cancel_sent) {
            // drain what is in flight, then post the cancel
            continue;
        }
    }
    for (hipEvent_t ev : inflight) {
        (void)hipEventSynchronize(ev);
        put_event(ev);
    }
    if (status != LSR_OK) return status;
    lsr::JobState fin;
    std::memcpy(&fin, (const void*)mir, sizeof fin);
    int last = 0;
    lsr_status rs = finish_fused(j, fin, j->geom.tb, j->ctl, &last, stream);
    if (rs != LSR_OK) return rs;
    if (j->staged)
        HIP_TRY(hipMemcpy2DAsync(ug.data, ug.pitch * esz, j->buf[last], g.pitch * esz, g.cols * esz,
                                 g.rows, stage_kind(j, false), stream));
    else if (last)
        HIP_TRY(hipMemcpy2DAsync(j->buf[0], g.pitch * esz, j->buf[1], g.pitch * esz, g.cols * esz,
                                 g.rows, hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipEventRecord(j->ev_end, stream));
    HIP_TRY(hipEventSynchronize(j->ev_end));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, j->ev_begin, j->ev_end);
    lsr_job_result& r = j->result;
    r.iterations = fin.n;
    r.last_reduce = fin.r;
    r.last_count = fin.count;
    r.converged = fin.converged;
    r.stable_run = fin.run;
    r.sweeps_per_launch = j->geom.tb;
    r.checks = fin.checks;
    r.device_ms = ms;
    r.status = fin.status == lsr::ST_NUMERIC ? LSR_ENUMERIC
             : fin.status == lsr::ST_CANCELED ? LSR_ECANCELED : LSR_OK;
    return (lsr_status)r.status;
}

void lsr_ctx::drive() {
    (void)hipSetDevice(device);
    while (true) {
        Job* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            if (queue.empty()) return;
            j = queue.front();
            queue.pop_front();
            j->phase = Phase::Running;
        }
        lsr_status st = run_job(j);
        if (st != LSR_OK && st != LSR_ENUMERIC && st != LSR_ECANCELED) {
            j->error = g_last_error;
            (void)hipStreamSynchronize(stream);
            (void)hipEventRecord(j->ev_end, stream);
            j->result.status = st;
        }
        j->status = (lsr_status)j->result.status;
        if (j->exec) (void)hipGraphExecDestroy(j->exec);
        if (j->graph) (void)hipGraphDestroy(j->graph);
        j->exec = nullptr;
        j->graph = nullptr;
        j->release_scratch(pool);
        {
            std::lock_guard<std::mutex> lk(mu);
            if (j->slot >= 0) free_slots.push_back(j->slot);
            j->slot = -1;
            j->phase = Phase::Finished;
            done_q.push_back(j->id);
            --unfinished;
        }
        cv_done.notify_all();
    }
}

extern "C" {

const char* lsr_last_error(void) { return g_last_error.c_str(); }

const char* lsr_version(void) { return "lsr 0.1 (gfx950)"; }

lsr_status lsr_check_args(const lsr_grid* grid, int32_t stencil_id, int32_t reduce_op,
                          const lsr_cond* cond, int64_t max_iter) {
    return validate(grid, stencil_id, reduce_op, cond, max_iter);
}

lsr_status lsr_create(const lsr_config* cfg, lsr_ctx** out) {
    if (!cfg || !out) return fail(LSR_EINVAL, "cfg and out must not be NULL");
    *out = nullptr;
    if (cfg->flags & ~LSR_FLAG_BATCHED) return fail(LSR_EINVAL, "unknown flags 0x%x", cfg->flags);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(LSR_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(LSR_EINVAL, "device %d out of range", cfg->device);
    HIP_TRY(hipSetDevice(cfg->device));
    lsr_status ns = noalloc_setup(cfg->device);
    if (ns != LSR_OK) return ns;
    std::unique_ptr<lsr_ctx> c(new lsr_ctx());
    c->device = cfg->device;
    c->user_stream = static_cast<hipStream_t>(cfg->stream);
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    uint64_t budget = cfg->hbm_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIP_TRY(hipMemGetInfo(&fr, &tot));
        budget = (uint64_t)(0.9 * (double)fr);
    }
    c->pool.init(budget);
    HIP_TRY(hipHostMalloc((void**)&c->mirrors_host, sizeof(lsr::JobState) * kMirrorSlots,
                          hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostGetDevicePointer((void**)&c->mirrors_dev, c->mirrors_host, 0));
    std::memset(c->mirrors_host, 0, sizeof(lsr::JobState) * kMirrorSlots);
    for (int i = kMirrorSlots - 1; i >= 0; --i) c->free_slots.push_back(i);
    c->batched = (cfg->flags & LSR_FLAG_BATCHED) != 0;
    if (c->batched) {
        lsr_status st = c->engine_setup();
        if (st != LSR_OK) {
            c->engine_teardown();
            return st;
        }
    }
    lsr_ctx* raw = c.release();
    if (raw->batched) raw->driver = std::thread([raw] { raw->serve(); });
    else raw->driver = std::thread([raw] { raw->drive(); });
    *out = raw;
    return LSR_OK;
}

lsr_status lsr_set_tuning(lsr_ctx* ctx, const lsr_tuning* t) {
    if (!ctx) return fail(LSR_EINVAL, "ctx is NULL");
    if (t && (t->tile_rows < 0 || t->tb_depth < 0 || t->chunk < 0 || t->waves < 0 || t->unroll < 0))
        return fail(LSR_EINVAL, "tuning fields must be >= 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (t) ctx->tuning = *t;
    else ctx->tuning = lsr_tuning{};
    return LSR_OK;
}

lsr_status lsr_run(lsr_ctx* ctx, const lsr_grid* grid, int32_t stencil_id, int32_t reduce_op,
                   const lsr_cond* cond, int64_t max_iter, lsr_job* job_out) {
    return submit(ctx, grid, stencil_id, reduce_op, cond, max_iter, false, job_out);
}

lsr_status lsr_run_host(lsr_ctx* ctx, const lsr_grid* grid, int32_t stencil_id, int32_t reduce_op,
                        const lsr_cond* cond, int64_t max_iter, lsr_job* job_out) {
    return submit(ctx, grid, stencil_id, reduce_op, cond, max_iter, true, job_out);
}

lsr_status lsr_run_restore_host(lsr_ctx* ctx, const lsr_grid* y, void* u_out, int32_t u_dtype,
                                int32_t w_max, int32_t reduce_op, const lsr_cond* cond,
                                int64_t max_iter, lsr_job* job_out) {
    if (!ctx || !y || !u_out || !job_out) return fail(LSR_EINVAL, "NULL argument");
    if (!ctx->batched) return fail(LSR_EINVAL, "two-phase host jobs run on a batched context");
    if (!y->data || y->dtype != LSR_U8) return fail(LSR_EINVAL, "the frame is a U8 image");
    if (u_dtype != LSR_F32 && u_dtype != LSR_F64) return fail(LSR_EINVAL, "u_dtype is F32 or F64");
    if (w_max < 3 || w_max > 31 || w_max % 2 == 0) return fail(LSR_EINVAL, "w_max must be odd in [3, 31]");
    // the restoration job on the frame's shape; its mask is made on the device
    lsr_grid ug = *y;
    ug.dtype = u_dtype;
    ug.data = u_out;
    ug.env0 = y->data;
    lsr_status v = validate(&ug, LSR_ST_RESTORE, reduce_op, cond, max_iter);
    if (v != LSR_OK) return v;
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<Job> j(new Job());
    j->host = true;
    j->two_phase = true;
    j->w_max = w_max;
    j->in_host = y->data;
    j->out_host = u_out;
    j->host_pitch = y->pitch;
    j->grid = ug;
    j->xgrid = ug;
    j->stencil = LSR_ST_RESTORE;
    j->cond = *cond;
    j->max_iter = max_iter;
    j->ctl.reduce = reduce_op;
    return submit_batched(ctx, std::move(j), job_out);
}

}  // extern "C"

// Queues a job on a batched context (its descriptor from engine_submit).
lsr_status lsr_rt::submit_batched(lsr_ctx* ctx, std::unique_ptr<Job> j, lsr_job* job_out) {
    lsr_status s = ctx->engine_submit(j.get());
    if (s != LSR_OK) return s;
    if (hipEventCreateWithFlags(&j->ev_user, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&j->ev_begin) != hipSuccess || hipEventCreate(&j->ev_end) != hipSuccess ||
        hipEventRecord(j->ev_user, ctx->user_stream) != hipSuccess) {
        if (j->ev_user) (void)hipEventDestroy(j->ev_user);
        if (j->ev_begin) (void)hipEventDestroy(j->ev_begin);
        if (j->ev_end) (void)hipEventDestroy(j->ev_end);
        return fail(LSR_EDEVICE, "event setup failed");
    }
    j->t_submit = j->t_admit = Clock::now();
    Job* raw = j.get();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        raw->id = ctx->next_id++;
        ctx->jobs[raw->id] = std::move(j);
        ++ctx->unfinished;
        ctx->pending.push_back(raw);
    }
    ctx->cv_work.notify_one();
    *job_out = raw->id;
    return LSR_OK;
}

lsr_status lsr_rt::submit(lsr_ctx* ctx, const lsr_grid* grid, int32_t stencil_id, int32_t reduce_op,
                          const lsr_cond* cond, int64_t max_iter, bool host, lsr_job* job_out) {
    if (!ctx || !job_out) return fail(LSR_EINVAL, "ctx and job_out must not be NULL");
    lsr_status v = validate(grid, stencil_id, reduce_op, cond, max_iter);
    if (v != LSR_OK) return v;
    if (stencil_id == LSR_ST_HELMHOLTZ5_SEP && (host || ctx->batched))
        return fail(LSR_EINVAL, "the -i Helmholtz form runs on device buffers on a plain context");
    if ((stencil_id == LSR_ST_BOX || stencil_id == LSR_ST_LAPLACE7_3D) && ctx->batched)
        return fail(LSR_EINVAL, "box and 3D stencils run on a plain context");
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<Job> j(new Job());
    j->host = host;
    j->grid = *grid;
    j->xgrid = *grid;
    j->stencil = stencil_id;
    j->cond = *cond;
    j->max_iter = max_iter;
    if (ctx->batched) {
        j->ctl.reduce = reduce_op;
        return submit_batched(ctx, std::move(j), job_out);
    }
    lsr_tuning tun;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        tun = ctx->tuned_for(*grid, stencil_id, cond->check_every);
    }
    return submit_plain(ctx, std::move(j), grid, stencil_id, reduce_op, cond, max_iter, tun, job_out);
}

// The plain (one job at a time) path of lsr_run with the launch settings resolved.
lsr_status lsr_rt::plan_plain(Job* j, int reduce_op, const lsr_tuning& tun, int* nparts_out) {
    const lsr_grid& g = j->xgrid;
    const int stencil_id = j->stencil;
    // a check period of at least max_iter leaves only the check at the cap: the
    // same loop as a period of exactly max_iter
    const int check_every = (int)std::min<int64_t>(j->cond.check_every, j->max_iter);
    auto plan = [&](int want_depth) {
        switch (stencil_id) {
            case LSR_ST_LAPLACE5:
            case LSR_ST_HELMHOLTZ5:
            case LSR_ST_HELMHOLTZ5_SEP: {
                lsr::JacobiArgs a = jacobi_args(j, j->buf[0], j->buf[1]);
                int depth = 1, mc = 0;
                lsr::jacobi_tb_choose(a, check_every, j->max_iter, want_depth, &depth, &mc);
                j->geom = lsr::jacobi_geom(a, tun.tile_rows, tun.waves, tun.unroll, depth, mc);
                // unfused sweeps that replay a stop inside a fused launch
                j->replay_geom = lsr::jacobi_geom(a, 0);
                break;
            }
            case LSR_ST_LIFE: {
                lsr::LifeArgs a{};
                a.a = static_cast<const uint8_t*>(j->buf[0]);
                a.b = static_cast<uint8_t*>(j->buf[1]);
                a.rows = g.rows;
                a.cols = g.cols;
                a.pitch = g.pitch;
                a.torus = g.bc == LSR_BC_TORUS;
                a.padded = j->staged;
                const int depth = lsr::life_tb_choose(a, want_depth);
                j->geom = depth > 1 ? lsr::life_tb_geom(a, depth, tun.tile_rows)
                                    : lsr::life_geom(a, tun.tile_rows);
                // single generations that replay a stop inside a fused launch
                j->replay_geom = lsr::life_geom(a, 0);
                break;
            }
            case LSR_ST_SOBEL:
                j->geom = lsr::sobel_geom(g.rows, g.cols);
                break;
            case LSR_ST_BOX:
                j->geom = lsr::box_geom(g.rows, g.cols);
                break;
            case LSR_ST_LAPLACE7_3D:
                j->geom = lsr::laplace3d_geom(g.rows / (int64_t)g.param[0], (int64_t)g.param[0], g.cols);
                break;
            default: {
                lsr::RestoreArgs a{};
                a.rows = g.rows;
                a.cols = g.cols;
                j->geom = lsr::restore_geom(a, tun.tile_rows);
            }
        }
        return pick_chunk(&g, stencil_id, check_every, j->max_iter, tun.chunk, j->geom.tb);
    };
    int chunk = plan(tun.tb_depth);
    // a check period whose lcm with two fused launches is too long to capture:
    // unfused sweeps need only lcm(check_every, 2)
    if (chunk == 0 && j->geom.tb > 1) chunk = plan(1);
    if (chunk == 0)
        return fail(LSR_EINVAL, "check_every %d: a chunk of lcm(check_every, 2) sweeps exceeds %lld; "
                                "use a check period of at most %lld or at least max_iter",
                    j->cond.check_every, (long long)kMaxChunkBase, (long long)(kMaxChunkBase / 2));
    int nparts = j->geom.tiles;
    if (j->geom.mc) nparts = j->geom.tiles * j->geom.tb;   // one slice per level
    if (j->geom.tb > 1) nparts = std::max(nparts, j->replay_geom.tiles);
    if (stencil_id == LSR_ST_LIFE) nparts = std::max(nparts, lsr::count_u8_parts(g.rows, g.cols));
    *nparts_out = nparts;
    lsr::LoopCtl& c = j->ctl;
    c.max_iter = j->max_iter;
    c.check_every = check_every;
    c.chunk = chunk;
    c.reduce = reduce_op;
    c.cond = j->cond.kind;
    c.stable_window = j->cond.stable_window;
    c.nparts = j->geom.tiles;
    c.threshold = j->cond.threshold;
    c.mean_div = (double)g.rows * (double)g.cols;
    return LSR_OK;
}

// The plain (one job at a time) path of lsr_run with the launch settings resolved.
lsr_status lsr_rt::submit_plain(lsr_ctx* ctx, std::unique_ptr<Job> j, const lsr_grid* grid,
                                int32_t stencil_id, int32_t reduce_op, const lsr_cond* cond,
                                int64_t max_iter, const lsr_tuning& tun, lsr_job* job_out) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->free_slots.empty()) return fail(LSR_EBUSY, "too many jobs in flight");
        j->slot = ctx->free_slots.back();
        ctx->free_slots.pop_back();
    }
    auto give_back = [&] {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->free_slots.push_back(j->slot);
    };
    const size_t esz = dtype_size(grid->dtype);
    j->staged = j->host || needs_staging(*grid, stencil_id);
    if (j->staged) j->xgrid.pitch = stage_pitch(*grid);
    const size_t bytes = (size_t)grid->rows * (size_t)j->xgrid.pitch * esz;
    // geometry needs both buffers' alignment; the pool returns 256-byte aligned blocks
    lsr_status st = LSR_OK;
    if (j->staged) {
        st = ctx->pool.alloc(bytes, &j->buf[0]);
        if (st == LSR_OK && (stencil_id == LSR_ST_HELMHOLTZ5 || stencil_id == LSR_ST_RESTORE))
            st = ctx->pool.alloc((size_t)grid->rows * (size_t)j->xgrid.pitch * env_esz(j.get()),
                                 &j->stage_env);
        j->xgrid.data = j->buf[0];
        // the -i form's env arrays are the factor vectors, used in place
        if (stencil_id != LSR_ST_HELMHOLTZ5_SEP) j->xgrid.env0 = j->stage_env;
    } else {
        j->buf[0] = grid->data;
    }
    if (st == LSR_OK) st = ctx->pool.alloc(bytes, &j->buf[1]);
    if (st != LSR_OK) {
        if (j->staged) {
            ctx->pool.release(j->buf[0]);
            ctx->pool.release(j->stage_env);
        }
        ctx->pool.release(j->buf[1]);
        give_back();
        return st;
    }
    int nparts = 0;
    st = plan_plain(j.get(), reduce_op, tun, &nparts);
    if (st == LSR_OK) st = ctx->pool.alloc((size_t)std::max(nparts, 1) * 8, &j->partials);
    if (st == LSR_OK) st = ctx->pool.alloc(sizeof(lsr::JobState), (void**)&j->st);
    if (st != LSR_OK) {
        j->release_scratch(ctx->pool);
        give_back();
        return st;
    }
    j->use_graph = tun.use_graph >= 0;
    j->mirror_host = ctx->mirrors_host + j->slot;
    j->mirror_dev = ctx->mirrors_dev + j->slot;
    std::memset((void*)j->mirror_host, 0, sizeof(lsr::JobState));
    auto cleanup = [&] {
        j->release_scratch(ctx->pool);
        if (j->ev_user) (void)hipEventDestroy(j->ev_user);
        if (j->ev_begin) (void)hipEventDestroy(j->ev_begin);
        if (j->ev_end) (void)hipEventDestroy(j->ev_end);
        give_back();
    };
    if (hipEventCreateWithFlags(&j->ev_user, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&j->ev_begin) != hipSuccess || hipEventCreate(&j->ev_end) != hipSuccess ||
        hipEventRecord(j->ev_user, ctx->user_stream) != hipSuccess) {
        cleanup();
        return fail(LSR_EDEVICE, "event setup failed");
    }
    Job* raw = j.get();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        raw->id = ctx->next_id++;
        ctx->jobs[raw->id] = std::move(j);
        ++ctx->unfinished;
        ctx->queue.push_back(raw);
    }
    ctx->cv_work.notify_one();
    *job_out = raw->id;
    return LSR_OK;
}

extern "C" {

lsr_status lsr_result(lsr_ctx* ctx, lsr_job job, int32_t wait, lsr_job_result* out) {
    if (!ctx || !out) return fail(LSR_EINVAL, "ctx and out must not be NULL");
    std::unique_ptr<Job> j;
    {
        std::unique_lock<std::mutex> lk(ctx->mu);
        auto it = ctx->jobs.find(job);
        if (it == ctx->jobs.end()) return fail(LSR_ENOTFOUND, "unknown job %lld", (long long)job);
        Job* p = it->second.get();
        if (p->phase != Phase::Finished) {
            if (!wait) return fail(LSR_EBUSY, "job %lld is still running", (long long)job);
            ctx->cv_done.wait(lk, [&] { return p->phase == Phase::Finished; });
        }
        j = std::move(it->second);
        ctx->jobs.erase(it);
        // ids whose results were taken here stay in the completion queue until
        // lsr_wait_any skips them; drop them when they dominate it
        if (ctx->done_q.size() > 2 * ctx->jobs.size() + 1024) {
            std::deque<lsr_job> keep;
            for (lsr_job id : ctx->done_q)
                if (ctx->jobs.count(id)) keep.push_back(id);
            ctx->done_q.swap(keep);
        }
    }
    *out = j->result;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamWaitEvent(ctx->user_stream, j->ev_end, 0);
    (void)hipEventDestroy(j->ev_user);
    (void)hipEventDestroy(j->ev_begin);
    (void)hipEventDestroy(j->ev_end);
    const lsr_status s = (lsr_status)j->result.status;
    if (s == LSR_EDEVICE) g_last_error = j->error;
    else if (s == LSR_ENUMERIC) g_last_error = "reduce value became NaN or Inf";
    else if (s == LSR_ECANCELED) g_last_error = "job cancelled";
    return s;
}

lsr_status lsr_wait_any(lsr_ctx* ctx, int32_t wait, lsr_job* job_out) {
    if (!ctx || !job_out) return fail(LSR_EINVAL, "ctx and job_out must not be NULL");
    std::unique_lock<std::mutex> lk(ctx->mu);
    while (true) {
        while (!ctx->done_q.empty()) {
            const lsr_job id = ctx->done_q.front();
            ctx->done_q.pop_front();
            if (ctx->jobs.count(id)) {   // not yet taken by lsr_result
                *job_out = id;
                return LSR_OK;
            }
        }
        if (ctx->unfinished == 0) return fail(LSR_ENOTFOUND, "no job is outstanding");
        if (!wait) return fail(LSR_EBUSY, "no job has finished");
        ctx->cv_done.wait(lk);
    }
}

lsr_status lsr_get_stats(lsr_ctx* ctx, lsr_stats* out) {
    if (!ctx || !out) return fail(LSR_EINVAL, "ctx and out must not be NULL");
    lsr_stats s{};
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        s.pending = (int64_t)(ctx->batched ? ctx->pending.size() : ctx->queue.size());
        s.unfinished = ctx->unfinished;
        s.finished_untaken = (int64_t)ctx->jobs.size() - ctx->unfinished;
    }
    if (ctx->batched) {
        s.ingesting = ctx->pub_ingesting.load();
        s.active = ctx->pub_active.load();
        s.retiring = ctx->pub_retiring.load();
    } else {
        s.active = s.unfinished - s.pending;
    }
    ctx->pool.usage(&s.pool_live_bytes, &s.pool_cached_bytes);
    s.pool_budget_bytes = ctx->pool.budget();
    *out = s;
    return LSR_OK;
}

lsr_status lsr_cancel(lsr_ctx* ctx, lsr_job job) {
    if (!ctx) return fail(LSR_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end()) return fail(LSR_ENOTFOUND, "unknown job %lld", (long long)job);
    it->second->cancel.store(true);
    return LSR_OK;
}

lsr_status lsr_amf_detect(lsr_ctx* ctx, const lsr_grid* y, void* mask, void* u_init,
                          int32_t u_dtype, int32_t w_max) {
    if (!ctx || !y || !mask || !u_init || !y->data) return fail(LSR_EINVAL, "NULL argument");
    if (y->dtype != LSR_U8) return fail(LSR_EINVAL, "the image is U8");
    if (y->rows < 1 || y->cols < 1 || y->pitch < y->cols) return fail(LSR_EINVAL, "bad image shape");
    if (u_dtype != LSR_U8 && u_dtype != LSR_F32 && u_dtype != LSR_F64)
        return fail(LSR_EINVAL, "u_dtype is U8, F32 or F64");
    if (w_max < 3 || w_max > 31 || w_max % 2 == 0) return fail(LSR_EINVAL, "w_max must be odd in [3, 31]");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(lsr::launch_amf_detect(static_cast<const uint8_t*>(y->data), y->rows, y->cols, y->pitch,
                                   w_max, static_cast<uint8_t*>(mask), u_init, u_dtype,
                                   ctx->user_stream));
    return LSR_OK;
}

lsr_status lsr_probe_copy(lsr_ctx* ctx, void* dst, const void* src, uint64_t bytes, int32_t iters,
                          double* avg_ms) {
    if (!ctx || !dst || !src || !avg_ms || iters < 1) return fail(LSR_EINVAL, "bad probe arguments");
    if (bytes == 0 || bytes % 16 != 0 || ((reinterpret_cast<uintptr_t>(dst) |
                                            reinterpret_cast<uintptr_t>(src)) & 15) != 0)
        return fail(LSR_EINVAL, "probe needs 16-byte aligned buffers and a multiple of 16 bytes");
    HIP_TRY(hipSetDevice(ctx->device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = lsr::launch_copy16(src, dst, (int64_t)bytes, ctx->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < iters && e == hipSuccess; ++i)
        e = lsr::launch_copy16(src, dst, (int64_t)bytes, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(LSR_EDEVICE, "copy probe: %s", hipGetErrorString(e));
    *avg_ms = (double)ms / iters;
    return LSR_OK;
}

lsr_status lsr_destroy(lsr_ctx* ctx) {
    if (!ctx) return fail(LSR_EINVAL, "ctx is NULL");
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stopping = true;
    }
    ctx->cv_work.notify_all();
    if (ctx->driver.joinable()) ctx->driver.join();
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->batched) ctx->engine_teardown();
    for (auto& kv : ctx->jobs) {
        Job* j = kv.second.get();
        if (j->ev_user) (void)hipEventDestroy(j->ev_user);
        if (j->ev_begin) (void)hipEventDestroy(j->ev_begin);
        if (j->ev_end) (void)hipEventDestroy(j->ev_end);
    }
    ctx->jobs.clear();
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    ctx->pool.destroy();
    if (ctx->mirrors_host) (void)hipHostFree(ctx->mirrors_host);
    (void)hipStreamDestroy(ctx->capture);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return LSR_OK;
}

}  // extern "C"
