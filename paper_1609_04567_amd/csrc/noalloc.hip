// lsr_run_noalloc: lsr_run's loop for callers that cannot allocate device memory.
//
// The job's scratch (ping-pong partner grid, per-tile partials, 64 B loop state)
// lives in one file-scope device array of fixed size instead of the context's
// pool. Each device that loads the library holds its own copy of the array until
// the process ends; its device address is looked up once per device when a
// context is created there (lsr_create) and only that address is used from host
// code. The loop is driven synchronously on the caller's stream: sweep chunks
// are launched directly (no graph, no event, no pinned mirror), and the 64 B
// state is read back after each chunk to see whether the loop has stopped.
#include <mutex>

#include "runtime_internal.hpp"

// The scratch of every lsr_run_noalloc call on this device. In host code the
// name stands for a host-side shadow, never for device memory: kernels receive
// the address kept in g_scratch below.
static __device__ __align__(256) unsigned char scratch[(size_t)LSR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = (size_t)LSR_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

namespace lsr_rt {

// Called by lsr_create with `device` current: records the device address of the
// array on this device.
lsr_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(LSR_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return LSR_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(LSR_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[device] = p;
    return LSR_OK;
}

}  // namespace lsr_rt

using namespace lsr_rt;

extern "C" lsr_status lsr_run_noalloc(lsr_ctx* ctx, const lsr_grid* grid, int32_t stencil_id,
                                      int32_t reduce_op, const lsr_cond* cond, int64_t max_iter,
                                      lsr_job_result* out) {
    if (!ctx || !out) return fail(LSR_EINVAL, "ctx and out must not be NULL");
    lsr_status v = validate(grid, stencil_id, reduce_op, cond, max_iter);
    if (v != LSR_OK) return v;
    if (needs_staging(*grid, stencil_id))
        return fail(LSR_EINVAL, "lsr_run_noalloc needs grids the kernels sweep in place: 16-byte "
                                "aligned rows (Life: also a multiple of 16 cells per row)");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch[ctx->device];
    }
    if (!base) return fail(LSR_EDEVICE, "no scratch address for device %d", ctx->device);
    HIP_TRY(hipSetDevice(ctx->device));
    const auto t0 = Clock::now();

    // Layout: partner grid, then partials, then the loop state, each 256-byte aligned.
    Job j;
    j.grid = *grid;
    j.xgrid = *grid;
    j.stencil = stencil_id;
    j.cond = *cond;
    j.max_iter = max_iter;
    const lsr_grid& g = j.xgrid;
    const size_t esz = dtype_size(g.dtype);
    const size_t grid_bytes = (size_t)g.rows * (size_t)g.pitch * esz;
    if (grid_bytes > kScratchBytes)
        return fail(LSR_EINVAL, "a %lld x %lld grid (pitch %lld) needs %zu bytes of partner; the "
                                "no-alloc scratch holds %zu", (long long)g.rows, (long long)g.cols,
                    (long long)g.pitch, grid_bytes, kScratchBytes);
    j.buf[0] = grid->data;
    j.buf[1] = base;
    lsr_tuning tun;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        tun = ctx->tuned_for(*grid, stencil_id, cond->check_every);
    }
    int nparts = 0;
    lsr_status st = plan_plain(&j, reduce_op, tun, &nparts);
    if (st != LSR_OK) return st;
    const size_t parts_off = align256(grid_bytes);
    const size_t state_off = parts_off + align256((size_t)std::max(nparts, 1) * 8);
    if (state_off + sizeof(lsr::JobState) > kScratchBytes)
        return fail(LSR_EINVAL, "grid and partials need %zu bytes; the no-alloc scratch holds %zu",
                    state_off + sizeof(lsr::JobState), kScratchBytes);
    unsigned char* b = static_cast<unsigned char*>(base);
    j.partials = b + parts_off;
    j.st = reinterpret_cast<lsr::JobState*>(b + state_off);
    j.mirror_dev = nullptr;   // the state is read back with a copy instead

    hipStream_t s = ctx->user_stream;
    if (j.stencil != LSR_ST_LIFE) {
        // the partner holds the ring (Jacobi) and the unflagged pixels (restoration) too
        HIP_TRY(hipMemcpy2DAsync(j.buf[1], g.pitch * esz, j.buf[0], g.pitch * esz, g.cols * esz,
                                 g.rows, hipMemcpyDeviceToDevice, s));
        HIP_TRY(lsr::launch_init_state(j.st, nullptr, 0, s));
    } else {
        int np = 0;
        HIP_TRY(lsr::launch_count_u8(static_cast<uint8_t*>(j.buf[0]), g.rows, g.cols, g.pitch,
                                     j.partials, &np, s));
        HIP_TRY(lsr::launch_init_state(j.st, j.partials, np, s));
    }
    const int64_t chunks = (max_iter + j.ctl.chunk - 1) / j.ctl.chunk;
    lsr::JobState fin{};
    for (int64_t k = 0; k < chunks; ++k) {
        st = enqueue_chunk(&j, s);
        if (st != LSR_OK) return st;
        HIP_TRY(hipMemcpyAsync(&fin, j.st, sizeof fin, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (fin.done) break;
    }
    if (!fin.done) return fail(LSR_EDEVICE, "the loop did not stop at its cap");
    int last = 0;
    st = finish_fused(&j, fin, j.geom.tb, j.ctl, &last, s);
    if (st != LSR_OK) return st;
    if (last)
        HIP_TRY(hipMemcpy2DAsync(j.buf[0], g.pitch * esz, j.buf[1], g.pitch * esz, g.cols * esz,
                                 g.rows, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    lsr_job_result r{};
    r.iterations = fin.n;
    r.last_reduce = fin.r;
    r.last_count = fin.count;
    r.converged = fin.converged;
    r.stable_run = fin.run;
    r.sweeps_per_launch = j.geom.tb;
    r.checks = fin.checks;
    r.status = fin.status == lsr::ST_NUMERIC ? LSR_ENUMERIC : LSR_OK;
    r.latency_ms = r.device_ms = ms_between(t0, Clock::now());
    r.queue_ms = 0.0;
    *out = r;
    if (r.status == LSR_ENUMERIC) g_last_error = "reduce value became NaN or Inf";
    return (lsr_status)r.status;
}
