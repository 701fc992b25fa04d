// Autotuner: measures candidate launch settings for a job description on the
// device and keeps the fastest per key (stencil, dtype, size class, check
// period). lsr_run consults the table whenever the context's overrides leave
// the launch shape automatic, so a job's settings are a pure function of its key
// (and of the table), the same whatever else runs. The table round-trips as JSON
// text tagged with the device's architecture name.
#include <chrono>

#include "runtime_internal.hpp"

using namespace lsr_rt;

namespace lsr_rt {

namespace {

int bit_length(int64_t v) {
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

bool automatic_shape(const lsr_tuning& t) {
    return t.tile_rows == 0 && t.tb_depth == 0 && t.waves == 0 && t.unroll == 0;
}

// Candidate settings for one job description.
std::vector<lsr_tuning> candidates(int stencil) {
    std::vector<lsr_tuning> out;
    auto add = [&](int tile_rows, int depth, int waves, int unroll) {
        lsr_tuning t{};
        t.tile_rows = tile_rows;
        t.tb_depth = depth;
        t.waves = waves;
        t.unroll = unroll;
        out.push_back(t);
    };
    if (stencil == LSR_ST_LIFE) {
        for (int tr : {8, 16, 32, 64, 128}) add(tr, 1, 0, 0);
        // tile_rows 0: the band height the fused kernel derives from its occupancy
        for (int depth : {2, 3, 4, 5, 6, 8})
            for (int tr : {0, 16, 32, 64, 128}) add(tr, depth, 0, 0);
        return out;
    }
    static constexpr int kUnfused[][2] = {{1, 8}, {2, 8}, {4, 4}, {4, 8}, {4, 16}};
    for (const auto& s : kUnfused)
        for (int tr : {8, 16, 32}) add(tr, 1, s[0], s[1]);
    for (int depth : {2, 4, 5, 8, 10})
        for (int waves : {1, 2, 4})
            for (int tr : {0, 4, 8, 16, 32, 40, 48, 64}) add(tr, depth, waves, 0);
    return out;
}

// Candidates on a batched context: the engine's families take the fused depth
// (Jacobi: FP32 5 or 2, FP64 10, 5 or 2, kept only where it divides the check
// period; otherwise depth 5 with checks inside) and the band rows of a wavefront
// tile (Life: one generation per round, the SWAR tile, or 8, the fused tile,
// each with its band rows).
std::vector<lsr_tuning> candidates_batched(int stencil, int dtype, int check_every) {
    std::vector<lsr_tuning> out;
    auto add = [&](int tile_rows, int depth) {
        lsr_tuning t{};
        t.tile_rows = tile_rows;
        t.tb_depth = depth;
        out.push_back(t);
    };
    if (stencil == LSR_ST_LIFE) {
        for (int tr : {8, 16, 32, 64, 128}) add(tr, 1);
        for (int tr : {16, 32, 64, 128}) add(tr, 8);
        return out;
    }
    std::vector<int> depths;
    for (int k : dtype == LSR_F32 ? std::initializer_list<int>{5, 2} : std::initializer_list<int>{10, 5, 2})
        if (check_every % k == 0) depths.push_back(k);
    if (depths.empty()) depths.push_back(5);
    for (int k : depths)
        for (int tr : {8, 16, 24, 32, 48, 64}) add(tr, k);
    return out;
}

const char* arch_name(int device) {
    static thread_local char name[64];
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::snprintf(name, sizeof name, "%s", p.gcnArchName);
    // keep the base name (gfx950), not the feature suffixes
    for (char* c = name; *c; ++c)
        if (*c == ':') *c = 0;
    return name;
}

}  // namespace

TuneKey tune_key(int stencil, int dtype, int bc, int64_t rows, int64_t cols, int check_every) {
    return TuneKey{stencil, dtype, bc, bit_length(rows), bit_length(cols), check_every};
}

}  // namespace lsr_rt

lsr_tuning lsr_ctx::tuned_for(const lsr_grid& g, int stencil, int check_every) const {
    lsr_tuning t = tuning;
    if (!automatic_shape(t)) return t;
    auto it = tune_table.find(tune_key(stencil, g.dtype, g.bc, g.rows, g.cols, check_every));
    if (it == tune_table.end()) return t;
    const lsr_tuning& w = it->second.tuning;
    t.tile_rows = w.tile_rows;
    t.tb_depth = w.tb_depth;
    t.waves = w.waves;
    t.unroll = w.unroll;
    return t;
}

extern "C" {

lsr_status lsr_autotune(lsr_ctx* ctx, int32_t stencil_id, int32_t dtype, int64_t rows, int64_t cols,
                        int32_t check_every, int64_t max_iter, lsr_tuning* best_out) {
    if (!ctx) return fail(LSR_EINVAL, "ctx is NULL");
    if (stencil_id != LSR_ST_LAPLACE5 && stencil_id != LSR_ST_HELMHOLTZ5 && stencil_id != LSR_ST_LIFE)
        return fail(LSR_EINVAL, "the autotuner covers the Laplace, Helmholtz and Life sweeps");
    if (ctx->batched) {   // its candidates go through the context's overrides
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->unfinished > 0) return fail(LSR_EBUSY, "the batched context has jobs running");
    }
    if (rows < 1 || cols < 1 || rows > (1 << 20) || cols > (1 << 20))
        return fail(LSR_EINVAL, "rows and cols must be in [1, 2^20]");
    const size_t esz = dtype_size(dtype);
    const int64_t pitch = (cols * (int64_t)esz + 255) / 256 * 256 / (int64_t)esz;
    const size_t bytes = (size_t)rows * (size_t)pitch * esz;
    const bool helm = stencil_id == LSR_ST_HELMHOLTZ5;
    lsr_grid g{};
    g.rows = rows;
    g.cols = cols;
    g.pitch = pitch;
    g.dtype = dtype;
    g.bc = stencil_id == LSR_ST_LIFE ? LSR_BC_TORUS : LSR_BC_RING;
    g.param[0] = 1.0;
    g.param[1] = 1.0 / (double)std::max<int64_t>(rows - 1, 1);
    lsr_cond cond{};
    cond.kind = LSR_COND_NEVER;
    cond.check_every = check_every;
    cond.stable_window = 1;
    cond.threshold = 0.0;
    // a short run of the same loop: enough sweeps for several launches at every depth
    const double cells = (double)rows * (double)cols;
    int64_t sweeps = (int64_t)std::min(400.0, std::max(40.0, 2.0e9 / std::max(cells, 1.0)));
    // a fused Life launch takes tens of microseconds: 40 generations are a few
    // launches, too few to rank depths
    if (stencil_id == LSR_ST_LIFE) sweeps = std::max<int64_t>(sweeps, 240);
    sweeps = (sweeps + 39) / 40 * 40;
    if (max_iter > 0) sweeps = std::min<int64_t>(sweeps, max_iter);
    const int reduce = stencil_id == LSR_ST_LIFE ? LSR_RED_SUM : LSR_RED_MAX_ABS_DELTA;
    g.data = reinterpret_cast<void*>(16);   // validation only checks for NULL
    g.env0 = helm ? g.data : nullptr;
    lsr_status v = validate(&g, stencil_id, reduce, &cond, sweeps);
    if (v != LSR_OK) return v;

    HIP_TRY(hipSetDevice(ctx->device));
    // a batched context is measured under load: enough jobs of the key to hold
    // about 2^25 cells run together (8 to 256 jobs, each on its own grid, sharing
    // the read-only g), as the jobs of a stream fill the rounds, and a candidate is
    // ranked by the wall time of the whole batch (a job alone, or a few, favour
    // the most and smallest tiles, which a full round does not need: measured on
    // the mixed stream, tuning with 1 or 8 jobs lost 15-27 % of its jobs/s)
    const int copies = ctx->batched
        ? (int)std::min(256.0, std::max(8.0, std::ceil(33554432.0 / std::max(cells, 1.0))))
        : 1;
    std::vector<void*> grid_bufs(copies, nullptr);
    void* env_buf = nullptr;
    auto release_all = [&]() {
        for (void*& b : grid_bufs) {
            ctx->pool.release(b);
            b = nullptr;
        }
        ctx->pool.release(env_buf);
        env_buf = nullptr;
    };
    lsr_status st = LSR_OK;
    for (int c = 0; c < copies && st == LSR_OK; ++c) st = ctx->pool.alloc(bytes, &grid_bufs[c]);
    if (st == LSR_OK && helm) st = ctx->pool.alloc(bytes, &env_buf);
    if (st != LSR_OK) {
        release_all();
        return st;
    }
    g.data = grid_bufs[0];
    g.env0 = env_buf;
    hipError_t e = hipSuccess;
    for (int c = 0; c < copies && e == hipSuccess; ++c)
        e = hipMemsetAsync(grid_bufs[c], 0, bytes, ctx->user_stream);
    if (e == hipSuccess && env_buf) e = hipMemsetAsync(env_buf, 0, bytes, ctx->user_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->user_stream);
    if (e != hipSuccess) {
        release_all();
        return fail(LSR_EDEVICE, "autotune scratch: %s", hipGetErrorString(e));
    }

    lsr_tuning base;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        base = ctx->tuning;
    }
    // Life jobs key on their boundary too: both boundaries are measured
    const int bcs_life[] = {LSR_BC_TORUS, LSR_BC_BOTTOM};
    const int bcs_jac[] = {LSR_BC_RING};
    const int* bcs = stencil_id == LSR_ST_LIFE ? bcs_life : bcs_jac;
    const int nbc = stencil_id == LSR_ST_LIFE ? 2 : 1;
    lsr_tuning best_first{};
    for (int b = 0; b < nbc && st == LSR_OK; ++b) {
        g.bc = bcs[b];
        lsr_tuning best{};
        double best_ms = 1e300;
        const std::vector<lsr_tuning> cands = ctx->batched ? candidates_batched(stencil_id, dtype, check_every)
                                                           : candidates(stencil_id);
        for (const lsr_tuning& cand : cands) {
            lsr_tuning t = base;
            t.tile_rows = cand.tile_rows;
            t.tb_depth = cand.tb_depth;
            t.waves = cand.waves;
            t.unroll = cand.unroll;
            double ms = 1e300;
            for (int rep = 0; rep < 2 && st == LSR_OK; ++rep) {   // the first run also warms up
                lsr_job id = 0;
                if (ctx->batched) {
                    // the engine reads the context's overrides at submission: the
                    // candidate's jobs run in its rounds with this setting
                    const auto t0 = std::chrono::steady_clock::now();
                    std::vector<lsr_job> ids;
                    {
                        std::lock_guard<std::mutex> lk(ctx->mu);
                        ctx->tuning = t;
                    }
                    for (int c = 0; c < copies && st == LSR_OK; ++c) {
                        lsr_grid gc = g;
                        gc.data = grid_bufs[c];
                        st = submit(ctx, &gc, stencil_id, reduce, &cond, sweeps, false, &id);
                        if (st == LSR_OK) ids.push_back(id);
                    }
                    {
                        std::lock_guard<std::mutex> lk(ctx->mu);
                        ctx->tuning = base;
                    }
                    for (lsr_job jid : ids) {   // every submitted job is collected
                        lsr_job_result r{};
                        const lsr_status s2 = lsr_result(ctx, jid, 1, &r);
                        if (st == LSR_OK) st = s2;
                    }
                    if (st != LSR_OK) break;
                    ms = std::min(ms, std::chrono::duration<double, std::milli>(
                                          std::chrono::steady_clock::now() - t0).count());
                    continue;
                } else {
                    std::unique_ptr<Job> j(new Job());
                    j->grid = g;
                    j->xgrid = g;
                    j->stencil = stencil_id;
                    j->cond = cond;
                    j->max_iter = sweeps;
                    st = submit_plain(ctx, std::move(j), &g, stencil_id, reduce, &cond, sweeps, t, &id);
                }
                if (st != LSR_OK) break;
                lsr_job_result r{};
                st = lsr_result(ctx, id, 1, &r);
                if (st == LSR_OK) ms = std::min(ms, r.device_ms);
            }
            if (st != LSR_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        if (st != LSR_OK) break;
        std::lock_guard<std::mutex> lk(ctx->mu);
        TuneEntry& en = ctx->tune_table[tune_key(stencil_id, dtype, g.bc, rows, cols, check_every)];
        en.tuning = best;
        en.us_per_sweep = best_ms * 1e3 / (double)sweeps;
        if (b == 0) best_first = best;
    }
    (void)hipStreamSynchronize(ctx->user_stream);
    release_all();
    if (st != LSR_OK) return st;
    if (best_out) *best_out = best_first;
    return LSR_OK;
}

lsr_status lsr_tune_export(lsr_ctx* ctx, char* buf, uint64_t cap, uint64_t* len_out) {
    if (!ctx) return fail(LSR_EINVAL, "ctx is NULL");
    std::string s = "{\"arch\": \"";
    s += arch_name(ctx->device);
    s += "\", \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        bool first = true;
        for (const auto& kv : ctx->tune_table) {
            const TuneKey& k = kv.first;
            const lsr_tuning& t = kv.second.tuning;
            char line[512];
            std::snprintf(line, sizeof line,
                          "%s\n  {\"stencil\": %d, \"dtype\": %d, \"bc\": %d, \"rows_log2\": %d, "
                          "\"cols_log2\": %d, \"check_every\": %d, \"tile_rows\": %d, \"tb_depth\": %d, "
                          "\"waves\": %d, \"unroll\": %d, \"us_per_sweep\": %.6g}",
                          first ? "" : ",", k.stencil, k.dtype, k.bc, k.rows_log2, k.cols_log2,
                          k.check_every, t.tile_rows, t.tb_depth, t.waves, t.unroll,
                          kv.second.us_per_sweep);
            s += line;
            first = false;
        }
    }
    s += "\n]}\n";
    if (len_out) *len_out = s.size() + 1;
    if (!buf || cap < s.size() + 1) {
        if (buf) return fail(LSR_EINVAL, "buffer too small: %llu bytes needed", (unsigned long long)(s.size() + 1));
        return LSR_OK;
    }
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return LSR_OK;
}

lsr_status lsr_tune_import(lsr_ctx* ctx, const char* json) {
    if (!ctx || !json) return fail(LSR_EINVAL, "ctx and json must not be NULL");
    const std::string s(json);
    // "arch": "<name>" must match this device
    const std::string want = std::string("\"arch\": \"") + arch_name(ctx->device) + "\"";
    if (s.find(want) == std::string::npos)
        return fail(LSR_EINVAL, "tuning table is for another architecture (expected %s)", want.c_str());
    auto field = [](const std::string& obj, const char* name, double* v) {
        const std::string key = std::string("\"") + name + "\":";
        const size_t p = obj.find(key);
        if (p == std::string::npos) return false;
        char* end = nullptr;
        *v = std::strtod(obj.c_str() + p + key.size(), &end);
        return end != obj.c_str() + p + key.size();
    };
    std::map<TuneKey, TuneEntry> parsed;
    size_t pos = s.find('[');
    if (pos == std::string::npos) return fail(LSR_EINVAL, "no entries list");
    while (true) {
        const size_t a = s.find('{', pos);
        if (a == std::string::npos) break;
        const size_t b = s.find('}', a);
        if (b == std::string::npos) return fail(LSR_EINVAL, "unterminated entry");
        const std::string obj = s.substr(a, b - a + 1);
        const char* names[] = {"stencil", "dtype", "bc", "rows_log2", "cols_log2", "check_every",
                               "tile_rows", "tb_depth", "waves", "unroll", "us_per_sweep"};
        double v[11];
        for (int i = 0; i < 11; ++i)
            if (!field(obj, names[i], &v[i])) return fail(LSR_EINVAL, "entry lacks \"%s\"", names[i]);
        for (int i = 0; i < 10; ++i)
            if (!(v[i] >= -1.0 && v[i] <= 2147483647.0) || v[i] != std::floor(v[i]))
                return fail(LSR_EINVAL, "entry field \"%s\" is not an integer in range", names[i]);
        TuneKey k{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5]};
        TuneEntry en{};
        en.tuning.tile_rows = (int)v[6];
        en.tuning.tb_depth = (int)v[7];
        en.tuning.waves = (int)v[8];
        en.tuning.unroll = (int)v[9];
        en.us_per_sweep = v[10];
        const lsr_tuning& t = en.tuning;
        const bool jac = k.stencil == LSR_ST_LAPLACE5 || k.stencil == LSR_ST_HELMHOLTZ5;
        const bool life = k.stencil == LSR_ST_LIFE;
        if (!jac && !life) return fail(LSR_EINVAL, "entry for stencil %d, which has no launch shapes", k.stencil);
        if (jac ? (k.dtype != LSR_F64 && k.dtype != LSR_F32) || k.bc != LSR_BC_RING
                : k.dtype != LSR_U8 || (k.bc != LSR_BC_TORUS && k.bc != LSR_BC_BOTTOM))
            return fail(LSR_EINVAL, "entry's dtype or boundary does not fit stencil %d", k.stencil);
        if (k.rows_log2 < 1 || k.rows_log2 > 40 || k.cols_log2 < 1 || k.cols_log2 > 40 || k.check_every < 1)
            return fail(LSR_EINVAL, "entry has an out-of-range key field");
        const bool depth_ok = t.tb_depth == 0 || t.tb_depth == 1 ||
                              (jac ? lsr::jacobi_tb_depth_ok(t.tb_depth) : lsr::life_tb_depth_ok(t.tb_depth));
        if (!depth_ok) return fail(LSR_EINVAL, "entry's tb_depth %d is not a compiled depth", t.tb_depth);
        if (t.tile_rows < 0 || t.tile_rows > 65536)
            return fail(LSR_EINVAL, "entry's tile_rows %d is outside [0, 65536]", t.tile_rows);
        if (jac ? !(t.waves == 0 || t.waves == 1 || t.waves == 2 || t.waves == 4) ||
                      !(t.unroll == 0 || t.unroll == 4 || t.unroll == 8 || t.unroll == 16)
                : t.waves != 0 || t.unroll != 0)
            return fail(LSR_EINVAL, "entry's waves %d / unroll %d are not supported", t.waves, t.unroll);
        if (!(en.us_per_sweep >= 0.0)) return fail(LSR_EINVAL, "entry's us_per_sweep is negative");
        parsed[k] = en;
        pos = b + 1;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const auto& kv : parsed) ctx->tune_table[kv.first] = kv.second;
    return LSR_OK;
}

}  // extern "C"
