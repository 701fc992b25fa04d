// Game of Life B3/S23 sweep (the elemental function of the paper's Fig. 1) with
// the live-cell count fused in.
//
// Fast path (cols and pitch multiples of 16 bytes, 16-byte aligned buffers):
// each lane owns 16 consecutive cells held as four 32-bit words, one byte per
// cell (SWAR). Per row it forms the byte-wise column sums V = up + mid + down
// (<= 3 per byte, no carries), shifts V by one byte left and right (the missing
// edge bytes come from the neighbouring lanes by cross-lane shuffles, or from a
// halo byte loaded by the wavefront's edge lanes), and adds the three to get the
// 3x3 total T (<= 9). With the neighbour count being T - centre, the rule is
//   alive' = (T == 3) || (T == 4 && alive)
// evaluated on all four bytes of a word at once with a zero-byte test. The new
// word's popcount is the cell count. Wavefronts stream down `tile_rows` rows as
// in the Jacobi kernel, so each row is read from HBM once per tile (2 bytes per
// cell update in all).
//
// Generic path (any shape/pitch): one thread per cell, nine byte loads.
//
// Boundaries: torus wraps rows and columns; bottom treats outside cells as dead.
#include "kernels.hpp"

namespace lsr {
namespace {

__device__ __forceinline__ uint32_t nz_bytes(uint32_t x) {
    // 0x01 in every byte that is non-zero, 0x00 elsewhere
    return ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) >> 7) & 0x01010101u;
}

__device__ __forceinline__ uint32_t zero_bytes_hi(uint32_t x) {
    // 0x80 in every byte equal to zero, for byte values below 0x80
    return ~(x + 0x7F7F7F7Fu) & 0x80808080u;
}

template <int NW, int U, bool NT = false>
__global__ __launch_bounds__(NW * 64) void life_swar_kernel(
    const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t rows, int64_t cols,
    int64_t pitch, int torus, JobState* __restrict__ st, unsigned long long* __restrict__ partials,
    LoopCtl ctl, int j, int strips, int tiles, int tile_rows) {
    __shared__ unsigned long long lds[NW];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;

    const int band = t / strips, strip = t - band * strips;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cw = (int64_t)strip * (NW * 1024) + (int64_t)wave * 1024;
    const int64_t c = cw + (int64_t)lane * 16;
    const bool active = c < cols;
    int nact = 0;
    if (cw < cols) nact = (int)min<int64_t>(64, (cols - cw) / 16);
    const int last = nact - 1;
    int64_t wcol = cw - 1, ecol = cw + (int64_t)nact * 16;
    bool has_w = (lane == 0) && nact > 0, has_e = (lane == last) && nact > 0;
    if (wcol < 0) { if (torus) wcol += cols; else has_w = false; }
    if (ecol >= cols) { if (torus) ecol -= cols; else has_e = false; }

    const int64_t r0 = (int64_t)band * tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, rows);

    auto load = [&](int64_t r, uint32_t (&w)[4], uint32_t& hw, uint32_t& he) {
        w[0] = w[1] = w[2] = w[3] = 0;
        hw = he = 0;
        if (r < 0 || r >= rows) {
            if (!torus) return;
            r = (r + rows) % rows;
        }
        const uint8_t* p = a + r * pitch;
        if (active) {
            const uint4 x = *reinterpret_cast<const uint4*>(p + c);
            w[0] = nz_bytes(x.x);
            w[1] = nz_bytes(x.y);
            w[2] = nz_bytes(x.z);
            w[3] = nz_bytes(x.w);
        }
        if (has_w) hw = p[wcol] != 0;
        if (has_e) he = p[ecol] != 0;
    };

    uint32_t up[4], mid[4], up_w, up_e, mid_w, mid_e;
    load(r0 - 1, up, up_w, up_e);
    load(r0, mid, mid_w, mid_e);
    unsigned long long cnt = 0;

    for (int64_t r = r0; r < r1; r += U) {
        uint32_t dn[U][4], dn_w[U], dn_e[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (r + k < r1) load(r + k + 1, dn[k], dn_w[k], dn_e[k]);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (r + k < r1) {
                uint32_t V[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) V[m] = up[m] + mid[m] + dn[k][m];
                const uint32_t vw_h = up_w + mid_w + dn_w[k];
                const uint32_t ve_h = up_e + mid_e + dn_e[k];
                uint32_t wv = __shfl_up(V[3], 1, 64) >> 24;
                uint32_t ev = __shfl_down(V[0], 1, 64) & 0xFFu;
                if (lane == 0) wv = vw_h;
                if (lane == last) ev = ve_h;
                uint32_t out[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint32_t prev = (m > 0) ? (V[m - 1] >> 24) : wv;
                    const uint32_t next = (m < 3) ? (V[m + 1] & 0xFFu) : ev;
                    const uint32_t T = ((V[m] << 8) | prev) + V[m] + ((V[m] >> 8) | (next << 24));
                    const uint32_t eq3 = zero_bytes_hi(T ^ 0x03030303u);
                    const uint32_t eq4 = zero_bytes_hi(T ^ 0x04040404u);
                    const uint32_t alive = eq3 | (eq4 & (mid[m] << 7));
                    out[m] = alive >> 7;
                    cnt += (unsigned)__popc(alive);
                }
                if (active) {
                    typedef uint32_t W4 __attribute__((ext_vector_type(4)));
                    W4 o;
                    o[0] = out[0];
                    o[1] = out[1];
                    o[2] = out[2];
                    o[3] = out[3];
                    W4* dst = reinterpret_cast<W4*>(b + (r + k) * pitch + c);
                    if (NT) __builtin_nontemporal_store(o, dst);
                    else *dst = o;
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) { up[m] = mid[m]; mid[m] = dn[k][m]; }
                up_w = mid_w; up_e = mid_e;
                mid_w = dn_w[k]; mid_e = dn_e[k];
            }
        }
    }
    if (check) {
        const unsigned long long v = block_reduce_u64<NW>(active ? cnt : 0ull, lds);
        if (threadIdx.x == 0) partials[t] = v;
    }
}

constexpr int kGenericBlocks = 2048;

__global__ __launch_bounds__(256) void life_generic_kernel(
    const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t rows, int64_t cols,
    int64_t pitch, int torus, JobState* __restrict__ st, unsigned long long* __restrict__ partials,
    LoopCtl ctl, int j) {
    __shared__ unsigned long long lds[4];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    const bool check = is_check_sweep(n1, ctl);
    unsigned long long cnt = 0;
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / cols, cc = i - r * cols;
        int count = 0;
        for (int di = -1; di <= 1; ++di) {
            for (int dj = -1; dj <= 1; ++dj) {
                if (di == 0 && dj == 0) continue;
                int64_t rr = r + di, c2 = cc + dj;
                if (torus) {
                    rr = (rr + rows) % rows;
                    c2 = (c2 + cols) % cols;
                } else if (rr < 0 || c2 < 0 || rr >= rows || c2 >= cols) {
                    continue;
                }
                count += a[rr * pitch + c2] != 0;
            }
        }
        const int alive = a[r * pitch + cc] != 0;
        const uint8_t v = (count == 3 || (alive && count == 2)) ? 1 : 0;
        b[r * pitch + cc] = v;
        cnt += v;
    }
    if (check) {
        const unsigned long long v = block_reduce_u64<4>(cnt, lds);
        if (threadIdx.x == 0) partials[blockIdx.x] = v;
    }
}

constexpr int kWaves = 4;
constexpr int kUnroll = 4;

}  // namespace

SweepGeom life_geom(const LifeArgs& a, int tile_rows) {
    SweepGeom g;
    const bool al = ((reinterpret_cast<uintptr_t>(a.a) | reinterpret_cast<uintptr_t>(a.b)) & 15) == 0;
    if (a.cols % 16 == 0 && a.pitch % 16 == 0 && al) {
        g.vec = 16;
        g.waves = kWaves;
        g.tile_rows = tile_rows > 0 ? tile_rows : 64;
        const int64_t span = (int64_t)kWaves * 1024;
        g.strips = (int)((a.cols + span - 1) / span);
        g.bands = (int)((a.rows + g.tile_rows - 1) / g.tile_rows);
        g.tiles = g.strips * g.bands;
        g.blocks = pad_to_xcds(g.tiles);
    } else {
        g.vec = 0;
        g.waves = 4;
        const int64_t need = (a.rows * a.cols + 255) / 256;
        g.tiles = g.blocks = (int)(need < kGenericBlocks ? need : kGenericBlocks);
        g.strips = g.bands = 0;
        g.tile_rows = 0;
    }
    return g;
}

hipError_t launch_life(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                       const LoopCtl& c, int j, hipStream_t s) {
    auto* parts = static_cast<unsigned long long*>(partials);
    if (g.vec == 16) {
        hipLaunchKernelGGL((life_swar_kernel<kWaves, kUnroll>), dim3(g.blocks), dim3(kWaves * 64), 0,
                           s, a.a, a.b, a.rows, a.cols, a.pitch, a.torus, st, parts, c, j, g.strips,
                           g.tiles, g.tile_rows);
    } else {
        hipLaunchKernelGGL(life_generic_kernel, dim3(g.blocks), dim3(256), 0, s, a.a, a.b, a.rows,
                           a.cols, a.pitch, a.torus, st, parts, c, j);
    }
    return hipGetLastError();
}

}  // namespace lsr
