// Temporally blocked Game of Life: one launch advances the grid by K
// generations (the loop body of Sect. 3.1 applied K times between two reads of
// the grid), with the live-cell count of every checked generation fused in.
//
// Each wavefront owns a window of 992 columns (lanes 1..62, 16 cells per lane
// held as four 32-bit words, one byte per cell) and a band of rows. It loads
// 1024 columns: lanes 0 and 63 are halo lanes whose cells are computed but never
// stored or counted. A lane's edge bytes take the neighbouring lane's column sum
// by a DPP lane shift; at lanes 0 and 63 that shift brings in zero, so their
// outer cells go wrong, but the error moves inward by one cell per generation
// and does not leave the 16 cells of a halo lane for K <= 16.
// Rows stream through a register pipeline of K levels: level l holds its input
// rows (the output of level l - 1) i - l - 1 and i - l, and computes row i - l of
// generation n + l from them and the row level l - 1 produced in the same step.
// Neighbouring bands overlap by K rows, so every stored cell of generation n + K
// is computed from exactly the cells of generation n a plain sweep chain would
// read. A torus wraps rows and columns (any size, also below one window);
// outside cells of a dead border are zero at every level.
//
// Requirements (life_tb_ok): 16-byte aligned rows holding a multiple of 16
// cells, no padding. The cells hold 0 or 1 (the job's initial count pass
// normalises them).
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "kernels.hpp"

namespace lsr {
namespace {

constexpr int kWinLanes = 62;               // lanes of a window that are stored
constexpr int kWinCols = kWinLanes * 16;    // 992 columns per wavefront

constexpr int kDppShr1 = 0x138;   // wave_shr:1, lane l receives lane l-1 (lane 0 gets 0)
constexpr int kDppShl1 = 0x130;   // wave_shl:1, lane l receives lane l+1 (lane 63 gets 0)

template <int CTRL>
__device__ __forceinline__ uint32_t lane_shift_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ uint32_t zero_bytes_hi(uint32_t x) {
    // 0x80 in every byte equal to zero, for byte values below 0x80
    return ~(x + 0x7F7F7F7Fu) & 0x80808080u;
}

// One generation of 16 cells from the byte-wise column sums V of the lane's
// rows i-1, i, i+1 and its centre row c (bytes 0/1). With T the 3x3 total,
// B3/S23 is (T - c | c) == 3.
__device__ __forceinline__ void life_rule16(const uint32_t (&V)[4], const uint32_t (&c)[4],
                                            uint32_t (&out)[4]) {
    const uint32_t wv = lane_shift_u32<kDppShr1>(V[3]) >> 24;
    const uint32_t ev = lane_shift_u32<kDppShl1>(V[0]) & 0xFFu;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint32_t prev = (m > 0) ? (V[m - 1] >> 24) : wv;
        const uint32_t next = (m < 3) ? (V[m + 1] & 0xFFu) : ev;
        const uint32_t T = ((V[m] << 8) | prev) + V[m] + ((V[m] >> 8) | (next << 24));
        out[m] = zero_bytes_hi(((T - c[m]) | c[m]) ^ 0x03030303u) >> 7;
    }
}

// NW wavefronts per workgroup, each its own window (wave tile wt = t * NW + w,
// strip-major within a band); K generations; U = 3 rows per load group (one
// rotation of the row slots; two groups alternate, so the next group's loads are
// in flight while the current one is computed).
// check_mask bit l-1: generation n1 + l - 1 is checked; its count over the
// workgroup's windows goes to partials[(l - 1) * tiles + t].
template <int NW, int K, int U, bool TORUS>
__global__ __launch_bounds__(NW * 64) void life_tb_kernel(
    const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t rows, int64_t cols, int64_t pitch,
    JobState* __restrict__ st, unsigned long long* __restrict__ partials, LoopCtl ctl, int j,
    int strips, int wave_tiles, int tiles, int tile_rows) {
    static_assert(K >= 2 && K <= 16, "halo lanes cover at most 16 generations");
    __shared__ unsigned long long lds[K * NW];
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    // generations n1 .. n1 + K - 1 (those past the cap are computed and never kept:
    // the driver replays up to a stop inside the launch)
    const int64_t n1 = __hip_atomic_load(&st->n_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + j + 1;
    if (n1 > ctl.max_iter) return;
    uint32_t mask = 0;
#pragma unroll
    for (int lev = 1; lev <= K; ++lev) {
        const int64_t n = n1 + lev - 1;
        if (n <= ctl.max_iter && is_check_sweep(n, ctl)) mask |= 1u << (lev - 1);
    }
    const int t = xcd_logical_tile(blockIdx.x, gridDim.x);
    if (t >= tiles) return;
    // the wavefront index is uniform across a wavefront: readfirstlane tells the
    // compiler, so band and row bounds live in scalar registers and the per-row
    // tests below are scalar branches
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wt = t * NW + wave;
    uint32_t cnt[K];
#pragma unroll
    for (int l = 0; l < K; ++l) cnt[l] = 0;

    if (wt < wave_tiles) {
        const int band = wt / strips, strip = wt - band * strips;
        const int64_t col_raw = (int64_t)strip * kWinCols - 16 + (int64_t)lane * 16;
        const bool in_cols = col_raw >= 0 && col_raw < cols;
        int64_t col = col_raw;
        if (TORUS && !in_cols) {
            col %= cols;
            if (col < 0) col += cols;
        }
        const bool loads = TORUS || in_cols;
        const uint32_t own = (lane >= 1 && lane <= kWinLanes && col_raw < cols) ? 0xFFFFFFFFu : 0u;
        const uint32_t live = loads ? 0xFFFFFFFFu : 0u;   // dead columns of a dead border
        const int64_t r0 = (int64_t)band * tile_rows;
        const int64_t r1 = min(r0 + (int64_t)tile_rows, rows);
        const int64_t i_beg = r0 - K, i_end = r1 + K;

        // rows i0 .. i0 + U - 1 of generation n (those below i_end), zero outside a dead border
        auto load_group = [&](int64_t i0, uint32_t (&w)[U][4]) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                w[k][0] = w[k][1] = w[k][2] = w[k][3] = 0;
                int64_t r = i0 + k;
                if (r >= i_end) continue;
                if (r < 0 || r >= rows) {
                    if (!TORUS) continue;
                    r %= rows;
                    if (r < 0) r += rows;
                }
                if (!loads) continue;
                const uint4 x = *reinterpret_cast<const uint4*>(a + r * pitch + col);
                w[k][0] = x.x;
                w[k][1] = x.y;
                w[k][2] = x.z;
                w[k][3] = x.w;
            }
        };

        // R[l][s]: the last three rows of level l (l = 0: the loaded rows of generation
        // n), in slots by row phase: at step i (phase P = (i - i_beg) mod 3) level l
        // writes its row into slot P and level l + 1 reads rows i-l-2, i-l-1, i-l
        // from slots P+1, P+2, P (mod 3). Steps go in groups of three, so slot
        // numbers are compile-time constants and rows never move between registers.
        uint32_t R[K][3][4];
#pragma unroll
        for (int l = 0; l < K; ++l)
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int m = 0; m < 4; ++m) R[l][q][m] = 0;

        // the K levels of step i (input row i of generation n), then the store of row i - K
        auto step = [&](auto phase, int64_t i, const uint32_t (&row_in)[4]) {
            constexpr int P = decltype(phase)::value, PU = (P + 1) % 3, PM = (P + 2) % 3;
#pragma unroll
            for (int m = 0; m < 4; ++m) R[0][P][m] = row_in[m];
            uint32_t out[4];
#pragma unroll
            for (int l = 1; l <= K; ++l) {
                const int64_t row = i - l;   // row of generation n + l computed here
                const uint32_t(&src)[3][4] = R[l - 1];
                uint32_t V[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) V[m] = src[PU][m] + src[PM][m] + src[P][m];
                life_rule16(V, src[PM], out);
                if (!TORUS) {
                    const uint32_t lv = (row >= 0 && row < rows) ? live : 0u;
#pragma unroll
                    for (int m = 0; m < 4; ++m) out[m] &= lv;
                }
                if (((mask >> (l - 1)) & 1u) && row >= r0 && row < r1)
                    cnt[l - 1] += (uint32_t)(__popc(out[0]) + __popc(out[1]) + __popc(out[2]) +
                                             __popc(out[3])) & own;
                if (l < K) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) R[l][P][m] = out[m];
                }
            }
            const int64_t row = i - K;
            if (row >= r0 && row < r1 && own) {
                typedef uint32_t W4 __attribute__((ext_vector_type(4)));
                W4 o;
                o[0] = out[0];
                o[1] = out[1];
                o[2] = out[2];
                o[3] = out[3];
                __builtin_nontemporal_store(o, reinterpret_cast<W4*>(b + row * pitch + col_raw));
            }
        };
        static_assert(U == 3, "a load group is one rotation of the row slots");
        auto process_group = [&](int64_t i0, const uint32_t (&w)[U][4]) {
            step(std::integral_constant<int, 0>{}, i0, w[0]);
            if (i0 + 1 >= i_end) return;
            step(std::integral_constant<int, 1>{}, i0 + 1, w[1]);
            if (i0 + 2 >= i_end) return;
            step(std::integral_constant<int, 2>{}, i0 + 2, w[2]);
        };

        uint32_t ga[U][4], gb[U][4];
        load_group(i_beg, ga);
        for (int64_t i0 = i_beg; i0 < i_end; i0 += 2 * U) {
            load_group(i0 + U, gb);
            process_group(i0, ga);
            if (i0 + U >= i_end) break;
            load_group(i0 + 2 * U, ga);
            process_group(i0 + U, gb);
        }
    }
    if (mask == 0) return;
#pragma unroll
    for (int l = 0; l < K; ++l) {
        if ((mask >> l) & 1u) {
            const unsigned long long v = wave_sum_u64(cnt[l]);
            if (lane == 0) lds[l * NW + wave] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < K && ((mask >> threadIdx.x) & 1u)) {
        unsigned long long s = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += lds[threadIdx.x * NW + w];
        partials[(size_t)threadIdx.x * (size_t)tiles + t] = s;
    }
}

constexpr int kWaves = 4;
constexpr int kUnroll = 3;
constexpr int kDepths[] = {2, 3, 4, 5, 6, 8};
constexpr int kDefaultDepth = 8;   // 16384^2 torus: 2: 3.8, 4: 7.2, 6: 8.4, 8: 8.5 TLUP/s

constexpr int64_t kMaxAutoRows = 256;

// Workgroups of the depth-K kernel the whole device holds at once (occupancy
// times compute units), measured once per depth and boundary on the current
// device (the library's devices are all of one kind).
template <int K, bool TORUS>
int64_t resident_k() {
    static std::atomic<int64_t> cached{0};
    if (cached.load() > 0) return cached.load();
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, life_tb_kernel<kWaves, K, kUnroll, TORUS>,
                                                     kWaves * 64, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    cached.store((int64_t)per_cu * cus);
    return cached.load();
}

int64_t resident_workgroups(int depth, bool torus) {
    switch (depth) {
        case 2: return torus ? resident_k<2, true>() : resident_k<2, false>();
        case 3: return torus ? resident_k<3, true>() : resident_k<3, false>();
        case 4: return torus ? resident_k<4, true>() : resident_k<4, false>();
        case 5: return torus ? resident_k<5, true>() : resident_k<5, false>();
        case 6: return torus ? resident_k<6, true>() : resident_k<6, false>();
        case 8: return torus ? resident_k<8, true>() : resident_k<8, false>();
    }
    return 1024;
}

template <int K>
hipError_t launch_k(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                    const LoopCtl& c, int j, hipStream_t s) {
    auto* p = static_cast<unsigned long long*>(partials);
    if (a.torus)
        hipLaunchKernelGGL((life_tb_kernel<kWaves, K, kUnroll, true>), dim3(g.blocks), dim3(kWaves * 64),
                           0, s, a.a, a.b, a.rows, a.cols, a.pitch, st, p, c, j, g.strips,
                           g.strips * g.bands, g.tiles, g.tile_rows);
    else
        hipLaunchKernelGGL((life_tb_kernel<kWaves, K, kUnroll, false>), dim3(g.blocks), dim3(kWaves * 64),
                           0, s, a.a, a.b, a.rows, a.cols, a.pitch, st, p, c, j, g.strips,
                           g.strips * g.bands, g.tiles, g.tile_rows);
    return hipGetLastError();
}

}  // namespace

bool life_tb_ok(const LifeArgs& a) {
    const bool al = ((reinterpret_cast<uintptr_t>(a.a) | reinterpret_cast<uintptr_t>(a.b)) & 15) == 0;
    return al && a.pitch % 16 == 0 && a.cols % 16 == 0 && !a.padded;
}

bool life_tb_depth_ok(int depth) {
    for (int k : kDepths)
        if (k == depth) return true;
    return false;
}

int life_tb_choose(const LifeArgs& a, int requested) {
    if (requested == 1 || !life_tb_ok(a)) return 1;
    if (requested > 1) {
        for (int k : kDepths)
            if (k == requested) return k;
        return 1;
    }
    return kDefaultDepth;
}

SweepGeom life_tb_geom(const LifeArgs& a, int depth, int tile_rows) {
    SweepGeom g;
    g.vec = 16;
    g.waves = kWaves;
    g.unroll = kUnroll;
    g.tb = depth;
    g.mc = 1;   // every generation of a launch may be checked
    g.strips = (int)((a.cols + kWinCols - 1) / kWinCols);
    if (tile_rows > 0) {
        g.tile_rows = tile_rows;
    } else {
        // The launch is ALU-bound and its workgroups take equal time, so the
        // last partial wave of workgroups costs as much as a full one. Take the
        // most bands whose workgroups all fit on the device at once (one round;
        // more rounds only when a band would exceed kMaxAutoRows rows), and no
        // band below 2K rows, where the K-row overlaps would double the work.
        const int64_t slots = resident_workgroups(depth, a.torus != 0);
        int64_t t = 0;
        for (int64_t m = 1;; ++m) {
            const int64_t bands = std::max<int64_t>(1, m * slots * kWaves / g.strips);
            t = (a.rows + bands - 1) / bands;
            if (t <= kMaxAutoRows) break;
        }
        g.tile_rows = (int)std::max<int64_t>(t, 2 * depth);
    }
    g.bands = (int)((a.rows + g.tile_rows - 1) / g.tile_rows);
    g.tiles = (g.strips * g.bands + kWaves - 1) / kWaves;
    g.blocks = pad_to_xcds(g.tiles);
    return g;
}

hipError_t launch_life_tb(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                          const LoopCtl& c, int j, hipStream_t s) {
    if (!life_tb_ok(a) || g.waves != kWaves) return hipErrorInvalidValue;
    switch (g.tb) {
        case 2: return launch_k<2>(a, g, st, partials, c, j, s);
        case 3: return launch_k<3>(a, g, st, partials, c, j, s);
        case 4: return launch_k<4>(a, g, st, partials, c, j, s);
        case 5: return launch_k<5>(a, g, st, partials, c, j, s);
        case 6: return launch_k<6>(a, g, st, partials, c, j, s);
        case 8: return launch_k<8>(a, g, st, partials, c, j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lsr
