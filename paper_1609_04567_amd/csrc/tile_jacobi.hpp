// Tile body of the 5-point Jacobi sweep with the fused residual reduce (Laplace
// and the Helmholtz solver of Sect. 4.1), FP64 or FP32 storage. Shared by the
// single-job kernel (jacobi.hip) and the batched kernel (batch.hip).
//
// One workgroup = NW wavefronts side by side; each wavefront owns 64*VEC
// consecutive columns and streams down `tile_rows` rows of the grid, keeping
// the rows above/at/below the current one in registers (each row of the iterate
// is read from HBM once per tile, plus the two halo rows). Horizontal
// neighbours come from the adjacent lanes through cross-lane shuffles; only the
// first and last lane of a wavefront load one extra halo element per row. Loads
// of U rows are issued before any of them is used. The update never runs in
// place (a stencil cannot, Sect. 3.1): it reads `a` and writes `b`.
//
// Expression order is fixed (the build uses -ffp-contract=off):
//   Laplace   b = 0.25 * ((N + S) + (W + E))
//   Helmholtz b = (((N + S) + (W + E)) + g) * rd
// FP32 Helmholtz is compensated (still only FP32 operations): late in a slow
// solve g is ~1/n of the neighbour sum s, so a plain fl(s + g) quantises each
// sweep's increment to ulp(s) with a bias that is coherent over the smooth field,
// and fl(rd) misplaces the alpha h^2 part of 1/(4 + alpha h^2) by up to 10 %;
// both errors then accumulate over thousands of sweeps. So t = fl(s + g) keeps
// its exact rounding error e (TwoSum), rd is applied as 0.25 - rd_lo, and
//   x = 0.25 t + (0.25 e - rd_lo t)
// is rounded to FP32 stochastically: with p = |x - fl(x)| / ulp, the stored value
// moves one ulp from fl(x) towards x with probability p, drawn from a 32-bit hash
// of (row, column, sweep). Round-to-nearest errors of a smooth field are
// correlated between neighbours and feed the slowly decaying smooth mode;
// unbiased, decorrelated rounding does not (max error vs the FP64 solution at
// 1025^2 x 5000 sweeps: 3.3e-6 with round-to-nearest, 7.7e-7 stochastic). The
// draw depends only on the cell and the sweep, so results are reproducible.
// On a check sweep each lane accumulates delta = b - a in FP64 over its cells
// (max |delta|, sum delta^2 or sum |delta|); the workgroup folds the lanes in a
// fixed order and writes one partial per tile.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace lsr {

// NTL = non-temporal load (for data read exactly once per sweep, such as g).
template <typename T, int VEC, bool NTL = false>
__device__ __forceinline__ void load_row(const T* __restrict__ p, int64_t c, int64_t cols,
                                         T (&v)[VEC]) {
    if (VEC > 1 && c + VEC <= cols) {
        typedef T V __attribute__((ext_vector_type(VEC)));
        V x = NTL ? __builtin_nontemporal_load(reinterpret_cast<const V*>(p + c))
                  : *reinterpret_cast<const V*>(p + c);
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = x[e];
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = (c + e < cols) ? p[c + e] : T(0);
    }
}

// NT = non-temporal: the next iterate is not read again before the whole grid has
// streamed through, so keeping it out of L2/MALL leaves room for the halo rows.
template <typename T, int VEC, bool NT>
__device__ __forceinline__ void store_row(T* __restrict__ p, int64_t c, int64_t cols,
                                          const T (&v)[VEC]) {
    if (VEC > 1 && c + VEC <= cols) {
        typedef T V __attribute__((ext_vector_type(VEC)));
        V x;
#pragma unroll
        for (int e = 0; e < VEC; ++e) x[e] = v[e];
        if (NT) __builtin_nontemporal_store(x, reinterpret_cast<V*>(p + c));
        else *reinterpret_cast<V*>(p + c) = x;
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (c + e < cols) p[c + e] = v[e];
    }
}

// 32-bit integer hash ("lowbias32", C. Wellons, 2018: xorshift-multiply
// rounds with constants found by search for low bias).
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// fl(p + c) rounded stochastically by its exact remainder: one ulp towards
// p + c with probability |remainder| / ulp, resolved to 1/256 ulp by the byte
// `bits8` (u = (bits8 + 1/2) / 256). Needs |c| <= |p|, where Fast2Sum's
// remainder c - (fl(p + c) - p) is exact (Dekker, 1971).
__device__ __forceinline__ float add_round_stochastic(float p, float c, uint32_t bits8) {
    const float hi = p + c;
    const float rem = c - (hi - p);
    const float ulp = __uint_as_float(__float_as_uint(hi) & 0x7f800000u) * 1.1920928955078125e-7f;
    const float u = ((float)bits8 + 0.5f) * 3.90625e-3f;
    return (fabsf(rem) > u * ulp) ? hi + copysignf(ulp, rem) : hi;
}

// The 5-point update of one cell (row, col) at sweep number `sweep`; the only
// place the expression is written, shared by the plain and the blocked tiles.
template <typename T, bool HELM>
__device__ __forceinline__ T jacobi_update(T N, T S, T W, T E, T gv, T rd, T rd_lo, int64_t row,
                                           int64_t col, uint32_t sweep) {
    if constexpr (HELM && sizeof(T) == 8) {
        return (((N + S) + (W + E)) + gv) * rd;
    } else if constexpr (HELM) {
        const T sn = (N + S) + (W + E);
        const T tt = sn + gv, bb = tt - sn;
        const T te = (sn - (tt - bb)) + (gv - bb);  // exact: sn + gv = tt + te
        // one hash per (row, group of four columns, sweep), one byte of it per
        // column: a lane's four cells share the hash (the integer multiplies are
        // quarter-rate instructions)
        const uint32_t key = (uint32_t)row * 0x9e3779b1u ^ (uint32_t)(col >> 2) * 0x85ebca77u ^
                             sweep * 0xc2b2ae3du;
        const uint32_t bits8 = (hash32(key) >> (8 * (uint32_t)(col & 3))) & 0xFFu;
        // |rd_lo| <= 1/8 (checked at submission) keeps |0.25 te - rd_lo tt| below
        // |0.25 tt|, as the rounding add requires
        return add_round_stochastic(T(0.25) * tt, T(0.25) * te - rd_lo * tt, bits8);
    } else {
        return T(0.25) * ((N + S) + (W + E));
    }
}

__device__ __forceinline__ double jacobi_accum(int red, double acc, double d) {
    if (red == RED_MAX_ABS) return max_nan(acc, fabs(d));
    if (red == RED_L2) return acc + d * d;
    return acc + fabs(d);
}

// The right-hand side of the -i form (Sect. 3.1: the elemental function also sees
// the cell's index): g(i, j) = c2 * (c1 * (p[i] * q[j])) in FP64, then stored in T,
// evaluated per cell from its indices instead of read from an env array.
struct SepSource {
    const double* p;   // rows values
    const double* q;   // cols values
    double c1, c2;
};
template <typename T>
__device__ __forceinline__ T sep_value(const SepSource& s, double pi, double qj) {
    return (T)(s.c2 * (s.c1 * (pi * qj)));
}

// Tile t of a grid split into `strips` column strips and bands of `tile_rows`
// rows (band-major). The workgroup must have NW*64 threads; lds holds NW doubles.
// WT (wavefront tile): the calling wavefront alone owns tile t (NW must be 1);
// other wavefronts of the workgroup may run other tiles, so the reduce stays
// inside the wavefront and its lane 0 writes the partial.
// SEP: the -i form (HELM must be set): g comes from `sep`, not from `g`.
template <typename T, bool HELM, int VEC, int NW, int U, bool NT, bool NTG, bool NTU = false,
          bool WT = false, bool SEP = false>
__device__ __forceinline__ void jacobi5_tile(const T* __restrict__ a, T* __restrict__ b,
                                             const T* __restrict__ g, int64_t rows, int64_t cols,
                                             int64_t pitch, T rd, T rd_lo, uint32_t sweep,
                                             bool check, int red, int t,
                                             int strips, int tile_rows,
                                             double* __restrict__ partials, double* lds,
                                             SepSource sep = SepSource{}) {
    static_assert(!WT || NW == 1, "a wavefront tile has one wavefront");
    const int band = t / strips, strip = t - band * strips;
    // (the wavefront index stays a vector value here: made scalar, the edge
    // handling turns into branches and the 8192^2 FP64 sweep lost 10 %)
    const int lane = threadIdx.x & 63, wave = WT ? 0 : threadIdx.x >> 6;
    const int64_t cw = (int64_t)strip * (NW * 64 * VEC) + (int64_t)wave * (64 * VEC);
    const int64_t c = cw + (int64_t)lane * VEC;
    const int64_t r0 = 1 + (int64_t)band * tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, rows - 1);
    const int64_t ce = cw + 64 * VEC;           // first column after this wavefront
    // Halo elements exist only for wavefronts that own columns of the grid
    // (cw < cols); a wavefront past the last column loads nothing at all.
    const bool has_w = (lane == 0) && cw >= 1 && cw < cols;
    const bool has_e = (lane == 63) && ce < cols;

    T up[VEC], mid[VEC];
    T mid_w = T(0), mid_e = T(0);
    double qv[SEP ? VEC : 1];
    if constexpr (SEP) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) qv[e] = (c + e < cols) ? sep.q[c + e] : 0.0;
    }
    load_row<T, VEC>(a + (r0 - 1) * pitch, c, cols, up);
    load_row<T, VEC>(a + r0 * pitch, c, cols, mid);
    if (has_w) mid_w = a[r0 * pitch + cw - 1];
    if (has_e) mid_e = a[r0 * pitch + ce];

    double acc = 0.0;
    for (int64_t r = r0; r < r1; r += U) {
        T dn[U][VEC], dn_w[U], dn_e[U], gr[U][VEC];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (r + k < r1) {
                const T* prow = a + (r + k + 1) * pitch;
                load_row<T, VEC, NTU>(prow, c, cols, dn[k]);
                dn_w[k] = has_w ? prow[cw - 1] : T(0);
                dn_e[k] = has_e ? prow[ce] : T(0);
                if (HELM && !SEP) load_row<T, VEC, NTG>(g + (r + k) * pitch, c, cols, gr[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (r + k < r1) {
                T wl = __shfl_up(mid[VEC - 1], 1, 64);
                T er = __shfl_down(mid[0], 1, 64);
                if (lane == 0) wl = mid_w;
                if (lane == 63) er = mid_e;
                T out[VEC];
                const double prow = SEP ? sep.p[r + k] : 0.0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T W = (e > 0) ? mid[e - 1] : wl;
                    const T E = (e < VEC - 1) ? mid[e + 1] : er;
                    const T N = up[e], S = dn[k][e];
                    const T gv = SEP ? sep_value<T>(sep, prow, qv[e]) : HELM ? gr[k][e] : T(0);
                    const T nv = jacobi_update<T, HELM>(N, S, W, E, gv, rd, rd_lo, r + k, c + e,
                                                        sweep);
                    const int64_t col = c + e;
                    const bool inner = col >= 1 && col <= cols - 2;
                    out[e] = inner ? nv : mid[e];
                    if (check && inner) acc = jacobi_accum(red, acc, (double)nv - (double)mid[e]);
                }
                store_row<T, VEC, NT>(b + (r + k) * pitch, c, cols, out);
#pragma unroll
                for (int e = 0; e < VEC; ++e) { up[e] = mid[e]; mid[e] = dn[k][e]; }
                mid_w = dn_w[k];
                mid_e = dn_e[k];
            }
        }
    }
    if (check) {
        if (WT) {
            const double v = red == RED_MAX_ABS ? wave_max(acc) : wave_sum(acc);
            if (lane == 0) partials[t] = v;
        } else {
            const double v = block_reduce<NW>(acc, red == RED_MAX_ABS, lds);
            if (threadIdx.x == 0) partials[t] = v;
        }
    }
}


// ---------------------------------------------------------------------------
// Temporally blocked tile: K sweeps per launch (read u and g once, write the
// K-th iterate once: 24/K bytes per cell update in FP64).
//
// Each wavefront loads a window of 64*VEC columns starting at a 16-byte aligned
// column and writes only part of it: values next to a window edge that lies
// inside the grid are wrong after each level, and the wrong region grows by one
// column per level, so window w (starting at column w*OW, OW = 64*VEC - 2K
// rounded down to a multiple of VEC) writes columns [w*OW + K, w*OW + K + OW);
// consecutive windows overlap by 2K columns and tile the row exactly. A window
// that contains the boundary ring (column 0 or cols-1) writes up to it: ring
// cells keep their value at every level, so nothing spreads across them.
// Rows stream downwards: after level-0 row i is loaded, level j (1..K) computes
// its row i-j from the last three rows of level j-1, each level keeping its own
// three rows in registers. The g rows go through a per-wavefront ring of K rows
// in LDS (level j reads g row i-j), which keeps register moves out of the row
// loop. Level K rows in [r0, r1) are stored (and reduced on a check sweep,
// against level K-1, the previous sweep). Each level evaluates jacobi_update
// with that level's sweep number, so the K-th iterate is bit-identical to K
// single sweeps. Rows and columns outside the grid are zero-filled and never
// loaded; like the windows' inner edges they cannot reach an interior cell
// through the fixed ring.
//
// Horizontal neighbours move between lanes with DPP wave shifts (gfx9
// wave_shr:1 / wave_shl:1, a VALU move with no LDS round trip); lane 0 gets 0
// from the west and lane 63 gets 0 from the east, which only feeds columns that
// are never stored. Per-lane selects for the ring columns are only evaluated in
// the two windows that hold column 0 or cols-1; elsewhere a row is either
// updated or carried unchanged as a whole.
template <int VEC, int K>
constexpr int tb_out_width() { return (64 * VEC - 2 * K) / VEC * VEC; }

constexpr int kDppWaveShr1 = 0x138;  // lane l receives lane l-1
constexpr int kDppWaveShl1 = 0x130;  // lane l receives lane l+1

template <int CTRL>
__device__ __forceinline__ float lane_shift(float x) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double lane_shift(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// LDS the tile needs for the g ring, in elements of T.
template <int VEC, int NW, int K>
constexpr int tb_gring_elems() { return NW * K * 64 * VEC; }

// WT as for jacobi5_tile: the calling wavefront alone owns tile t (NW = 1); its
// g ring is still the slot of its own wavefront in the workgroup (gring holds
// one ring per wavefront of the workgroup).
// check_mask: bit j-1 set when level j's sweep (sweep0 + j - 1) is a check sweep.
// Without MC only bit K-1 may be set and the tile's partial goes to partials[t];
// with MC (several checks per launch) level j's partial goes to
// partials[(j-1) * tiles + t], its delta taken against level j-1.
// SEP: the -i form (HELM must be set): level j computes g of its row from `sep`
// (no g rows are loaded and gring is unused).
// VERT: the workgroup's NW wavefronts take NW consecutive bands of one window
// (tile t = band group t / strips, window t % strips) instead of NW windows of
// one band. Odd wavefronts stream their band upwards (from row r1 + K - 1 down to
// r0 - K in index), so each pair of neighbouring bands reaches the 2K rows both
// read at about the same time and the second read is served by the cache instead
// of HBM. The N + S sum is commutative, so a band streamed upwards computes the
// same values bit for bit; only the order of a lane's delta sum changes.
// GA > 0: the g rows of the next GA levels are read from the ring ahead of their
// use, so a level does not wait for its own LDS read.
// Band groups per dispatch chunk of a vertical-tile launch (8192^2 FP64 Helmholtz,
// depth 10: 1, 4, 8, 16, 32 -> 1387, 1381, 1401, 1393, 1365 GLUP/s; fetched bytes
// -2 % at 8, +10 % at 32, where a chunk's windows no longer run together).
constexpr int kTbChunk = 8;

// RED >= 0: the reduce op is that constant (red is ignored), so the delta sums
// carry no selects between the reduce kinds.
template <typename T, bool HELM, int VEC, int NW, int K, bool NT, bool NTG, bool WT = false,
          bool MC = false, bool SEP = false, bool VERT = false, int GA = 0, int RED = -1>
__device__ __forceinline__ void jacobi5_tb_tile(const T* __restrict__ a, T* __restrict__ b,
                                                const T* __restrict__ g, int64_t rows,
                                                int64_t cols, int64_t pitch, T rd, T rd_lo,
                                                uint32_t sweep0, uint32_t check_mask, int red_arg,
                                                int t, int strips, int tiles, int tile_rows,
                                                double* __restrict__ partials, double* lds,
                                                T* gring, SepSource sep = SepSource{}) {
    constexpr bool GRING = HELM && !SEP;   // g rows stream through the LDS ring
    const int red = RED >= 0 ? RED : red_arg;
    static_assert(!WT || NW == 1, "a wavefront tile has one wavefront");
    typedef T V __attribute__((ext_vector_type(VEC)));
    constexpr int OW = tb_out_width<VEC, K>();
    static_assert(!VERT || !WT, "vertical band groups are workgroup tiles");
    const bool check = (check_mask >> (K - 1)) & 1u;
    int tband, strip;
    if (VERT) {
        // band groups in chunks of kTbChunk: a chunk's tiles go window by window,
        // its band groups innermost, so the groups above and below a seam start
        // together and read the seam's 2K rows from L2 the second time
        const int bands = tiles / strips, span = strips * kTbChunk;
        const int ch = t / span, r = t - ch * span;
        const int hb = min(kTbChunk, bands - ch * kTbChunk);
        strip = r / hb;
        tband = ch * kTbChunk + (r - strip * hb);
    } else {
        tband = t / strips;
        strip = t - tband * strips;
    }
    const int lane = threadIdx.x & 63;
    // the wavefront's slot in the workgroup (a wavefront tile of the batched kernel
    // is NW = 1 in a workgroup of several); readfirstlane keeps it scalar
    const int hw_wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wave = WT ? 0 : hw_wave;
    const int band = VERT ? tband * NW + wave : tband;
    const bool up = VERT && (wave & 1);
    const int64_t cw = (VERT ? (int64_t)strip : (int64_t)strip * NW + wave) * OW;   // window start (aligned)
    const int64_t c = cw + (int64_t)lane * VEC;
    const int64_t olo = (cw == 0) ? 1 : cw + K;                  // output columns [olo, ohi)
    const int64_t ohi = min(cw + K + (int64_t)OW, cols - 1);
    const int64_t r0 = 1 + (int64_t)band * tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, rows - 1);   // r0 >= r1: no rows (VERT)
    // level-0 rows r0-K .. r1+K-1 stream through, three per iteration, from
    // i_first (r0-K downwards, r1+K-1 upwards); the rows past the far end that
    // round the count up are computed and never stored
    const int64_t nstream = (r1 - r0 + 2 * K + 2) / 3 * 3;
    const int64_t i_first = up ? r1 + K - 1 : r0 - K;
    // the window holds a ring column: per-lane selects needed
    const bool edge = (cw == 0) || (cw + 64 * VEC > cols - 1);
    // every row a level computes is interior and every row loaded (level-0 row
    // i, g row i -+ 1) is in the grid: no row or column tests at all. Computed
    // rows: r0-2K .. i_first+nstream-2 downwards, i_first-nstream+2 .. r1+2K-1
    // upwards.
    const bool fast = !edge && (up ? i_first - nstream + 1 >= 0 && r1 + 2 * K + 1 <= rows
                                   : r0 - 2 * K >= 1 && i_first + nstream <= rows);
    const bool vec_ok = c + VEC <= cols;
    const bool store_vec = c >= olo && c + VEC <= ohi;
    V* ring = reinterpret_cast<V*>(gring) + (size_t)hw_wave * K * 64 + lane;  // slot s at ring[s * 64]
    double qv[SEP ? VEC : 1];
    if constexpr (SEP) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) qv[e] = (c + e < cols) ? sep.q[c + e] : 0.0;
    }

    // W[j][s]: three rows of level j in registers; the slot that receives a
    // level's new row rotates with the row index (phase P = step % 3), so the
    // rows never move between registers
    T W[K][3][VEC];
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2)
#pragma unroll
            for (int e = 0; e < VEC; ++e) W[j][s2][e] = T(0);
    if (GRING) {
        V z;
#pragma unroll
        for (int e = 0; e < VEC; ++e) z[e] = T(0);
#pragma unroll
        for (int s2 = 0; s2 < K; ++s2) ring[s2 * 64] = z;
    }
    double acc = 0.0;
    double accs[MC ? K : 1];   // per-level deltas (MC)
#pragma unroll
    for (int k = 0; k < (MC ? K : 1); ++k) accs[k] = 0.0;
    int slot = 0;   // ring slot of g row (i -+ 1) at step i

    auto load = [&](auto fast_tag, const T* __restrict__ base, int64_t row, T (&v)[VEC], bool nt) {
        constexpr bool FAST = decltype(fast_tag)::value;
        const T* p = base + row * pitch;
        if (FAST) {
            const V x = nt ? __builtin_nontemporal_load(reinterpret_cast<const V*>(p + c))
                           : *reinterpret_cast<const V*>(p + c);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = x[e];
            return;
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = T(0);
        if (row < 0 || row >= rows) return;
        if (vec_ok) {
            const V x = nt ? __builtin_nontemporal_load(reinterpret_cast<const V*>(p + c))
                           : *reinterpret_cast<const V*>(p + c);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = x[e];
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (c + e < cols) v[e] = p[c + e];
        }
    };

    // one stream step: level-0 row i arrives in slot P of every level's triple;
    // level j computes row i - j (downwards) or i + j (upwards)
    auto step = [&](auto fast_tag, auto dir_tag, auto phase, int64_t i, const T (&inrow)[VEC],
                    const T (&grow)[VEC]) {
        constexpr bool FAST = decltype(fast_tag)::value;
        constexpr bool UP = decltype(dir_tag)::value;
        constexpr int P = decltype(phase)::value;
        constexpr int PN = (P + 1) % 3, PC = (P + 2) % 3;   // older rows: north, centre
#pragma unroll
        for (int e = 0; e < VEC; ++e) W[0][P][e] = inrow[e];
        // ring slot of the g row level jj reads at this step
        auto gslot = [&](int jj) { int s2 = slot - (jj - 1); return s2 < 0 ? s2 + K : s2; };
        V gb[GA > 0 ? GA : 1];   // g rows of the next GA levels, read ahead of their use
        if (GRING) {
            V x;
#pragma unroll
            for (int e = 0; e < VEC; ++e) x[e] = grow[e];
            ring[slot * 64] = x;   // g row i -+ 1
            if (GA > 0) {
                gb[0] = x;
#pragma unroll
                for (int d = 1; d < GA; ++d)
                    if (1 + d <= K) gb[d] = ring[gslot(1 + d) * 64];
            }
        }
#pragma unroll
        for (int j = 1; j <= K; ++j) {
            const int64_t row = UP ? i + j : i - j;
            const T(&src)[3][VEC] = W[j - 1];
            const T wl = lane_shift<kDppWaveShr1>(src[PC][VEC - 1]);
            const T er = lane_shift<kDppWaveShl1>(src[PC][0]);
            T gv[VEC];
            if (SEP) {
                // rows outside the grid only feed cells that are never stored
                const double pr = (row >= 0 && row < rows) ? sep.p[row] : 0.0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) gv[e] = sep_value<T>(sep, pr, qv[e]);
            } else if (HELM) {
                V x;   // g row i -+ j
                if (GA > 0) {
                    x = gb[(j - 1) % (GA > 0 ? GA : 1)];
                    if (j + GA <= K) gb[(j - 1) % (GA > 0 ? GA : 1)] = ring[gslot(j + GA) * 64];
                } else {
                    x = ring[gslot(j) * 64];
                }
#pragma unroll
                for (int e = 0; e < VEC; ++e) gv[e] = x[e];
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) gv[e] = T(0);
            }
            T nv[VEC];
            if (FAST || (row >= 1 && row <= rows - 2)) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T Wv = (e > 0) ? src[PC][e - 1] : wl;
                    const T Ev = (e < VEC - 1) ? src[PC][e + 1] : er;
                    nv[e] = jacobi_update<T, HELM>(src[PN][e], src[P][e], Wv, Ev, gv[e], rd, rd_lo,
                                                   row, c + e, sweep0 + (uint32_t)(j - 1));
                }
                if (!FAST && edge) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int64_t col = c + e;
                        if (col < 1 || col > cols - 2) nv[e] = src[PC][e];
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) nv[e] = src[PC][e];
            }
            if (MC && j < K && ((check_mask >> (j - 1)) & 1u) && row >= r0 && row < r1) {
                // a check inside the launch: delta of level j over this tile's cells
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int64_t col = c + e;
                    if (store_vec || (col >= olo && col < ohi))
                        accs[j - 1] = jacobi_accum(red, accs[j - 1], (double)nv[e] - (double)src[PC][e]);
                }
            }
            if (j < K) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) W[j][P][e] = nv[e];
            } else if (row >= r0 && row < r1) {
                T* p = b + row * pitch;
                if (store_vec) {
                    V x;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) x[e] = nv[e];
                    if (NT) __builtin_nontemporal_store(x, reinterpret_cast<V*>(p + c));
                    else *reinterpret_cast<V*>(p + c) = x;
                    if (check) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            acc = jacobi_accum(red, acc, (double)nv[e] - (double)src[PC][e]);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int64_t col = c + e;
                        if (col >= olo && col < ohi) {
                            p[col] = nv[e];
                            if (check) acc = jacobi_accum(red, acc, (double)nv[e] - (double)src[PC][e]);
                        }
                    }
                }
            }
        }
        slot = (slot + 1 == K) ? 0 : slot + 1;
    };

    // rows come in groups of three, each group's loads issued just before it is
    // computed. (Keeping the next group's loads in flight in a second register
    // buffer cost 24 VGPRs, and with them the third wavefront per SIMD at depth
    // 10: 8192^2 FP64 Helmholtz 1190 -> 1320 GLUP/s without it.)
    auto stream = [&](auto fast_tag, auto dir_tag) {
        constexpr int D = decltype(dir_tag)::value ? -1 : 1;   // row step of the stream
        for (int64_t n = 0; n < nstream; n += 3) {
            const int64_t i0 = i_first + D * n;
            T in[3][VEC], gin[3][VEC];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                load(fast_tag, a, i0 + D * q, in[q], false);
                if (GRING) load(fast_tag, g, i0 + D * (q - 1), gin[q], NTG);
            }
            step(fast_tag, dir_tag, std::integral_constant<int, 0>{}, i0, in[0], gin[0]);
            step(fast_tag, dir_tag, std::integral_constant<int, 1>{}, i0 + D, in[1], gin[1]);
            step(fast_tag, dir_tag, std::integral_constant<int, 2>{}, i0 + 2 * D, in[2], gin[2]);
        }
    };
    if (r0 < r1) {
        if constexpr (VERT) {
            if (up) {
                if (fast) stream(std::true_type{}, std::true_type{});
                else stream(std::false_type{}, std::true_type{});
            } else {
                if (fast) stream(std::true_type{}, std::false_type{});
                else stream(std::false_type{}, std::false_type{});
            }
        } else {
            if (fast) stream(std::true_type{}, std::false_type{});
            else stream(std::false_type{}, std::false_type{});
        }
    }

    auto reduce_out = [&](double v, int slot_index) {
        if (WT) {
            v = red == RED_MAX_ABS ? wave_max(v) : wave_sum(v);
            if (lane == 0) partials[slot_index] = v;
        } else {
            v = block_reduce<NW>(v, red == RED_MAX_ABS, lds);
            if (threadIdx.x == 0) partials[slot_index] = v;
            if (NW > 1) __syncthreads();   // lds is reused by the next reduce
        }
    };
    if (MC) {
        accs[K - 1] = acc;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if ((check_mask >> k) & 1u) reduce_out(accs[k], k * tiles + t);
    } else if (check) {
        reduce_out(acc, t);
    }
}

}  // namespace lsr
