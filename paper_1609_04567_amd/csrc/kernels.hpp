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
};
// tile_rows / waves / unroll of 0 (or an unsupported pair) select the measured default.
SweepGeom jacobi_geom(const JacobiArgs& a, int tile_rows, int waves = 0, int unroll = 0);
hipError_t launch_jacobi(const JacobiArgs& a, const SweepGeom& g, JobState* st, void* partials,
                         const LoopCtl& c, int j, hipStream_t s);

// Game of Life B3/S23 --------------------------------------------------------
struct LifeArgs {
    const uint8_t* a;
    uint8_t* b;
    int64_t rows, cols, pitch;
    int torus;
};
SweepGeom life_geom(const LifeArgs& a, int tile_rows);
hipError_t launch_life(const LifeArgs& a, const SweepGeom& g, JobState* st, void* partials,
                       const LoopCtl& c, int j, hipStream_t s);
// Live-cell count of a u8 grid into partials (one per block); returns the partial count.
hipError_t launch_count_u8(const uint8_t* a, int64_t rows, int64_t cols, int64_t pitch,
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

// HBM copy probe: bytes must be a multiple of 16, buffers 16-byte aligned.
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s);

// Loop control ---------------------------------------------------------------
hipError_t launch_init_state(JobState* st, const void* count_parts, int nparts, hipStream_t s);
hipError_t launch_finalize(JobState* st, const void* partials, const LoopCtl& c, int j,
                           JobState* mirror, hipStream_t s);
hipError_t launch_cancel(JobState* st, JobState* mirror, hipStream_t s);

}  // namespace lsr
