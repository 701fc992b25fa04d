// Plain HBM copy kernel: the measured denominator of the roofline and the
// calibration of the FETCH_SIZE / WRITE_SIZE counters (a copy of B bytes reads
// B and writes B). 16-byte loads/stores, grid-stride, XCD-agnostic.
#include "kernels.hpp"

namespace lsr {
namespace {

__global__ __launch_bounds__(256) void copy16_kernel(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    const int64_t want = (n16 + 255) / 256;
    const int blocks = (int)(want < 256 * 32 ? want : 256 * 32);
    hipLaunchKernelGGL(copy16_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace lsr
