// Plain HBM copy kernel: the measured denominator of the roofline and the
// calibration of the FETCH_SIZE / WRITE_SIZE counters (a copy of B bytes reads
// B and writes B). Each thread issues four 16-byte loads before its four
// non-temporal 16-byte stores; grid-stride over the buffer.
#include "kernels.hpp"

namespace lsr {
namespace {

typedef uint32_t W4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(256) void copy16_kernel(const W4* __restrict__ src, W4* __restrict__ dst,
                                                     int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256 * kCopyUnroll;
    for (int64_t i = (int64_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x; i < n16; i += stride) {
        W4 v[kCopyUnroll];
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) {
            const int64_t idx = i + (int64_t)k * 256;
            if (idx < n16) v[k] = src[idx];
        }
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) {
            const int64_t idx = i + (int64_t)k * 256;
            if (idx < n16) __builtin_nontemporal_store(v[k], dst + idx);
        }
    }
}

}  // namespace

hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    const int64_t want = (n16 + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    const int blocks = (int)(want < 256 * 64 ? want : 256 * 64);
    hipLaunchKernelGGL(copy16_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s,
                       static_cast<const W4*>(src), static_cast<W4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace lsr
