// Measurement hook: a plain device copy of known size whose loads and stores have a chosen width
// (8 or 16 bytes per lane), so that hardware traffic counters (bytes fetched from and written to HBM
// per dispatch) can be scaled against a kernel that moves exactly the bytes it is given.
#include "hs_common.h"

namespace hs {

typedef unsigned int hs_u4v __attribute__((ext_vector_type(4)));
typedef unsigned int hs_u2v __attribute__((ext_vector_type(2)));

template <class V>
__global__ __launch_bounds__(256) void k_calib_copy(const V* __restrict__ src, V* __restrict__ dst, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const V v = *(const HS_GLOBAL V*)(src + i);
        *(HS_GLOBAL V*)(dst + i) = v;
    }
}

bool launch_calib_copy(const void* src, void* dst, int64_t bytes, int width, hipStream_t s) {
    if (width == 16) {
        const int64_t n = bytes / 16;
        const int blocks = (int)std::min<int64_t>(8192, (n + 255) / 256);
        hipLaunchKernelGGL((k_calib_copy<hs_u4v>), dim3(blocks), dim3(256), 0, s, (const hs_u4v*)src, (hs_u4v*)dst, n);
        return true;
    }
    if (width == 8) {
        const int64_t n = bytes / 8;
        const int blocks = (int)std::min<int64_t>(8192, (n + 255) / 256);
        hipLaunchKernelGGL((k_calib_copy<hs_u2v>), dim3(blocks), dim3(256), 0, s, (const hs_u2v*)src, (hs_u2v*)dst, n);
        return true;
    }
    return false;
}

}  // namespace hs
