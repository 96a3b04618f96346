// Device-memory streaming ceiling.  A plain copy with 16-byte non-temporal
// loads and stores over a grid-stride loop: the rate at which it moves its
// bytes in and out is the practical HBM bound that the step kernels are
// measured against (beside the published peak).
#include "common.h"

namespace {
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const u4v* src, u4v* dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const u4v v = __builtin_nontemporal_load(src + i);
        __builtin_nontemporal_store(v, dst + i);
    }
}
}  // namespace

extern "C" int rbffd_stream_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    if (!src || !dst || bytes < 0 || (bytes % 16) || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
        return RBFFD_EINVAL;
    const int64_t n16 = bytes / 16;
    if (n16 == 0) return RBFFD_OK;
    const int64_t grid = std::min<int64_t>(cdiv(n16, 256), (int64_t)1 << 20);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, (const u4v*)src,
                       (u4v*)dst, n16);
    return hipGetLastError() == hipSuccess ? RBFFD_OK : RBFFD_EHIP;
}
