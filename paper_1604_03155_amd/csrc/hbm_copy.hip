// Streaming device-to-device copy: the reference kernel for attainable HBM
// bandwidth and for scaling hardware byte counters.
#include "common.h"
#include "../../include/vg.h"

namespace vg {
vg_status fail(vg_status st, const std::string& msg);
vg_status from_hip(hipError_t e, const char* what);

namespace {
__global__ void __launch_bounds__(256) copy16_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}
}  // namespace
}  // namespace vg

extern "C" vg_status vg_hbm_copy(void* dst, const void* src, size_t bytes, void* stream) {
    using namespace vg;
    if (!dst || !src || (bytes % 16) != 0) return fail(VG_ERR_INVALID_ARG, "copy needs device pointers and bytes % 16 == 0");
    const long long n = (long long)(bytes / 16);
    if (n == 0) return VG_OK;
    long long blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;  // 64 workgroups per CU, grid-stride beyond
    hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n);
    return from_hip(hipGetLastError(), "vg_hbm_copy");
}
