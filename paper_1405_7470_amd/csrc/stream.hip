// Streaming probe kernels: measured HBM rate and byte-counter calibration.
#include <hip/hip_runtime.h>

#include "lpx_internal.h"

namespace lpx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// y[r*n + t] = x[t] for r < fanout: one read stream, `fanout` write streams
// (fanout 1 is a plain copy).  n4 = n / 4 float4 chunks, one per thread:
// the grid covers the array, which streams faster on this GPU than a
// persistent grid-stride loop.
__global__ __launch_bounds__(256) void stream_kernel(const f4* __restrict__ x,
                                                     f4* __restrict__ y, int64_t n4,
                                                     int fanout) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const f4 v = x[t];
    for (int r = 0; r < fanout; ++r) y[r * n4 + t] = v;
}

}  // namespace
}  // namespace lpx

using namespace lpx;

extern "C" lpx_status lpx_stream_probe(const float* x, float* y, int64_t n, int32_t fanout,
                                       void* stream) {
    clear_error();
    if (n < 0 || fanout < 1 || fanout > 8)
        return set_error(LPX_ERR_INVALID_ARG, "need n >= 0 and 1 <= fanout <= 8");
    if (n == 0) return LPX_OK;
    if (n % 4 || !x || !y || (reinterpret_cast<uintptr_t>(x) & 15) ||
        (reinterpret_cast<uintptr_t>(y) & 15))
        return set_error(LPX_ERR_INVALID_ARG, "n must be a multiple of 4, pointers 16-byte aligned");
    if (n > INT64_MAX / 4 / fanout) return set_error(LPX_ERR_INVALID_ARG, "n too large");
    const int64_t nb = n * 4, ynb = nb * fanout;
    auto px = reinterpret_cast<uintptr_t>(x), py = reinterpret_cast<uintptr_t>(y);
    if (px < py + (uintptr_t)ynb && py < px + (uintptr_t)nb)
        return set_error(LPX_ERR_ALIAS, "y overlaps x");
    DeviceInfo dev;
    lpx_status s = current_device_info(&dev);
    if (s != LPX_OK) return s;
    const int64_t n4 = n / 4;
    const int64_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7fffffff) return set_error(LPX_ERR_INVALID_ARG, "n too large for one launch");
    hipLaunchKernelGGL(stream_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream),
                       reinterpret_cast<const f4*>(x), reinterpret_cast<f4*>(y), n4, fanout);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "stream probe: %s", hipGetErrorString(e));
    return LPX_OK;
}
