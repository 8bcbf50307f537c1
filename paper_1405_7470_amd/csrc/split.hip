// Split-precision conversion x -> (hi, lo) bfloat16 planes.
#include <hip/hip_runtime.h>

#include "lpx_internal.h"

namespace lpx {
namespace {

__device__ __forceinline__ unsigned short bits(__bf16 h) {
    return __builtin_bit_cast(unsigned short, h);
}

__global__ __launch_bounds__(256) void split_bf16_kernel(const float* __restrict__ x,
                                                         uint16_t* __restrict__ hi,
                                                         uint16_t* __restrict__ lo,
                                                         int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[t];
        const __bf16 h = (__bf16)v;  // round to nearest even (v_cvt_pk_bf16_f32)
        hi[t] = bits(h);
        lo[t] = bits((__bf16)(v - (float)h));
    }
}

}  // namespace

lpx_status launch_split_bf16(const float* x, uint16_t* hi, uint16_t* lo, int64_t n,
                             void* stream) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), x, hi, lo, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(LPX_ERR_HIP, "split launch: %s", hipGetErrorString(e));
    return LPX_OK;
}

}  // namespace lpx
