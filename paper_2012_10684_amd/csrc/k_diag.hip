// k_diag.hip -- the FP32 base-2 logarithm the threshold search evaluates
// (v_log_f32), exposed so that its error against an exact log2 can be
// measured: the search's FP32 error bound assumes at most LOG2_ERR_UNITS
// units of 2^-24 * max(1, |log2 x|) for normal inputs.
#include <algorithm>

#include "common.h"

namespace ts {

__global__ void __launch_bounds__(256) k_log2_f32(const float *__restrict__ x, float *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        y[i] = __builtin_amdgcn_logf(x[i]);
}

ts_status launch_log2_f32(const float *x, float *y, int64_t n, hipStream_t st)
{
    const int64_t grid = (n + 255) / 256;
    if (grid > 0x7fffffff)
        return fail(TS_ERR_INVALID_ARG, "ts_log2_f32: n too large for one launch");
    hipLaunchKernelGGL(k_log2_f32, dim3((unsigned)grid), dim3(256), 0, st, x, y, n);
    return check_launch("ts_log2_f32");
}

} // namespace ts
