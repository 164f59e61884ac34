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


// Issue-rate probe: every lane runs `iters` blocks of independent VALU
// instructions (no result feeds another inside the loop, so nothing waits on
// a dependency): op 0 eight v_add_f32, op 1 eight v_log_f32, op 2 two
// v_log_f32 and twelve v_add_f32 (the mix of one FP32 class term of the
// search).  Timing a launch that fills every SIMD gives the chip's issue
// rate of plain FP32 VALU instructions and of the transcendental unit, the
// peaks the search's roofline is taken against.
template <int OP>
__global__ void __launch_bounds__(256) k_issue(float a, int iters, float *__restrict__ out)
{
    const float x0 = a + (float)threadIdx.x, x1 = x0 + 1.0f, x2 = x0 + 2.0f;
    float r0 = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0, r5 = 0, r6 = 0, r7 = 0;
    for (int i = 0; i < iters; ++i) {
        if (OP == 0)
            asm volatile("v_add_f32 %0, %8, %9\n\tv_add_f32 %1, %9, %10\n\tv_add_f32 %2, %8, %10\n\t"
                         "v_add_f32 %3, %10, %8\n\tv_add_f32 %4, %9, %8\n\tv_add_f32 %5, %10, %9\n\t"
                         "v_add_f32 %6, %8, %8\n\tv_add_f32 %7, %9, %9"
                         : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
                         : "v"(x0), "v"(x1), "v"(x2));
        else if (OP == 1)
            asm volatile("v_log_f32 %0, %8\n\tv_log_f32 %1, %9\n\tv_log_f32 %2, %10\n\tv_log_f32 %3, %8\n\t"
                         "v_log_f32 %4, %9\n\tv_log_f32 %5, %10\n\tv_log_f32 %6, %8\n\tv_log_f32 %7, %9"
                         : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
                         : "v"(x0), "v"(x1), "v"(x2));
        else
            asm volatile("v_log_f32 %0, %8\n\tv_add_f32 %1, %9, %10\n\tv_add_f32 %2, %8, %10\n\t"
                         "v_add_f32 %3, %10, %8\n\tv_add_f32 %4, %9, %8\n\tv_add_f32 %5, %10, %9\n\t"
                         "v_add_f32 %6, %8, %8\n\tv_log_f32 %7, %9\n\tv_add_f32 %1, %9, %8\n\t"
                         "v_add_f32 %2, %10, %10\n\tv_add_f32 %3, %8, %9\n\tv_add_f32 %4, %10, %8\n\t"
                         "v_add_f32 %5, %9, %10\n\tv_add_f32 %6, %8, %10"
                         : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
                         : "v"(x0), "v"(x1), "v"(x2));
    }
    asm volatile("s_nop 7" ::: "memory"); // transcendental results settle before they are read
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = ((r0 + r1) + (r2 + r3)) + ((r4 + r5) + (r6 + r7));
}

ts_status launch_issue_rate(int op, int blocks, int iters, float *out, hipStream_t st)
{
    if (op == 0)
        hipLaunchKernelGGL(k_issue<0>, dim3(blocks), dim3(256), 0, st, 1.5f, iters, out);
    else if (op == 1)
        hipLaunchKernelGGL(k_issue<1>, dim3(blocks), dim3(256), 0, st, 1.5f, iters, out);
    else
        hipLaunchKernelGGL(k_issue<2>, dim3(blocks), dim3(256), 0, st, 1.5f, iters, out);
    return check_launch("ts_issue_rate");
}

} // namespace ts
