// hist_dev.h -- device code of the histogram count shared by the histogram
// pass and the fused segmentation kernel: the gray levels of 8 int16 voxels
// (one 16-byte vector) counted into an LDS histogram with R replicas of every
// bin, laid out bin-major (bin * R + replica).
#pragma once

#include "common.h"

namespace ts {

typedef int v4i __attribute__((ext_vector_type(4)));

template <int R, int MAP>
__device__ __forceinline__ void count8(uint32_t *lds, const v4i &w, const BinMap &bm, uint32_t rep)
{
    const uint32_t u[4] = {(uint32_t)w.x, (uint32_t)w.y, (uint32_t)w.z, (uint32_t)w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int v0 = (int)(int16_t)(u[j] & 0xffffu);
        int v1 = (int)(int16_t)(u[j] >> 16);
        atomicAdd(&lds[bin_of_t<MAP>(v0, bm) * R + rep], 1u);
        atomicAdd(&lds[bin_of_t<MAP>(v1, bm) * R + rep], 1u);
    }
}

// The same count with 2^lr replicas chosen at run time (the shift and add
// are one instruction).
template <int MAP>
__device__ __forceinline__ void count8_rt(uint32_t *lds, const v4i &w, const BinMap &bm, int lr, uint32_t rep)
{
    const uint32_t u[4] = {(uint32_t)w.x, (uint32_t)w.y, (uint32_t)w.z, (uint32_t)w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int v0 = (int)(int16_t)(u[j] & 0xffffu);
        int v1 = (int)(int16_t)(u[j] >> 16);
        atomicAdd(&lds[(bin_of_t<MAP>(v0, bm) << lr) + rep], 1u);
        atomicAdd(&lds[(bin_of_t<MAP>(v1, bm) << lr) + rep], 1u);
    }
}

} // namespace ts
