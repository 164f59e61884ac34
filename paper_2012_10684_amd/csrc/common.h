// common.h -- internal helpers shared by the HIP translation units of libts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ts.h"

namespace ts {

constexpr int WAVE = 64;
constexpr int MAX_BINS = 4096;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
ts_status fail(ts_status st, const std::string &msg);
ts_status check_launch(const char *what);
int device_cu_count();

// ---------------------------------------------------------------- tuning
struct Tune {
    int hist_block, hist_replicas, hist_wg_per_cu;
    int label_block, label_wg_per_cu;
    int search_cols, search_rows;
    int min_chunk;
    int search_path, search_block;
};
ts_status resolve_tuning(const ts_tuning *t, int nbins, Tune *out);

// ---------------------------------------------------------------- bin map
// b(d) = (d * mul) >> shift for the in-window offset d = v - lo, with the
// constants chosen on the host and checked there for every d in [0, W).
struct BinMap {
    int32_t lo, hi, L;
    uint32_t mul;   // multiplier
    uint32_t shift; // right shift
    int32_t wide;   // 1: use the 32x32 high product of (d*L) with mul
    int32_t narrow; // 1: window narrower than L (values above hi need a select)
};
ts_status make_binmap(const ts_binning &bin, BinMap *bm);

// MAP selects the multiply at compile time: bit 0 = wide, bit 1 = narrow
// window (values above hi need the explicit select).
template <int MAP>
__device__ __forceinline__ int bin_of_t(int v, const BinMap &bm)
{
    int vc = min(max(v, bm.lo), bm.hi);
    uint32_t d = (uint32_t)(vc - bm.lo);
    uint32_t b;
    if (MAP & 1)
        b = __umulhi(d * (uint32_t)bm.L, bm.mul) >> bm.shift;
    else
        b = __umul24(d, bm.mul) >> bm.shift;
    if ((MAP & 2) && v > bm.hi)
        b = (uint32_t)(bm.L - 1);
    return (int)b;
}

__device__ __forceinline__ int bin_of(int v, const BinMap &bm)
{
    switch ((bm.wide ? 1 : 0) | (bm.narrow ? 2 : 0)) {
    case 0: return bin_of_t<0>(v, bm);
    case 1: return bin_of_t<1>(v, bm);
    case 2: return bin_of_t<2>(v, bm);
    default: return bin_of_t<3>(v, bm);
    }
}

inline int map_kind(const BinMap &bm) { return (bm.wide ? 1 : 0) | (bm.narrow ? 2 : 0); }

// Pointers read from a device table are generic; the voxel and label arrays
// always live in global memory, and saying so lets the compiler use global
// (not flat) loads and stores, which do not wait on LDS traffic.
#define TS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const TS_GLOBAL T *gp(const T *p)
{
    return (const TS_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ TS_GLOBAL T *gpw(T *p)
{
    return (TS_GLOBAL T *)p;
}

// ---------------------------------------------------------------- batch walk
// Index of the problem containing flattened position pos: the largest s with
// offs[s] <= pos (binary search; offs non-decreasing, nseg >= 1).
__device__ __forceinline__ int find_segment(const int64_t *offs, int nseg, int64_t pos)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= pos)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

// order-preserving map of a float onto int32 (for atomicMax on floats)
__device__ __forceinline__ int float_to_ordered(float f)
{
    int b = __float_as_int(f);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float ordered_to_float(int e)
{
    return __int_as_float(e ^ ((e >> 31) & 0x7fffffff));
}

// ---------------------------------------------------------------- launches
ts_status launch_histogram(const ts_batch &b, const BinMap &bm, uint32_t *hist, const Tune &t, hipStream_t s);
ts_status launch_prefix(const uint32_t *hist, int nseg, int L, double q, double *P, double *Q, hipStream_t s);
ts_status launch_label(const ts_batch &b, const BinMap &bm, const int32_t *thr, int k, uint8_t *const *out,
                       const Tune &t, hipStream_t s);

struct SearchPlan;
size_t search_workspace_bytes(int nseg, int L, int k, int mode, int cols);
ts_status launch_search(const double *P, const double *Q, int nseg, int L, int k, double q, int mode, void *ws,
                        size_t ws_bytes, int32_t *thr, double *obj, int32_t *status, const Tune &t,
                        hipStream_t s);

} // namespace ts
