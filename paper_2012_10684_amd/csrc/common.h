// common.h -- internal helpers shared by the HIP translation units of libts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ts.h"

namespace ts {

constexpr int WAVE = 64;
// v_log_f32 error bound used by the FP32 search keys' error bounds, in units
// of 2^-24 * max(1, |log2 x|); ts_log2_f32 applies the same instruction so
// that the bound can be checked against an FP64 log2.
constexpr double LOG2_ERR_UNITS = 4.0;
constexpr int MAX_BINS = 4096;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
ts_status fail(ts_status st, const std::string &msg);
ts_status check_launch(const char *what);
int device_cu_count();
// Let kernel fn use `bytes` of dynamic LDS (more than the default 64 KiB) on
// the current device: the attribute is set once per kernel and device and
// kept (setting it on every launch stalled the host behind queued work).
void allow_dynamic_lds(const void *fn, size_t bytes);

// ---------------------------------------------------------------- tuning
struct Tune {
    int hist_block, hist_replicas, hist_wg_per_cu;
    int label_block, label_vecs;
    int search_cols, search_rows;
    int min_chunk;
    int search_path, search_block;
    int segment_parts, segment_block;
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

// Workgroup barrier that orders LDS accesses only: global stores and atomics
// issued before it stay in flight (__syncthreads also waits for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// A guess at the segment holding flattened position pos (0 <= pos < total),
// exact for segments of equal size: callers check it with the two offsets
// around it (loaded together with whatever they load for that segment) and
// fall back to find_segment when it is wrong.
__device__ __forceinline__ int guess_segment(int nseg, int64_t total, int64_t pos)
{
    const double f = (double)pos / (double)total * (double)nseg; // rounding only costs the fallback
    return (int)min((double)(nseg - 1), f);
}

// ---------------------------------------------------------------- reductions
// Wavefront reductions with DPP lane moves (full-rate VALU; no LDS round
// trips): swaps within quads, mirrors within half-rows and rows, then the
// row broadcasts of lanes 15 and 31 leave the result in lane 63, which is
// read back as a wavefront-uniform value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xF, false);
}

__device__ __forceinline__ float wave_max(float v)
{
#define TS_DPP_MAX(C, M) v = fmaxf(v, __int_as_float(dpp_i32<C, M>(__float_as_int(v))))
    TS_DPP_MAX(0xB1, 0xF);  // quad_perm [1,0,3,2]
    TS_DPP_MAX(0x4E, 0xF);  // quad_perm [2,3,0,1]
    TS_DPP_MAX(0x141, 0xF); // row_half_mirror
    TS_DPP_MAX(0x140, 0xF); // row_mirror
    TS_DPP_MAX(0x142, 0xA); // row_bcast15 into rows 1 and 3
    TS_DPP_MAX(0x143, 0xC); // row_bcast31 into rows 2 and 3
#undef TS_DPP_MAX
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <int C, int M>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<C, M>((int)(b & 0xffffffffLL));
    const int hi = dpp_i32<C, M>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_min_f64(double v)
{
    v = fmin(v, dpp_f64<0xB1, 0xF>(v));
    v = fmin(v, dpp_f64<0x4E, 0xF>(v));
    v = fmin(v, dpp_f64<0x141, 0xF>(v));
    v = fmin(v, dpp_f64<0x140, 0xF>(v));
    v = fmin(v, dpp_f64<0x142, 0xA>(v));
    v = fmin(v, dpp_f64<0x143, 0xC>(v));
    const long long b = __double_as_longlong(v);
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
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
ts_status launch_prefix(const uint32_t *hist, int nseg, int L, int nq, const double *q, double *P, double *Q,
                        hipStream_t s);
// Threshold rows and output tables of the sets labelled by one launch.
struct LabelSets {
    const int32_t *thr[TS_MAX_LABEL_SETS];
    uint8_t *const *out[TS_MAX_LABEL_SETS];
};
ts_status launch_fill_u32(uint32_t *p, int64_t n, hipStream_t st); // zero n words (k_histogram.hip)
size_t hist2d_lds_bytes(int L, int H, int W);
ts_status launch_hist2d(const ts_batch &b, int H, int W, const BinMap &bm, uint32_t *hist, hipStream_t st);
size_t search2d_workspace_bytes(int nseg, int nq, int L);
size_t dp_workspace_bytes(int nprob, int L, int k);
size_t open2d_workspace_bytes(int nseg, int H, int W);
ts_status launch_open2d(const ts_batch &b, int H, int W, const BinMap &bm, int r, uint8_t *eroded,
                        uint8_t *opened, uint8_t *residue, int16_t *residue16, hipStream_t st);
ts_status launch_dp(const double *P, const double *Q, int nseg, int L, int k, int nq, const double *q, void *ws,
                    int32_t *thr, double *obj, int32_t *status, hipStream_t st);
ts_status launch_search2d(const uint32_t *hist, int nseg, int L, int nq, const double *q, void *ws, int32_t *thr,
                          double *obj, int32_t *status, hipStream_t st);
ts_status launch_log2_f32(const float *x, float *y, int64_t n, hipStream_t st);
ts_status launch_issue_rate(int op, int blocks, int iters, float *out, hipStream_t st);
ts_status launch_label(const ts_batch &b, const BinMap &bm, const LabelSets &sets, int nsets, int k, const Tune &t,
                       hipStream_t st);

struct SearchPlan;
size_t search_workspace_bytes(int nseg, int L, int k, int mode, int cols);
// workspace bytes the search touches for these sizes and this tuning (0 on
// the one-workgroup-per-problem path, which keeps everything in LDS)
size_t search_need_bytes(int nprob, int L, int k, int mode, const Tune &t);
// argument checks shared by the search entry points
ts_status check_search_args(const char *fn, const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                            int32_t nq, const double *q, int32_t mode, int32_t *thr, double *obj, int32_t *status);
ts_status launch_search(const double *P, const double *Q, int nseg, int L, int k, int nq, const double *q, int mode,
                        void *ws, size_t ws_bytes, int32_t *thr, double *obj, int32_t *status, const Tune &t,
                        hipStream_t st);
size_t segment_workspace_bytes(int nseg, int L, int k, int nq, int mode, bool labels);
ts_status launch_segment(const ts_batch &b, const BinMap &bm, int k, int nq, const double *q, int mode,
                         uint32_t *hist, int32_t *thr, double *obj, int32_t *status, const LabelSets *sets, void *ws,
                         const Tune &t, hipStream_t st);

} // namespace ts
