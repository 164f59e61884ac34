// k_label.hip -- the thresholding kernel function (Algorithm 1) generalised
// to k thresholds, fused with the bin map: label(v) = #{j : b(v) > t_j}.
//
// No bin index is materialised.  For the window rule of ts_binning,
// b(v) > t  <=>  v >= cut(t) = lo + ceil((t + 1) * W / L)   (W = hi - lo + 1),
// which also covers values outside the window (below lo: bin 0, never above a
// threshold; above hi: bin L-1, above every threshold since cut(t) <= hi + 1).
// So each voxel costs k integer compares.  Streaming layout as in the
// histogram: a persistent grid splits the flattened batch into equal ranges;
// 16-byte loads of 8 voxels and 8-byte stores of 8 labels where the input and
// output phases agree, element-wise code elsewhere.
#include <algorithm>

#include "common.h"

namespace ts {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

struct Cuts {
    int c0, c1, c2; // label = [v >= c0] + [v >= c1] + [v >= c2]
};

// Cut values of problem s; a row that is not a strictly ascending tuple in
// [0, L-2] (e.g. the -1 row of a degenerate problem) gives no cuts (all 0).
__device__ __forceinline__ Cuts make_cuts(const int32_t *thr, int k, const BinMap &bm)
{
    const int NEVER = 0x7fffffff;
    Cuts c = {NEVER, NEVER, NEVER};
    int t[3] = {-1, -1, -1};
    bool ok = true;
    for (int j = 0; j < k; ++j) {
        t[j] = thr[j];
        ok = ok && t[j] >= 0 && t[j] <= bm.L - 2 && (j == 0 || t[j] > t[j - 1]);
    }
    if (!ok)
        return c;
    const int64_t W = (int64_t)bm.hi - bm.lo + 1;
    int cc[3] = {NEVER, NEVER, NEVER};
    for (int j = 0; j < k; ++j)
        cc[j] = bm.lo + (int)(((int64_t)(t[j] + 1) * W + bm.L - 1) / bm.L);
    c.c0 = cc[0];
    c.c1 = cc[1];
    c.c2 = cc[2];
    return c;
}

__device__ __forceinline__ uint32_t lab1(int v, const Cuts &c)
{
    return (uint32_t)(v >= c.c0) + (uint32_t)(v >= c.c1) + (uint32_t)(v >= c.c2);
}

// labels of the two int16 in a dword, packed as bytes 0 and 1 of the result
__device__ __forceinline__ uint32_t lab2(uint32_t w, const Cuts &c)
{
    int v0 = (int)(int16_t)(w & 0xffffu);
    int v1 = (int)(int16_t)(w >> 16);
    return lab1(v0, c) | (lab1(v1, c) << 8);
}

__device__ __forceinline__ v2u lab8(const v4i &w, const Cuts &c)
{
    uint32_t a = lab2((uint32_t)w.x, c) | (lab2((uint32_t)w.y, c) << 16);
    uint32_t b = lab2((uint32_t)w.z, c) | (lab2((uint32_t)w.w, c) << 16);
    v2u r;
    r.x = a;
    r.y = b;
    return r;
}

// Up to TS_MAX_LABEL_SETS threshold sets labelled in one pass: each 16-byte
// load of 8 voxels feeds one 8-byte store per set.
template <int NS>
__device__ __forceinline__ void label_vec(const TS_GLOBAL v4i *vp, TS_GLOBAL v2u *const (&op)[NS],
                                          const Cuts (&cuts)[NS], int64_t nvec)
{
    const int64_t st = blockDim.x;
    int64_t j = threadIdx.x;
    // pairs of vectors per thread; the next pair is in flight while the
    // current one is labelled and stored
    bool have = j + st < nvec;
    v4i a0 = {0, 0, 0, 0}, a1 = a0;
    if (have) {
        a0 = __builtin_nontemporal_load(vp + j);
        a1 = __builtin_nontemporal_load(vp + j + st);
    }
    while (have) {
        const int64_t jn = j + 2 * st;
        const bool nxt = jn + st < nvec;
        v4i b0 = a0, b1 = a1;
        if (nxt) {
            b0 = __builtin_nontemporal_load(vp + jn);
            b1 = __builtin_nontemporal_load(vp + jn + st);
        }
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            __builtin_nontemporal_store(lab8(a0, cuts[u]), op[u] + j);
            __builtin_nontemporal_store(lab8(a1, cuts[u]), op[u] + j + st);
        }
        a0 = b0;
        a1 = b1;
        j = jn;
        have = nxt;
    }
    for (; j < nvec; j += st) {
        const v4i a = __builtin_nontemporal_load(vp + j);
#pragma unroll
        for (int u = 0; u < NS; ++u)
            __builtin_nontemporal_store(lab8(a, cuts[u]), op[u] + j);
    }
}

template <int NS>
__global__ void __launch_bounds__(1024) k_label(const int16_t *const *__restrict__ vox,
                                                const int64_t *__restrict__ offs, int nseg, int64_t total,
                                                int64_t chunk, BinMap bm, LabelSets sets, int k)
{
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(total, beg + chunk);
    if (beg >= end)
        return;
    int s = find_segment(offs, nseg, beg);
    int64_t pos = beg;
    while (pos < end) {
        while (s + 1 < nseg && offs[s + 1] <= pos)
            ++s;
        const int64_t s0 = offs[s];
        const int64_t s1 = min(offs[s + 1], end);
        const TS_GLOBAL int16_t *src = gp(vox[s]);
        TS_GLOBAL uint8_t *dst[NS];
        Cuts cuts[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            dst[u] = gpw(sets.out[u][s]);
            cuts[u] = make_cuts(sets.thr[u] + (int64_t)s * k, k, bm);
        }
        const int64_t i0 = pos - s0, i1 = s1 - s0;
        const uintptr_t ain = (uintptr_t)(src + i0);
        // element phase of 16-byte input alignment; every output must have
        // the same phase for 8-byte alignment
        const int64_t hin = (int64_t)(((16u - (ain & 15u)) & 15u) >> 1);
        bool vec = (ain & 1u) == 0;
#pragma unroll
        for (int u = 0; u < NS; ++u)
            vec = vec && (int64_t)((8u - ((uintptr_t)(dst[u] + i0) & 7u)) & 7u) == hin;
        if (vec) {
            const int64_t head = min(hin, i1 - i0);
            if (threadIdx.x < head) {
                const int v = src[i0 + threadIdx.x];
#pragma unroll
                for (int u = 0; u < NS; ++u)
                    dst[u][i0 + threadIdx.x] = (uint8_t)lab1(v, cuts[u]);
            }
            const int64_t vb = i0 + head;
            const int64_t nvec = (i1 - vb) >> 3;
            TS_GLOBAL v2u *op[NS];
#pragma unroll
            for (int u = 0; u < NS; ++u)
                op[u] = reinterpret_cast<TS_GLOBAL v2u *>(dst[u] + vb);
            label_vec<NS>(reinterpret_cast<const TS_GLOBAL v4i *>(src + vb), op, cuts, nvec);
            const int64_t tb = vb + (nvec << 3);
            if (threadIdx.x < i1 - tb) {
                const int v = src[tb + threadIdx.x];
#pragma unroll
                for (int u = 0; u < NS; ++u)
                    dst[u][tb + threadIdx.x] = (uint8_t)lab1(v, cuts[u]);
            }
        } else {
            for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
                const int v = src[i];
#pragma unroll
                for (int u = 0; u < NS; ++u)
                    dst[u][i] = (uint8_t)lab1(v, cuts[u]);
            }
        }
        pos = s0 + i1;
        ++s;
    }
}

ts_status launch_label(const ts_batch &b, const BinMap &bm, const LabelSets &sets, int nsets, int k, const Tune &t,
                       hipStream_t st)
{
    if (b.total == 0)
        return TS_OK;
    const int64_t max_wg = (int64_t)device_cu_count() * t.label_wg_per_cu;
    int64_t grid = std::min<int64_t>(max_wg, (b.total + t.min_chunk - 1) / t.min_chunk);
    if (grid < 1)
        grid = 1;
    int64_t chunk = (b.total + grid - 1) / grid;
    chunk = (chunk + 63) & ~(int64_t)63;
    grid = (b.total + chunk - 1) / chunk;
    const dim3 g((unsigned)grid), blk(t.label_block);
    switch (nsets) {
    case 1: hipLaunchKernelGGL(k_label<1>, g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, chunk, bm, sets, k); break;
    case 2: hipLaunchKernelGGL(k_label<2>, g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, chunk, bm, sets, k); break;
    case 3: hipLaunchKernelGGL(k_label<3>, g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, chunk, bm, sets, k); break;
    default: hipLaunchKernelGGL(k_label<4>, g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, chunk, bm, sets, k); break;
    }
    return check_launch("ts_label");
}

} // namespace ts
