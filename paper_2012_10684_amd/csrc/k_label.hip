// k_label.hip -- the thresholding kernel function (Algorithm 1) generalised
// to k thresholds, fused with the bin map: label(v) = #{j : b(v) > t_j}.
//
// No bin index is materialised.  For the window rule of ts_binning,
// b(v) > t  <=>  v >= cut(t) = lo + ceil((t + 1) * W / L)   (W = hi - lo + 1),
// which also covers values outside the window (below lo: bin 0, never above a
// threshold; above hi: bin L-1, above every threshold since cut(t) <= hi + 1).
// So each voxel costs k integer compares; on the vector path two voxels
// share each operation (packed 16-bit arithmetic).  One-shot grid over tiles
// of the flattened batch; 16-byte loads of 8 voxels and 8-byte stores of 8
// labels where the input and output phases agree, element-wise code
// elsewhere.
#include <algorithm>

#include "common.h"
#include "label_dev.h"

namespace ts {

// Cut values of problem s for every set, computed by one lane per (set,
// threshold) and broadcast through readlane (wavefront-uniform results).
// (t+1) W <= 4095 * 65536 < 2^32, so the ceiling division is exact in uint32.
// NS * KM <= 64 lanes.
template <int NS, int KM>
__device__ __forceinline__ void wave_cuts(const LabelSets &sets, int s, int k, const BinMap &bm,
                                          Cuts<KM> (&cuts)[NS])
{
    static_assert(NS * KM <= 64, "one lane per (set, threshold)");
    const int lane = threadIdx.x & 63;
    const int u = lane / KM, j = lane % KM;
    int c = 0x7fffffff;
    if (u < NS && j < k) {
        const int32_t *t = sets.thr[u] + (int64_t)s * k;
        bool ok = true;
        for (int i = 0; i < k; ++i) // the whole row must be a strictly ascending tuple in [0, L-2]
            ok = ok && t[i] >= 0 && t[i] <= bm.L - 2 && (i == 0 || t[i] > t[i - 1]);
        if (ok) {
            const uint32_t W = (uint32_t)((int64_t)bm.hi - bm.lo + 1);
            c = bm.lo + (int)(((uint32_t)(t[j] + 1) * W + (uint32_t)bm.L - 1) / (uint32_t)bm.L);
        }
    }
#pragma unroll
    for (int u2 = 0; u2 < NS; ++u2) {
#pragma unroll
        for (int j2 = 0; j2 < KM; ++j2) // up to 64 values: vector registers beyond the 3-cut case
            cuts[u2].c[j2] = KM <= 3 ? __builtin_amdgcn_readlane(c, KM * u2 + j2) : __shfl(c, KM * u2 + j2, 64);
    }
}

// One workgroup per tile of blockDim * 8 * U voxels of the flattened batch,
// one pass over the voxels for NS threshold sets (up to TS_MAX_LABEL_SETS):
// each 16-byte load of 8 voxels feeds one 8-byte store per set.  A tile inside
// one segment whose input and outputs share the 16/8-byte alignment phase is
// labelled with vector accesses; any other tile voxel by voxel.  A one-shot
// grid keeps the voxels in flight at any time in one window of HBM, which
// streams faster on MI355X than long per-workgroup ranges.
template <int NS, int U, int KM>
__global__ void __launch_bounds__(1024) k_label(const int16_t *const *__restrict__ vox,
                                                const int64_t *__restrict__ offs, int nseg, int64_t total, BinMap bm,
                                                LabelSets sets, int k)
{
    const int64_t T = (int64_t)blockDim.x * 8 * U;
    const int64_t t0 = (int64_t)blockIdx.x * T;
    const int64_t t1 = min(total, t0 + T);
    // everything the tile needs from the guessed segment is loaded in one
    // round trip; a wrong guess (uneven segments) is corrected afterwards
    int s = guess_segment(nseg, total, t0);
    int64_t o0 = offs[s], o1 = offs[s + 1];
    const int16_t *vs = vox[s];
    uint8_t *os[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u)
        os[u] = sets.out[u][s];
    Cuts<KM> cuts[NS];
    wave_cuts<NS, KM>(sets, s, k, bm, cuts);
    if (!(o0 <= t0 && t0 < o1)) {
        s = find_segment(offs, nseg, t0);
        while (s + 1 < nseg && offs[s + 1] <= t0) // skip empty segments
            ++s;
        o0 = offs[s];
        o1 = offs[s + 1];
        vs = vox[s];
#pragma unroll
        for (int u = 0; u < NS; ++u)
            os[u] = sets.out[u][s];
        wave_cuts<NS, KM>(sets, s, k, bm, cuts);
    }
    if (t1 <= o1) { // the whole tile lies in segment s
        const TS_GLOBAL int16_t *src = gp(vs) + (t0 - o0);
        TS_GLOBAL uint8_t *dst[NS];
        bool vec = ((uintptr_t)src & 15u) == 0;
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            dst[u] = gpw(os[u]) + (t0 - o0);
            vec = vec && ((uintptr_t)dst[u] & 7u) == 0;
        }
        const int n = (int)(t1 - t0);
        if (vec) {
            PCuts<KM> pc[NS];
#pragma unroll
            for (int u = 0; u < NS; ++u)
                pc[u] = pack_cuts(cuts[u]);
            const TS_GLOBAL v4i *vp = reinterpret_cast<const TS_GLOBAL v4i *>(src);
            const int nvec = n >> 3;
            v4i w[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int i = threadIdx.x + j * blockDim.x;
                w[j] = i < nvec ? __builtin_nontemporal_load(vp + i) : v4i{0, 0, 0, 0};
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int i = threadIdx.x + j * blockDim.x;
                if (i < nvec) {
#pragma unroll
                    for (int u = 0; u < NS; ++u)
                        __builtin_nontemporal_store(lab8(w[j], pc[u]),
                                                    reinterpret_cast<TS_GLOBAL v2u *>(dst[u]) + i);
                }
            }
            const int tb = nvec << 3; // ragged end of the segment
            if ((int)threadIdx.x < n - tb) {
                const int v = src[tb + threadIdx.x];
#pragma unroll
                for (int u = 0; u < NS; ++u)
                    dst[u][tb + threadIdx.x] = (uint8_t)lab1p(v, pc[u]);
            }
        } else {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int v = src[i];
#pragma unroll
                for (int u = 0; u < NS; ++u)
                    dst[u][i] = (uint8_t)lab1(v, cuts[u]);
            }
        }
        return;
    }
    // the tile crosses segment ends: voxel by voxel, segments walked forward
    for (int64_t pos = t0 + threadIdx.x; pos < t1; pos += blockDim.x) {
        int sv = s;
        while (offs[sv + 1] <= pos)
            ++sv;
        const int64_t i = pos - offs[sv];
        const int v = gp(vox[sv])[i];
#pragma unroll
        for (int u = 0; u < NS; ++u)
            gpw(sets.out[u][sv])[i] = (uint8_t)lab1(v, make_cuts<KM>(sets.thr[u] + (int64_t)sv * k, k, bm));
    }
}

template <int NS, int KM>
static void launch_label_ns(int U, dim3 g, dim3 blk, hipStream_t st, const ts_batch &b, const BinMap &bm,
                            const LabelSets &sets, int k)
{
    if (U == 1)
        hipLaunchKernelGGL((k_label<NS, 1, KM>), g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, bm, sets, k);
    else if (U == 2)
        hipLaunchKernelGGL((k_label<NS, 2, KM>), g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, bm, sets, k);
    else
        hipLaunchKernelGGL((k_label<NS, 4, KM>), g, blk, 0, st, b.vox, b.offs, b.nseg, b.total, bm, sets, k);
}

template <int KM>
static void launch_label_km(int nsets, int U, dim3 g, dim3 blk, hipStream_t st, const ts_batch &b, const BinMap &bm,
                            const LabelSets &sets, int k)
{
    switch (nsets) {
    case 1: launch_label_ns<1, KM>(U, g, blk, st, b, bm, sets, k); break;
    case 2: launch_label_ns<2, KM>(U, g, blk, st, b, bm, sets, k); break;
    case 3: launch_label_ns<3, KM>(U, g, blk, st, b, bm, sets, k); break;
    default: launch_label_ns<4, KM>(U, g, blk, st, b, bm, sets, k); break;
    }
}

ts_status launch_label(const ts_batch &b, const BinMap &bm, const LabelSets &sets, int nsets, int k, const Tune &t,
                       hipStream_t st)
{
    if (b.total == 0)
        return TS_OK;
    const int64_t T = (int64_t)t.label_block * 8 * t.label_vecs;
    const int64_t grid = (b.total + T - 1) / T;
    if (grid > 0x7fffffff)
        return fail(TS_ERR_INVALID_ARG, "ts_label: batch too large for one launch");
    const dim3 g((unsigned)grid), blk(t.label_block);
    switch (k) { // as many cut values as thresholds up to 3, else the 16-cut instance
    case 1: launch_label_km<1>(nsets, t.label_vecs, g, blk, st, b, bm, sets, k); break;
    case 2: launch_label_km<2>(nsets, t.label_vecs, g, blk, st, b, bm, sets, k); break;
    case 3: launch_label_km<3>(nsets, t.label_vecs, g, blk, st, b, bm, sets, k); break;
    default: launch_label_km<LABEL_MAX_K>(nsets, t.label_vecs, g, blk, st, b, bm, sets, k); break;
    }
    return check_launch("ts_label");
}

} // namespace ts
