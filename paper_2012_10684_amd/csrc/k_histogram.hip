// k_histogram.hip -- per-problem histograms of gray levels (Thresholding
// section: the histogram of brightness levels is the measurement space; the
// levels come from the linear intensity map of the Pre-processing section).
//
// Design (HBM-bound streaming reduction):
//  * a persistent grid of workgroups splits the flattened voxel stream of the
//    whole batch into equal contiguous ranges, so uneven problems share one
//    launch;
//  * each workgroup keeps a private histogram in LDS with R replicas of every
//    bin, laid out bin-major (bin * R + lane % R).  With R = 32 the 32 lanes
//    of a half-wave always hit 32 distinct banks, so even a bin that takes
//    40 % of all voxels (the clamp bin of a narrow window) never serialises;
//  * voxels are read as 16-byte vectors (8 x int16) from the first 16-byte
//    aligned element of each piece, with a scalar head and tail;
//  * when the range crosses into the next problem, and at the end, the
//    workgroup folds its replicas and adds the non-zero bins to the global
//    histogram with device-scope atomics (integer adds, so the result does
//    not depend on their order).
#include <algorithm>

#include "common.h"
#include "hist_dev.h"

namespace ts {

// Zero n words: the words before the first 16-byte boundary, then 16-byte
// stores, then the last n mod 4 words (p is 4-byte aligned).
__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n)
{
    const int64_t head = min(n, (int64_t)(((16u - ((uintptr_t)p & 15u)) & 15u) >> 2));
    const int64_t nv = (n - head) >> 2;
    uint4 *v = reinterpret_cast<uint4 *>(p + head);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < nv; j += stride)
        v[j] = make_uint4(0u, 0u, 0u, 0u);
    if (i < head)
        p[i] = 0u;
    const int64_t t0 = head + (nv << 2);
    if (i < n - t0)
        p[t0 + i] = 0u;
}

ts_status launch_fill_u32(uint32_t *p, int64_t n, hipStream_t st)
{
    if (n <= 0)
        return TS_OK;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4096, ((n >> 2) + 255) / 256));
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, st, p, n);
    return check_launch("zero fill");
}

template <int R>
__device__ void flush(uint32_t *lds, int L, uint32_t *__restrict__ hist_row)
{
    __syncthreads();
    for (int b = threadIdx.x; b < L; b += blockDim.x) {
        uint32_t s = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s += lds[b * R + r];
            lds[b * R + r] = 0u;
        }
        if (s)
            atomicAdd(&hist_row[b], s);
    }
    __syncthreads();
}

template <int R, int MAP>
__global__ void __launch_bounds__(1024) k_histogram(const int16_t *const *__restrict__ vox,
                                                    const int64_t *__restrict__ offs, int nseg, int64_t total,
                                                    int64_t chunk, BinMap bm, uint32_t *__restrict__ hist)
{
    extern __shared__ uint32_t lds[];
    const int L = bm.L;
    for (int i = threadIdx.x; i < L * R; i += blockDim.x)
        lds[i] = 0u;
    __syncthreads();

    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(total, beg + chunk);
    if (beg >= end)
        return;
    const uint32_t rep = threadIdx.x % R;
    // the segment of the first voxel: an arithmetic guess checked with two
    // offsets in one round trip (a binary search only when it is wrong)
    int s = guess_segment(nseg, total, beg);
    if (!(offs[s] <= beg && beg < offs[s + 1]))
        s = find_segment(offs, nseg, beg);
    int64_t pos = beg;
    while (pos < end) {
        // skip empty problems that start at pos
        while (s + 1 < nseg && offs[s + 1] <= pos)
            ++s;
        const int64_t s0 = offs[s];
        const int64_t s1 = min(offs[s + 1], end);
        const TS_GLOBAL int16_t *base = gp(vox[s]);
        int64_t i0 = pos - s0, i1 = s1 - s0; // local element range [i0, i1)
        // elements before the first 16-byte aligned one
        const uintptr_t a0 = (uintptr_t)(base + i0);
        int64_t head = (int64_t)(((16u - (a0 & 15u)) & 15u) >> 1);
        if (head > i1 - i0)
            head = i1 - i0;
        if (threadIdx.x < head)
            atomicAdd(&lds[bin_of_t<MAP>(base[i0 + threadIdx.x], bm) * R + rep], 1u);
        const int64_t vb = i0 + head;        // first aligned element
        const int64_t nvec = (i1 - vb) >> 3; // whole 8-element vectors
        const TS_GLOBAL v4i *vp = reinterpret_cast<const TS_GLOBAL v4i *>(base + vb);
        const int64_t st = blockDim.x;
        int64_t j = threadIdx.x;
        // groups of four vectors per thread; the next group is in flight
        // while the current one is counted
        bool have = j + 3 * st < nvec;
        v4i a0v = {0, 0, 0, 0}, a1v = a0v, a2v = a0v, a3v = a0v;
        if (have) {
            a0v = __builtin_nontemporal_load(vp + j);
            a1v = __builtin_nontemporal_load(vp + j + st);
            a2v = __builtin_nontemporal_load(vp + j + 2 * st);
            a3v = __builtin_nontemporal_load(vp + j + 3 * st);
        }
        while (have) {
            const int64_t jn = j + 4 * st;
            const bool nxt = jn + 3 * st < nvec;
            v4i b0 = a0v, b1 = a1v, b2 = a2v, b3 = a3v;
            if (nxt) {
                b0 = __builtin_nontemporal_load(vp + jn);
                b1 = __builtin_nontemporal_load(vp + jn + st);
                b2 = __builtin_nontemporal_load(vp + jn + 2 * st);
                b3 = __builtin_nontemporal_load(vp + jn + 3 * st);
            }
            count8<R, MAP>(lds, a0v, bm, rep);
            count8<R, MAP>(lds, a1v, bm, rep);
            count8<R, MAP>(lds, a2v, bm, rep);
            count8<R, MAP>(lds, a3v, bm, rep);
            a0v = b0;
            a1v = b1;
            a2v = b2;
            a3v = b3;
            j = jn;
            have = nxt;
        }
        for (; j < nvec; j += st)
            count8<R, MAP>(lds, __builtin_nontemporal_load(vp + j), bm, rep);
        const int64_t tb = vb + (nvec << 3); // tail elements [tb, i1)
        if (threadIdx.x < i1 - tb)
            atomicAdd(&lds[bin_of_t<MAP>(base[tb + threadIdx.x], bm) * R + rep], 1u);
        pos = s0 + i1;
        flush<R>(lds, L, hist + (int64_t)s * L);
        ++s;
    }
}

template <int R, int MAP>
static void launch_rm(int grid, int block, size_t lds, hipStream_t st, const ts_batch &b, int64_t chunk,
                      const BinMap &bm, uint32_t *hist)
{
    allow_dynamic_lds((const void *)k_histogram<R, MAP>, lds);
    hipLaunchKernelGGL((k_histogram<R, MAP>), dim3(grid), dim3(block), lds, st, b.vox, b.offs, b.nseg, b.total,
                       chunk, bm, hist);
}

template <int R>
static void launch_r(int grid, int block, size_t lds, hipStream_t st, const ts_batch &b, int64_t chunk,
                     const BinMap &bm, uint32_t *hist)
{
    switch (map_kind(bm)) {
    case 0: launch_rm<R, 0>(grid, block, lds, st, b, chunk, bm, hist); break;
    case 1: launch_rm<R, 1>(grid, block, lds, st, b, chunk, bm, hist); break;
    case 2: launch_rm<R, 2>(grid, block, lds, st, b, chunk, bm, hist); break;
    default: launch_rm<R, 3>(grid, block, lds, st, b, chunk, bm, hist); break;
    }
}

ts_status launch_histogram(const ts_batch &b, const BinMap &bm, uint32_t *hist, const Tune &t, hipStream_t st)
{
    const int64_t nh = (int64_t)b.nseg * bm.L;
    {
        ts_status e = launch_fill_u32(hist, nh, st);
        if (e != TS_OK)
            return e;
    }
    if (b.total == 0)
        return TS_OK;
    const int64_t max_wg = (int64_t)device_cu_count() * t.hist_wg_per_cu;
    int64_t grid = std::min<int64_t>(max_wg, (b.total + t.min_chunk - 1) / t.min_chunk);
    if (grid < 1)
        grid = 1;
    int64_t chunk = (b.total + grid - 1) / grid;
    chunk = (chunk + 63) & ~(int64_t)63;
    grid = (b.total + chunk - 1) / chunk;
    const size_t lds = (size_t)bm.L * t.hist_replicas * sizeof(uint32_t);
    switch (t.hist_replicas) {
    case 1: launch_r<1>((int)grid, t.hist_block, lds, st, b, chunk, bm, hist); break;
    case 2: launch_r<2>((int)grid, t.hist_block, lds, st, b, chunk, bm, hist); break;
    case 4: launch_r<4>((int)grid, t.hist_block, lds, st, b, chunk, bm, hist); break;
    case 8: launch_r<8>((int)grid, t.hist_block, lds, st, b, chunk, bm, hist); break;
    case 16: launch_r<16>((int)grid, t.hist_block, lds, st, b, chunk, bm, hist); break;
    default: launch_r<32>((int)grid, t.hist_block, lds, st, b, chunk, bm, hist); break;
    }
    return check_launch("ts_histogram");
}

} // namespace ts
