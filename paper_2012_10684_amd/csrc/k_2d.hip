// k_2d.hip -- the paper's two-dimensional Tsallis thresholding (Tsallis-
// entropy section, the 2D form): the 3x3 average image g = floor(mean of the
// 3x3 gray levels, edge pixels repeated), the 2D histogram h(i, j) of
// (gray level, average gray level), the classes {i <= t, j <= s} and
// {i > t, j > s} (quadrants 1 and 3) and the arg max over (t, s) of the
// pseudo-additive objective.  Only t thresholds the image (ts_label, k = 1).
//
// k_hist2d: one workgroup per band of at most 65535 pixels of one image, in
// chunks of about 4096 pixels: the 8-bit gray levels of a chunk's rows and
// its two halo rows are staged in LDS in one pass, so each pixel's 3x3 sum
// reads LDS only.  The whole L x L plane is counted in LDS as 16-bit cells
// (two per word; 128 KiB at L = 256), which cannot overflow within the
// band; the two clamp corners (0, 0) and (L-1, L-1), which take a large share
// of the pixels under a narrow window, count in per-lane LDS words instead of
// one hot address.  At the end the non-zero cells are added to the global 2D
// histogram.
//
// k_search2d: one workgroup per (q index, problem), one thread per column s.
// Class 2 sums are accumulated bottom-up over rows and its log term
// sgn(1-q) (ln Q_2 - q ln w_2) is stored per cell in the workspace (FP64);
// then class 1 sums are accumulated top-down, the stored class 2 term of
// (t+1, s+1) is added and the first best pair is kept (t outermost).  Row
// sums along s are fixed-order block scans, and an empty cell takes the row
// sum of the last (first, for suffixes) occupied cell, so a whole empty
// column or row leaves every class sum unchanged bit for bit and the pairs
// it separates tie exactly.  FP64 throughout: the reported pair is the FP64
// arg max.  q = 1 is the Shannon limit, as in the one-dimensional search.
#include <math.h>

#include <algorithm>

#include "common.h"

namespace ts {

constexpr int H2_THREADS = 1024;
constexpr int H2_MAX_W = 4096;    // row length held in the LDS ring
constexpr int H2_MAX_L = 256;     // 2D histograms up to 256 x 256
constexpr int S2_THREADS = 256;   // one thread per column s (L <= 256)

// ------------------------------------------------------------------ histogram

template <int MAP>
__global__ void __launch_bounds__(H2_THREADS) k_hist2d(const int16_t *const *__restrict__ vox, int nseg, int H,
                                                       int W, int rows_per_wg, int chunk_rows, BinMap bm,
                                                       uint32_t *__restrict__ hist)
{
    extern __shared__ uint32_t sm[];
    const int L = bm.L;
    const int nw2 = (L * L + 1) / 2;                       // packed 16-bit cells
    uint32_t *plane = sm;                                  // [nw2]: cell c in half (c & 1) of word c >> 1
    uint32_t *hot = plane + nw2;                           // [2 * 64]: (0,0), (L-1,L-1) per lane
    uint8_t *rows = reinterpret_cast<uint8_t *>(hot + 128); // [(chunk_rows + 2) * W] gray levels (L <= 256)
    const int lane = threadIdx.x & 63;
    const int bands = (H + rows_per_wg - 1) / rows_per_wg;
    const int s = blockIdx.x / bands;
    const int r0 = (blockIdx.x % bands) * rows_per_wg;
    const int r1 = min(H, r0 + rows_per_wg);
    const TS_GLOBAL int16_t *img = gp(vox[s]);
    uint32_t *hs = hist + (int64_t)s * L * L;
    for (int i = threadIdx.x; i < nw2 + 128; i += blockDim.x)
        sm[i] = 0u;
    // chunks of chunk_rows image rows: the gray levels of rows r-1 .. r+n
    // (edge rows repeated) are staged in LDS in one pass, then every pixel of
    // rows r .. r+n-1 is counted
    for (int r = r0; r < r1; r += chunk_rows) {
        const int n = min(chunk_rows, r1 - r);
        __syncthreads(); // previous chunk fully counted
        for (int i = threadIdx.x; i < (n + 2) * W; i += blockDim.x) {
            const int k = i / W, x = i - k * W;
            const int y = min(max(r - 1 + k, 0), H - 1);
            rows[i] = (uint8_t)bin_of_t<MAP>(img[(int64_t)y * W + x], bm);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n * W; i += blockDim.x) {
            const int k = i / W + 1, x = i - (k - 1) * W;
            const int xl = max(x - 1, 0), xr = min(x + 1, W - 1);
            const uint8_t *up = rows + (k - 1) * W, *cu = rows + k * W, *dn = rows + (k + 1) * W;
            const int sum = (int)up[xl] + up[x] + up[xr] + cu[xl] + cu[x] + cu[xr] + dn[xl] + dn[x] + dn[xr];
            const int f = cu[x];
            const int g = (int)((uint32_t)sum / 9u);
            const int c = f * L + g;
            const bool corner = f == g && (f == 0 || f == L - 1);
            uint32_t *a = corner ? hot + (f == 0 ? 0 : 64) + lane : plane + (c >> 1);
            atomicAdd(a, corner ? 1u : (1u << ((c & 1) << 4)));
        }
    }
    __syncthreads();
    // every cell count is at most the workgroup's pixel count (<= 65535): no
    // half-word overflows.  Add the non-zero cells to the global histogram.
    for (int i = threadIdx.x; i < nw2; i += blockDim.x) {
        uint32_t w2 = plane[i];
        if (i == 0 || i == (L * L - 1) >> 1) { // the clamp corners' per-lane counters
            for (int j = 0; j < 2; ++j) {
                const int cell = j == 0 ? 0 : L * L - 1;
                if ((cell >> 1) != i)
                    continue;
                uint32_t cc = 0;
                for (int l = 0; l < 64; ++l)
                    cc += hot[j * 64 + l];
                atomicAdd(&hs[cell], cc); // global directly: the sum may exceed 16 bits
            }
        }
        if (w2 & 0xffffu)
            atomicAdd(&hs[2 * i], w2 & 0xffffu);
        if ((w2 >> 16) && 2 * i + 1 < L * L)
            atomicAdd(&hs[2 * i + 1], w2 >> 16);
    }
}

static int hist2d_chunk_rows(int W) { return std::max(1, 4096 / W); }

size_t hist2d_lds_bytes(int L, int W)
{
    return ((size_t)(L * L + 1) / 2 + 128) * sizeof(uint32_t) + (size_t)(hist2d_chunk_rows(W) + 2) * W;
}

ts_status launch_hist2d(const ts_batch &b, int H, int W, const BinMap &bm, uint32_t *hist, hipStream_t st)
{
    if (W > H2_MAX_W || bm.L > H2_MAX_L)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: width or nbins beyond the LDS layout");
    const int64_t n = (int64_t)b.nseg * bm.L * bm.L;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, st, hist,
                       n);
    // at most 65535 pixels per workgroup (16-bit cell counters in LDS)
    const int rows = std::max(1, std::min(H, 65535 / std::max(W, 1)));
    const int bands = (H + rows - 1) / rows;
    const int chunk = hist2d_chunk_rows(W);
    const size_t lds = hist2d_lds_bytes(bm.L, W);
    const dim3 g((unsigned)((int64_t)b.nseg * bands)), blk(H2_THREADS);
#define TS_H2(M)                                                                                                    \
    (void)hipFuncSetAttribute((const void *)k_hist2d<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
    hipLaunchKernelGGL(k_hist2d<M>, g, blk, lds, st, b.vox, b.nseg, H, W, rows, chunk, bm, hist)
    switch (map_kind(bm)) {
    case 0: TS_H2(0); break;
    case 1: TS_H2(1); break;
    case 2: TS_H2(2); break;
    default: TS_H2(3); break;
    }
#undef TS_H2
    return check_launch("ts_histogram2d");
}

// ------------------------------------------------------------------ search

struct Q2List {
    double q[TS_MAX_Q];
};

// Row prefix (DIR = +1) or suffix (DIR = -1) along s of one 2D histogram
// row, in a fixed order: scan position p = threadIdx.x is column p (prefix)
// or column L-1-p (suffix); c is that column's count, loaded by the caller.
// Returns the exact integer count sum and the FP64 sum of p^q (or p ln p) up
// to the position, where an empty cell repeats the value of the nearest
// occupied cell before it in scan order.  ws* hold one entry per wavefront.
struct RowSums {
    uint64_t c;
    double q;
};

__device__ __forceinline__ double pterm(uint32_t c, double N, double q)
{
    if (!c)
        return 0.0;
    const double p = (double)c / N;
    return q == 1.0 ? p * log(p) : pow(p, q);
}

// Per-wavefront totals of one row scan: count, FP64 sum, last occupied scan
// position of the wavefront (or -1) and the inclusive sum there.
struct WaveTot {
    uint64_t c;
    double v;
    int occ;
    double occv;
};

__device__ __forceinline__ RowSums row_scan(uint32_t c, double pv, WaveTot *wt)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t ic = c;
    double iv = pv; // p^q (or p ln p) of this cell
    int occ = c ? (int)threadIdx.x : -1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t tc = __shfl_up(ic, o, 64);
        const double tv = __shfl_up(iv, o, 64);
        const int to = __shfl_up(occ, o, 64);
        if (lane >= o) {
            ic += tc;
            iv = tv + iv;
            occ = max(occ, to);
        }
    }
    // inclusive sum at this wavefront's last occupied position so far
    const double ivocc = __shfl(iv, occ < 0 ? 0 : (occ & 63), 64);
    if (lane == 63) // ivocc of lane 63: the sum at the wavefront's last occupied position
        wt[w] = WaveTot{ic, iv, occ, ivocc};
    __syncthreads();
    // totals of the earlier wavefronts, combined in order
    uint64_t bc = 0;
    double bv = 0.0;
    int bo = -1;
    double bov = 0.0;
    for (int i = 0; i < w; ++i) {
        const WaveTot t = wt[i];
        bc += t.c;
        if (t.occ >= 0) {
            bo = t.occ;
            bov = bv + t.occv; // the sum at that position, as its own wavefront formed it after the base
        }
        bv = bv + t.v;
    }
    RowSums r;
    r.c = bc + ic;
    // empty cells take the sum at the last occupied position in scan order
    if (occ >= 0)
        r.q = bv + ivocc;
    else
        r.q = bo >= 0 ? bov : 0.0;
    return r;
}

// sgn(1-q) (ln Q - q ln w) for Tsallis, ln w - E / w for q = 1; -inf when
// the class is empty; clamped to [0, hmax]
__device__ __forceinline__ double class_term2(uint64_t c, double sumq, double N, double q, double sgn, double hmax)
{
    if (c == 0)
        return -INFINITY;
    const double w = (double)c / N;
    const double h = sgn == 0.0 ? log(w) - sumq / w : sgn * (log(sumq) - q * log(w));
    return fmin(fmax(h, 0.0), hmax);
}

__global__ void __launch_bounds__(S2_THREADS) k_search2d(const uint32_t *__restrict__ hist, int nseg, int L, Q2List ql,
                                                         double *__restrict__ lb, int32_t *__restrict__ thr,
                                                         double *__restrict__ obj, int32_t *__restrict__ status)
{
    __shared__ uint64_t wu[S2_THREADS / 64 + 1];
    __shared__ WaveTot wt[2][S2_THREADS / 64]; // alternate rows: one barrier per row scan
    __shared__ double br[S2_THREADS / 64];
    __shared__ long long bc[S2_THREADS / 64];
    const int prob = blockIdx.x, s0 = prob % nseg, j = prob / nseg;
    const double q = ql.q[j];
    const double sgn = q == 1.0 ? 0.0 : (q < 1.0 ? 1.0 : -1.0);
    const double hmax = (q == 1.0 ? 1.0 : fabs(1.0 - q)) * 2.0 * log((double)L); // a class holds at most L^2 cells
    const uint32_t *h = hist + (int64_t)s0 * L * L;
    double *lbp = lb + (int64_t)prob * L * L;
    const int s = threadIdx.x;
    // N
    uint64_t n = 0;
    for (int i = threadIdx.x; i < L * L; i += blockDim.x)
        n += h[i];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0)
        wu[threadIdx.x >> 6] = n;
    __syncthreads();
    uint64_t N = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
        N += wu[i];
    __syncthreads();
    // thr is [nq][2][nseg]: t at row 0, s at row 1 of this q
    int32_t *thr_t = thr + (int64_t)(2 * j) * nseg + s0, *thr_s = thr_t + nseg;
    if (N == 0) {
        if (threadIdx.x == 0) {
            *thr_t = *thr_s = -1;
            obj[prob] = NAN;
            status[prob] = TS_PROBLEM_EMPTY;
        }
        return;
    }
    const double Nd = (double)N;
    // class 2, bottom-up: B(t, s) = sums over {i >= t, j >= s}; thread p
    // holds column L-1-p (suffix order); each row's counts are loaded one
    // row ahead
    const int cb = L - 1 - s; // this thread's column in the suffix pass
    uint64_t bcnt = 0;
    double bq = 0.0;
    uint32_t cn = (s < L) ? h[(int64_t)(L - 1) * L + cb] : 0u;
    for (int t = L - 1; t >= 1; --t) {
        const uint32_t c = cn;
        if (t > 1)
            cn = (s < L) ? h[(int64_t)(t - 1) * L + cb] : 0u;
        const RowSums r = row_scan(c, pterm(c, Nd, q), wt[t & 1]);
        bcnt += r.c;
        bq = bq + r.q;
        if (s < L)
            lbp[(int64_t)t * L + cb] = class_term2(bcnt, bq, Nd, q, sgn, hmax);
    }
    // class 1, top-down: A(t, s) = sums over {i <= t, j <= s}, thread s holds
    // column s; the pair (t, s) adds class 2 at (t+1, s+1), written above by
    // another thread of the workgroup
    __syncthreads();
    uint64_t acnt = 0;
    double aq = 0.0;
    double best = -INFINITY;
    long long code = 0x7fffffffffffffffLL;
    cn = (s < L) ? h[s] : 0u;
    for (int t = 0; t <= L - 2; ++t) {
        const uint32_t c = cn;
        cn = (s < L) ? h[(int64_t)(t + 1) * L + s] : 0u;
        const double lbv = s <= L - 2 ? lbp[(int64_t)(t + 1) * L + s + 1] : -INFINITY;
        const RowSums r = row_scan(c, pterm(c, Nd, q), wt[t & 1]);
        acnt += r.c;
        aq = aq + r.q;
        if (s <= L - 2) {
            const double la = class_term2(acnt, aq, Nd, q, sgn, hmax);
            const double lam = la + lbv;
            const long long cd = ((long long)t << 12) | s;
            if (lam > -INFINITY && (lam > best || (lam == best && cd < code))) {
                best = lam;
                code = cd;
            }
        }
    }
    // first best pair of the workgroup
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double b2 = __shfl_xor(best, o, 64);
        const long long c2 = __shfl_xor(code, o, 64);
        if (b2 > best || (b2 == best && c2 < code)) {
            best = b2;
            code = c2;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        br[threadIdx.x >> 6] = best;
        bc[threadIdx.x >> 6] = code;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
            if (br[i] > best || (br[i] == best && bc[i] < code)) {
                best = br[i];
                code = bc[i];
            }
        if (!(best > -INFINITY)) {
            *thr_t = *thr_s = -1;
            obj[prob] = NAN;
            status[prob] = TS_PROBLEM_DEGENERATE;
        } else {
            *thr_t = (int32_t)(code >> 12);
            *thr_s = (int32_t)(code & 4095);
            obj[prob] = sgn == 0.0 ? best : expm1(sgn * best) / (1.0 - q);
            status[prob] = TS_PROBLEM_OK;
        }
    }
}

size_t search2d_workspace_bytes(int nprob, int L) { return (size_t)nprob * L * L * sizeof(double); }

ts_status launch_search2d(const uint32_t *hist, int nseg, int L, int nq, const double *q, void *ws, int32_t *thr,
                          double *obj, int32_t *status, hipStream_t st)
{
    Q2List ql;
    for (int i = 0; i < TS_MAX_Q; ++i)
        ql.q[i] = q[i < nq ? i : 0];
    hipLaunchKernelGGL(k_search2d, dim3((unsigned)(nseg * nq)), dim3(S2_THREADS), 0, st, hist, nseg, L, ql,
                       (double *)ws, thr, obj, status);
    return check_launch("ts_threshold_search2d");
}

} // namespace ts
