// k_2d.hip -- the paper's two-dimensional Tsallis thresholding (Tsallis-
// entropy section, the 2D form): the 3x3 average image g = floor(mean of the
// 3x3 gray levels, edge pixels repeated), the 2D histogram h(i, j) of
// (gray level, average gray level), the classes {i <= t, j <= s} and
// {i > t, j > s} (quadrants 1 and 3) and the arg max over (t, s) of the
// pseudo-additive objective.  Only t thresholds the image (ts_label, k = 1).
//
// k_hist2d: one workgroup per band of rows of one image.  The gray levels of
// three consecutive rows sit in an LDS ring, so each pixel's 3x3 sum is a
// column sum of the ring plus its two neighbours.  CT neighbourhoods are
// smooth, so (f, g) stays near the diagonal: cells with |f - g| <= BAND go to
// an LDS histogram of the band, the two clamp corners (0, 0) and (L-1, L-1)
// to per-lane LDS counters (under a narrow window they take a large share of
// the pixels), and the rest straight to the global 2D histogram with
// atomics.  The LDS atomic is issued for every pixel (cells outside the
// LDS band land on a per-lane dummy), so its address, not a branch, selects
// the target.
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

constexpr int H2_THREADS = 256;
constexpr int H2_BAND = 31;       // |f - g| <= BAND counted in LDS
constexpr int H2_MAX_W = 4096;    // row length held in the LDS ring
constexpr int H2_MAX_L = 256;     // 2D histograms up to 256 x 256
constexpr int S2_THREADS = 256;   // one thread per column s (L <= 256)

// ------------------------------------------------------------------ histogram

template <int MAP>
__global__ void __launch_bounds__(H2_THREADS) k_hist2d(const int16_t *const *__restrict__ vox, int nseg, int H,
                                                       int W, int rows_per_wg, BinMap bm, uint32_t *__restrict__ hist)
{
    extern __shared__ uint32_t sm[];
    const int L = bm.L;
    const int BW = 2 * H2_BAND + 1;
    uint32_t *band = sm;                                  // [L * BW]
    uint32_t *hot = band + L * BW;                        // [2 * 64]: (0,0), (L-1,L-1) per lane
    uint32_t *dummy = hot + 128;                          // [64]
    int *ring = reinterpret_cast<int *>(dummy + 64);      // [3 * W] gray levels of rows r-1, r, r+1
    const int lane = threadIdx.x & 63;
    const int bands = (H + rows_per_wg - 1) / rows_per_wg;
    const int s = blockIdx.x / bands;
    const int r0 = (blockIdx.x % bands) * rows_per_wg;
    const int r1 = min(H, r0 + rows_per_wg);
    const TS_GLOBAL int16_t *img = gp(vox[s]);
    uint32_t *hs = hist + (int64_t)s * L * L;
    for (int i = threadIdx.x; i < L * BW + 192; i += blockDim.x)
        sm[i] = 0u;
    // ring slot of image row y: y mod 3 (rows r0-1 .. r1 are loaded in order)
    auto load_row = [&](int y) {
        const int yc = min(max(y, 0), H - 1);
        int *dst = ring + ((y + 3) % 3) * W;
        for (int x = threadIdx.x; x < W; x += blockDim.x)
            dst[x] = bin_of_t<MAP>(img[(int64_t)yc * W + x], bm);
    };
    load_row(r0 - 1);
    load_row(r0);
    for (int r = r0; r < r1; ++r) {
        load_row(r + 1);
        __syncthreads();
        const int *up = ring + ((r + 2) % 3) * W, *cu = ring + ((r + 3) % 3) * W, *dn = ring + ((r + 4) % 3) * W;
        for (int x = threadIdx.x; x < W; x += blockDim.x) {
            const int xl = max(x - 1, 0), xr = min(x + 1, W - 1);
            const int sum = up[xl] + up[x] + up[xr] + cu[xl] + cu[x] + cu[xr] + dn[xl] + dn[x] + dn[xr];
            const int f = cu[x];
            const int g = (int)((uint32_t)sum / 9u);
            const int d = g - f;
            const bool inb = d >= -H2_BAND && d <= H2_BAND;
            uint32_t *a = inb ? band + f * BW + (d + H2_BAND) : dummy + lane;
            if (f == g && (f == 0 || f == L - 1))
                a = hot + (f == 0 ? 0 : 64) + lane;
            atomicAdd(a, 1u);
            if (!inb) // rare: far from the diagonal
                atomicAdd(&hs[(int64_t)f * L + g], 1u);
        }
        __syncthreads(); // the ring slot of row r-1 is reloaded next
    }
    // fold the clamp-corner counters into the band, then add the band
    if (threadIdx.x < 2) {
        uint32_t c = 0;
        for (int i = 0; i < 64; ++i)
            c += hot[threadIdx.x * 64 + i];
        const int f = threadIdx.x == 0 ? 0 : L - 1;
        atomicAdd(&band[f * BW + H2_BAND], c);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L * BW; i += blockDim.x) {
        const uint32_t c = band[i];
        if (c) {
            const int f = i / BW, g = f + i % BW - H2_BAND;
            atomicAdd(&hs[(int64_t)f * L + g], c);
        }
    }
}

size_t hist2d_lds_bytes(int L, int W)
{
    return ((size_t)L * (2 * H2_BAND + 1) + 192) * sizeof(uint32_t) + (size_t)3 * W * sizeof(int);
}

ts_status launch_hist2d(const ts_batch &b, int H, int W, const BinMap &bm, uint32_t *hist, hipStream_t st)
{
    if (W > H2_MAX_W || bm.L > H2_MAX_L)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: width or nbins beyond the LDS layout");
    const int64_t n = (int64_t)b.nseg * bm.L * bm.L;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, st, hist,
                       n);
    const int rows = std::max(1, std::min(H, (int)((int64_t)65536 / std::max(W, 1)))); // ~64k pixels per workgroup
    const int bands = (H + rows - 1) / rows;
    const size_t lds = hist2d_lds_bytes(bm.L, W);
    const dim3 g((unsigned)((int64_t)b.nseg * bands)), blk(H2_THREADS);
    switch (map_kind(bm)) {
    case 0:
        (void)hipFuncSetAttribute((const void *)k_hist2d<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_hist2d<0>, g, blk, lds, st, b.vox, b.nseg, H, W, rows, bm, hist);
        break;
    case 1:
        (void)hipFuncSetAttribute((const void *)k_hist2d<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_hist2d<1>, g, blk, lds, st, b.vox, b.nseg, H, W, rows, bm, hist);
        break;
    case 2:
        (void)hipFuncSetAttribute((const void *)k_hist2d<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_hist2d<2>, g, blk, lds, st, b.vox, b.nseg, H, W, rows, bm, hist);
        break;
    default:
        (void)hipFuncSetAttribute((const void *)k_hist2d<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_hist2d<3>, g, blk, lds, st, b.vox, b.nseg, H, W, rows, bm, hist);
        break;
    }
    return check_launch("ts_histogram2d");
}

// ------------------------------------------------------------------ search

struct Q2List {
    double q[TS_MAX_Q];
};

// Row prefix (dir = +1) or suffix (dir = -1) along s of one 2D histogram row
// for the thread's column s = threadIdx.x, in a fixed order: the exact
// integer count c and the FP64 sum of p^q (or p ln p), where an empty cell
// repeats the value of the nearest occupied cell on the side it is summed
// from.  ws* hold one entry per wavefront (+1).
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

template <int DIR>
__device__ __forceinline__ RowSums row_scan(const uint32_t *__restrict__ hrow, int L, double N, double q,
                                            uint64_t *wu, double *wd, int *wi, double *rq)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // position along the scan direction
    const int s = threadIdx.x;
    const bool in = s < L;
    const uint32_t c = in ? hrow[s] : 0u;
    const double v = in ? pterm(c, N, q) : 0.0;
    // the scan index: ascending s for prefixes, descending for suffixes
    // (lanes are reversed for suffixes so that every scan runs over lanes in
    // ascending order)
    const int pos = DIR > 0 ? s : (blockDim.x - 1 - s);
    // exchange through LDS so that lane order is scan order
    __shared__ uint32_t xc[S2_THREADS];
    __shared__ double xv[S2_THREADS];
    xc[pos] = c;
    xv[pos] = v;
    __syncthreads();
    const uint32_t mc = xc[threadIdx.x];
    const double mv = xv[threadIdx.x];
    __syncthreads();
    uint64_t ic = mc;
    double iv = mv;
    int occ = mc ? (int)threadIdx.x : -1;
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
    if (lane == 63) {
        wu[w] = ic;
        wd[w] = iv;
        wi[w] = occ;
    }
    __syncthreads();
    if (threadIdx.x == 0) { // sequential over the wavefront totals
        uint64_t rc = 0;
        double rv = 0.0;
        int ro = -1;
        for (int i = 0; i < nw; ++i) {
            const uint64_t a = wu[i];
            const double b = wd[i];
            const int o2 = wi[i];
            wu[i] = rc;
            wd[i] = rv;
            wi[i] = ro;
            rc += a;
            rv = rv + b;
            ro = max(ro, o2);
        }
    }
    __syncthreads();
    ic += wu[w];
    iv = wd[w] + iv;
    occ = max(occ, wi[w]);
    // empty cells take the sum at the last occupied scan position
    rq[threadIdx.x] = iv;
    __syncthreads();
    const double fixed = occ < 0 ? 0.0 : rq[occ];
    __syncthreads();
    // back to column order
    __shared__ uint64_t yc[S2_THREADS];
    __shared__ double yv[S2_THREADS];
    yc[threadIdx.x] = ic;
    yv[threadIdx.x] = fixed;
    __syncthreads();
    RowSums r;
    r.c = yc[pos];
    r.q = yv[pos];
    __syncthreads();
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
    __shared__ double wd[S2_THREADS / 64 + 1];
    __shared__ int wi[S2_THREADS / 64 + 1];
    __shared__ double rq[S2_THREADS];
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
    // class 2, bottom-up: B(t, s) = sums over {i >= t, j >= s}
    uint64_t bcnt = 0;
    double bq = 0.0;
    for (int t = L - 1; t >= 1; --t) {
        const RowSums r = row_scan<-1>(h + (int64_t)t * L, L, Nd, q, wu, wd, wi, rq);
        bcnt += r.c;
        bq = bq + r.q;
        if (s < L)
            lbp[(int64_t)t * L + s] = class_term2(bcnt, bq, Nd, q, sgn, hmax);
    }
    // class 1, top-down: A(t, s) = sums over {i <= t, j <= s}; pair (t, s)
    // adds class 2 at (t+1, s+1)
    uint64_t acnt = 0;
    double aq = 0.0;
    double best = -INFINITY;
    long long code = 0x7fffffffffffffffLL;
    for (int t = 0; t <= L - 2; ++t) {
        const RowSums r = row_scan<1>(h + (int64_t)t * L, L, Nd, q, wu, wd, wi, rq);
        acnt += r.c;
        aq = aq + r.q;
        if (s <= L - 2) {
            const double la = class_term2(acnt, aq, Nd, q, sgn, hmax);
            const double lbv = lbp[(int64_t)(t + 1) * L + s + 1];
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
