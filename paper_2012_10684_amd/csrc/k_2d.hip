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
// k_search2d: one workgroup of four wavefronts per (q index, problem); the
// rows holding counts are split into four blocks, one per wavefront, four
// columns per lane.  Class 2 sums are accumulated bottom-up over rows and
// class 1 sums top-down; a wavefront starts its block from the carried sums
// of the blocks before it in that direction (each block's column totals,
// summed along s, exchanged through LDS), so the four walk their rows at
// once.  FP32 keys of every pair, then an FP64 re-check of the rows whose
// best key is within the keys' error bound of the maximum, from the same
// sums; the first best FP64 pair wins (t outermost).  Sums along s are
// fixed-order scans, and an empty cell (or an empty column of a block's
// totals) takes the sum of the last occupied one, so a whole empty column or
// row leaves every class sum unchanged bit for bit and the pairs it
// separates tie exactly.  q = 1 is the Shannon limit, as in the
// one-dimensional search.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace ts {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int H2_THREADS = 1024;
constexpr int H2_MAX_W = 4096;    // row length held in the LDS ring
constexpr int H2_MAX_L = 256;     // 2D histograms up to 256 x 256
constexpr int H2_LDS = 160 * 1024; // LDS of one workgroup: the plane (128 KiB at L = 256) and staged rows
constexpr int S2_WAVES = 4;       // wavefronts per (q, image), each a block of the rows
constexpr int S2_THREADS = 64 * S2_WAVES;
constexpr int S2_CPL = 4;         // columns per lane (L <= 256)
constexpr int S2_TAB = 2048;      // p^q (or p ln p) of counts below this from an LDS table
constexpr int S2_RING = 3;        // rows of counts in flight ahead of the row being summed

// ------------------------------------------------------------------ histogram

// LDS layout of k_hist2d: the packed plane, the per-lane corner counters,
// then the staged gray levels (16-byte aligned).
__host__ __device__ inline int hist2d_rows_offset(int L) { return (((L * L + 1) / 2 + 128) * 4 + 15) & ~15; }

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
    uint8_t *rows = reinterpret_cast<uint8_t *>(sm) + hist2d_rows_offset(L); // [(chunk_rows + 2) * W]
    const int lane = threadIdx.x & 63;
    const int bands = (H + rows_per_wg - 1) / rows_per_wg;
    const int s = blockIdx.x / bands;
    const int r0 = (blockIdx.x % bands) * rows_per_wg;
    const int r1 = min(H, r0 + rows_per_wg);
    const TS_GLOBAL int16_t *img = gp(vox[s]);
    uint32_t *hs = hist + (int64_t)s * L * L;
    const bool vec = (W % 8) == 0 && ((uintptr_t)img & 15) == 0;
    for (int i = threadIdx.x; i < nw2 + 128; i += blockDim.x)
        sm[i] = 0u;
    // one count: (f, g) = (gray level, floor of the 3x3 mean); the clamp
    // corners count in per-lane words, every other cell in its half-word
    auto count = [&](int f, int sum) {
        const int g = (int)((uint32_t)sum / 9u);
        const int c = f * L + g;
        const bool corner = f == g && (f == 0 || f == L - 1);
        uint32_t *a = corner ? hot + (f == 0 ? 0 : 64) + lane : plane + (c >> 1);
        atomicAdd(a, corner ? 1u : (1u << ((c & 1) << 4)));
    };
    // chunks of chunk_rows image rows: the gray levels of rows r-1 .. r+n
    // (edge rows repeated) are staged in LDS in one pass, then every pixel of
    // rows r .. r+n-1 is counted
    for (int r = r0; r < r1; r += chunk_rows) {
        const int n = min(chunk_rows, r1 - r);
        __syncthreads(); // previous chunk fully counted
        if (vec) { // 8 pixels per 16-byte load, 8 gray levels per 8-byte LDS store
            const int nv = (n + 2) * W / 8;
            for (int i = threadIdx.x; i < nv; i += blockDim.x) {
                const int e = i * 8, k = e / W, x = e - k * W;
                const int y = min(max(r - 1 + k, 0), H - 1);
                const v4i v = *reinterpret_cast<const TS_GLOBAL v4i *>(img + (int64_t)y * W + x);
                const uint32_t w4[4] = {(uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2], (uint32_t)v[3]};
                uint32_t b[2] = {0u, 0u};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int16_t h16 = (int16_t)(w4[j >> 1] >> ((j & 1) * 16));
                    b[j >> 2] |= (uint32_t)bin_of_t<MAP>(h16, bm) << ((j & 3) * 8);
                }
                *reinterpret_cast<uint2 *>(rows + e) = make_uint2(b[0], b[1]);
            }
        } else {
            for (int i = threadIdx.x; i < (n + 2) * W; i += blockDim.x) {
                const int k = i / W, x = i - k * W;
                const int y = min(max(r - 1 + k, 0), H - 1);
                rows[i] = (uint8_t)bin_of_t<MAP>(img[(int64_t)y * W + x], bm);
            }
        }
        __syncthreads();
        if ((W & 3) == 0) { // 4 pixels per thread: one aligned word and its two neighbours per row
            const int n4 = n * W / 4;
            for (int i = threadIdx.x; i < n4; i += blockDim.x) {
                const int e = i * 4, k = e / W + 1, x = e - (k - 1) * W;
                int hsum[3][4];
                int fcen[4];
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const uint8_t *row = rows + (k - 1 + dy) * W;
                    const uint32_t wd = *reinterpret_cast<const uint32_t *>(row + x);
                    int b[6];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        b[j + 1] = (wd >> (8 * j)) & 0xff;
                    b[0] = x > 0 ? row[x - 1] : b[1];          // edge pixel repeated
                    b[5] = x + 4 < W ? row[x + 4] : b[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        hsum[dy][j] = b[j] + b[j + 1] + b[j + 2];
                    if (dy == 1) {
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            fcen[j] = b[j + 1];
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    count(fcen[j], hsum[0][j] + hsum[1][j] + hsum[2][j]);
            }
        } else {
            for (int i = threadIdx.x; i < n * W; i += blockDim.x) {
                const int k = i / W + 1, x = i - (k - 1) * W;
                const int xl = max(x - 1, 0), xr = min(x + 1, W - 1);
                const uint8_t *up = rows + (k - 1) * W, *cu = rows + k * W, *dn = rows + (k + 1) * W;
                count(cu[x], (int)up[xl] + up[x] + up[xr] + cu[xl] + cu[x] + cu[xr] + dn[xl] + dn[x] + dn[xr]);
            }
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

// Band and chunk sizes: bands of at most 65535 pixels (16-bit cells),
// balanced over the image's rows; chunks as large as the LDS left beside the
// plane allows, balanced over the band.
struct Hist2dShape {
    int rows_per_wg, chunk_rows;
    size_t lds;
};

static Hist2dShape hist2d_shape(int L, int H, int W)
{
    Hist2dShape sh;
    const int max_rows = std::max(1, std::min(H, 65535 / std::max(W, 1)));
    const int bands = (H + max_rows - 1) / max_rows;
    sh.rows_per_wg = (H + bands - 1) / bands;
    const int base = hist2d_rows_offset(L);
    const int fit = std::max(3, (H2_LDS - base) / std::max(W, 1)); // staged rows that fit (>= 3 by the launch check)
    int chunk = std::max(1, std::min(fit - 2, sh.rows_per_wg));
    const int nch = (sh.rows_per_wg + chunk - 1) / chunk;
    chunk = (sh.rows_per_wg + nch - 1) / nch;
    sh.chunk_rows = chunk;
    sh.lds = (size_t)base + (size_t)(chunk + 2) * W;
    return sh;
}

size_t hist2d_lds_bytes(int L, int H, int W) { return hist2d_shape(L, H, W).lds; }

ts_status launch_hist2d(const ts_batch &b, int H, int W, const BinMap &bm, uint32_t *hist, hipStream_t st)
{
    if (W > H2_MAX_W || bm.L > H2_MAX_L)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: width or nbins beyond the LDS layout");
    const int64_t n = (int64_t)b.nseg * bm.L * bm.L;
    {
        ts_status e = launch_fill_u32(hist, n, st);
        if (e != TS_OK)
            return e;
    }
    const Hist2dShape sh = hist2d_shape(bm.L, H, W);
    const int rows = sh.rows_per_wg, chunk = sh.chunk_rows;
    const size_t lds = sh.lds;
    const int bands = (H + rows - 1) / rows;
    const dim3 g((unsigned)((int64_t)b.nseg * bands)), blk(H2_THREADS);
#define TS_H2(M)                                                                                                    \
    allow_dynamic_lds((const void *)k_hist2d<M>, lds);                                                            \
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

// With p_ij = c_ij / N the class term sgn(1-q) (ln Q - q ln w) equals
// sgn(1-q) (ln sum c^q - q ln C) for a class of C pixels, and the Shannon
// term ln w - E / w equals ln C - (sum c ln c) / C: N cancels, so the search
// works on raw counts.  cterm(c) is c^q (c ln c for q = 1), 0 for c = 0.
__device__ __forceinline__ double cterm(uint32_t c, double q)
{
    if (!c)
        return 0.0;
    const double x = (double)c;
    return q == 1.0 ? x * log(x) : pow(x, q);
}

// out of line for the rare counts past the table (small code in the row loops)
__device__ __noinline__ double cterm_big(uint32_t c, double q) { return cterm(c, q); }

// Cross-lane moves within the wavefront (DPP): lanes without a source, or in
// rows masked off, receive 0, the identity of the sums below.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    const uint32_t lo = dpp32<CTRL, ROWS>((uint32_t)v), hi = dpp32<CTRL, ROWS>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dppv(T v)
{
    if constexpr (std::is_same<T, double>::value)
        return __longlong_as_double((long long)dpp64<CTRL, ROWS>((uint64_t)__double_as_longlong(v)));
    else if constexpr (sizeof(T) == 4)
        return (T)dpp32<CTRL, ROWS>((uint32_t)v);
    else
        return (T)dpp64<CTRL, ROWS>((uint64_t)v);
}

// Exclusive sum over the lanes of the wavefront in a fixed order: a
// Hillis-Steele scan within each row of 16 lanes, then the rows carried by
// broadcasts of lanes 15 and 31, then a shift by one lane.
template <typename T>
__device__ __forceinline__ T wave_excl_sum(T v)
{
    v = v + dppv<0x111, 0xf>(v); // row_shr:1
    v = v + dppv<0x112, 0xf>(v); // row_shr:2
    v = v + dppv<0x114, 0xf>(v); // row_shr:4
    v = v + dppv<0x118, 0xf>(v); // row_shr:8
    v = v + dppv<0x142, 0xa>(v); // row_bcast:15 into rows 1 and 3
    v = v + dppv<0x143, 0xc>(v); // row_bcast:31 into rows 2 and 3
    return dppv<0x138, 0xf>(v);  // wave_shr:1: lane 0 gets 0
}

// Sums along s of one 2D histogram row, S2_CPL cells per lane: scan position
// p = S2_CPL * lane + u (u = 0 .. S2_CPL-1) is column p (prefix order) or
// column L-1-p (suffix order).  For every position the exact count sum and
// the FP64 sum of cterm up to it: within the lane sequentially, after the
// lane's exclusive base.  An empty position takes the value at the nearest
// occupied position before it in scan order, so an all-empty column never
// changes a class sum (bit for bit) and the pairs it separates tie.
template <typename CT>
__device__ __forceinline__ void row_sums(const uint32_t (&c)[S2_CPL], const double *tab, double q,
                                         CT (&rc)[S2_CPL], double (&rq)[S2_CPL])
{
    const int lane = threadIdx.x & 63;
    CT lc = 0;
    double lq = 0.0;
    int first = S2_CPL; // first occupied position of this lane
    CT pc[S2_CPL];
    double pq[S2_CPL];
    // cterm from the table tab[c] for small counts (the table holds the
    // identical expression, so both give the same bits); a count past the
    // table anywhere in the row takes the out-of-line path
    double t[S2_CPL];
    bool big = false;
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        t[u] = tab[min(c[u], (uint32_t)S2_TAB - 1u)];
        big |= c[u] >= (uint32_t)S2_TAB;
    }
    if (__ballot(big)) {
#pragma unroll
        for (int u = 0; u < S2_CPL; ++u)
            if (c[u] >= (uint32_t)S2_TAB)
                t[u] = cterm_big(c[u], q);
    }
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        lc += (CT)c[u];
        lq = lq + t[u]; // an empty cell adds +0.0: bits unchanged
        pc[u] = lc;
        pq[u] = lq;
        if (c[u] && first == S2_CPL)
            first = u;
    }
    const uint64_t occ = __ballot(lc != 0);
    const CT bc = wave_excl_sum<CT>(lc);
    const double bq = wave_excl_sum<double>(lq);
    const double last = bq + lq; // the value at this lane's last occupied position
    const uint64_t before = occ & ((1ull << lane) - 1ull);
    const int src = before ? 63 - __clzll((long long)before) : lane;
    const double prev_raw = __shfl(last, src, 64);
    const double prev = before ? prev_raw : 0.0;
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        rc[u] = bc + pc[u];
        rq[u] = u >= first ? bq + pq[u] : prev;
    }
}

// The same scan for per-position values given directly (cc counts, cq sums
// of cterm; a block's column totals): exact count prefix, FP64 prefix in
// the lane then after its exclusive base, an empty position taking the
// value at the nearest occupied position before it.
__device__ __forceinline__ void pos_sums(const uint64_t (&cc)[S2_CPL], const double (&cq)[S2_CPL],
                                         uint64_t (&rc)[S2_CPL], double (&rq)[S2_CPL])
{
    const int lane = threadIdx.x & 63;
    uint64_t lc = 0;
    double lq = 0.0;
    int first = S2_CPL;
    uint64_t pc[S2_CPL];
    double pq[S2_CPL];
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        lc += cc[u];
        lq = lq + cq[u];
        pc[u] = lc;
        pq[u] = lq;
        if (cc[u] && first == S2_CPL)
            first = u;
    }
    const uint64_t occ = __ballot(lc != 0);
    const uint64_t bc = wave_excl_sum<uint64_t>(lc);
    const double bq = wave_excl_sum<double>(lq);
    const double last = bq + lq;
    const uint64_t before = occ & ((1ull << lane) - 1ull);
    const int src = before ? 63 - __clzll((long long)before) : lane;
    const double prev_raw = __shfl(last, src, 64);
    const double prev = before ? prev_raw : 0.0;
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        rc[u] = bc + pc[u];
        rq[u] = u >= first ? bq + pq[u] : prev;
    }
}

// FP64 class term from the class sums: sgn(1-q) (ln S - q ln C) for Tsallis,
// ln C - S / C for q = 1 (S = sum of cterm, C = pixels); -inf for an empty
// class; clamped to [0, hmax].  Called only for the few rows the FP64
// re-check visits: kept out of line so that its registers do not burden the
// FP32 passes.
__device__ __noinline__ double class_term2(uint64_t c, double sumq, double q, double sgn, double hmax)
{
    if (c == 0)
        return -INFINITY;
    const double C = (double)c;
    const double h = sgn == 0.0 ? log(C) - sumq / C : sgn * (log(sumq) - q * log(C));
    return fmin(fmax(h, 0.0), hmax);
}

// Per-problem constants of the search.
struct S2 {
    const uint32_t *h; // the L x L histogram
    int L;
    bool vec;          // rows load as 16-byte vectors (L % 4 == 0, aligned)
    double q, sgn, hmax;
    const double *tab; // cterm of counts below S2_TAB
    const uint32_t *band; // per row: lowest | highest column holding counts << 16 (LDS)
    float mq;          // -q rounded to FP32 (Tsallis)
    float sg;          // sgn(1-q) as +-1 (Tsallis)
    float gmax;        // hmax / ln 2 rounded up
};

// The same class term in log2 units in FP32, from the FP64 class sums: the
// key of the search.  Its error against class_term2 / ln 2 is bounded in
// s2_delta.  sgn(1-q) (log2 S - q log2 C) is formed as the fma
// log2 S - q log2 C times +-1 (exact).
template <typename CT>
__device__ __forceinline__ float class_key32(CT c, double sumq, const S2 &p)
{
    const float lc = __builtin_amdgcn_logf((float)c);
    float g;
    if (p.sgn == 0.0) { // Shannon: log2 C - (S / C) log2 e
        const float r = (float)(sumq / (double)c);
        g = fmaf(r, -1.44269504f, lc);
    } else {
        g = fmaf(p.mq, lc, __builtin_amdgcn_logf((float)sumq)) * p.sg;
    }
    g = __builtin_amdgcn_fmed3f(g, 0.0f, p.gmax);
    return c ? g : -INFINITY;
}

// Bound on |key32 - key64 / ln 2| for every pair of one problem (key32 the
// sum of the two FP32 class keys, key64 the FP64 sum of class_term2 from the
// same class sums) for an image of N pixels.  Per class: the casts of C and
// S (or S / C) to FP32 (2^-24 relative each, 1.5 * 2^-24 after the log2),
// v_log_f32 (LOG2_ERR_UNITS * 2^-24 * max(1, |log2 x|)), q or log2 e rounded
// to FP32, the fma; then the FP32 sum of the two clamped terms, and the
// clamp at gmax instead of hmax / ln 2.  Magnitudes: 1 <= C <= N; a class of
// m <= L^2 occupied cells has 1 <= S <= max(C^q, m^(1-q) C^q), so
// 0 <= log2 S <= q log2 N + 2 |1-q| log2 L; 0 <= S / C <= ln N for q = 1.
// Infinity when S could leave the FP32 range: every pair is then re-checked
// in FP64.
__device__ __forceinline__ double s2_delta(const S2 &p, double N)
{
    const double u = 0x1p-24;
    const double lN = log2(N) * 1.0001 + 1e-6;
    const double q = p.q;
    double e1;
    if (p.sgn == 0.0) {
        const double r = lN * 0.6931471805599453 * 1.0001; // S / C <= ln N
        e1 = 1.5 * u + LOG2_ERR_UNITS * u * fmax(1.0, lN) + 2.0 * u * 1.4426950408889634 * r +
             u * (lN + 1.4426950408889634 * r);
    } else {
        const double Ux = q * lN + 2.0 * fabs(1.0 - q) * log2((double)p.L) * 1.0001 + 1e-6, Vy = lN;
        if (Ux > 120.0)
            return INFINITY;
        e1 = 1.5 * u * (1.0 + q) + LOG2_ERR_UNITS * u * (fmax(1.0, Ux) + q * fmax(1.0, Vy)) + u * q * Vy +
             u * (Ux + q * Vy);
    }
    return (2.0 * e1 + 2.0 * u * (double)p.gmax + 2.0 * 0x1p-20 * (double)p.gmax) * 1.01 + 1e-12;
}

// Counts of row t in the lane's scan positions (DIR = +1: column
// S2_CPL * lane + u; DIR = -1: column L-1-(S2_CPL * lane + u)); zero past
// the row's ends.  t must be a valid row.  The loads are unconditional
// (clamped addresses, masked values) so that several rows' loads can be in
// flight at once.
template <int DIR>
__device__ __forceinline__ void load_row(const uint32_t *h, int L, bool vec, int t, uint32_t (&c)[S2_CPL],
                                         const uint32_t *band)
{
    const int lane = threadIdx.x & 63;
    const uint32_t *row = h + (int64_t)t * L;
    // columns outside the row's band hold no counts: those lanes load nothing
    // (band null: every column)
    const uint32_t bd = band ? band[t] : 0xffff0000u;
    const int jlo = (int)(bd & 0xffffu), jhi = (int)(bd >> 16);
    const int c0 = DIR > 0 ? S2_CPL * lane : L - S2_CPL - S2_CPL * lane; // the lane's lowest column (vec)
    if (vec) {
        const bool ok = S2_CPL * lane < L && c0 <= jhi && c0 + S2_CPL - 1 >= jlo;
        const uint4 v = ok ? *reinterpret_cast<const uint4 *>(row + c0) : make_uint4(0u, 0u, 0u, 0u);
        if (DIR > 0) {
            c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
        } else {
            c[0] = v.w; c[1] = v.z; c[2] = v.y; c[3] = v.x;
        }
    } else {
#pragma unroll
        for (int u = 0; u < S2_CPL; ++u) {
            const int col = DIR > 0 ? S2_CPL * lane + u : L - 1 - (S2_CPL * lane + u);
            const bool ok = col >= 0 && col < L && col >= jlo && col <= jhi;
            c[u] = ok ? row[col] : 0u;
        }
    }
}

// Visits n >= 0 rows of the compacted list of rows holding counts, rows[k0],
// rows[k0 + DIR], ..., with each row's sums along s (row_sums, in DIR's scan
// order) and S2_CPL auxiliary values aux(k, .) per lane (stored keys the row
// needs); the counts and auxiliary values of the next S2_RING rows are in
// flight meanwhile.  Past the last row the ring reloads the last row and its
// sums are discarded.
template <int DIR, typename CT, typename A, typename F>
__device__ __forceinline__ void for_rows(const S2 &p, const int *rows, int k0, int n, A &&aux, F &&f)
{
    if (n <= 0)
        return;
    uint32_t ring[S2_RING][S2_CPL];
    float xr[S2_RING][S2_CPL];
#pragma unroll
    for (int d = 0; d < S2_RING; ++d) {
        const int kk = k0 + DIR * min(d, n - 1);
        load_row<DIR>(p.h, p.L, p.vec, rows[kk], ring[d], p.band);
        aux(kk, xr[d]);
    }
    for (int i0 = 0; i0 < n; i0 += S2_RING) {
#pragma unroll
        for (int d = 0; d < S2_RING; ++d) {
            const int i = i0 + d;
            uint32_t c[S2_CPL];
            float x[S2_CPL];
#pragma unroll
            for (int u = 0; u < S2_CPL; ++u) {
                c[u] = ring[d][u];
                x[u] = xr[d][u];
            }
            const int kk = k0 + DIR * min(i + S2_RING, n - 1);
            load_row<DIR>(p.h, p.L, p.vec, rows[kk], ring[d], p.band);
            aux(kk, xr[d]);
            CT rc[S2_CPL];
            double rq[S2_CPL];
            row_sums<CT>(c, p.tab, p.q, rc, rq);
            if (i < n)
                f(k0 + DIR * i, rc, rq, x);
        }
    }
}

// Column totals of the listed rows rows[k0], rows[k0 + DIR], ... (n >= 0 of
// them) in DIR's scan positions: count sums and sums of cterm, added in
// walking order; the next S2_RING rows' loads in flight.
template <int DIR>
__device__ __forceinline__ void block_totals(const S2 &p, const int *rows, int k0, int n, uint64_t (&cc)[S2_CPL],
                                             double (&cq)[S2_CPL])
{
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        cc[u] = 0;
        cq[u] = 0.0;
    }
    if (n <= 0)
        return;
    uint32_t ring[S2_RING][S2_CPL];
#pragma unroll
    for (int d = 0; d < S2_RING; ++d)
        load_row<DIR>(p.h, p.L, p.vec, rows[k0 + DIR * min(d, n - 1)], ring[d], p.band);
    for (int i0 = 0; i0 < n; i0 += S2_RING) {
#pragma unroll
        for (int d = 0; d < S2_RING; ++d) {
            const int i = i0 + d;
            uint32_t c[S2_CPL];
#pragma unroll
            for (int u = 0; u < S2_CPL; ++u)
                c[u] = ring[d][u];
            load_row<DIR>(p.h, p.L, p.vec, rows[k0 + DIR * min(i + S2_RING, n - 1)], ring[d], p.band);
            if (i < n) {
                double t[S2_CPL];
                bool big = false;
#pragma unroll
                for (int u = 0; u < S2_CPL; ++u) {
                    t[u] = p.tab[min(c[u], (uint32_t)S2_TAB - 1u)];
                    big |= c[u] >= (uint32_t)S2_TAB;
                }
                if (__ballot(big)) {
#pragma unroll
                    for (int u = 0; u < S2_CPL; ++u)
                        if (c[u] >= (uint32_t)S2_TAB)
                            t[u] = cterm_big(c[u], p.q);
                }
#pragma unroll
                for (int u = 0; u < S2_CPL; ++u) {
                    cc[u] += c[u];
                    cq[u] = cq[u] + t[u];
                }
            }
        }
    }
}

// Maximum over the wavefront by DPP moves (no LDS round trips): within rows
// of 16 lanes, then carried by the broadcasts of lanes 15 and 31; lanes
// without a source read -inf.  The result is read from lane 63.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_max_step(float v)
{
    const int ninf = __float_as_int(-INFINITY);
    const float o = __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), CTRL, ROWS, 0xf, false));
    return fmaxf(v, o);
}

__device__ __forceinline__ float wave_max_f32(float v)
{
    v = dpp_max_step<0x111, 0xf>(v); // row_shr:1
    v = dpp_max_step<0x112, 0xf>(v); // row_shr:2
    v = dpp_max_step<0x114, 0xf>(v); // row_shr:4
    v = dpp_max_step<0x118, 0xf>(v); // row_shr:8
    v = dpp_max_step<0x142, 0xa>(v); // row_bcast:15
    v = dpp_max_step<0x143, 0xc>(v); // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// LDS of one (q index, problem).
struct S2Lds {
    double tab[S2_TAB];                   // cterm of counts below S2_TAB
    uint32_t band[H2_MAX_L];              // each row's band of columns holding counts
    int rows[H2_MAX_L];                   // rows holding counts, increasing
    float rmax[H2_MAX_L];                 // best pair key of each listed row
    uint64_t tc[2][S2_WAVES][H2_MAX_L];   // block totals along s: [0] class 2 blocks, [1] class 1 blocks
    double tq[2][S2_WAVES][H2_MAX_L];
    float wm[S2_WAVES];                   // per-wavefront maxima
    double wb[S2_WAVES];                  // per-wavefront best FP64 pair
    long long wcode[S2_WAVES];
};

// Block w of n listed rows starting at k0 in one of S2_WAVES equal parts.
__device__ __forceinline__ int s2_block(int k0, int n, int w) { return k0 + (int)(((int64_t)n * w) / S2_WAVES); }

// This wavefront's block totals along s (its lane's scan positions) into
// LDS, from its rows rows[k0], rows[k0 + DIR], ... (n of them).
template <int DIR>
__device__ __forceinline__ void store_block_totals(const S2 &p, const int *rows, int k0, int n, uint64_t *tc,
                                                   double *tq)
{
    const int lane = threadIdx.x & 63;
    uint64_t cc[S2_CPL], rc[S2_CPL];
    double cq[S2_CPL], rq[S2_CPL];
    block_totals<DIR>(p, rows, k0, n, cc, cq);
    pos_sums(cc, cq, rc, rq);
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        const int pos = S2_CPL * lane + u;
        if (pos < H2_MAX_L) {
            tc[pos] = rc[u];
            tq[pos] = rq[u];
        }
    }
}

// The sums carried into block w: the block totals of blocks v0, v0 + dv, ...
// up to (not including) w, added in that order.
template <typename CT>
__device__ __forceinline__ void carry_in(const uint64_t (*tc)[H2_MAX_L], const double (*tq)[H2_MAX_L], int v0,
                                         int dv, int w, CT (&ac)[S2_CPL], double (&aq)[S2_CPL])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        ac[u] = 0;
        aq[u] = 0.0;
    }
    for (int v = v0; v != w; v += dv) {
#pragma unroll
        for (int u = 0; u < S2_CPL; ++u) {
            const int pos = min(S2_CPL * lane + u, H2_MAX_L - 1);
            ac[u] += (CT)tc[v][pos];
            aq[u] = aq[u] + tq[v][pos];
        }
    }
}

// One (q index, problem) per workgroup of S2_WAVES wavefronts; CT is the type
// of in-row count sums (uint32_t when the image holds fewer than 2^32
// pixels).  R >= 1 rows hold counts, listed in rows[] in increasing order.
// A row without counts (t >= 1) leaves the class 1 sums unchanged and
// B(t+1, .) = B(t, .): its pairs tie exactly with those of row t-1, which
// come first, so only listed rows are visited, and the class 2 partner of
// the listed row rows[k] is rows[k+1].
//  1. class 2 keys, bottom-up: B(t, s) = sums over {i >= t, j >= s} (scan
//     position p is column L-1-p); the listed rows kB .. R-1 in S2_WAVES
//     blocks, each started from the totals of the blocks below it; FP32 key
//     of every listed row t >= 1 into k2 (workspace, [L][L] floats);
//  2. class 1, top-down: A(t, s) = sums over {i <= t, j <= s}, the listed
//     rows 0 .. R-2 in blocks, each started from the totals of the blocks
//     above it; the pair key is the FP32 class 1 key plus k2 at
//     (rows[k+1], s+1); row maxima rmax[k] and the maximum M;
//  3. rows with rmax >= M - 2 delta (the FP64 arg max is among them): the
//     FP64 class 2 terms of their partner rows into t2 (workspace, doubles),
//     from the same sums as in 1;
//  4. the FP64 value of every pair of those rows whose key is >= M - 2
//     delta, from the same sums as in 2; the first best pair (t outermost).
template <typename CT>
__device__ __forceinline__ void search2d_body(const S2 &p, double N, int R, S2Lds &sh, float *k2, double *t2,
                                              int32_t *thr_t, int32_t *thr_s, double *obj_p, int32_t *status_p)
{
    const int lane = threadIdx.x & 63, L = p.L;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int *rows = sh.rows;
    float *rmax = sh.rmax;
    int colB[S2_CPL], colA[S2_CPL];
#pragma unroll
    for (int u = 0; u < S2_CPL; ++u) {
        colB[u] = L - 1 - (S2_CPL * lane + u);
        colA[u] = S2_CPL * lane + u;
    }
    const int kB = rows[0] == 0 ? 1 : 0; // class 2 starts at row 1 at the earliest
    // pairs exist for listed rows k with k + 1 < R (rows[k] <= L - 2 follows)
    const int npair = R - 1;
    // this wavefront's blocks: [b0, b1) of kB .. R-1 (class 2), [a0, a1) of
    // 0 .. npair-1 (class 1)
    const int b0 = s2_block(kB, R - kB, w), b1 = s2_block(kB, R - kB, w + 1);
    const int a0 = s2_block(0, npair, w), a1 = s2_block(0, npair, w + 1);
    auto none = [](int, float(&)[S2_CPL]) {};
    // the stored class 2 keys at (rows[k + 1], s + 1) for the lane's columns s
    auto partner = [&](int k, float(&x)[S2_CPL]) {
        const float *row2 = k2 + (int64_t)rows[k + 1] * L; // k <= R - 2 in the pass that uses it
#pragma unroll
        for (int u = 0; u < S2_CPL; ++u) {
            const float v = row2[min(colA[u] + 1, L - 1)]; // unconditional load, masked below
            x[u] = colA[u] <= L - 2 ? v : -INFINITY;
        }
    };

    // block totals of both directions, then the carries into this block
    store_block_totals<-1>(p, rows, b1 - 1, b1 - b0, sh.tc[0][w], sh.tq[0][w]);
    store_block_totals<1>(p, rows, a0, a1 - a0, sh.tc[1][w], sh.tq[1][w]);
    __syncthreads();
    // the sums carried into this wavefront's blocks (the blocks below it for
    // class 2, above it for class 1) are re-read from LDS at the start of
    // each walk rather than held in registers across the passes

    // 1. class 2 keys
    {
        CT bc[S2_CPL];
        double bq[S2_CPL];
        carry_in<CT>(sh.tc[0], sh.tq[0], S2_WAVES - 1, -1, w, bc, bq);
        for_rows<-1, CT>(p, rows, b1 - 1, b1 - b0, none, [&](int k, const CT(&rc)[S2_CPL], const double(&rq)[S2_CPL],
                                                            const float(&)[S2_CPL]) {
            float *row = k2 + (int64_t)rows[k] * L;
#pragma unroll
            for (int u = 0; u < S2_CPL; ++u) {
                bc[u] += rc[u];
                bq[u] = bq[u] + rq[u];
                if (colB[u] >= 0)
                    row[colB[u]] = class_key32(bc[u], bq[u], p);
            }
        });
    }
    __syncthreads();
    // 2. pair keys, row maxima
    {
        float M = -INFINITY;
        CT ac[S2_CPL];
        double aq[S2_CPL];
        carry_in<CT>(sh.tc[1], sh.tq[1], 0, 1, w, ac, aq);
        for_rows<1, CT>(p, rows, a0, a1 - a0, partner, [&](int k, const CT(&rc)[S2_CPL], const double(&rq)[S2_CPL],
                                                          const float(&x)[S2_CPL]) {
            float m = -INFINITY;
#pragma unroll
            for (int u = 0; u < S2_CPL; ++u) {
                ac[u] += rc[u];
                aq[u] = aq[u] + rq[u];
                if (colA[u] <= L - 2)
                    m = fmaxf(m, class_key32(ac[u], aq[u], p) + x[u]);
            }
            m = wave_max_f32(m);
            if (lane == 0)
                rmax[k] = m;
            M = fmaxf(M, m);
        });
        if (lane == 0)
            sh.wm[w] = M;
    }
    __syncthreads();
    float M = -INFINITY;
    for (int v = 0; v < S2_WAVES; ++v)
        M = fmaxf(M, sh.wm[v]);
    const double delta = s2_delta(p, N);
    const bool all = !(delta < INFINITY);
    if (!all && !(M > -INFINITY)) { // every key finite for a valid pair: none is valid
        if (threadIdx.x == 0) {
            *thr_t = *thr_s = -1;
            *obj_p = NAN;
            *status_p = TS_PROBLEM_DEGENERATE;
        }
        return;
    }
    const double T = all ? -INFINITY : (double)M - 2.0 * delta;
    // 3. FP64 class 2 terms of the partner rows rows[k], k - 1 a candidate,
    // k in this wavefront's class 2 block: walked from the block's bottom up
    // to the highest such row
    {
        int kmin = b1;
        for (int k = b0 + lane; k < b1; k += 64)
            if (k >= 1 && (all || (double)rmax[k - 1] >= T))
                kmin = min(kmin, k);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            kmin = min(kmin, __shfl_xor(kmin, o, 64));
        if (kmin < b1) {
            CT bc[S2_CPL];
            double bq[S2_CPL];
            carry_in<CT>(sh.tc[0], sh.tq[0], S2_WAVES - 1, -1, w, bc, bq);
            for_rows<-1, CT>(p, rows, b1 - 1, b1 - kmin, none,
                             [&](int k, const CT(&rc)[S2_CPL], const double(&rq)[S2_CPL], const float(&)[S2_CPL]) {
#pragma unroll
                                 for (int u = 0; u < S2_CPL; ++u) {
                                     bc[u] += rc[u];
                                     bq[u] = bq[u] + rq[u];
                                 }
                                 if (k >= 1 && (all || (double)rmax[k - 1] >= T)) {
                                     double *row = t2 + (int64_t)rows[k] * L;
#pragma unroll
                                     for (int u = 0; u < S2_CPL; ++u)
                                         if (colB[u] >= 0)
                                             row[colB[u]] = class_term2(bc[u], bq[u], p.q, p.sgn, p.hmax);
                                 }
                             });
        }
    }
    __syncthreads();
    // 4. FP64 values of the candidate pairs of this wavefront's class 1 block
    double best = -INFINITY;
    long long code = 0x7fffffffffffffffLL;
    {
        int kmax = a0 - 1;
        for (int k = a0 + lane; k < a1; k += 64)
            if (all || (double)rmax[k] >= T)
                kmax = max(kmax, k);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            kmax = max(kmax, __shfl_xor(kmax, o, 64));
        if (kmax >= a0) {
            CT ac[S2_CPL];
            double aq[S2_CPL];
            carry_in<CT>(sh.tc[1], sh.tq[1], 0, 1, w, ac, aq);
            for_rows<1, CT>(p, rows, a0, kmax - a0 + 1, none,
                            [&](int k, const CT(&rc)[S2_CPL], const double(&rq)[S2_CPL], const float(&)[S2_CPL]) {
#pragma unroll
                                for (int u = 0; u < S2_CPL; ++u) {
                                    ac[u] += rc[u];
                                    aq[u] = aq[u] + rq[u];
                                }
                                if (!(all || (double)rmax[k] >= T))
                                    return;
                                const int t = rows[k], r2 = rows[k + 1];
                                const float *row2 = k2 + (int64_t)r2 * L;
                                const double *row2d = t2 + (int64_t)r2 * L;
#pragma unroll
                                for (int u = 0; u < S2_CPL; ++u) {
                                    if (colA[u] <= L - 2) {
                                        const float key = class_key32(ac[u], aq[u], p) + row2[colA[u] + 1];
                                        if (all || (double)key >= T) {
                                            const double lam = class_term2(ac[u], aq[u], p.q, p.sgn, p.hmax) +
                                                               row2d[colA[u] + 1];
                                            const long long cd = ((long long)t << 12) | colA[u];
                                            if (lam > -INFINITY && (lam > best || (lam == best && cd < code))) {
                                                best = lam;
                                                code = cd;
                                            }
                                        }
                                    }
                                }
                            });
        }
    }
    // first best pair of the wavefront, then of the workgroup
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double b2 = __shfl_xor(best, o, 64);
        const long long c2 = __shfl_xor(code, o, 64);
        if (b2 > best || (b2 == best && c2 < code)) {
            best = b2;
            code = c2;
        }
    }
    if (lane == 0) {
        sh.wb[w] = best;
        sh.wcode[w] = code;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 0; v < S2_WAVES; ++v)
            if (sh.wb[v] > best || (sh.wb[v] == best && sh.wcode[v] < code)) {
                best = sh.wb[v];
                code = sh.wcode[v];
            }
        if (!(best > -INFINITY)) {
            *thr_t = *thr_s = -1;
            *obj_p = NAN;
            *status_p = TS_PROBLEM_DEGENERATE;
        } else {
            *thr_t = (int32_t)(code >> 12);
            *thr_s = (int32_t)(code & 4095);
            *obj_p = p.sgn == 0.0 ? best : expm1(p.sgn * best) / (1.0 - p.q);
            *status_p = TS_PROBLEM_OK;
        }
    }
}

// Which rows of each image hold counts, the image's pixel count and each
// row's band of columns holding counts: one wavefront per group of 16 rows,
// all 16 rows' loads in flight together.  mask[s][g] bit d: row 16 g + d
// holds counts; cnt[s][g]: its pixels; band[s][t]: the lowest column holding
// counts in row t | the highest << 16 (0xffff | 0 << 16 for an empty row).
__global__ void __launch_bounds__(64) k_rows2d(const uint32_t *__restrict__ hist, int L, int groups,
                                               uint16_t *__restrict__ mask, uint64_t *__restrict__ cnt,
                                               uint32_t *__restrict__ band)
{
    const int s0 = blockIdx.x / groups, g = blockIdx.x % groups, lane = threadIdx.x & 63;
    const uint32_t *h = hist + (int64_t)s0 * L * L;
    const bool vec = (L % S2_CPL) == 0 && ((uintptr_t)h & 15) == 0;
    uint32_t c[16][S2_CPL];
#pragma unroll
    for (int d = 0; d < 16; ++d) // rows past L reload row L-1 and count as empty
        load_row<1>(h, L, vec, min(16 * g + d, L - 1), c[d], nullptr);
    uint32_t bits = 0;
    uint64_t n = 0;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        uint64_t r = 0;
#pragma unroll
        for (int u = 0; u < S2_CPL; ++u)
            r += c[d][u];
        if (16 * g + d >= L)
            r = 0;
        n += r;
        if (__ballot(r != 0))
            bits |= 1u << d;
        int lo = 0xffff, hi = 0;
#pragma unroll
        for (int u = S2_CPL - 1; u >= 0; --u)
            if (c[d][u])
                lo = S2_CPL * lane + u;
#pragma unroll
        for (int u = 0; u < S2_CPL; ++u)
            if (c[d][u])
                hi = S2_CPL * lane + u;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
        }
        if (lane == 0 && 16 * g + d < L)
            band[(int64_t)s0 * L + 16 * g + d] = (bits >> d) & 1u ? (uint32_t)lo | ((uint32_t)hi << 16) : 0xffffu;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        n += __shfl_xor(n, o, 64);
    if (threadIdx.x == 0) {
        mask[(int64_t)s0 * 16 + g] = (uint16_t)bits;
        cnt[(int64_t)s0 * 16 + g] = n;
    }
}

// Workgroup b takes image s0 = 8 (b / 8 / nq) + b % 8 and q index (b / 8) %
// nq: the nq workgroups of an image are 8 apart, so they land on the same XCD
// (workgroups go to the 8 XCDs in turn) and share its L2 for the image's
// rows; workgroups with s0 >= nseg do nothing.
__global__ void __launch_bounds__(S2_THREADS) k_search2d(const uint32_t *__restrict__ hist, int nseg, int nq, int L,
                                                         Q2List ql, float *__restrict__ k2all,
                                                         double *__restrict__ t2all, const uint16_t *__restrict__ mask,
                                                         const uint64_t *__restrict__ cnt,
                                                         const uint32_t *__restrict__ band, int32_t *__restrict__ thr,
                                                         double *__restrict__ obj, int32_t *__restrict__ status)
{
    __shared__ S2Lds sh;
    __shared__ int nrows;
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x >> 3, s0 = (slot / nq) * 8 + (blockIdx.x & 7), j = slot % nq;
    if (s0 >= nseg)
        return;
    const int prob = j * nseg + s0;
    S2 p;
    p.h = hist + (int64_t)s0 * L * L;
    p.L = L;
    p.vec = (L % S2_CPL) == 0 && ((uintptr_t)p.h & 15) == 0;
    p.q = ql.q[j];
    p.sgn = p.q == 1.0 ? 0.0 : (p.q < 1.0 ? 1.0 : -1.0);
    p.hmax = (p.q == 1.0 ? 1.0 : fabs(1.0 - p.q)) * 2.0 * log((double)L); // a class holds at most L^2 cells
    p.mq = (float)(-p.q);
    p.sg = p.q < 1.0 ? 1.0f : -1.0f;
    p.gmax = (float)(p.hmax * 1.4426950408889634 * (1.0 + 0x1p-20));
    p.tab = sh.tab;
    p.band = sh.band;
    // the image's pixel count (every wavefront) and its rows holding counts,
    // in increasing order (wavefront 0): lane l looks at rows 4l .. 4l+3
    // (groups past the last hold no rows below L)
    const int groups = (L + 15) / 16;
    uint64_t n = lane < groups ? cnt[(int64_t)s0 * 16 + lane] : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        n += __shfl_xor(n, o, 64);
    if (threadIdx.x < 64) {
        const uint32_t g16 = (4 * lane) / 16 < groups ? mask[(int64_t)s0 * 16 + (4 * lane) / 16] : 0u;
        uint32_t nib = (g16 >> ((4 * lane) % 16)) & 0xfu;
        if (4 * lane + 4 > L)
            nib &= (4 * lane < L) ? (1u << (L - 4 * lane)) - 1u : 0u;
        const uint32_t pos = wave_excl_sum<uint32_t>((uint32_t)__popc(nib));
        uint32_t w = pos;
#pragma unroll
        for (int d = 0; d < 4; ++d)
            if (nib & (1u << d))
                sh.rows[w++] = 4 * lane + d;
        const int R = __shfl(w, 63, 64);
        if (lane == 0)
            nrows = R;
    }
    // thr is [nq][2][nseg]: t at row 0, s at row 1 of this q
    int32_t *thr_t = thr + (int64_t)(2 * j) * nseg + s0, *thr_s = thr_t + nseg;
    if (n == 0) {
        if (threadIdx.x == 0) {
            *thr_t = *thr_s = -1;
            obj[prob] = NAN;
            status[prob] = TS_PROBLEM_EMPTY;
        }
        return;
    }
    for (int i = threadIdx.x; i < S2_TAB; i += blockDim.x)
        sh.tab[i] = cterm((uint32_t)i, p.q);
    for (int i = threadIdx.x; i < L; i += blockDim.x)
        sh.band[i] = band[(int64_t)s0 * L + i];
    __syncthreads();
    const int R = nrows;
    float *k2 = k2all + (int64_t)prob * L * L;
    double *t2 = t2all + (int64_t)prob * L * L;
    if (n >> 32)
        search2d_body<uint64_t>(p, (double)n, R, sh, k2, t2, thr_t, thr_s, obj + prob, status + prob);
    else
        search2d_body<uint32_t>(p, (double)n, R, sh, k2, t2, thr_t, thr_s, obj + prob, status + prob);
}

// Workspace: FP64 terms [nprob][L][L], FP32 keys [nprob][L][L], row masks
// uint16 [nseg][16], pixel counts uint64 [nseg][16] and row bands uint32
// [nseg][L], each part starting 256-byte aligned (the workspace itself must
// be 8-byte aligned).
static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t search2d_workspace_bytes(int nseg, int nq, int L)
{
    const size_t cells = (size_t)nseg * nq * L * L;
    return up256(cells * sizeof(double)) + up256(cells * sizeof(float)) + up256((size_t)nseg * 16 * 2) +
           up256((size_t)nseg * 16 * 8) + (size_t)nseg * L * 4;
}

ts_status launch_search2d(const uint32_t *hist, int nseg, int L, int nq, const double *q, void *ws, int32_t *thr,
                          double *obj, int32_t *status, hipStream_t st)
{
    Q2List ql;
    for (int i = 0; i < TS_MAX_Q; ++i)
        ql.q[i] = q[i < nq ? i : 0];
    const size_t cells = (size_t)nseg * nq * L * L;
    char *w = (char *)ws;
    double *t2 = (double *)w;
    float *k2 = (float *)(w + up256(cells * sizeof(double)));
    uint16_t *mask = (uint16_t *)(w + up256(cells * sizeof(double)) + up256(cells * sizeof(float)));
    uint64_t *cnt = (uint64_t *)((char *)mask + up256((size_t)nseg * 16 * 2));
    uint32_t *band = (uint32_t *)((char *)cnt + up256((size_t)nseg * 16 * 8));
    const int groups = (L + 15) / 16;
    hipLaunchKernelGGL(k_rows2d, dim3((unsigned)(nseg * groups)), dim3(64), 0, st, hist, L, groups, mask, cnt, band);
    const unsigned nblk = (unsigned)((nseg + 7) / 8 * 8 * nq);
    hipLaunchKernelGGL(k_search2d, dim3(nblk), dim3(S2_THREADS), 0, st, hist, nseg, nq, L, ql, k2, t2, mask, cnt, band,
                       thr, obj, status);
    return check_launch("ts_threshold_search2d");
}

} // namespace ts
