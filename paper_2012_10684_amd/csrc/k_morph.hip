// k_morph.hip -- the paper's morphology step (Morphology section): gray-scale
// erosion (minimum) and dilation (maximum) of the gray-level image under a
// flat disk B = {(dx, dy) : dx^2 + dy^2 <= r^2}, the opening (dilation of the
// erosion) and the residue original - opened that removes the large bright
// chest structures.  Pixels outside the image take no part.
//
// One workgroup per 64 x 64 output tile of one image; each thread owns a
// pair of adjacent output columns.  The tile and a halo of r rows and R
// columns (R = r rounded up to even) are staged in LDS as gray levels, two
// per 32-bit word (outside the image the neutral value, 255 for the minimum
// and 0 for the maximum), with a fixed row stride, so that a thread's staged
// rows sit at constant offsets.  The disk is the union over row offsets dy
// of horizontal runs of half-width w(dy) = floor(sqrt(r^2 - dy^2)); w grows
// as |dy| falls, so each thread holds the horizontal minimum (maximum) of its
// staged rows' pair in registers and widens it one unit of width at a time:
// the neighbours at distance d are the word d / 2 away (d even) or the two
// halves of the words (d - 1) / 2 and (d + 1) / 2 away joined by one byte
// align (d odd), so each new word is read once and serves two widths, and
// each step is two packed 16-bit min (max) operations for two pixels.  After
// each distinct w the rows are published in a row buffer H (pairs too), and
// each output pair takes the minimum (maximum) of H at rows y - |dy| and
// y + |dy| when w = w(dy).  Per output pixel and pass: about r/2 (1 + 2r/64)
// LDS word reads and 3r/2 (1 + 2r/64) packed operations to widen, r + 1
// word reads and r + 1 packed operations to combine.
#include "common.h"

namespace ts {

constexpr int MO_TX = 64, MO_TY = 64, MO_THREADS = 256;
constexpr int MO_PAIRS = MO_TX / 2;                   // column pairs per tile row
constexpr int MO_PH = MO_THREADS / MO_PAIRS;          // row phases: rows yb, yb + 8, ...
constexpr int MO_PER = MO_TY / MO_PH;                 // output pairs per thread
constexpr int MO_SWW = (MO_TX + 2 * TS_MORPH_MAX_RADIUS) / 2; // staged row stride in words
constexpr int MO_SH = MO_TY + 2 * TS_MORPH_MAX_RADIUS;        // largest staged column
constexpr int MO_ROWS = MO_SH / MO_PH;                        // staged rows per thread, at most
constexpr int MO_STG = MO_SH / (MO_THREADS / 64);             // staging rows per thread, at most

// Staged rows allocated for sh staged rows: the rows a thread's last group of
// four may touch, sh rounded up to MO_PH * 4.
__host__ __device__ inline int morph_rows_alloc(int sh) { return (sh + 4 * MO_PH - 1) / (4 * MO_PH) * (4 * MO_PH); }
static_assert(TS_MORPH_MAX_RADIUS % 2 == 0, "the staged halo is rounded up to even");

typedef unsigned short mo_u16x2 __attribute__((ext_vector_type(2)));

// Two 16-bit lanes min (MAXOP: max): v_pk_min_u16 / v_pk_max_u16.
template <bool MAXOP>
__device__ __forceinline__ uint32_t pk(uint32_t a, uint32_t b)
{
    const mo_u16x2 x = __builtin_bit_cast(mo_u16x2, a), y = __builtin_bit_cast(mo_u16x2, b);
    return __builtin_bit_cast(uint32_t, MAXOP ? __builtin_elementwise_max(x, y) : __builtin_elementwise_min(x, y));
}

// floor(sqrt(n)) from a guess g >= 0 (wavefront-uniform integers: scalar code)
__device__ __forceinline__ int isqrt_from(int n, int g)
{
    while (g * g > n)
        --g;
    while ((g + 1) * (g + 1) <= n)
        ++g;
    return g;
}

// MAXOP = false: erosion of the gray levels of the int16 images (src16,
// binned) into dst; MAXOP = true: dilation of the uint8 images src8 into dst
// and/or the residue gray(src16) - dilation into res (uint8) and res16
// (int16).
template <bool MAXOP, int MAP>
__global__ void __launch_bounds__(MO_THREADS) k_morph(const int16_t *const *__restrict__ src16,
                                                      const uint8_t *__restrict__ src8, int H, int W, int r,
                                                      BinMap bm, uint8_t *__restrict__ dst, uint8_t *__restrict__ res,
                                                      int16_t *__restrict__ res16)
{
    extern __shared__ uint32_t mo_lds[]; // staged rows [morph_rows_alloc(sh)][MO_SWW], then H [sh][MO_PAIRS]
    const int tiles_x = (W + MO_TX - 1) / MO_TX, tiles_y = (H + MO_TY - 1) / MO_TY;
    const int s = blockIdx.x / (tiles_x * tiles_y);
    const int tile = blockIdx.x % (tiles_x * tiles_y);
    const int x0 = (tile % tiles_x) * MO_TX, y0 = (tile / tiles_x) * MO_TY;
    const int R = (r + 1) & ~1;                      // column halo, even
    const int nw = MO_PAIRS + R, sh = MO_TY + 2 * r; // staged words per row, staged rows
    uint32_t *in = mo_lds, *hr = mo_lds + morph_rows_alloc(sh) * MO_SWW;
    const uint32_t neutral = MAXOP ? 0u : 255u;
    const int64_t img_off = (int64_t)s * H * W;
    const TS_GLOBAL int16_t *img16 = gp(src16[s]);
    // stage word j of row rho: pixels x = x0 - R + 2j and x + 1 of row y0 - r
    // + rho; every load of the thread is issued before the first is used.
    // With an even width and aligned rows (pairs) the two pixels of a word are
    // both inside or both outside the image and load as one access.
    const bool pairs = (W & 1) == 0 && (MAXOP ? ((uintptr_t)(src8 + img_off) & 1) == 0 : ((uintptr_t)img16 & 3) == 0);
    {
        const int j = threadIdx.x & 63, rw = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); // rows rw, rw + 4, ...
        const int x = x0 - R + 2 * j;
        const bool xin0 = j < nw && x >= 0 && x < W, xin1 = j < nw && x + 1 >= 0 && x + 1 < W;
        uint32_t stg[MO_STG][2];
        if (pairs) {
#pragma unroll
            for (int i = 0; i < MO_STG; ++i) {
                const int y = y0 - r + rw + 4 * i;
                const bool in2 = rw + 4 * i < sh && y >= 0 && y < H && xin0;
                if (MAXOP) {
                    const uint16_t *row8 = reinterpret_cast<const uint16_t *>(src8 + img_off + (int64_t)y * W);
                    const uint32_t v = in2 ? (uint32_t)row8[x >> 1] : neutral | (neutral << 8);
                    stg[i][0] = v & 0xffu;
                    stg[i][1] = v >> 8;
                } else {
                    const TS_GLOBAL uint32_t *row16 =
                        reinterpret_cast<const TS_GLOBAL uint32_t *>(img16 + (int64_t)y * W);
                    const uint32_t v = in2 ? row16[x >> 1] : 0u;
                    stg[i][0] = v & 0xffffu;
                    stg[i][1] = v >> 16;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < MO_STG; ++i) {
                const int y = y0 - r + rw + 4 * i;
                const bool yin = rw + 4 * i < sh && y >= 0 && y < H;
                // the row's base is the same in the wavefront; the column a 32-bit offset
                if (MAXOP) {
                    const uint8_t *row8 = src8 + img_off + (int64_t)y * W;
                    stg[i][0] = yin && xin0 ? (uint32_t)row8[x] : neutral;
                    stg[i][1] = yin && xin1 ? (uint32_t)row8[x + 1] : neutral;
                } else {
                    const TS_GLOBAL int16_t *row16 = img16 + (int64_t)y * W;
                    stg[i][0] = yin && xin0 ? (uint32_t)(uint16_t)row16[x] : 0u;
                    stg[i][1] = yin && xin1 ? (uint32_t)(uint16_t)row16[x + 1] : 0u;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < MO_STG; ++i) {
            const int rho = rw + 4 * i, y = y0 - r + rho;
            if (rho < sh && j < nw) {
                uint32_t v0 = stg[i][0], v1 = stg[i][1];
                if (!MAXOP) {
                    const bool yin = y >= 0 && y < H;
                    v0 = yin && xin0 ? (uint32_t)bin_of_t<MAP>((int)(int16_t)v0, bm) : neutral;
                    v1 = yin && xin1 ? (uint32_t)bin_of_t<MAP>((int)(int16_t)v1, bm) : neutral;
                }
                in[rho * MO_SWW + j] = v0 | (v1 << 16);
            }
        }
    }
    // this thread: column pair l, staged rows yb + 8 i, i < nr (the same for
    // both half-waves of a wavefront: nr changes only at yb = sh mod 8, which
    // is even); rows of the last group of four past sh read staged memory that
    // is never used
    const int l = threadIdx.x % MO_PAIRS, yb = threadIdx.x / MO_PAIRS;
    const int nr = __builtin_amdgcn_readfirstlane((sh - yb + MO_PH - 1) / MO_PH);
    const uint32_t *cin = in + yb * MO_SWW + l + R / 2; // the thread's own pair in row yb
    constexpr int RS = MO_PH * MO_SWW;                  // words between a thread's staged rows
    uint32_t hv[MO_ROWS], pl[MO_ROWS], pr[MO_ROWS];
    __syncthreads();
#pragma unroll
    for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
        if (i0 < nr) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                hv[i0 + u] = pl[i0 + u] = pr[i0 + u] = cin[(i0 + u) * RS]; // half-width 0
        }
    // publish the rows at their current half-width into hr
    auto publish = [&]() {
#pragma unroll
        for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
            if (i0 < nr) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + u < nr)
                        hr[(yb + (i0 + u) * MO_PH) * MO_PAIRS + l] = hv[i0 + u];
            }
    };
    publish();
    // output pairs at rows yb + 8 i, i < MO_PER
    uint32_t out[MO_PER];
#pragma unroll
    for (int i = 0; i < MO_PER; ++i)
        out[i] = neutral | (neutral << 16);
    int cur = 0, wg = 0;
    __syncthreads(); // hr at half-width 0
    for (int a = r; a >= 0; --a) {
        const int w = wg = isqrt_from(r * r - a * a, wg);
        if (w > cur) { // widen every staged row of the thread from half-width cur to w
            for (int d = cur + 1; d <= w; ++d) {
                if (d & 1) { // the words k = (d + 1) / 2 away, each side; pl, pr hold those k - 1 away
                    const int k = (d + 1) >> 1;
                    const uint32_t *ql = cin - k, *qr = cin + k;
#pragma unroll
                    for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
                        if (i0 < nr) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int i = i0 + u;
                                const uint32_t lk = ql[i * RS], rk = qr[i * RS];
                                const uint32_t lft = __builtin_amdgcn_alignbyte(pl[i], lk, 2); // pixels -d, -d+1
                                const uint32_t rgt = __builtin_amdgcn_alignbyte(rk, pr[i], 2); // pixels d, d+1 past the pair's first
                                hv[i] = pk<MAXOP>(hv[i], pk<MAXOP>(lft, rgt));
                                pl[i] = lk;
                                pr[i] = rk;
                            }
                        }
                } else { // the words d / 2 away, loaded at d - 1
#pragma unroll
                    for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
                        if (i0 < nr) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int i = i0 + u;
                                hv[i] = pk<MAXOP>(hv[i], pk<MAXOP>(pl[i], pr[i]));
                            }
                        }
                }
            }
            __syncthreads(); // the combine steps before have read hr
            publish();
            cur = w;
            __syncthreads();
        }
        // rows y - a and y + a of every output take half-width w(a); output
        // i sits 8 i staged rows below output 0 (immediate LDS offsets)
        const uint32_t *plo = hr + (yb + r - a) * MO_PAIRS + l, *phi = hr + (yb + r + a) * MO_PAIRS + l;
#pragma unroll
        for (int i = 0; i < MO_PER; ++i)
            out[i] = pk<MAXOP>(out[i], pk<MAXOP>(plo[MO_PH * MO_PAIRS * i], phi[MO_PH * MO_PAIRS * i]));
    }
    // the residue's input values are all loaded before the first store (the
    // outputs may alias the input as far as the compiler knows)
    int f[MO_PER][2];
    const bool opairs = (W & 1) == 0 && ((uintptr_t)img16 & 3) == 0 && ((uintptr_t)dst & 1) == 0 &&
                        ((uintptr_t)res & 1) == 0 && ((uintptr_t)res16 & 3) == 0;
    if (MAXOP && (res || res16)) {
        if (opairs) {
#pragma unroll
            for (int i = 0; i < MO_PER; ++i) {
                const int y = y0 + yb + MO_PH * i, x = x0 + 2 * l;
                const uint32_t v =
                    y < H && x < W ? reinterpret_cast<const TS_GLOBAL uint32_t *>(img16 + (int64_t)y * W)[x >> 1] : 0u;
                f[i][0] = (int)(int16_t)(v & 0xffffu);
                f[i][1] = (int)(int16_t)(v >> 16);
            }
        } else {
#pragma unroll
            for (int i = 0; i < MO_PER; ++i)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int y = y0 + yb + MO_PH * i, x = x0 + 2 * l + e;
                    f[i][e] = y < H && x < W ? (int)img16[(int64_t)y * W + x] : 0;
                }
        }
    }
    if (opairs) { // both pixels of a pair inside or both outside: one store per output and pair
#pragma unroll
        for (int i = 0; i < MO_PER; ++i) {
            const int y = y0 + yb + MO_PH * i, x = x0 + 2 * l;
            if (y >= H || x >= W)
                continue;
            const uint32_t v0 = out[i] & 0xffffu, v1 = out[i] >> 16;
            const int64_t o = img_off + (int64_t)y * W + x;
            if (dst)
                *reinterpret_cast<uint16_t *>(dst + o) = (uint16_t)(v0 | (v1 << 8));
            if (MAXOP && (res || res16)) {
                const int g0 = bin_of_t<MAP>(f[i][0], bm) - (int)v0, g1 = bin_of_t<MAP>(f[i][1], bm) - (int)v1;
                if (res)
                    *reinterpret_cast<uint16_t *>(res + o) = (uint16_t)((g0 & 0xff) | ((g1 & 0xff) << 8));
                if (res16)
                    *reinterpret_cast<uint32_t *>(res16 + o) = (uint32_t)(g0 & 0xffff) | ((uint32_t)(g1 & 0xffff) << 16);
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < MO_PER; ++i) {
        const int y = y0 + yb + MO_PH * i;
        if (y >= H)
            continue;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int x = x0 + 2 * l + e;
            if (x >= W)
                continue;
            const int v = (int)((out[i] >> (16 * e)) & 0xffffu);
            const int64_t o = img_off + (int64_t)y * W + x;
            if (dst)
                dst[o] = (uint8_t)v;
            if (MAXOP && (res || res16)) {
                const int g = bin_of_t<MAP>(f[i][e], bm);
                if (res)
                    res[o] = (uint8_t)(g - v);
                if (res16)
                    res16[o] = (int16_t)(g - v);
            }
        }
    }
}

size_t open2d_workspace_bytes(int nseg, int H, int W) { return (size_t)nseg * H * W; }

static size_t morph_lds_bytes(int r)
{
    const int sh = MO_TY + 2 * r;
    return ((size_t)morph_rows_alloc(sh) * MO_SWW + (size_t)sh * MO_PAIRS) * sizeof(uint32_t);
}

ts_status launch_open2d(const ts_batch &b, int H, int W, const BinMap &bm, int r, uint8_t *eroded,
                        uint8_t *opened, uint8_t *residue, int16_t *residue16, hipStream_t st)
{
    const int tiles = ((W + MO_TX - 1) / MO_TX) * ((H + MO_TY - 1) / MO_TY);
    const dim3 g((unsigned)((int64_t)b.nseg * tiles)), blk(MO_THREADS);
    const size_t lds = morph_lds_bytes(r);
#define TS_MO(M)                                                                                                     \
    hipLaunchKernelGGL((k_morph<false, M>), g, blk, lds, st, b.vox, nullptr, H, W, r, bm, eroded, nullptr, nullptr); \
    hipLaunchKernelGGL((k_morph<true, M>), g, blk, lds, st, b.vox, eroded, H, W, r, bm, opened, residue, residue16)
    switch (map_kind(bm)) {
    case 0: TS_MO(0); break;
    case 1: TS_MO(1); break;
    case 2: TS_MO(2); break;
    default: TS_MO(3); break;
    }
#undef TS_MO
    return check_launch("ts_open2d");
}

} // namespace ts
