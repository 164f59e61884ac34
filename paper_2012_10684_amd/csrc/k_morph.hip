// k_morph.hip -- the paper's morphology step (Morphology section): gray-scale
// erosion (minimum) and dilation (maximum) of the gray-level image under a
// flat disk B = {(dx, dy) : dx^2 + dy^2 <= r^2}, the opening (dilation of the
// erosion) and the residue original - opened that removes the large bright
// chest structures.  Pixels outside the image take no part.
//
// One workgroup per 64 x 64 output tile of one image.  The tile and a halo of
// r pixels are staged in LDS (gray levels; outside the image the neutral
// value, 255 for the minimum and 0 for the maximum) with a fixed row stride,
// so that a thread's staged rows sit at constant offsets from each other.
// The disk is the union over row offsets dy of horizontal runs of half-width
// w(dy) = floor(sqrt(r^2 - dy^2)); w grows as |dy| falls, so each thread
// holds the horizontal minimum (maximum) of its staged rows in registers and
// widens them one distinct w at a time (two LDS byte reads and one min3 per
// row and unit of width), then publishes them in a row buffer H; each output
// takes the minimum (maximum) of H at rows y - |dy| and y + |dy| when w =
// w(dy).  Per output pixel and pass: about 2r (1 + 2r / 64) LDS reads to
// widen and 2r + 2 to combine.
#include "common.h"

namespace ts {

constexpr int MO_TX = 64, MO_TY = 64, MO_THREADS = 256;
constexpr int MO_PER = MO_TX * MO_TY / MO_THREADS; // outputs per thread
constexpr int MO_SW = MO_TX + 2 * TS_MORPH_MAX_RADIUS;  // staged row stride (the largest staged row)
constexpr int MO_SH = MO_TY + 2 * TS_MORPH_MAX_RADIUS;  // largest staged column
constexpr int MO_PH = MO_THREADS / MO_TX;               // row phases: thread rows yb, yb + 4, ...
constexpr int MO_ROWS = MO_SH / MO_PH;                  // staged rows per thread, at most

// min (MAXOP: max) of three values as one v_min3_u32 / v_max3_u32 (the
// compiler would split it into a 16-bit and a 32-bit operation)
template <bool MAXOP>
__device__ __forceinline__ unsigned op3(unsigned a, unsigned b, unsigned c)
{
    unsigned r;
    if (MAXOP)
        asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    else
        asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
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
    __shared__ uint8_t in[MO_SH * MO_SW];
    __shared__ uint8_t hr[MO_SH * MO_TX];
    const int tiles_x = (W + MO_TX - 1) / MO_TX, tiles_y = (H + MO_TY - 1) / MO_TY;
    const int s = blockIdx.x / (tiles_x * tiles_y);
    const int tile = blockIdx.x % (tiles_x * tiles_y);
    const int x0 = (tile % tiles_x) * MO_TX, y0 = (tile / tiles_x) * MO_TY;
    const int sw = MO_TX + 2 * r, sh = MO_TY + 2 * r;
    const uint8_t neutral = MAXOP ? 0 : 255;
    const int64_t img_off = (int64_t)s * H * W;
    const TS_GLOBAL int16_t *img16 = gp(src16[s]);
    const int c = threadIdx.x % MO_TX, yb = threadIdx.x / MO_TX; // lane column, row phase (0..3)
    // stage the tile and its halo: rows yb, yb + 4, ..., columns c, c + 64
    for (int row = yb; row < sh; row += MO_PH) {
        const int y = y0 - r + row;
        const bool yin = y >= 0 && y < H;
        for (int col = c; col < sw; col += MO_TX) {
            const int x = x0 - r + col;
            int v = neutral;
            if (yin && x >= 0 && x < W) {
                if (MAXOP)
                    v = src8[img_off + (int64_t)y * W + x];
                else
                    v = bin_of_t<MAP>(img16[(int64_t)y * W + x], bm);
            }
            in[row * MO_SW + col] = (uint8_t)v;
        }
    }
    // this thread's staged rows yb + 4 i, i < nr, in groups of four (rows of
    // the last group past sh read staged memory that is never used)
    const int nr = __builtin_amdgcn_readfirstlane((sh - yb + MO_PH - 1) / MO_PH); // the same in the wavefront
    const uint8_t *cin = in + yb * MO_SW + c + r; // row yb, column c of the tile
    unsigned hv[MO_ROWS];
    __syncthreads();
#pragma unroll
    for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
        if (i0 < nr) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                hv[i0 + u] = cin[(i0 + u) * MO_PH * MO_SW]; // half-width 0: the staged pixel itself
        }
    // publish the rows at their current half-width into hr
    auto publish = [&]() {
#pragma unroll
        for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
            if (i0 < nr) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + u < nr)
                        hr[(yb + (i0 + u) * MO_PH) * MO_TX + c] = (uint8_t)hv[i0 + u];
            }
    };
    publish();
    // outputs (yb + 4 i, c), i < MO_PER
    int out[MO_PER];
#pragma unroll
    for (int i = 0; i < MO_PER; ++i)
        out[i] = neutral;
    int cur = 0, wg = 0;
    __syncthreads(); // hr at half-width 0
    for (int a = r; a >= 0; --a) {
        const int w = wg = isqrt_from(r * r - a * a, wg);
        if (w > cur) { // widen every staged row of the thread from half-width cur to w
            for (int d = cur + 1; d <= w; ++d) {
                const uint8_t *pl = cin - d, *pr = cin + d;
#pragma unroll
                for (int i0 = 0; i0 < MO_ROWS; i0 += 4)
                    if (i0 < nr) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int o = (i0 + u) * MO_PH * MO_SW;
                            hv[i0 + u] = op3<MAXOP>(hv[i0 + u], pl[o], pr[o]);
                        }
                    }
            }
            __syncthreads(); // the combine steps before have read hr
            publish();
            cur = w;
            __syncthreads();
        }
        // rows y - a and y + a of every output take half-width w(a); output
        // i sits 4 i staged rows below output 0 (immediate LDS offsets)
        const uint8_t *plo = hr + (yb + r - a) * MO_TX + c, *phi = hr + (yb + r + a) * MO_TX + c;
#pragma unroll
        for (int i = 0; i < MO_PER; ++i) {
            const int lo = plo[4 * MO_TX * i], hi = phi[4 * MO_TX * i];
            out[i] = MAXOP ? max(out[i], max(lo, hi)) : min(out[i], min(lo, hi));
        }
    }
    const int x = x0 + c;
    if (x >= W)
        return;
#pragma unroll
    for (int i = 0; i < MO_PER; ++i) {
        const int y = y0 + yb + 4 * i;
        if (y >= H)
            continue;
        const int64_t o = img_off + (int64_t)y * W + x;
        if (dst)
            dst[o] = out[i];
        if (MAXOP && (res || res16)) {
            const int f = bin_of_t<MAP>(img16[(int64_t)y * W + x], bm);
            if (res)
                res[o] = (uint8_t)(f - (int)out[i]);
            if (res16)
                res16[o] = (int16_t)(f - (int)out[i]);
        }
    }
}

size_t open2d_workspace_bytes(int nseg, int H, int W) { return (size_t)nseg * H * W; }

ts_status launch_open2d(const ts_batch &b, int H, int W, const BinMap &bm, int r, uint8_t *eroded,
                        uint8_t *opened, uint8_t *residue, int16_t *residue16, hipStream_t st)
{
    const int tiles = ((W + MO_TX - 1) / MO_TX) * ((H + MO_TY - 1) / MO_TY);
    const dim3 g((unsigned)((int64_t)b.nseg * tiles)), blk(MO_THREADS);
#define TS_MO(M)                                                                                                     \
    hipLaunchKernelGGL((k_morph<false, M>), g, blk, 0, st, b.vox, nullptr, H, W, r, bm, eroded, nullptr, nullptr);  \
    hipLaunchKernelGGL((k_morph<true, M>), g, blk, 0, st, b.vox, eroded, H, W, r, bm, opened, residue, residue16)
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
