// morph_dev.h -- the paper's morphology step (Morphology section): gray-scale
// erosion (minimum) and dilation (maximum) of the gray-level image under a
// flat disk B = {(dx, dy) : dx^2 + dy^2 <= r^2}, the opening (dilation of the
// erosion) and the residue original - opened that removes the large bright
// chest structures.  Pixels outside the image take no part.
//
// Decomposition.  The disk is the union over column offsets a = |dx| of
// vertical runs of half-height h(a) = floor(sqrt(r^2 - a^2)), so with
// V_h(x, y) = min over |dy| <= h of I(x, y + dy),
//     erosion(x, y) = min over |a| <= r of V_h(|a|)(x + a, y)
// (max for the dilation).  h is a step function of a: r + 1 offsets share a
// handful of distinct heights (7 at r = 10).
//
// Order of the gray-level map.  The map from stored values to gray levels is
// non-decreasing, so it commutes with min and max: the erosion runs on the
// raw int16 values and maps only its result, one map per output pixel
// instead of one per staged pixel.
//
// Layout.  One workgroup per tile of MV_TY rows and up to 2 * MV_THREADS
// columns of one image; each thread owns one pair of adjacent columns, two
// 16-bit values per 32-bit register (packed min/max: one instruction for two
// pixels).  A thread loads its column pair over the tile's rows and r rows
// above and below into registers (all loads in flight before the first is
// used) and grows V_h one unit of height at a time: two packed operations
// per row and unit, no cross-lane traffic.  At each distinct height the rows
// of V go to an LDS plane (two planes alternate, so one barrier per height
// suffices) and every thread folds in the offsets a with that height from
// its neighbours' words: a word d / 2 away for even d, the halves of two
// words joined by one byte align for odd d.  Images up to 2 * MV_THREADS
// pixels wide are one tile wide with no halo columns (outside the image the
// neutral value); wider images take tiles of 2 * (MV_THREADS - 2 ceil(r/2))
// output columns with ceil(r/2) halo column pairs each side.  The radius is
// a template parameter (every radius the entry point takes has its own
// kernel), so every row and offset index is a constant and the loops unroll.
// Workgroups of the same image run on the same XCD (its own L2), where tiles
// above and below re-read each other's halo rows.
#pragma once
#include "common.h"

namespace ts {

constexpr int MV_THREADS = 256; // threads per workgroup: one column pair each
// Output rows per tile.  A thread holds its column pair over MV_TY + 2r rows
// in registers; taller tiles load fewer halo rows per output row (the
// neighbours' halo rows mostly come from L2) but hold more registers and fit
// fewer wavefronts per SIMD.  Eight rows (68-76 VGPRs at r = 10, six or seven
// wavefronts) measured never more than 8 % slower than the fastest of 4, 6,
// 8, 12 and 16 rows at radii from 1 to 32 on 512- and 2048-wide images, and
// up to 37 % faster than 16 rows.
constexpr int MV_TY = 8;

// floor(sqrt(n)), n >= 0, at compile time
constexpr int mv_isqrt(int n)
{
    int g = 0;
    while ((g + 1) * (g + 1) <= n)
        ++g;
    return g;
}
// half-height of the disk of radius R at column offset a
constexpr int mv_chord(int R, int a) { return mv_isqrt(R * R - a * a); }
// whether some offset a in 0..R has half-height h, and how many distinct
// heights below h exist (the LDS plane parity of height h)
constexpr bool mv_is_level(int R, int h)
{
    for (int a = 0; a <= R; ++a)
        if (mv_chord(R, a) == h)
            return true;
    return false;
}
constexpr int mv_levels_below(int R, int h)
{
    int n = 0;
    for (int j = 0; j < h; ++j)
        n += mv_is_level(R, j) ? 1 : 0;
    return n;
}

typedef short mv_i16x2 __attribute__((ext_vector_type(2)));

// Two signed 16-bit lanes: min (MAXOP: max), v_pk_min_i16 / v_pk_max_i16.
template <bool MAXOP>
__device__ __forceinline__ uint32_t mv_op(uint32_t a, uint32_t b)
{
    const mv_i16x2 x = __builtin_bit_cast(mv_i16x2, a), y = __builtin_bit_cast(mv_i16x2, b);
    return __builtin_bit_cast(uint32_t, MAXOP ? __builtin_elementwise_max(x, y) : __builtin_elementwise_min(x, y));
}

struct MorphArgs {
    const int16_t *const *src16; // the images (int16 values)
    const uint8_t *src8;         // dilation: the eroded gray levels [nseg][H][W]
    int H, W;
    BinMap bm;
    int mapk;              // map_kind(bm)
    int tiles_x, tiles;    // tiles per image row band, per image
    int tp, hw;            // output column pairs per tile, halo column pairs left of them
    int ntiles;            // nseg * tiles
    uint8_t *dst;          // erosion: eroded gray levels; dilation: opened (or null)
    uint8_t *res;          // dilation: residue (or null)
    int16_t *res16;        // dilation: residue as int16 (or null)
};

// Buffer resource over one image of `bytes` bytes: loads and stores through
// it take the row's byte offset in a scalar register and the thread's byte
// offset within the row in a vector register (no 64-bit address arithmetic
// per lane, no row addresses held in registers).  Every offset the kernel
// forms lies inside the image.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mv_rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, 0x00020000);
}

// The tile's outputs from O (rows y0 ..): erosion, the gray levels of the
// minima of the raw values; dilation, the opened gray levels and the residue
// gray(original) - opened, the originals F loaded before the compute.
template <bool MAXOP, int MAP>
__device__ __forceinline__ void mv_epilogue(const MorphArgs &g, const uint32_t (&O)[MV_TY], const uint32_t (&F)[MV_TY],
                                            int64_t img, int y0, int x, bool out, bool pairs)
{
    const int H = g.H, W = g.W, npix = H * W;
    const int xo = max(x, 0);
    const __amdgpu_buffer_rsrc_t d8 = mv_rsrc(g.dst + img, npix), r8 = mv_rsrc(g.res + img, npix),
                                 r16 = mv_rsrc(g.res16 + img, 2 * npix);
    const bool want_res = MAXOP && (g.res || g.res16);
#pragma unroll
    for (int i = 0; i < MV_TY; ++i) {
        const int y = y0 + i;
        if (!out || y >= H)
            continue;
        const int ro = y * W;
        int v0, v1, g0 = 0, g1 = 0;
        if (!MAXOP) {
            v0 = bin_of_t<MAP>((int)(int16_t)(O[i] & 0xffffu), g.bm);
            v1 = bin_of_t<MAP>((int)(int16_t)(O[i] >> 16), g.bm);
        } else {
            v0 = (int)(O[i] & 0xffffu);
            v1 = (int)(O[i] >> 16);
            if (want_res) {
                g0 = bin_of_t<MAP>((int)(int16_t)(F[i] & 0xffffu), g.bm) - v0;
                g1 = bin_of_t<MAP>((int)(int16_t)(F[i] >> 16), g.bm) - v1;
            }
        }
        if (pairs) {
            if (g.dst)
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(v0 | (v1 << 8)), d8, xo, ro, 0);
            if (MAXOP && g.res)
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)((g0 & 0xff) | ((g1 & 0xff) << 8)), r8, xo, ro,
                                                      0);
            if (MAXOP && g.res16)
                __builtin_amdgcn_raw_buffer_store_b32((g0 & 0xffff) | ((uint32_t)(g1 & 0xffff) << 16), r16, 2 * xo,
                                                      2 * ro, 0);
        } else {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (x + e >= W)
                    continue;
                const int v = e ? v1 : v0, gr = e ? g1 : g0;
                if (g.dst)
                    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)v, d8, xo + e, ro, 0);
                if (MAXOP && g.res)
                    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)gr, r8, xo + e, ro, 0);
                if (MAXOP && g.res16)
                    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)gr, r16, 2 * (xo + e), 2 * ro, 0);
            }
        }
    }
}

// Fold the offsets a = A..R with half-height HH into O from the plane p (the
// thread's own word at p[0]; V holds the same rows in registers).
template <bool MAXOP, int R, int HH, int PS, int A = 0>
__device__ __forceinline__ void mv_combine(uint32_t (&O)[MV_TY], const uint32_t (&V)[MV_TY], const uint32_t *p)
{
    if constexpr (A <= R) {
        if constexpr (mv_chord(R, A) == HH) {
#pragma unroll
            for (int i = 0; i < MV_TY; ++i) {
                const uint32_t *q = p + i * PS;
                if constexpr (A == 0) {
                    O[i] = mv_op<MAXOP>(O[i], V[i]);
                } else if constexpr ((A & 1) == 0) {
                    constexpr int k = A >> 1;
                    O[i] = mv_op<MAXOP>(O[i], mv_op<MAXOP>(q[-k], q[k]));
                } else {
                    // pixels 2t - A, 2t + 1 - A: the high half of the word k
                    // away on the left, the low half of the word k - 1 away;
                    // mirrored on the right
                    constexpr int k = (A + 1) >> 1;
                    const uint32_t l0 = q[-k], l1 = k == 1 ? V[i] : q[1 - k];
                    const uint32_t r0 = k == 1 ? V[i] : q[k - 1], r1 = q[k];
                    const uint32_t lft = __builtin_amdgcn_alignbyte(l1, l0, 2);
                    const uint32_t rgt = __builtin_amdgcn_alignbyte(r1, r0, 2);
                    O[i] = mv_op<MAXOP>(O[i], mv_op<MAXOP>(lft, rgt));
                }
            }
        }
        mv_combine<MAXOP, R, HH, PS, A + 1>(O, V, p);
    }
}

// whether a neighbour's offset (a > 0) has half-height h: only then do the
// rows of that height go through LDS
constexpr bool mv_needs_plane(int R, int h)
{
    for (int a = 1; a <= R; ++a)
        if (mv_chord(R, a) == h)
            return true;
    return false;
}

// Heights HH..R: grow V by one unit of height, and at each distinct height
// publish V and fold in its offsets.
template <bool MAXOP, int R, int HH, int NI, int PS>
__device__ __forceinline__ void mv_levels(uint32_t (&O)[MV_TY], uint32_t (&V)[MV_TY], const uint32_t (&I)[NI],
                                          uint32_t *planes, int c)
{
    if constexpr (HH > 0) {
#pragma unroll
        for (int i = 0; i < MV_TY; ++i)
            V[i] = mv_op<MAXOP>(V[i], mv_op<MAXOP>(I[i + R - HH], I[i + R + HH]));
    }
    if constexpr (mv_is_level(R, HH)) {
        constexpr int B = mv_levels_below(R, HH) & 1;
        uint32_t *p = planes + B * (MV_TY * PS) + c;
        if constexpr (mv_needs_plane(R, HH)) {
#pragma unroll
            for (int i = 0; i < MV_TY; ++i)
                p[i * PS] = V[i];
            __syncthreads();
        }
        mv_combine<MAXOP, R, HH, PS>(O, V, p);
    }
    if constexpr (HH < R)
        mv_levels<MAXOP, R, HH + 1, NI, PS>(O, V, I, planes, c);
}

// MAXOP = false: erosion of the raw values of the int16 images (src16) into
// the gray levels dst; MAXOP = true: dilation of the gray levels src8 into
// dst (opened) and/or the residue gray(src16) - opened into res (uint8) and
// res16 (int16).
template <bool MAXOP, int R>
__global__ void __launch_bounds__(MV_THREADS) k_morph(MorphArgs g)
{
    constexpr int HP = (R + 1) / 2;             // plane padding words each side
    constexpr int PS = MV_THREADS + 2 * HP;     // plane row stride in words
    constexpr int NI = MV_TY + 2 * R;           // rows a thread loads
    constexpr uint32_t NEUT = MAXOP ? 0x80008000u : 0x7fff7fffu;
    __shared__ uint32_t planes[2 * MV_TY * PS];
    // workgroup b runs on XCD b mod 8: give each XCD a contiguous range of
    // tiles (vertical neighbours share halo rows through that XCD's L2)
    const int per = (int)(gridDim.x >> 3);
    const int lb = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    if (lb >= g.ntiles)
        return;
    const int s = lb / g.tiles, tl = lb % g.tiles;
    const int tx = tl % g.tiles_x, ty = tl / g.tiles_x;
    const int H = g.H, W = g.W;
    const int y0 = ty * MV_TY, t = threadIdx.x;
    const int x = tx * 2 * g.tp + 2 * (t - g.hw); // first pixel column of the thread's pair
    const bool out = t >= g.hw && t < g.hw + g.tp && x < W;
    const int64_t img = (int64_t)s * H * W;
    const TS_GLOBAL int16_t *img16 = gp(g.src16[s]);
    // with an even width and aligned images the two pixels of a pair are both
    // inside or both outside the image and load and store as one access
    bool pairs = (W & 1) == 0 && (((uintptr_t)img16) & 3) == 0;
    if (MAXOP)
        pairs = pairs && ((uintptr_t)(g.src8 + img) & 1) == 0 && ((uintptr_t)g.dst & 1) == 0 &&
                ((uintptr_t)g.res & 1) == 0 && ((uintptr_t)g.res16 & 3) == 0;
    else
        pairs = pairs && ((uintptr_t)g.dst & 1) == 0;
    // neutral padding left and right of every plane row (never overwritten)
    if constexpr (HP > 0) {
        for (int i = t; i < 2 * MV_TY * 2 * HP; i += MV_THREADS) {
            const int j = i % (2 * HP), row = i / (2 * HP);
            planes[row * PS + (j < HP ? j : MV_THREADS + j)] = NEUT;
        }
    }
    // the thread's column pair over rows y0 - R .. y0 + MV_TY - 1 + R (rows
    // and columns outside the image clamped for the load, then neutral), and
    // for the dilation's residue the original values of its output rows
    const int npix = H * W;
    const __amdgpu_buffer_rsrc_t b16 = mv_rsrc((const void *)img16, 2 * npix);
    const __amdgpu_buffer_rsrc_t b8 = mv_rsrc(g.src8 + img, npix);
    uint32_t I[NI], F[MV_TY];
    const bool xin0 = x >= 0 && x < W, xin1 = x + 1 >= 0 && x + 1 < W;
    const bool want_f = MAXOP && (g.res || g.res16);
    if (pairs) {
        const int xo = min(max(x, 0), W - 2);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ro = min(max(y0 - R + i, 0), H - 1) * W;
            if (MAXOP)
                I[i] = __builtin_amdgcn_perm(0u, (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(b8, xo, ro, 0),
                                             0x0c010c00u); // bytes b0, 0, b1, 0
            else
                I[i] = __builtin_amdgcn_raw_buffer_load_b32(b16, 2 * xo, 2 * ro, 0);
        }
        if (want_f) {
#pragma unroll
            for (int i = 0; i < MV_TY; ++i)
                F[i] = __builtin_amdgcn_raw_buffer_load_b32(b16, 2 * xo, 2 * min(y0 + i, H - 1) * W, 0);
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int y = y0 - R + i;
            I[i] = (y >= 0 && y < H && xin0) ? I[i] : NEUT;
        }
    } else {
        const int xo0 = min(max(x, 0), W - 1), xo1 = min(max(x + 1, 0), W - 1);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ro = min(max(y0 - R + i, 0), H - 1) * W;
            uint32_t v0, v1;
            if (MAXOP) {
                v0 = __builtin_amdgcn_raw_buffer_load_b8(b8, xo0, ro, 0);
                v1 = __builtin_amdgcn_raw_buffer_load_b8(b8, xo1, ro, 0);
            } else {
                v0 = __builtin_amdgcn_raw_buffer_load_b16(b16, 2 * xo0, 2 * ro, 0);
                v1 = __builtin_amdgcn_raw_buffer_load_b16(b16, 2 * xo1, 2 * ro, 0);
            }
            const bool yin = y0 - R + i >= 0 && y0 - R + i < H;
            v0 = yin && xin0 ? v0 : (NEUT & 0xffffu);
            v1 = yin && xin1 ? v1 : (NEUT & 0xffffu);
            I[i] = v0 | (v1 << 16);
        }
        if (want_f) {
#pragma unroll
            for (int i = 0; i < MV_TY; ++i) {
                const int ro = 2 * min(y0 + i, H - 1) * W;
                F[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(b16, 2 * xo0, ro, 0) |
                       ((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(b16, 2 * xo1, ro, 0) << 16);
            }
        }
    }
    uint32_t V[MV_TY], O[MV_TY];
#pragma unroll
    for (int i = 0; i < MV_TY; ++i) {
        V[i] = I[i + R];
        O[i] = NEUT;
    }
    mv_levels<MAXOP, R, 0, NI, PS>(O, V, I, planes, HP + t);
    switch (g.mapk) {
    case 0: mv_epilogue<MAXOP, 0>(g, O, F, img, y0, x, out, pairs); break;
    case 1: mv_epilogue<MAXOP, 1>(g, O, F, img, y0, x, out, pairs); break;
    case 2: mv_epilogue<MAXOP, 2>(g, O, F, img, y0, x, out, pairs); break;
    default: mv_epilogue<MAXOP, 3>(g, O, F, img, y0, x, out, pairs); break;
    }
}

// Both passes of the opening for radius R on stream st.
template <int R>
static void launch_morph_r(dim3 grid, hipStream_t st, const MorphArgs &ero, const MorphArgs &dil)
{
    hipLaunchKernelGGL((k_morph<false, R>), grid, dim3(MV_THREADS), 0, st, ero);
    hipLaunchKernelGGL((k_morph<true, R>), grid, dim3(MV_THREADS), 0, st, dil);
}

// The passes for radius r if R0 <= r <= R1 (returns whether it launched).
template <int R0, int R1>
static bool launch_morph_range(int r, dim3 grid, hipStream_t st, const MorphArgs &ero, const MorphArgs &dil)
{
    if constexpr (R0 <= R1) {
        if (r == R0) {
            launch_morph_r<R0>(grid, st, ero, dil);
            return true;
        }
        return launch_morph_range<R0 + 1, R1>(r, grid, st, ero, dil);
    }
    return false;
}

// The kernels of each range of radii live in a source file of their own
// (k_morph_rNN.hip: radius NN and up), so that they compile in parallel.
#define TS_MORPH_RANGES(X) X(0, 12) X(13, 18) X(19, 23) X(24, 27) X(28, 30) X(31, 32)
#define TS_MORPH_DECL(a, b) bool launch_morph_##a##_##b(int r, dim3 grid, hipStream_t st, const MorphArgs &ero, const MorphArgs &dil);
TS_MORPH_RANGES(TS_MORPH_DECL)
#undef TS_MORPH_DECL

} // namespace ts

