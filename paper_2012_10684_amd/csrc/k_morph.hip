// k_morph.hip -- host side of the morphology step (Morphology section): tile
// shape and launch of the opening's two passes (erosion, then dilation with
// the residue).  The kernels and their design are in morph_dev.h.
#include <string>

#include "morph_dev.h"

namespace ts {

static_assert(TS_MORPH_MAX_RADIUS == 32, "the ranges of radii with kernels end at 32");

size_t open2d_workspace_bytes(int nseg, int H, int W) { return (size_t)nseg * H * W; }

ts_status launch_open2d(const ts_batch &b, int H, int W, const BinMap &bm, int r, uint8_t *eroded,
                        uint8_t *opened, uint8_t *residue, int16_t *residue16, hipStream_t st)
{
    MorphArgs a = {};
    a.src16 = b.vox;
    a.H = H;
    a.W = W;
    a.bm = bm;
    a.mapk = map_kind(bm);
    if (W <= 2 * MV_THREADS) { // one tile across, no halo columns
        a.tiles_x = 1;
        a.tp = MV_THREADS;
        a.hw = 0;
    } else {
        a.hw = (r + 1) / 2;
        a.tp = MV_THREADS - 2 * a.hw;
        a.tiles_x = (W + 2 * a.tp - 1) / (2 * a.tp);
    }
    a.tiles = a.tiles_x * ((H + MV_TY - 1) / MV_TY);
    const int64_t nt = (int64_t)b.nseg * a.tiles;
    if (nt > (int64_t)INT32_MAX - 8)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: too many tiles for one launch");
    a.ntiles = (int)nt;
    const dim3 grid((unsigned)((nt + 7) & ~(int64_t)7));
    MorphArgs ero = a, dil = a;
    ero.dst = eroded;
    dil.src8 = eroded;
    dil.dst = opened;
    dil.res = residue;
    dil.res16 = residue16;
    bool done = false;
#define TS_MORPH_CALL(a, b) done = done || launch_morph_##a##_##b(r, grid, st, ero, dil);
    TS_MORPH_RANGES(TS_MORPH_CALL)
#undef TS_MORPH_CALL
    if (!done)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: radius must be in 0.." + std::to_string(TS_MORPH_MAX_RADIUS));
    return check_launch("ts_open2d");
}

} // namespace ts
