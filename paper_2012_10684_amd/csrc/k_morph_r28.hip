// k_morph_r28.hip -- the opening's kernels for disk radii 28..30 (the
// kernels are in morph_dev.h; one source file per range of radii so that the
// fully unrolled kernels compile in parallel).
#include "morph_dev.h"

namespace ts {

bool launch_morph_28_30(int r, dim3 grid, hipStream_t st, const MorphArgs &ero, const MorphArgs &dil)
{
    return launch_morph_range<28, 30>(r, grid, st, ero, dil);
}

} // namespace ts
