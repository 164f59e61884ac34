// k_morph_r00.hip -- the opening's kernels for disk radii 0..12 (the
// kernels are in morph_dev.h; one source file per range of radii so that the
// fully unrolled kernels compile in parallel).
#include "morph_dev.h"

namespace ts {

bool launch_morph_0_12(int r, dim3 grid, hipStream_t st, const MorphArgs &ero, const MorphArgs &dil)
{
    return launch_morph_range<0, 12>(r, grid, st, ero, dil);
}

} // namespace ts
