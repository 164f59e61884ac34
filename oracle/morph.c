/*
 * morph.c -- plain CPU oracle for the paper's morphology step (Morphology
 * section: erosion A (-) B = {z | (B)_z contained in A}, dilation
 * A (+) B = {z | (B^)_z meets A}, opening = dilation of the erosion, and the
 * chest removed by a subtraction involving the opened image).
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c (built into the same library): it
 * shares nothing with the GPU library, and only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  Every pixel is
 * computed from its definition by plain loops; speed is not a goal.
 *
 * Readings adopted here (the paper is silent or ambiguous):
 *  - A is the gray-level image (the same bin map as the histogram), so the
 *    operations are the gray-scale ones: erosion = minimum and dilation =
 *    maximum of the image under the structuring element;
 *  - B is a flat disk of radius r pixels, {(dx, dy) : dx^2 + dy^2 <= r^2}
 *    ("size 10" read as the radius), symmetric, so B^ = B;
 *  - pixels outside the image take no part in the minimum or maximum;
 *  - the chest is removed by original - opened (the opening never exceeds
 *    the original, so the printed order opened - original would be <= 0
 *    everywhere): the residue keeps the structures narrower than the disk.
 */
#include <stdint.h>

/* Gray-scale erosion (take_max = 0) or dilation (take_max = 1) of the
   H x W image f by the disk of radius r. */
void or_morph(const int32_t *f, int32_t H, int32_t W, int32_t r, int32_t take_max, int32_t *out)
{
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x) {
            int32_t best = f[(int64_t)y * W + x]; /* the centre is in B */
            for (int32_t dy = -r; dy <= r; ++dy)
                for (int32_t dx = -r; dx <= r; ++dx) {
                    if (dx * dx + dy * dy > r * r)
                        continue; /* outside the disk */
                    const int32_t yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue; /* outside the image */
                    const int32_t v = f[(int64_t)yy * W + xx];
                    if (take_max ? v > best : v < best)
                        best = v;
                }
            out[(int64_t)y * W + x] = best;
        }
}

/* Opening (erosion, then dilation of the result) and the residue
   original - opened.  tmp holds the eroded image. */
void or_open(const int32_t *f, int32_t H, int32_t W, int32_t r, int32_t *tmp, int32_t *opened, int32_t *residue)
{
    or_morph(f, H, W, r, 0, tmp);
    or_morph(tmp, H, W, r, 1, opened);
    for (int64_t i = 0; i < (int64_t)H * W; ++i)
        residue[i] = f[i] - opened[i];
}
