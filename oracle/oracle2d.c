/*
 * oracle2d.c -- plain, slow FP64 CPU oracle for the paper's two-dimensional
 * Tsallis thresholding (Tsallis-entropy section: the 3x3 average image, the
 * 2D histogram of (gray level, average gray level), the threshold pair
 * (t, s), the class entropies H1, H2 over quadrants 1 and 3, and the arg max
 * of H1 + H2 + (1 - alpha) H1 H2; only t is used to threshold the image).
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c (built into the same library): it
 * shares nothing with the GPU library, and only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  Every routine
 * follows the definitions literally; speed is not a goal.
 *
 * Readings adopted here (the paper is silent or garbled):
 *  - the average image is the floor (the paper's "decimal part" is read as
 *    the integer part) of the mean of the 3x3 neighbourhood of gray levels,
 *    with f(x+i, y+j) for the printed f(x+i, y+i);
 *  - at the image border the neighbourhood repeats the nearest edge pixel;
 *  - gray levels come from the same bin map as the one-dimensional path;
 *  - class 1 is {i <= t, j <= s}, class 2 is {i > t, j > s} (quadrants 1 and
 *    3); the other two quadrants are ignored; t, s range over 0..L-2;
 *  - p_ij = h(i, j) / N; the printed P(i) inside the class sums is read as
 *    p_ij (the one-dimensional P(i) does not fit a double sum);
 *  - a class with zero mass makes the pair invalid; ties go to the first
 *    pair with t outermost; q = 1 is the Shannon (Kapur) limit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR2_OK 0
#define OR2_DEGENERATE 1
#define OR2_EMPTY 2
#define OR2_BADARG 3

#define OR2_MODE_DIRECT 0 /* region sums evaluated literally, O(L^2) per pair */
#define OR2_MODE_PREFIX 1 /* region sums from sequential 2-D prefix sums, O(1) */
#define OR2_MODE_KAPUR 2  /* Shannon (q -> 1) limit, literal sums */

int32_t or_bin(int32_t v, int32_t lo, int32_t hi, int32_t L); /* oracle.c */

/* The average gray image g of the gray-level image f (H rows of W). */
void or2_mean3x3(const int32_t *f, int32_t H, int32_t W, int32_t *g)
{
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x) {
            int64_t sum = 0;
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    int32_t yy = y + dy, xx = x + dx;
                    if (yy < 0)
                        yy = 0;
                    if (yy > H - 1)
                        yy = H - 1;
                    if (xx < 0)
                        xx = 0;
                    if (xx > W - 1)
                        xx = W - 1;
                    sum += f[(int64_t)yy * W + xx];
                }
            g[(int64_t)y * W + x] = (int32_t)(sum / 9); /* sum >= 0: division floors */
        }
}

/* The 2D histogram h(i, j) = #{(x, y) : f(x, y) = i and g(x, y) = j} of one
 * H x W image (counts; p_ij = h / N).  h is L*L, row i = gray level. */
void or2_histogram(const int16_t *img, int32_t H, int32_t W, int32_t lo, int32_t hi, int32_t L, uint32_t *h)
{
    const int64_t n = (int64_t)H * W;
    int32_t *f = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *g = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        f[i] = or_bin(img[i], lo, hi, L);
    or2_mean3x3(f, H, W, g);
    memset(h, 0, sizeof(uint32_t) * (size_t)L * (size_t)L);
    for (int64_t i = 0; i < n; ++i)
        h[(int64_t)f[i] * L + g[i]] += 1u;
    free(f);
    free(g);
}

/* Class entropy of the region [i0, i1] x [j0, j1] by literal sums. */
static double region_tsallis_direct(const uint32_t *h, int32_t L, double N, int32_t i0, int32_t i1, int32_t j0,
                                    int32_t j1, double q, double *mass)
{
    double w = 0.0;
    for (int32_t i = i0; i <= i1; ++i)
        for (int32_t j = j0; j <= j1; ++j)
            w += (double)h[(int64_t)i * L + j] / N;
    *mass = w;
    if (!(w > 0.0))
        return NAN;
    double s = 0.0;
    for (int32_t i = i0; i <= i1; ++i)
        for (int32_t j = j0; j <= j1; ++j) {
            const double p = (double)h[(int64_t)i * L + j] / N;
            if (p > 0.0)
                s += pow(p / w, q);
        }
    return (1.0 - s) / (q - 1.0);
}

static double region_shannon_direct(const uint32_t *h, int32_t L, double N, int32_t i0, int32_t i1, int32_t j0,
                                    int32_t j1, double *mass)
{
    double w = 0.0;
    for (int32_t i = i0; i <= i1; ++i)
        for (int32_t j = j0; j <= j1; ++j)
            w += (double)h[(int64_t)i * L + j] / N;
    *mass = w;
    if (!(w > 0.0))
        return NAN;
    double s = 0.0;
    for (int32_t i = i0; i <= i1; ++i)
        for (int32_t j = j0; j <= j1; ++j) {
            const double p = (double)h[(int64_t)i * L + j] / N;
            if (p > 0.0)
                s -= (p / w) * log(p / w);
        }
    return s;
}

/* Sequential 2-D prefix sums from both corners: for class 1 the rows of
 * (c, p^q) are summed left to right and then the row sums top to bottom; for
 * class 2 right to left and bottom to top.  Counts are exact integers. */
typedef struct {
    int32_t L;
    double N, q;
    int64_t *CA, *CB; /* [L*L] counts of {i <= t, j <= s} and {i >= t, j >= s} */
    double *QA, *QB;  /* [L*L] sums of p^q over the same regions */
} sat_t;

static int sat_init(sat_t *z, const uint32_t *h, int32_t L, double q)
{
    const size_t n = (size_t)L * (size_t)L;
    z->L = L;
    z->q = q;
    z->CA = (int64_t *)calloc(n, sizeof(int64_t));
    z->CB = (int64_t *)calloc(n, sizeof(int64_t));
    z->QA = (double *)calloc(n, sizeof(double));
    z->QB = (double *)calloc(n, sizeof(double));
    if (!z->CA || !z->CB || !z->QA || !z->QB)
        return 0;
    int64_t N = 0;
    for (size_t i = 0; i < n; ++i)
        N += h[i];
    z->N = (double)N;
    for (int32_t i = 0; i < L; ++i) { /* row prefix, left to right */
        int64_t c = 0;
        double s = 0.0;
        for (int32_t j = 0; j < L; ++j) {
            const uint32_t hij = h[(int64_t)i * L + j];
            c += hij;
            s += hij ? pow((double)hij / z->N, q) : 0.0;
            z->CA[(int64_t)i * L + j] = c;
            z->QA[(int64_t)i * L + j] = s;
        }
    }
    for (int32_t i = 1; i < L; ++i) /* then down the columns */
        for (int32_t j = 0; j < L; ++j) {
            z->CA[(int64_t)i * L + j] += z->CA[(int64_t)(i - 1) * L + j];
            z->QA[(int64_t)i * L + j] += z->QA[(int64_t)(i - 1) * L + j];
        }
    for (int32_t i = L - 1; i >= 0; --i) { /* row suffix, right to left */
        int64_t c = 0;
        double s = 0.0;
        for (int32_t j = L - 1; j >= 0; --j) {
            const uint32_t hij = h[(int64_t)i * L + j];
            c += hij;
            s += hij ? pow((double)hij / z->N, q) : 0.0;
            z->CB[(int64_t)i * L + j] = c;
            z->QB[(int64_t)i * L + j] = s;
        }
    }
    for (int32_t i = L - 2; i >= 0; --i) /* then up the columns */
        for (int32_t j = 0; j < L; ++j) {
            z->CB[(int64_t)i * L + j] += z->CB[(int64_t)(i + 1) * L + j];
            z->QB[(int64_t)i * L + j] += z->QB[(int64_t)(i + 1) * L + j];
        }
    return 1;
}

static void sat_free(sat_t *z)
{
    free(z->CA);
    free(z->CB);
    free(z->QA);
    free(z->QB);
}

/* Class entropy from a region's count and sum of p^q: sum (p/w)^q = Q / w^q. */
static double region_tsallis_prefix(int64_t C, double Q, double N, double q, double *mass)
{
    const double w = (double)C / N;
    *mass = w;
    if (!(w > 0.0))
        return NAN;
    return (1.0 - Q / pow(w, q)) / (q - 1.0);
}

/* The objective of the pair (t, s); NaN if a class is empty. */
static double pair_objective(const uint32_t *h, int32_t L, double N, double q, int32_t mode, const sat_t *z,
                             int32_t t, int32_t s)
{
    double H1, H2, w1, w2;
    if (mode == OR2_MODE_PREFIX) {
        H1 = region_tsallis_prefix(z->CA[(int64_t)t * L + s], z->QA[(int64_t)t * L + s], N, q, &w1);
        H2 = region_tsallis_prefix(z->CB[(int64_t)(t + 1) * L + s + 1], z->QB[(int64_t)(t + 1) * L + s + 1], N, q,
                                   &w2);
    } else if (mode == OR2_MODE_KAPUR) {
        H1 = region_shannon_direct(h, L, N, 0, t, 0, s, &w1);
        H2 = region_shannon_direct(h, L, N, t + 1, L - 1, s + 1, L - 1, &w2);
    } else {
        H1 = region_tsallis_direct(h, L, N, 0, t, 0, s, q, &w1);
        H2 = region_tsallis_direct(h, L, N, t + 1, L - 1, s + 1, L - 1, q, &w2);
    }
    if (!(w1 > 0.0) || !(w2 > 0.0))
        return NAN;
    if (mode == OR2_MODE_KAPUR)
        return H1 + H2;
    return H1 + H2 + (1.0 - q) * H1 * H2;
}

static int args2_ok(int32_t L, double q, int32_t mode)
{
    if (L < 2 || L > 4096)
        return 0;
    if (mode != OR2_MODE_DIRECT && mode != OR2_MODE_PREFIX && mode != OR2_MODE_KAPUR)
        return 0;
    if (mode != OR2_MODE_KAPUR && (!(q > 0.0) || q == 1.0 || !isfinite(q)))
        return 0;
    return 1;
}

double or2_objective(const uint32_t *h, int32_t L, double q, int32_t mode, int32_t t, int32_t s)
{
    if (!args2_ok(L, q, mode) || t < 0 || s < 0 || t > L - 2 || s > L - 2)
        return NAN;
    sat_t z;
    memset(&z, 0, sizeof(z));
    double N = 0.0;
    for (int64_t i = 0; i < (int64_t)L * L; ++i)
        N += h[i];
    if (mode == OR2_MODE_PREFIX && !sat_init(&z, h, L, q)) {
        sat_free(&z);
        return NAN;
    }
    const double S = N > 0.0 ? pair_objective(h, L, N, q, mode, &z, t, s) : NAN;
    sat_free(&z);
    return S;
}

/* Exhaustive arg max over (t, s), t outermost; strict > keeps the first of
 * equal values.  second = the best objective over the other valid pairs. */
int32_t or2_search(const uint32_t *h, int32_t L, double q, int32_t mode, int32_t *t_out, int32_t *s_out,
                   double *obj, double *second)
{
    *t_out = -1;
    *s_out = -1;
    *obj = NAN;
    *second = NAN;
    if (!args2_ok(L, q, mode))
        return OR2_BADARG;
    double N = 0.0;
    for (int64_t i = 0; i < (int64_t)L * L; ++i)
        N += h[i];
    if (!(N > 0.0))
        return OR2_EMPTY;
    sat_t z;
    memset(&z, 0, sizeof(z));
    if (mode == OR2_MODE_PREFIX && !sat_init(&z, h, L, q)) {
        sat_free(&z);
        return OR2_BADARG;
    }
    double best = -INFINITY, sec = -INFINITY;
    int found = 0;
    for (int32_t t = 0; t <= L - 2; ++t)
        for (int32_t s = 0; s <= L - 2; ++s) {
            const double S = pair_objective(h, L, N, q, mode, &z, t, s);
            if (isnan(S))
                continue;
            if (!found || S > best) {
                if (found)
                    sec = best > sec ? best : sec;
                best = S;
                *t_out = t;
                *s_out = s;
                found = 1;
            } else if (S > sec) {
                sec = S;
            }
        }
    sat_free(&z);
    if (!found)
        return OR2_DEGENERATE;
    *obj = best;
    *second = sec;
    return OR2_OK;
}
