/*
 * oracle.c -- plain, slow FP64 CPU oracle for maximum-Tsallis-entropy
 * thresholding of CT intensity data (Chang & Sheu, arXiv 2012.10684).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  It shares no code, header, table or constant with the
 * GPU library, and nothing in the product path may link or call it: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it.  Every routine below follows the paper's definitions literally and in
 * the paper's order; speed is not a goal.
 *
 * Readings of the paper adopted here (the paper is silent or ambiguous):
 *  - bin map: inclusive HU window [lo,hi] of width W = hi-lo+1 split into L
 *    equal integer-floor bins; values below/above the window go to the first
 *    /last bin (Pre-processing section: levels are linearly mapped onto the
 *    gray-level range).
 *  - index ranges: class 1 holds bins 0..t and class 2 bins t+1..L-1, so a
 *    threshold ranges over 0..L-2 (Tsallis-entropy section, the sums that
 *    define H1, H2, P1, P2).
 *  - more than two classes: the pseudo-additive composition rule of the
 *    objective phi is applied recursively, T <- T + S_j + (1-q) T S_j.
 *    A second composition, the multilevel form used elsewhere in the
 *    literature, sum_j S_j + (1-q) prod_j S_j, is offered beside it
 *    (or_search_c / or_objective_c with OR_COMP_SUMPROD); both equal the
 *    paper's H1 + H2 + (1-q) H1 H2 for one threshold.
 *  - a class with zero probability mass makes the tuple invalid.
 *  - bins with p_i = 0 contribute nothing to the sum of (p_i/w)^q.
 *  - ties: the first tuple in lexicographic order (t1 outermost) wins.
 *  - labels: a voxel in bin b gets #{j : b > t_j}; for one threshold this is
 *    the thresholding kernel function (Algorithm 1) with T = t+1 in bin units.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_DEGENERATE 1
#define OR_EMPTY 2
#define OR_BADARG 3

#define OR_MODE_DIRECT 0 /* class sums evaluated literally, O(L) per class */
#define OR_MODE_PREFIX 1 /* class sums from sequential prefix sums, O(1) */
#define OR_MODE_KAPUR 2  /* Shannon (q -> 1) limit, literal sums */

#define OR_COMP_RECURSIVE 0 /* T <- T + S_j + (1-q) T S_j */
#define OR_COMP_SUMPROD 1   /* sum_j S_j + (1-q) prod_j S_j */

/* ------------------------------------------------------------------ */
/* Pre-processing section: linear map of intensity levels to L gray levels. */
int32_t or_bin(int32_t v, int32_t lo, int32_t hi, int32_t L)
{
    if (v < lo)
        return 0;
    if (v > hi)
        return L - 1;
    int64_t W = (int64_t)hi - (int64_t)lo + 1;
    return (int32_t)(((int64_t)v - (int64_t)lo) * (int64_t)L / W);
}

void or_bin_map(const int16_t *vox, int64_t n, int32_t lo, int32_t hi, int32_t L, int32_t *bins)
{
    for (int64_t i = 0; i < n; ++i)
        bins[i] = or_bin(vox[i], lo, hi, L);
}

/* Thresholding section: the histogram of brightness levels is the
   measurement space, c_i = number of voxels whose level is i. */
void or_histogram(const int16_t *vox, int64_t n, int32_t lo, int32_t hi, int32_t L, uint32_t *hist)
{
    for (int32_t i = 0; i < L; ++i)
        hist[i] = 0;
    for (int64_t i = 0; i < n; ++i)
        hist[or_bin(vox[i], lo, hi, L)] += 1u;
}

/* ------------------------------------------------------------------ */
/* Tsallis-entropy section: the probability set p_i = c_i / N, and the
   class masses P(t) = sum_{i<=t} p_i.  Also Q(t) = sum_{i<=t} p_i^q, both
   summed left to right. */
void or_prefix(const uint32_t *hist, int32_t L, double q, double *P, double *Q)
{
    int64_t N = 0;
    for (int32_t i = 0; i < L; ++i)
        N += hist[i];
    int64_t C = 0;
    double acc = 0.0;
    for (int32_t i = 0; i < L; ++i) {
        C += hist[i];
        if (N == 0) {
            P[i] = 0.0;
            Q[i] = 0.0;
            continue;
        }
        P[i] = (double)C / (double)N;
        if (hist[i] > 0)
            acc += pow((double)hist[i] / (double)N, q);
        Q[i] = acc;
    }
}

/* Class Tsallis entropy of the bins a..b (inclusive), evaluated literally:
   w = sum p_i,  S = (1 - sum_{p_i>0} (p_i / w)^q) / (q - 1).
   Returns NAN when w == 0 (the tuple is invalid). */
static double class_tsallis_direct(const double *p, int32_t a, int32_t b, double q)
{
    double w = 0.0;
    for (int32_t i = a; i <= b; ++i)
        w += p[i];
    if (!(w > 0.0))
        return NAN;
    double s = 0.0;
    for (int32_t i = a; i <= b; ++i)
        if (p[i] > 0.0)
            s += pow(p[i] / w, q);
    return (1.0 - s) / (q - 1.0);
}

/* Shannon entropy of the bins a..b normalised by their mass (the q -> 1
   limit of the class Tsallis entropy). */
static double class_shannon_direct(const double *p, int32_t a, int32_t b)
{
    double w = 0.0;
    for (int32_t i = a; i <= b; ++i)
        w += p[i];
    if (!(w > 0.0))
        return NAN;
    double s = 0.0;
    for (int32_t i = a; i <= b; ++i)
        if (p[i] > 0.0) {
            double r = p[i] / w;
            s -= r * log(r);
        }
    return s;
}

/* Same class entropy from the prefix sums: w = (C(b) - C(a-1)) / N and
   sum (p_i / w)^q = (Q(b) - Q(a-1)) / w^q. */
static double class_tsallis_prefix(const int64_t *C, const double *Q, int64_t N, int32_t a, int32_t b, double q)
{
    int64_t cnt = C[b] - (a > 0 ? C[a - 1] : 0);
    if (cnt <= 0)
        return NAN;
    double w = (double)cnt / (double)N;
    double dq = Q[b] - (a > 0 ? Q[a - 1] : 0.0);
    return (1.0 - dq / pow(w, q)) / (q - 1.0);
}

/* Objective phi: pseudo-additive composition of the class entropies,
   T <- T + S_j + (1 - q) T S_j (Tsallis-entropy section, the bracket inside
   the arg max); for the Kapur limit the composition is the plain sum. */
static double compose(const double *S, int32_t ncls, double q, int kapur)
{
    double T = S[0];
    for (int32_t j = 1; j < ncls; ++j) {
        if (kapur)
            T = T + S[j];
        else
            T = T + S[j] + (1.0 - q) * T * S[j];
    }
    return T;
}

/* The multilevel variant: the plain sum of the class entropies plus (1 - q)
   times their product (for the Kapur limit, the plain sum). */
static double compose_sumprod(const double *S, int32_t ncls, double q, int kapur)
{
    double sum = 0.0, prod = 1.0;
    for (int32_t j = 0; j < ncls; ++j) {
        sum += S[j];
        prod *= S[j];
    }
    return kapur ? sum : sum + (1.0 - q) * prod;
}

typedef struct {
    int32_t L;
    double q;
    int32_t mode;
    int64_t N;
    double *p;      /* [L] probabilities (direct / kapur) */
    int64_t *C;     /* [L] count prefix (prefix mode) */
    double *Q;      /* [L] prefix of p^q (prefix mode) */
    double *table;  /* [L*L] class entropies memoised by (a,b) (prefix mode, k >= 2) */
    int32_t comp;   /* OR_COMP_* */
} ctx_t;

static double class_entropy(const ctx_t *cx, int32_t a, int32_t b)
{
    if (cx->mode == OR_MODE_DIRECT)
        return class_tsallis_direct(cx->p, a, b, cx->q);
    if (cx->mode == OR_MODE_KAPUR)
        return class_shannon_direct(cx->p, a, b);
    if (cx->table)
        return cx->table[(int64_t)a * cx->L + b];
    return class_tsallis_prefix(cx->C, cx->Q, cx->N, a, b, cx->q);
}

/* Objective of one tuple t_1 < ... < t_k: classes [0,t_1], [t_1+1,t_2], ...,
   [t_k+1, L-1].  NAN when a class is empty. */
static double tuple_objective(const ctx_t *cx, const int32_t *t, int32_t k)
{
    double S[16] = {NAN};
    int32_t a = 0;
    for (int32_t j = 0; j <= k; ++j) {
        int32_t b = (j < k) ? t[j] : cx->L - 1;
        S[j] = class_entropy(cx, a, b);
        if (isnan(S[j]))
            return NAN;
        a = b + 1;
    }
    if (cx->comp == OR_COMP_SUMPROD)
        return compose_sumprod(S, k + 1, cx->q, cx->mode == OR_MODE_KAPUR);
    return compose(S, k + 1, cx->q, cx->mode == OR_MODE_KAPUR);
}

static int ctx_init(ctx_t *cx, const uint32_t *hist, int32_t L, int32_t k, double q, int32_t mode)
{
    memset(cx, 0, sizeof(*cx));
    cx->L = L;
    cx->q = q;
    cx->mode = mode;
    for (int32_t i = 0; i < L; ++i)
        cx->N += hist[i];
    if (cx->N == 0)
        return OR_EMPTY;
    if (mode == OR_MODE_DIRECT || mode == OR_MODE_KAPUR) {
        cx->p = (double *)malloc(sizeof(double) * L);
        for (int32_t i = 0; i < L; ++i)
            cx->p[i] = (double)hist[i] / (double)cx->N;
        return OR_OK;
    }
    cx->C = (int64_t *)malloc(sizeof(int64_t) * L);
    cx->Q = (double *)malloc(sizeof(double) * L);
    double *P = (double *)malloc(sizeof(double) * L);
    or_prefix(hist, L, q, P, cx->Q);
    free(P);
    int64_t c = 0;
    for (int32_t i = 0; i < L; ++i) {
        c += hist[i];
        cx->C[i] = c;
    }
    if (k >= 2) {
        /* memoise every class (a,b); each is evaluated by the same formula */
        cx->table = (double *)malloc(sizeof(double) * (size_t)L * (size_t)L);
        if (!cx->table)
            return OR_BADARG;
        for (int32_t a = 0; a < L; ++a)
            for (int32_t b = a; b < L; ++b)
                cx->table[(int64_t)a * L + b] = class_tsallis_prefix(cx->C, cx->Q, cx->N, a, b, q);
    }
    return OR_OK;
}

static void ctx_free(ctx_t *cx)
{
    free(cx->p);
    free(cx->C);
    free(cx->Q);
    free(cx->table);
}

static int args_ok(int32_t L, int32_t k, double q, int32_t mode)
{
    if (k < 1 || k > 15 || L < 2 || L > 65536)
        return 0;
    if (mode < 0 || mode > 2)
        return 0;
    if (mode != OR_MODE_KAPUR && (!(q > 0.0) || q == 1.0 || !isfinite(q)))
        return 0;
    return 1;
}

/* Exhaustive arg max of the objective over every tuple t_1 < ... < t_k with
   t_j in [0, L-2], visited in lexicographic order; the first strictly
   greater value wins (arg max of phi, Tsallis-entropy section).
   Outputs: thr[k] (all -1 when no tuple is valid), *best, and *second = the
   largest objective over all valid tuples other than the winner (NAN if
   there is none).  Returns OR_OK, OR_DEGENERATE, OR_EMPTY or OR_BADARG. */
int32_t or_search_c(const uint32_t *hist, int32_t L, int32_t k, double q, int32_t mode, int32_t comp,
                    int32_t *thr, double *best, double *second)
{
    for (int32_t j = 0; j < k && j < 16; ++j)
        thr[j] = -1;
    *best = NAN;
    *second = NAN;
    if (!args_ok(L, k, q, mode))
        return OR_BADARG;
    if (k > L - 1)
        return OR_DEGENERATE;
    if (comp != OR_COMP_RECURSIVE && comp != OR_COMP_SUMPROD)
        return OR_BADARG;
    ctx_t cx;
    int st = ctx_init(&cx, hist, L, k, q, mode);
    cx.comp = comp;
    if (st != OR_OK) {
        ctx_free(&cx);
        return st;
    }
    int32_t t[16];
    for (int32_t j = 0; j < k; ++j)
        t[j] = j;
    int found = 0;
    double b1 = -INFINITY, b2 = -INFINITY;
    int have2 = 0;
    for (;;) {
        double S = tuple_objective(&cx, t, k);
        if (!isnan(S)) {
            if (!found || S > b1) {
                if (found) {
                    b2 = b1;
                    have2 = 1;
                }
                b1 = S;
                found = 1;
                for (int32_t j = 0; j < k; ++j)
                    thr[j] = t[j];
            } else if (!have2 || S > b2) {
                b2 = S;
                have2 = 1;
            }
        }
        /* next tuple in lexicographic order */
        int32_t j = k - 1;
        while (j >= 0 && t[j] >= (L - 2) - (k - 1 - j))
            --j;
        if (j < 0)
            break;
        t[j] += 1;
        for (int32_t m = j + 1; m < k; ++m)
            t[m] = t[m - 1] + 1;
    }
    ctx_free(&cx);
    if (!found)
        return OR_DEGENERATE;
    *best = b1;
    *second = have2 ? b2 : NAN;
    return OR_OK;
}

int32_t or_search(const uint32_t *hist, int32_t L, int32_t k, double q, int32_t mode,
                  int32_t *thr, double *best, double *second)
{
    return or_search_c(hist, L, k, q, mode, OR_COMP_RECURSIVE, thr, best, second);
}

/* Objective of one given tuple (NAN if invalid or out of range). */
double or_objective_c(const uint32_t *hist, int32_t L, int32_t k, double q, int32_t mode, int32_t comp,
                      const int32_t *thr)
{
    if (!args_ok(L, k, q, mode) || (comp != OR_COMP_RECURSIVE && comp != OR_COMP_SUMPROD))
        return NAN;
    for (int32_t j = 0; j < k; ++j) {
        if (thr[j] < 0 || thr[j] > L - 2)
            return NAN;
        if (j > 0 && thr[j] <= thr[j - 1])
            return NAN;
    }
    ctx_t cx;
    int st = ctx_init(&cx, hist, L, 1, q, mode); /* no table: one tuple only */
    cx.comp = comp;
    double S = NAN;
    if (st == OR_OK)
        S = tuple_objective(&cx, thr, k);
    ctx_free(&cx);
    return S;
}

double or_objective(const uint32_t *hist, int32_t L, int32_t k, double q, int32_t mode, const int32_t *thr)
{
    return or_objective_c(hist, L, k, q, mode, OR_COMP_RECURSIVE, thr);
}

/* Dynamic programme for many thresholds, where the exhaustive search cannot
   finish (e.g. four thresholds over 1024 levels: 4.5e10 tuples).  The
   recursive composition T <- T + S_j + (1-q) T S_j multiplies the factors
   1 + (1-q) S_j (1 + (1-q) T' = (1 + (1-q) T)(1 + (1-q) S_j)), so phi is a
   strictly increasing function of F = sum_j f_j with
   f_j = sgn(1-q) ln(1 + (1-q) S_j) (for the Kapur limit f_j = S_j and F = T):
   the arg max of phi over the tuples is the arg max of F, a sum over
   consecutive classes.  With W_m(a) the best F of the bins a..L-1 split into
   m + 1 classes,
       W_0(a) = f(a, L-1),   W_m(a) = max_t [ f(a, t) + W_{m-1}(t + 1) ],
   the maximum is W_k(0), and the first tuple attaining it (t_1 outermost) is
   rebuilt forward by taking the smallest t whose term equals the table value
   exactly (the same sums in the same order).  S_j are the class entropies of
   the prefix mode (or the literal Shannon sums); an empty class is invalid.
   Outputs thr[k] and *best = phi at the optimum (expm1(sgn F) / (1 - q), or F
   for Kapur).  Returns OR_OK, OR_DEGENERATE, OR_EMPTY or OR_BADARG. */
int32_t or_search_dp(const uint32_t *hist, int32_t L, int32_t k, double q, int32_t mode, int32_t *thr,
                     double *best)
{
    for (int32_t j = 0; j < k && j < 16; ++j)
        thr[j] = -1;
    *best = NAN;
    if (!args_ok(L, k, q, mode) || mode == OR_MODE_DIRECT)
        return OR_BADARG;
    if (k > L - 1)
        return OR_DEGENERATE;
    ctx_t cx;
    int st = ctx_init(&cx, hist, L, 2, q, mode); /* every class (a, b) memoised (prefix mode) */
    if (st != OR_OK) {
        ctx_free(&cx);
        return st;
    }
    const int kapur = mode == OR_MODE_KAPUR;
    const double sgn = q < 1.0 ? 1.0 : -1.0;
    double *f = (double *)malloc(sizeof(double) * (size_t)L * (size_t)L); /* f[a * L + b], a <= b */
    double *W = (double *)malloc(sizeof(double) * (size_t)(k + 1) * (size_t)L);
    for (int32_t a = 0; a < L; ++a)
        for (int32_t b = a; b < L; ++b) {
            const double S = class_entropy(&cx, a, b);
            f[(int64_t)a * L + b] = isnan(S) ? -INFINITY : (kapur ? S : sgn * log(1.0 + (1.0 - q) * S));
        }
    for (int32_t a = 0; a < L; ++a)
        W[a] = f[(int64_t)a * L + (L - 1)];
    for (int32_t m = 1; m <= k; ++m)
        for (int32_t a = 0; a < L; ++a) {
            double v = -INFINITY;
            /* class [a, t], then m more classes of at least one bin each */
            for (int32_t t = a; t <= L - 1 - m; ++t) {
                const double x = f[(int64_t)a * L + t] + W[(size_t)(m - 1) * L + t + 1];
                if (x > v)
                    v = x;
            }
            W[(size_t)m * L + a] = v;
        }
    const double F = W[(size_t)k * L];
    if (!(F > -INFINITY)) {
        free(f);
        free(W);
        ctx_free(&cx);
        return OR_DEGENERATE;
    }
    int32_t a = 0;
    for (int32_t m = k; m >= 1; --m) {
        const double want = W[(size_t)m * L + a];
        int32_t t = a;
        while (t <= L - 1 - m && !(f[(int64_t)a * L + t] + W[(size_t)(m - 1) * L + t + 1] == want))
            ++t;
        thr[k - m] = t;
        a = t + 1;
    }
    *best = kapur ? F : expm1(sgn * F) / (1.0 - q);
    free(f);
    free(W);
    ctx_free(&cx);
    return OR_OK;
}

/* Thresholding kernel function (Algorithm 1) generalised to k thresholds:
   label = number of thresholds strictly below the voxel's bin.  A tuple
   whose first entry is negative (no valid tuple) labels everything 0. */
void or_label(const int16_t *vox, int64_t n, int32_t lo, int32_t hi, int32_t L,
              const int32_t *thr, int32_t k, uint8_t *out)
{
    int degenerate = (k < 1) || thr[0] < 0;
    for (int64_t i = 0; i < n; ++i) {
        if (degenerate) {
            out[i] = 0;
            continue;
        }
        int32_t b = or_bin(vox[i], lo, hi, L);
        uint8_t c = 0;
        for (int32_t j = 0; j < k; ++j)
            if (b > thr[j])
                ++c;
        out[i] = c;
    }
}
