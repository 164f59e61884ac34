/*
 * ts.h -- C ABI of the MI355X (gfx950) library for maximum-Tsallis-entropy
 * threshold segmentation of CT volumes (Chang & Sheu, arXiv 2012.10684).
 *
 * The path is four calls, each following one step of the paper's statement of
 * the problem:
 *   ts_histogram        histogram of brightness levels, the "measurement
 *                       space" of thresholding (Thresholding section), after
 *                       the linear map of intensities onto gray levels
 *                       (Pre-processing section);
 *   ts_prefix           the probability set p_i and the class masses
 *                       P(t) = sum_{i<=t} p_i, plus Q(t) = sum_{i<=t} p_i^q
 *                       (Tsallis-entropy section, the sums defining H1, H2,
 *                       P1, P2);
 *   ts_threshold_search arg max of the pseudo-additive objective
 *                       H1 + H2 + (1-q) H1 H2 (Tsallis-entropy section),
 *                       extended to k = 1..3 thresholds by applying the
 *                       composition rule recursively;
 *   ts_label            the thresholding kernel function (Algorithm 1),
 *                       extended to k thresholds.
 *   ts_label_sets       ts_label for several threshold sets in one pass;
 *   ts_log2_f32         diagnostic: the FP32 logarithm of the search keys;
 *   ts_histogram2d,     the paper's two-dimensional form: 2D histogram of
 *   ts_threshold_search2d  (gray level, 3x3 average gray level) and the
 *                       arg max over threshold pairs (t, s).
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE pointers unless marked [host].  The caller allocates
 *    and owns every buffer; no call allocates device memory.  Scratch memory
 *    for the search is passed in as a workspace.
 *  - Every call is asynchronous on `stream` (a hipStream_t, or NULL for the
 *    default stream) and does not synchronise the host.
 *  - Argument errors are detected on the host before any launch and returned
 *    synchronously; nothing is launched then.  TS_ERR_HIP reports a failed
 *    launch; faults inside kernels surface at the caller's next
 *    synchronisation of the stream.  ts_last_error() gives a text for the
 *    last non-OK status returned on the calling thread.
 *  - The device contents of a ts_batch (pointers and offsets) cannot be
 *    checked on the host: offsets must be non-decreasing with offs[0] = 0
 *    and offs[nseg] = total, and every pointer must address at least its
 *    problem's voxel count.  Violations are undefined behaviour.
 *  - Results are bit-identical across runs, tunings and batch compositions.
 */
#ifndef TS_H
#define TS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ts_stream_t; /* a hipStream_t; NULL = the default stream */

/* Largest number of entropic indices q that ts_prefix and
 * ts_threshold_search take in one call. */
#define TS_MAX_Q 8

typedef enum {
    TS_OK = 0,
    TS_ERR_INVALID_ARG = 1, /* bad sizes, null pointers, bad q/k/window */
    TS_ERR_UNSUPPORTED = 2, /* valid request the library does not implement (none at present) */
    TS_ERR_WORKSPACE = 3,   /* workspace smaller than ts_search_workspace_bytes() */
    TS_ERR_HIP = 4          /* a HIP runtime call or kernel launch failed */
} ts_status;

/* [host] Intensity window and number of gray levels (bins).  A voxel v in
 * [lo, hi] goes to bin floor((v - lo) * nbins / (hi - lo + 1)); v < lo goes
 * to bin 0 and v > hi to bin nbins - 1.  Requires lo <= hi, both within
 * int16, and 2 <= nbins <= 4096. */
typedef struct {
    int32_t lo;
    int32_t hi;
    int32_t nbins;
} ts_binning;

/* A batch of nseg independent problems (slices, slabs or volumes).  Problem s
 * is the offs[s+1] - offs[s] contiguous int16 voxels at vox[s].
 *   vox   device array [nseg] of device pointers (2-byte aligned);
 *   offs  device array [nseg + 1], offs[0] = 0, non-decreasing;
 *   nseg  number of problems (>= 0);
 *   total [host] copy of offs[nseg] (sizes the launch). */
typedef struct {
    const int16_t *const *vox;
    const int64_t *offs;
    int32_t nseg;
    int64_t total;
} ts_batch;

/* Search modes. */
enum {
    TS_SEARCH_FP32_TIECHECK = 0, /* FP32 exhaustive keys, then an FP64 re-check of every
                                    tuple within the FP32 error bound (default; exact) */
    TS_SEARCH_FP32_ONLY = 1,     /* FP32 keys only: first tuple with the largest FP32 key */
    TS_SEARCH_FP64 = 2,          /* FP64 exhaustive keys */
    TS_SEARCH_PLAIN = 3,         /* one thread per tuple, all classes evaluated directly in
                                    FP64, one launch per problem: the simple GPU form */
    TS_SEARCH_SUMPROD = 4,       /* a different objective: the multilevel form
                                    sum_j S_j + (1-q) prod_j S_j of the class entropies
                                    (equal to the paper's for k = 1), FP64 exhaustive, all
                                    problems in one launch; obj is that value */
    TS_SEARCH_PLAIN_FP32 = 5     /* one thread per tuple, every class term evaluated directly in
                                    FP32 (the keys of TS_SEARCH_FP32_ONLY, from the prefix sums
                                    split into two floats), one launch per problem: the simple
                                    GPU form in single precision; the first tuple with the
                                    largest key; obj is its FP64 objective */
};

/* Per-problem outcome written by ts_threshold_search. */
enum {
    TS_PROBLEM_OK = 0,
    TS_PROBLEM_DEGENERATE = 1, /* no valid tuple: fewer than k+1 occupied bins */
    TS_PROBLEM_EMPTY = 2,      /* the problem has no voxels */
    TS_PROBLEM_SYNC_FAILED = 3 /* ts_segment's one-problem path: a wait between its workgroups gave up
                                  (never expected: the launch keeps them all resident); outputs invalid */
};

/* [host] Optional launch shapes (NULL, or 0 in a field, selects the built-in
 * default).  Tunings never change any output bit. */
typedef struct {
    int32_t hist_block;      /* threads per histogram workgroup: 64..1024, multiple of 64 */
    int32_t hist_replicas;   /* LDS copies of every bin: 1, 2, 4, 8, 16 or 32 */
    int32_t hist_wg_per_cu;  /* persistent histogram workgroups per compute unit: 1..16 */
    int32_t label_block;     /* threads per label workgroup: 64..1024, multiple of 64 */
    int32_t label_vecs;      /* 16-byte vectors (8 voxels) per label thread: 1, 2 or 4 */
    int32_t search_cols;     /* threshold columns held per lane in a search tile: 1, 2 or 4 */
    int32_t search_rows;     /* rows (first-threshold values) per k=2 search tile: 16..4096, multiple of 4 */
    int32_t min_chunk;       /* minimum voxels per histogram workgroup: >= 512 */
    int32_t search_path;     /* 1: one workgroup per problem (k <= 2, nbins <= 1024, or k = 1),
                                2: one launch per search phase; 0: chosen from the sizes */
    int32_t search_block;    /* threads per workgroup on the one-workgroup path: 256, 512 or 1024 */
    int32_t segment_parts;   /* ts_segment: workgroups per problem, 1..64 (1: the whole path of a
                                problem in one workgroup and one launch) */
    int32_t segment_block;   /* ts_segment: threads per workgroup: 256, 512 or 1024 (raised to what
                                the prefix scan of nbins needs) */
} ts_tuning;

/* ts_histogram -- per-problem histograms of gray levels (Thresholding
 * section: histogram of brightness levels; Pre-processing section: linear
 * map of intensities to gray levels, here the window rule of ts_binning).
 *   batch  problems to count;
 *   bin    [host] window and number of bins L;
 *   hist   out: uint32 [nseg][L], overwritten; row s counts problem s.
 *          Counts are exact (a problem may hold up to 2^32 - 1 voxels).
 * Errors: TS_ERR_INVALID_ARG for nseg < 0, total < 0, null pointers when
 * nseg > 0, or an invalid binning. */
ts_status ts_histogram(ts_batch batch, ts_binning bin, uint32_t *hist, const ts_tuning *tune,
                       ts_stream_t stream);

/* ts_prefix -- probabilities and prefix sums (Tsallis-entropy section:
 * p_i = c_i / N with N = sum c_i, class masses P(t) = sum_{i<=t} p_i, and
 * Q(t) = sum_{i<=t} p_i^q, the sum whose differences give the class sums of
 * p_i^q in H1 and H2), for nq entropic indices at once (the same section
 * leaves the index alpha as a parameter to tune, so a caller may search
 * several values on the same image).
 *   hist   uint32 [nseg][nbins] from ts_histogram;
 *   nq, q  [host] nq (1..TS_MAX_Q) entropic indices (the paper's alpha),
 *          each finite and > 0; q = 1 selects the Shannon limit (below);
 *   P      out: double [nseg][nbins], P(t) = C(t)/N with C(t) the exact
 *          integer count prefix (one rounding); P(nbins-1) = 1 exactly.
 *          P does not depend on q;
 *   Q      out: double [nq][nseg][nbins], row (j, s) for q[j]: Q(t) =
 *          sum_{i<=t} p_i^q, or sum_{i<=t} p_i ln p_i for q = 1 (the limit
 *          q -> 1 of the Tsallis class entropy is the Shannon entropy, whose
 *          class sums need p ln p).  Q is summed so that an empty bin repeats
 *          the previous value bit for bit.  A problem with N = 0 gets
 *          P = Q = 0.
 * Errors: TS_ERR_INVALID_ARG for nseg < 0, nbins outside [2, 4096], nq out
 * of range, null pointers when nseg > 0, a q not finite or <= 0. */
ts_status ts_prefix(const uint32_t *hist, int32_t nseg, int32_t nbins, int32_t nq, const double *q, double *P,
                    double *Q, ts_stream_t stream);

/* [host] Bytes of workspace ts_threshold_search needs for these sizes
 * (0 for invalid sizes). */
size_t ts_search_workspace_bytes(int32_t nseg, int32_t nbins, int32_t k, int32_t nq, int32_t mode);

/* ts_threshold_search -- exhaustive arg max of the Tsallis objective
 * (Tsallis-entropy section: phi = arg max [H1 + H2 + (1-q) H1 H2]) over every
 * tuple 0 <= t_1 < ... < t_k <= nbins-2 of thresholds.  Classes are
 * [0,t_1], [t_1+1,t_2], ..., [t_k+1, nbins-1]; the k+1 class entropies are
 * composed by the pseudo-additive rule applied recursively, which equals
 * S = expm1(Lambda)/(1-q) with Lambda = sum_j [ln Q_j - q ln w_j] (Q_j the
 * class sum of p_i^q, w_j the class mass).  A tuple with an empty class is
 * invalid.  Ties go to the first tuple in lexicographic order.  The nq x nseg
 * problems (one per entropic index and histogram) are searched in one pass.
 *   P, Q    double [nseg][nbins] and [nq][nseg][nbins] from ts_prefix with
 *           the same q array;
 *   k       1, 2 or 3;
 *   nq, q   [host] nq (1..TS_MAX_Q) entropic indices, each finite and > 0.
 *           q = 1 is the Shannon limit (Kapur's objective): class entropies
 *           S_j = -sum (p_i/w_j) ln(p_i/w_j) composed by addition, S = sum S_j;
 *   mode    TS_SEARCH_*;
 *   ws      device workspace of ws_bytes >= ts_search_workspace_bytes(...);
 *           its contents on entry are ignored;
 *   thr     out: int32 [nq][nseg][k], ascending, or all -1 if no valid tuple;
 *   obj     out: double [nq][nseg], the objective S at thr in FP64 (NaN if
 *           none): expm1(Lambda)/(1-q), or sum S_j for q = 1;
 *   status  out: int32 [nq][nseg], TS_PROBLEM_*.
 * A degenerate or empty problem does not affect the others in the batch.
 * Errors: TS_ERR_INVALID_ARG (sizes, pointers, k, nq, q, mode),
 * TS_ERR_WORKSPACE. */
ts_status ts_threshold_search(const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                              int32_t nq, const double *q, int32_t mode, void *ws, size_t ws_bytes, int32_t *thr,
                              double *obj, int32_t *status, const ts_tuning *tune, ts_stream_t stream);

/* [host] Bytes of workspace ts_segment needs for these sizes (labels: whether
 * it writes labels); 0 if the sizes are invalid. */
size_t ts_segment_workspace_bytes(int32_t nseg, int32_t nbins, int32_t k, int32_t nq, int32_t mode, int32_t labels);

/* ts_segment -- the whole path in one call: per problem the histogram of
 * gray levels (as ts_histogram), the prefix sums (as ts_prefix), the arg max
 * threshold tuple for every q (as ts_threshold_search) and the labels (as
 * ts_label_sets).  Every output is bit-identical to those calls'.  For
 * k <= 2 in the FP32 modes (nbins <= 4096 for k = 1, <= 1024 for k = 2;
 * nq <= TS_MAX_LABEL_SETS when labelling) and at least twice as many
 * problems as the GPU has compute units (or tune->segment_parts >= 1) the
 * steps run fused: with one workgroup per problem the whole path of a
 * problem is one workgroup of one launch (its voxels read twice, nothing
 * else leaves the chip but the histogram and the results); with several
 * workgroups per problem (tune->segment_parts > 1) the last one to finish
 * counting does the prefix sums and the search, then one label launch.
 * One problem with k = 1, one q and FP32_TIECHECK (up to 4,194,304 voxels,
 * nbins <= 4096, no tune->segment_parts) runs as one launch of up to 64
 * workgroups that share the histogram, the prefix sums (each computing one
 * 64-thread group of the scan in the prefix pass's summation order), the
 * FP64 objective of every threshold and the labels, with three grid-wide
 * waits between the stages; status TS_PROBLEM_SYNC_FAILED reports a wait
 * that gave up (not expected: the workgroups are few enough to be resident
 * at once).  Otherwise the separate passes run, in this one call.
 *   batch, bin, k, nq, q, mode   as for ts_histogram / ts_threshold_search;
 *   hist    out: uint32 [nseg][L];
 *   thr, obj, status   out: as ts_threshold_search ([nq][nseg][k], [nq][nseg]);
 *   out     [host] array [nq] of device tables of [nseg] device pointers (as
 *           ts_label_sets), or NULL for no labels;
 *   ws      device workspace of ws_bytes >= ts_segment_workspace_bytes(...);
 *           its contents on entry are ignored (the per-problem tickets that
 *           find the last workgroup of a problem are tagged with a value
 *           that changes with every call).  Concurrent calls must not share
 *           a workspace.
 * Errors: as the separate calls; TS_ERR_WORKSPACE for a workspace too small. */
ts_status ts_segment(ts_batch batch, ts_binning bin, int32_t k, int32_t nq, const double *q, int32_t mode,
                     uint32_t *hist, int32_t *thr, double *obj, int32_t *status, uint8_t *const *const *out,
                     void *ws, size_t ws_bytes, const ts_tuning *tune, ts_stream_t stream);

/* Bytes of the library-owned device scratch behind
 * ts_threshold_search_noalloc (one array per GPU, held until the process
 * ends). */
#define TS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* ts_threshold_search_noalloc -- ts_threshold_search for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * ts_threshold_search, without the workspace: the kernels that need one use
 * a fixed library-owned device array of TS_NOALLOC_SCRATCH_BYTES per GPU.
 * Nothing is allocated by this call (no hipMalloc, no library allocator).
 * The scratch is shared by every call on one GPU and keeps the last call's
 * contents (the kernels initialise every word they read); calls that overlap
 * on one GPU (different streams or threads) race on it and must be
 * serialised by the caller.
 * Errors: as ts_threshold_search, and TS_ERR_WORKSPACE when these sizes need
 * more than TS_NOALLOC_SCRATCH_BYTES of scratch (the one-workgroup-per-problem
 * path needs none), TS_ERR_HIP when the scratch's device address cannot be
 * obtained. */
ts_status ts_threshold_search_noalloc(const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                                      int32_t nq, const double *q, int32_t mode, int32_t *thr, double *obj,
                                      int32_t *status, const ts_tuning *tune, ts_stream_t stream);

/* Largest number of thresholds ts_threshold_search_dp finds and ts_label /
 * ts_label_sets apply. */
#define TS_DP_MAX_K 16

/* ts_label -- thresholding kernel function (Algorithm 1) with k thresholds:
 * a voxel whose gray level (ts_binning rule) is b gets the label
 * #{j : b > t_j} (0..k); for k = 1 this is 1 iff b >= T with T = t + 1.
 *   batch  problems to label (same layout as for ts_histogram);
 *   bin    [host] the binning used for the histogram;
 *   k      1..TS_DP_MAX_K;
 *   thr    int32 [nseg][k] from ts_threshold_search(_dp).  A row that is not
 *          strictly ascending within [0, nbins-2] (e.g. the all -1 row of a
 *          degenerate problem) labels its whole problem 0;
 *   out    device array [nseg] of device pointers; problem s writes
 *          offs[s+1]-offs[s] uint8 labels at out[s], in voxel order.
 * Errors: TS_ERR_INVALID_ARG for bad sizes, k, binning or null pointers. */
ts_status ts_label(ts_batch batch, ts_binning bin, const int32_t *thr, int32_t k, uint8_t *const *out,
                   const ts_tuning *tune, ts_stream_t stream);

/* ts_histogram2d -- 2D histograms of the two-dimensional method
 * (Tsallis-entropy section, 2D form): for every pixel of every image, the
 * gray level f (ts_binning rule) and the average gray level
 * g = floor(sum of f over the 3x3 neighbourhood / 9), the neighbourhood
 * repeating the nearest edge pixel at the image border; h(i, j) counts the
 * pixels with f = i and g = j.
 *   batch   nseg images, each height x width int16 pixels in row-major order
 *           (offs[s+1] - offs[s] = height * width for every s; the host
 *           checks total = nseg * height * width);
 *   height, width  image size; 1 <= width <= 4096;
 *   bin     [host] the binning; nbins <= 256;
 *   hist    out: uint32 [nseg][nbins][nbins] (row = gray level, column =
 *           average gray level), overwritten.
 * Errors: TS_ERR_INVALID_ARG for bad sizes, binning or null pointers. */
ts_status ts_histogram2d(ts_batch batch, int32_t height, int32_t width, ts_binning bin, uint32_t *hist,
                         ts_stream_t stream);

/* [host] Bytes of workspace ts_threshold_search2d needs (0 if invalid). */
size_t ts_search2d_workspace_bytes(int32_t nseg, int32_t nbins, int32_t nq);

/* ts_threshold_search2d -- arg max over threshold pairs (t, s), t, s in
 * [0, nbins-2], of H1 + H2 + (1-q) H1 H2 for the classes {i <= t, j <= s}
 * and {i > t, j > s} of the 2D histogram (Tsallis-entropy section, 2D
 * form; the other two quadrants are ignored).  A pair with an empty class is
 * invalid; ties go to the first pair with t outermost; q = 1 is the Shannon
 * limit (sum of the two class Shannon entropies).  The class sums come
 * from 2-D prefix sums formed inside the call, pairs are ranked by FP32
 * keys, and every pair whose key lies within twice the keys' proven error
 * bound of the best key is evaluated in FP64: the result is the FP64 arg
 * max.
 *   hist    uint32 [nseg][nbins][nbins] from ts_histogram2d;
 *   nq, q   [host] 1..TS_MAX_Q entropic indices, finite, > 0;
 *   ws      device workspace of ws_bytes >= ts_search2d_workspace_bytes(),
 *           8-byte aligned; overwritten;
 *   thr     out: int32 [nq][2][nseg]: t in row 0, s in row 1 of each q
 *           (-1 if no valid pair); only t thresholds the image, and row 0
 *           is the [nseg][1] threshold array of ts_label with k = 1;
 *   obj     out: double [nq][nseg], the objective at (t, s) (NaN if none);
 *   status  out: int32 [nq][nseg], TS_PROBLEM_*.
 * Errors: TS_ERR_INVALID_ARG (also for a workspace that is not 8-byte
 * aligned), TS_ERR_WORKSPACE. */
ts_status ts_threshold_search2d(const uint32_t *hist, int32_t nseg, int32_t nbins, int32_t nq, const double *q,
                                void *ws, size_t ws_bytes, int32_t *thr, double *obj, int32_t *status,
                                ts_stream_t stream);

/* [host] Bytes of workspace ts_threshold_search_dp needs (0 if invalid):
 * k * nq * nseg * nbins doubles. */
size_t ts_search_dp_workspace_bytes(int32_t nseg, int32_t nbins, int32_t k, int32_t nq);

/* ts_threshold_search_dp -- the arg max of ts_threshold_search (same
 * objective, classes, validity and first-tuple rule) by dynamic programming
 * over the class boundaries instead of enumerating tuples, for any k in
 * 1..TS_DP_MAX_K (Tsallis-entropy section: with 1 + (1-q) S = prod_j
 * Q_j / w_j^q the arg max of S is the arg max of a sum of class terms, which
 * is separable over consecutive classes).  k (nbins-1)^2 / 2 FP64 class
 * terms per problem instead of C(nbins-1, k) tuples.  The maximum is exact
 * for the per-tuple sums formed right to left in FP64 (the exhaustive
 * search forms them left to right: the two can differ in the last bits, so
 * of two tuples within a few ulps either may be reported); among the tuples
 * reaching it, the first in lexicographic order is returned, and tuples that
 * differ only inside runs of empty bins tie exactly.
 *   P, Q, nq, q   as for ts_threshold_search;
 *   k             1..TS_DP_MAX_K, nbins >= k + 1;
 *   ws            device workspace of ws_bytes >= ts_search_dp_workspace_bytes(),
 *                 8-byte aligned; overwritten;
 *   thr           out: int32 [nq][nseg][k], ascending, or all -1;
 *   obj           out: double [nq][nseg], the objective S (NaN if none);
 *   status        out: int32 [nq][nseg], TS_PROBLEM_*.
 * Errors: TS_ERR_INVALID_ARG, TS_ERR_WORKSPACE. */
ts_status ts_threshold_search_dp(const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                                 int32_t nq, const double *q, void *ws, size_t ws_bytes, int32_t *thr, double *obj,
                                 int32_t *status, ts_stream_t stream);

/* Largest disk radius ts_open2d takes. */
#define TS_MORPH_MAX_RADIUS 32
/* Largest image ts_open2d takes, in pixels (its int16 bytes fit a signed 32-bit offset). */
#define TS_MORPH_MAX_PIXELS 1073741823

/* [host] Bytes of workspace ts_open2d needs: one byte per pixel. */
size_t ts_open2d_workspace_bytes(int32_t nseg, int32_t height, int32_t width);

/* ts_open2d -- the morphology step before thresholding (Morphology section):
 * gray-scale opening of each image's gray levels (the ts_binning rule) by a
 * flat disk of the given radius, B = {(dx, dy) : dx^2 + dy^2 <= radius^2}:
 * erosion (the minimum under B), then dilation (the maximum under B) of the
 * result; pixels outside the image take no part.  The residue
 * gray - opened (>= 0) is the image with the structures wider than the disk
 * (the chest) removed.
 *   batch   nseg images of height x width int16 pixels, row-major (one
 *           pointer per image; total = nseg * height * width);
 *   bin     [host] the binning; nbins <= 256;
 *   radius  0..TS_MORPH_MAX_RADIUS (the paper's disk: 10);
 *   ws      device workspace of ws_bytes >= ts_open2d_workspace_bytes()
 *           (the eroded images); overwritten;
 *   opened    out: uint8 [nseg][height][width], or NULL;
 *   residue   out: uint8 [nseg][height][width], or NULL;
 *   residue16 out: the residue as int16 [nseg][height][width], or NULL: gray
 *             levels that ts_histogram / ts_label take directly with the
 *             binning {0, nbins-1, nbins} (each level its own bin), so the
 *             threshold is selected on the image after the morphology step,
 *             as the paper's segmentation does (at least one output).
 * Errors: TS_ERR_INVALID_ARG (also for an image of more than
 * TS_MORPH_MAX_PIXELS pixels), TS_ERR_WORKSPACE. */
ts_status ts_open2d(ts_batch batch, int32_t height, int32_t width, ts_binning bin, int32_t radius, void *ws,
                    size_t ws_bytes, uint8_t *opened, uint8_t *residue, int16_t *residue16, ts_stream_t stream);

/* Largest number of threshold sets ts_label_sets takes in one call. */
#define TS_MAX_LABEL_SETS 4

/* ts_label_sets -- ts_label for several threshold sets of one batch (e.g.
 * the thresholds found for several values of the tunable entropic index,
 * Tsallis-entropy section), in one pass over the voxels: each voxel is read
 * once and one label is written per set.  Labels are bit-identical to nsets
 * separate ts_label calls (Algorithm 1 applied once per set).
 *   nsets  1..TS_MAX_LABEL_SETS;
 *   thr    [host] array of nsets device pointers, each int32 [nseg][k]
 *          (same rules as ts_label's thr);
 *   out    [host] array of nsets device arrays [nseg] of device pointers
 *          (same layout as ts_label's out).  The outputs of different sets
 *          must not overlap.
 * Errors: as ts_label, and TS_ERR_INVALID_ARG for nsets out of range. */
ts_status ts_label_sets(ts_batch batch, ts_binning bin, int32_t nsets, const int32_t *const *thr, int32_t k,
                        uint8_t *const *const *out, const ts_tuning *tune, ts_stream_t stream);

/* ts_log2_f32 -- diagnostic: y[i] = the FP32 base-2 logarithm that the
 * FP32 search keys use (the hardware v_log_f32).  The bound on the FP32 key
 * error that decides which tuples the FP64 tie check revisits takes this
 * logarithm to be within 4 units of 2^-24 * max(1, |log2 x|) of log2(x) for
 * normal x; this call lets that be measured against an exact log2.
 *   x, y   device float [n]; n >= 0.
 * Errors: TS_ERR_INVALID_ARG for n < 0 or null pointers when n > 0. */
ts_status ts_log2_f32(const float *x, float *y, int64_t n, ts_stream_t stream);

/* ts_issue_rate -- diagnostic: one launch of `blocks` workgroups of 256
 * threads in which every lane issues `iters` blocks of independent FP32
 * vector instructions: op 0 eight v_add_f32 (plain FP32 issue), op 1 eight
 * v_log_f32 (the transcendental unit the FP32 search keys use), op 2 two
 * v_log_f32 and twelve v_add_f32 (one class term of the search).  The caller
 * times the launch; instructions per lane / time gives the issue peaks that
 * the search's throughput is compared with (its class terms are the O(1)
 * evaluation of the Tsallis objective, Tsallis-entropy section).
 *   out    device float [blocks * 256], overwritten with values that keep
 *          the instructions live (no meaning).
 * Errors: TS_ERR_INVALID_ARG for op outside 0..2, blocks or iters < 1, or a
 * null out. */
ts_status ts_issue_rate(int32_t op, int32_t blocks, int32_t iters, float *out, ts_stream_t stream);

/* [host] Text describing the last non-OK status returned on this thread
 * ("" if none).  The pointer stays valid until the next call on this thread. */
const char *ts_last_error(void);

/* [host] ABI version of this header (increments on incompatible change). */
int32_t ts_abi_version(void);

#define TS_ABI_VERSION 3

#ifdef __cplusplus
}
#endif

#endif /* TS_H */
