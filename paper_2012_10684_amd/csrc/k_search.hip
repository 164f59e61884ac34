// k_search.hip -- exhaustive arg max of the Tsallis objective over threshold
// tuples (Tsallis-entropy section: phi = arg max [H1 + H2 + (1-q) H1 H2],
// composed recursively for k = 2, 3).
//
// Objective in product/log form.  For a class (a, b] with mass w = P(b) - P(a)
// and Q_j = Q(b) - Q(a):  1 + (1-q) H_j = Q_j / w^q, and the composition rule
// multiplies these factors, so  S = expm1(Lambda) / (1 - q)  with
// Lambda = sum_j [ln Q_j - q ln w_j].  S is strictly increasing in
// Lambda / (1 - q) for q < 1 and for q > 1, hence arg max S = arg max of
// sgn(1-q) * Lambda.  Each class therefore contributes one signed term
//     g(a, b) = sgn(1-q) * (log Q_j - q log w_j)   in [0, |1-q| log L]
// (the range follows from Q_j / w^q lying between 1 and m^(1-q) for a class of
// m bins), and an empty class (w = 0) makes the tuple invalid (-inf, applied
// after the sign).  The expm1 form avoids the cancellation of 1 - sum(p/w)^q
// near q = 1; it is used once per problem, for the reported value.
//
// FP32 search with FP64 tie check (default mode):
//   setup   one workgroup per problem: head(t) = g(-1, t), tail(t) = g(t, L-1)
//           in FP32 (log2 units), and a per-problem bound delta on the
//           difference between any FP32 key and the FP64 value computed from
//           the same prefix sums;
//   pairs   (k = 3) rows A_t2(t1) = head(t1) + g(t1, t2) and
//           R_t2(t3) = g(t2, t3) + tail(t3), stored in the workspace;
//   phase 1 every tuple's FP32 key, one tile per wavefront: lanes hold the
//           last threshold(s) in registers, the earlier threshold is a
//           wavefront-uniform loop whose operands come through scalar loads;
//           wavefront max -> tile max, atomic max -> problem max M.
//           k = 3 reuses the whole R row for every t1: one add and one max
//           per tuple;
//   phase 2 tiles whose max is >= M - 2 delta re-evaluate their tuples; every
//           tuple with an FP32 key >= M - 2 delta is evaluated in FP64 and the
//           best (FP64 value, then lexicographically first tuple) is kept.
//           The FP64 arg max is always in that set, so the result is the FP64
//           arg max;
//   final   one workgroup per problem reduces the tile bests, writes the tuple,
//           S = expm1(Lambda)/(1-q) and the status.
// FP64 mode evaluates every key in FP64 directly (A/R rows in FP64 for k=3).
//
// q = 1 is the Shannon limit (Kapur's objective): class entropies
// S_j = ln w_j - E_j / w_j with E_j the class sum of p ln p (the prefix Q then
// holds sum p ln p), composed by plain addition; S_j lies in [0, ln m] for a
// class of m bins.  It runs through the same kernels with sgn = 0 (SGN = 0 in
// the FP32 templates): one log and one reciprocal per class term.
// Plain mode is the simple form: one thread per tuple (rank decoded into the
// tuple), every class evaluated from P and Q in global memory in FP64, a block
// reduction and a second reduction pass, one problem per launch.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <chrono>

#include "common.h"
#include "hist_dev.h"
#include "label_dev.h"
#include "prefix_dev.h"

namespace ts {

constexpr int PLAIN_BLOCKS = 65536;
constexpr int K3_THREADS = 256;                // k = 3 rows kernel
constexpr int K3_COLS = 4;                     // columns per lane
constexpr int K3_CHUNK = K3_THREADS * K3_COLS; // columns per workgroup
constexpr int K3_GROUP = 32;                   // rows per recorded maximum
constexpr int FUSED_THREADS = 1024; // upper bound; the launch picks 256, 512 or 1024
constexpr int FUSED_MAX_L = 4096;  // k = 1
constexpr int FUSED_MAX_L2 = 1024; // k = 2 (P and Q staged in LDS)
constexpr int FUSED_MAX_TILES = 4096;


struct Meta {
    int menc;    // ordered-int encoding of the problem's FP32 max key
    float delta; // bound on |key32 - key64 / ln 2|
    float pthr;  // k = 3: phase 1 skips row groups whose key bound is below this (-inf: none)
    int pad1;
};

struct Best {
    double rank; // value the arg max is taken over
    double lam;  // FP64 signed Lambda (natural log) of the tuple
    long long code;
    long long pad;
};

__device__ __forceinline__ bool better(double r1, long long c1, double r2, long long c2)
{
    return r1 > r2 || (r1 == r2 && c1 < c2);
}

// ---------------------------------------------------------------- plan

struct Plan {
    int L, k, mode, cols, CW, Lp, T1;
    int NB, NC, tiles; // column blocks, row groups, tiles per problem
    size_t off_meta, off_hl, off_head, off_tail, off_A, off_R, off_tmax, off_best, off_plain, bytes;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int64_t tuples_of(int L, int k)
{
    const int64_t n = L - 1;
    return k == 1 ? n : (k == 2 ? n * (n - 1) / 2 : n * (n - 1) * (n - 2) / 6);
}

// Workgroups per problem of the sum-product search: about 8 tuples per thread.
static int sumprod_blocks(int L, int k)
{
    return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (tuples_of(L, k) + 2047) / 2048));
}

static Plan make_plan(int nseg, int L, int k, int mode, int cols, int T1)
{
    Plan p;
    p.L = L;
    p.k = k;
    p.mode = mode;
    p.cols = cols;
    p.CW = 64 * cols;
    p.Lp = (L + 255) & ~255;
    p.T1 = T1;
    const int n = L - 1; // threshold positions 0..L-2
    if (k == 1) {
        p.NB = (n + p.CW - 1) / p.CW;
        p.NC = 1;
    } else if (k == 2) {
        p.NB = (n + p.CW - 1) / p.CW;
        p.NC = (std::max(L - 2, 1) + T1 - 1) / T1;
    } else if (mode == TS_SEARCH_FP64 || mode == TS_SEARCH_PLAIN) {
        p.NB = (n + p.CW - 1) / p.CW;
        p.NC = std::max(L - 3, 1); // one row per t2 in [1, L-3]
    } else {
        // (row t2, chunk of K3_CHUNK columns, wavefront) tiles of k_rows3
        p.NC = (std::max(L - 3, 1) + K3_CHUNK - 1) / K3_CHUNK; // chunks per row
        p.NB = K3_THREADS / 64 * std::max(L - 3, 1);          // wavefronts per chunk x rows
        p.T1 = (L + K3_GROUP - 1) / K3_GROUP;                 // row groups per wavefront tile
    }
    p.tiles = p.NB * p.NC;
    const bool f64 = mode == TS_SEARCH_FP64;
    const size_t es = f64 ? 8 : 4;
    size_t o = 0;
    p.off_meta = o;
    o = align256(o + (size_t)nseg * sizeof(Meta));
    p.off_hl = o;
    if (mode == TS_SEARCH_FP32_TIECHECK || mode == TS_SEARCH_FP32_ONLY)
        o = align256(o + (size_t)nseg * p.Lp * sizeof(float4));
    p.off_head = o;
    o = align256(o + (size_t)nseg * p.Lp * es);
    p.off_tail = o;
    o = align256(o + (size_t)nseg * p.Lp * es);
    p.off_A = o;
    p.off_R = o;
    if (k == 3 && mode == TS_SEARCH_FP64) {
        o = align256(o + (size_t)nseg * L * p.Lp * es);
        p.off_R = o;
        o = align256(o + (size_t)nseg * L * p.Lp * es);
    }
    p.off_tmax = o;
    if (mode == TS_SEARCH_FP32_TIECHECK || mode == TS_SEARCH_FP32_ONLY)
        o = align256(o + (size_t)nseg * p.tiles * (k == 3 ? p.T1 : 1) * sizeof(float));
    p.off_best = o;
    if (mode != TS_SEARCH_PLAIN && mode != TS_SEARCH_PLAIN_FP32 && mode != TS_SEARCH_SUMPROD)
        o = align256(o + (size_t)nseg * p.tiles * sizeof(Best));
    p.off_plain = o;
    if (mode == TS_SEARCH_PLAIN || mode == TS_SEARCH_PLAIN_FP32)
        o = align256(o + (size_t)PLAIN_BLOCKS * sizeof(Best));
    if (mode == TS_SEARCH_SUMPROD)
        o = align256(o + (size_t)nseg * sumprod_blocks(L, k) * sizeof(Best));
    p.bytes = o;
    return p;
}

size_t search_workspace_bytes(int nseg, int L, int k, int mode, int)
{
    // the largest plan over every tuning the library accepts
    size_t m = 0;
    for (int cols : {1, 2, 4})
        m = std::max(m, make_plan(nseg, L, k, mode, cols, 16).bytes);
    return m;
}

// ---------------------------------------------------------------- class terms

// Each FP64 prefix value X is also kept as a pair of floats, hi = fl32(X) and
// lo = fl32(X - hi) (x, y: P; z, w: Q), so a class difference is formed in
// FP32 as (hi_b - hi_a) + (lo_b - lo_a), within 2^-23 relative (plus
// 2^-46 X_max / difference) of the FP64 difference, at FP32 rate.
__device__ __forceinline__ float4 split_hl(double P, double Q)
{
    const float ph = (float)P, qh = (float)Q;
    return make_float4(ph, (float)(P - (double)ph), qh, (float)(Q - (double)qh));
}

// Signed FP32 class term in log2 units for the class (a, b] from the split
// prefixes at b and a (a = -1: all zero).  Valid iff the class mass is > 0.
template <int SGN>
__device__ __forceinline__ float cls32(const float4 &hb, const float4 &ha, float mq, float gmax)
{
    const float dp = (hb.x - ha.x) + (hb.y - ha.y);
    const float dq = (hb.z - ha.z) + (hb.w - ha.w);
    float g;
    if (SGN == 0) { // Shannon: log2 w - (E / w) log2(e)
        const float ly = __builtin_amdgcn_logf(dp);
        const float r = dq * __builtin_amdgcn_rcpf(dp);
        g = fmaf(r, -1.44269504f, ly);
    } else {
        const float lx = __builtin_amdgcn_logf(dq);
        const float ly = __builtin_amdgcn_logf(dp);
        g = fmaf(mq, ly, SGN > 0 ? lx : -lx); // mq = -sgn * q
    }
    g = __builtin_amdgcn_fmed3f(g, 0.0f, gmax);
    return dp > 0.0f ? g : -INFINITY;
}

// Signed FP64 class term in natural-log units.
__device__ __forceinline__ double cls64(double dP, double dQ, double q, double sgn, double hmax)
{
    if (!(dP > 0.0))
        return -INFINITY;
    const double h = sgn == 0.0 ? log(dP) - dQ / dP : sgn * (log(dQ) - q * log(dP));
    return fmin(fmax(h, 0.0), hmax);
}

// FP64 signed Lambda of the tuple t[0..k-1] directly from the prefix sums.
// The classes go through a rolled loop with one call site of log: the tie
// check runs for a handful of tuples per problem, so small code (few
// instruction-cache misses on its first run in each workgroup) matters more
// than instruction-level parallelism.  Same operations and order as cls64.
template <int K>
__device__ __forceinline__ double lambda64_k(const double *P, const double *Q, int L, const int *t, double q,
                                             double sgn, double hmax)
{
    const int t0 = t[0], t1 = K > 1 ? t[1] : 0, t2 = K > 2 ? t[2] : 0;
    double acc = 0.0;
    double pa = 0.0, qa = 0.0;
#pragma unroll 1
    for (int j = 0; j <= K; ++j) {
        const int b = j == K ? L - 1 : (j == 0 ? t0 : (j == 1 ? t1 : t2));
        const double pb = P[b], qb = Q[b];
        const double dP = pb - pa, dQ = qb - qa;
        if (!(dP > 0.0))
            return -INFINITY;
        double lg[2];
        if (sgn == 0.0) { // Shannon
            lg[1] = log(dP);
            lg[0] = dQ / dP;
        } else {
#pragma unroll 1
            for (int i = 0; i < 2; ++i)
                lg[i] = log(i == 0 ? dQ : dP);
        }
        const double h = sgn == 0.0 ? lg[1] - lg[0] : sgn * (lg[0] - q * lg[1]);
        acc += fmin(fmax(h, 0.0), hmax);
        pa = pb;
        qa = qb;
    }
    return acc;
}

__device__ __forceinline__ double lambda64(const double *P, const double *Q, int L, int k, const int *t, double q,
                                           double sgn, double hmax)
{
    if (k == 1)
        return lambda64_k<1>(P, Q, L, t, q, sgn, hmax);
    if (k == 2)
        return lambda64_k<2>(P, Q, L, t, q, sgn, hmax);
    return lambda64_k<3>(P, Q, L, t, q, sgn, hmax);
}

__device__ __forceinline__ long long make_code(int k, const int *t)
{
    long long c = 0;
    for (int j = 0; j < k; ++j)
        c = (c << 12) | (long long)t[j];
    return c;
}

// Best (rank desc, code asc) candidate of the wavefront, returned in every
// lane.  DPP moves as in wave_max; skipped when no lane holds a candidate.
template <int C, int M>
__device__ __forceinline__ void best_step(double &r, double &l, long long &c)
{
    const double r2 = dpp_f64<C, M>(r);
    const double l2 = dpp_f64<C, M>(l);
    const long long c2 = __double_as_longlong(dpp_f64<C, M>(__longlong_as_double(c)));
    if (better(r2, c2, r, c)) {
        r = r2;
        l = l2;
        c = c2;
    }
}

__device__ __forceinline__ double readlane63_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ void wave_best(double &r, double &l, long long &c)
{
    if (!__any(r > -INFINITY))
        return; // no lane holds a candidate
    best_step<0xB1, 0xF>(r, l, c);
    best_step<0x4E, 0xF>(r, l, c);
    best_step<0x141, 0xF>(r, l, c);
    best_step<0x140, 0xF>(r, l, c);
    best_step<0x142, 0xA>(r, l, c);
    best_step<0x143, 0xC>(r, l, c);
    r = readlane63_f64(r);
    l = readlane63_f64(l);
    c = __double_as_longlong(readlane63_f64(__longlong_as_double(c)));
}

// Constants of one entropic index q.
struct QConst {
    double q, sgn, hmax; // hmax = |1-q| ln L
    float mq, gmax;      // mq = -sgn * fl32(q), gmax = |1-q| log2 L (rounded up)
    float cw;            // |1-q| (1 for q = 1) rounded up: a class of n bins has g <= cw log2 n
};

// Problem p of a launch uses index q_{p / nseg}, P row p % nseg and Q row p;
// every per-problem output and workspace row is indexed by p.
struct Args {
    const double *P, *Q;
    int nseg, nprob, L, Lp, k, mode;
    QConst qc[TS_MAX_Q];
    int CW, NB, NC, T1, tiles;
    Meta *meta;
    float4 *hl; // [nseg][Lp] split prefixes (multi-launch paths)
    void *head, *tail, *A, *R;
    float *tmax;
    Best *best;
};

// ---------------------------------------------------------------- setup

// Smallest positive step of P and of Q over consecutive bins of one problem
// (block-wide minima; every thread returns them).  red holds 2 doubles per
// wavefront.  Any positive class mass is >= pmin, and any positive
// difference of stored Q values is >= dqmin (a difference of two stored
// non-decreasing prefix values is at least the largest step between them).
struct Steps {
    double pmin, dqmin;
};

__device__ __forceinline__ Steps block_steps(const double *P, const double *Q, int L, double *red)
{
    double pm = 1.0, qm = INFINITY;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const double dp = P[t] - (t ? P[t - 1] : 0.0);
        const double dq = fabs(Q[t] - (t ? Q[t - 1] : 0.0)); // Shannon: Q falls
        if (dp > 0.0)
            pm = fmin(pm, dp);
        if (dq > 0.0)
            qm = fmin(qm, dq);
    }
    pm = wave_min_f64(pm);
    qm = wave_min_f64(qm);
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = pm;
        red[nw + (threadIdx.x >> 6)] = qm;
    }
    __syncthreads();
    Steps r = {red[0], red[nw]};
    for (int i = 1; i < nw; ++i) {
        r.pmin = fmin(r.pmin, red[i]);
        r.dqmin = fmin(r.dqmin, red[nw + i]);
    }
    __syncthreads();
    return r;
}

// Bound on |key32 - key64 / ln 2| over every tuple of one problem, where
// key32 is the FP32 key and key64 the FP64 value from the same prefix sums.
// Per class term: the two casts to FP32 (2^-24 relative each), the error of
// v_log_f32 on both logs (LOG2_ERR_UNITS * 2^-24 * max(1, |log2 x|)), q
// rounded to FP32, the fma; then k additions of terms bounded by gmax.
// Magnitudes: |log2 w| <= |log2 pmin| and |log2 Q_j| <= max(|log2 Q_tot|,
// |log2 dqmin|) for every valid class (see block_steps); they are taken from
// v_log_f32 and inflated by 1 % + 1.  The result is doubled.  Infinity when a
// class sum could leave the normal FP32 range: every tuple is then re-checked
// in FP64.
__device__ __forceinline__ float problem_delta(const Args &a, const QConst &c, Steps st, double qtot)
{
    if (a.mode == TS_SEARCH_FP32_ONLY)
        return 0.0f;
    qtot = fabs(qtot); // Shannon: Q(L-1) = sum p ln p <= 0
    if (!(qtot > 0.0) || !(st.dqmin > 1e-36) || !(st.pmin > 1e-36) || qtot > 1e36)
        return INFINITY;
    const float u = 0x1p-24f;
    const float q = (float)c.q;
    const float lq = fmaxf(fabsf(__builtin_amdgcn_logf((float)qtot)), fabsf(__builtin_amdgcn_logf((float)st.dqmin)));
    const float lp = fabsf(__builtin_amdgcn_logf((float)st.pmin));
    const float Ux = lq * 1.01f + 1.0f, Vy = lp * 1.01f + 1.0f;
    const float gm = c.gmax;
    // split FP32 differences: relative error <= 2u + 4u^2 X_max / (smallest difference)
    const float rp = 2.0f * u + 4.0f * u * u / (float)st.pmin;
    const float rq = 2.0f * u + 4.0f * u * u * (float)(qtot / st.dqmin);
    if (!(rp < 1e-3f) || !(rq < 1e-3f))
        return INFINITY;
    float ec;
    if (c.sgn == 0.0) {
        // Shannon term log2 w - (E/w) log2 e: |E/w| <= max |ln p_i| <= ln(1/pmin)
        // = Vy ln 2 nats; the ratio carries the relative errors of both class
        // sums, of the reciprocal (2u) and of the product (u), the constant
        // log2 e its rounding (u); then the fma
        ec = rp * 1.5f                                      // w cast into the log
             + (float)LOG2_ERR_UNITS * u * Vy               // v_log_f32
             + Vy * (rq + rp + 4.1f * u)                    // E / w
             + u * (2.0f * Vy + gm + 1.0f);                 // fma + clamp
    } else {
        ec = (rq + q * rp) * 1.5f                                     // FP32 class sums
             + (float)LOG2_ERR_UNITS * u * (Ux + q * Vy)              // v_log_f32
             + (float)fabs((double)(-c.sgn * c.mq) - c.q) * Vy        // q rounded to FP32
             + u * (gm + 1.0f);                                       // fma + clamp
    }
    const float kk = (float)a.k;
    const float d = 2.0f * ((kk + 1.0f) * ec + kk * (kk + 1.0f) * u * (gm + 1.0f)) + 1e-9f * (kk + 1.0f) * (gm + 1.0f);
    return d * 1.0001f;
}

// FP32 head(t) = g(-1, t) and tail(t) = g(t, L-1) for t in [0, Lp); entries
// past L-2 are -inf.
template <int SGN>
__device__ __forceinline__ Steps head_tail32(const Args &a, const QConst &c, const double *P, const double *Q,
                                             float *hd, float *tl, float4 *hl, double *red, double *pl = nullptr,
                                             double *ql = nullptr)
{
    const int L = a.L;
    const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const double PL = P[L - 1], QL = Q[L - 1];
    const float4 last = split_hl(PL, QL);
    double pm = 1.0, qm = INFINITY;
    for (int t = threadIdx.x; t < a.Lp; t += blockDim.x) {
        const int ti = min(t, L - 1);
        const double p = P[ti], q = Q[ti];
        const double p0 = ti ? P[ti - 1] : 0.0, q0 = ti ? Q[ti - 1] : 0.0;
        if (t < L) {
            if (p - p0 > 0.0)
                pm = fmin(pm, p - p0);
            const double dqs = fabs(q - q0); // Shannon: Q falls
            if (dqs > 0.0)
                qm = fmin(qm, dqs);
        }
        const float4 h4 = split_hl(p, q);
        float h = -INFINITY, g = -INFINITY;
        if (t <= L - 2) {
            h = cls32<SGN>(h4, zero, c.mq, c.gmax);
            g = cls32<SGN>(last, h4, c.mq, c.gmax);
        }
        hd[t] = h;
        tl[t] = g;
        if (hl)
            hl[t] = h4;
        if (pl) {
            pl[t] = p;
            ql[t] = q;
        }
    }
    pm = wave_min_f64(pm);
    qm = wave_min_f64(qm);
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = pm;
        red[nw + (threadIdx.x >> 6)] = qm;
    }
    __syncthreads();
    Steps r = {red[0], red[nw]};
    for (int i = 1; i < nw; ++i) {
        r.pmin = fmin(r.pmin, red[i]);
        r.dqmin = fmin(r.dqmin, red[nw + i]);
    }
    return r;
}

// Ms - 3 delta rounded down; -inf (nothing pruned) unless both are finite.
__device__ __forceinline__ float prune_threshold(float Ms, float delta)
{
    if (!(Ms > -INFINITY) || !(delta < INFINITY))
        return -INFINITY;
    const double t64 = (double)Ms - 3.0 * (double)delta;
    float t = (float)t64;
    if ((double)t > t64)
        t = nextafterf(t, -INFINITY);
    return t;
}

__global__ void __launch_bounds__(256) k_setup(Args a)
{
    const int s = blockIdx.x; // problem
    const QConst &c = a.qc[s / a.nseg];
    const double *P = a.P + (int64_t)(s % a.nseg) * a.L;
    const double *Q = a.Q + (int64_t)s * a.L;
    const int L = a.L, Lp = a.Lp;
    __shared__ double red[8];
    Steps stp;
    if (a.mode == TS_SEARCH_FP64)
        stp = block_steps(P, Q, L, red);
    else if (c.sgn > 0)
        stp = head_tail32<1>(a, c, P, Q, (float *)a.head + (int64_t)s * Lp, (float *)a.tail + (int64_t)s * Lp,
                             a.hl + (int64_t)s * Lp, red);
    else if (c.sgn < 0)
        stp = head_tail32<-1>(a, c, P, Q, (float *)a.head + (int64_t)s * Lp, (float *)a.tail + (int64_t)s * Lp,
                              a.hl + (int64_t)s * Lp, red);
    else
        stp = head_tail32<0>(a, c, P, Q, (float *)a.head + (int64_t)s * Lp, (float *)a.tail + (int64_t)s * Lp,
                             a.hl + (int64_t)s * Lp, red);
    // k = 3 with the FP64 re-check: the largest FP32 key of a coarse grid of
    // tuples (seeds) gives the threshold below which k_rows3 skips row groups
    // (rows3_body); the rows written above are visible after the barrier
    float ms = -INFINITY;
    if (a.k == 3 && a.mode == TS_SEARCH_FP32_TIECHECK) {
        __syncthreads();
        const float *hd = (const float *)a.head + (int64_t)s * Lp, *tl = (const float *)a.tail + (int64_t)s * Lp;
        const float4 *hl = a.hl + (int64_t)s * Lp;
        constexpr int G = 16; // grid positions over [0, L - 2]
        const int S = (L - 1 + G - 1) / G;
        const int i = threadIdx.x / G, j = threadIdx.x % G;
        const int t1 = min(i * S + S / 2, L - 2), t2 = min(j * S + S / 2, L - 2);
        if (i < G && t1 < t2) {
            const float4 h1 = hl[t1], h2 = hl[t2];
            const float ar = hd[t1] + (c.sgn > 0 ? cls32<1>(h2, h1, c.mq, c.gmax)
                                                  : (c.sgn < 0 ? cls32<-1>(h2, h1, c.mq, c.gmax)
                                                               : cls32<0>(h2, h1, c.mq, c.gmax)));
            for (int m = j + 1; m < G; ++m) {
                const int t3 = min(m * S + S / 2, L - 2);
                if (t3 <= t2)
                    continue;
                const float4 h3 = hl[t3];
                const float g3 = c.sgn > 0 ? cls32<1>(h3, h2, c.mq, c.gmax)
                                           : (c.sgn < 0 ? cls32<-1>(h3, h2, c.mq, c.gmax)
                                                        : cls32<0>(h3, h2, c.mq, c.gmax));
                ms = fmaxf(ms, ar + (g3 + tl[t3])); // the A row term plus the column term, as in phase 1
            }
        }
        ms = wave_max(ms);
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = (double)ms;
        __syncthreads();
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            ms = fmaxf(ms, (float)red[w]);
    }
    if (threadIdx.x == 0) {
        Meta m;
        m.menc = float_to_ordered(-INFINITY);
        m.pad1 = 0;
        m.delta = problem_delta(a, c, stp, Q[L - 1]);
        m.pthr = a.k == 3 && a.mode == TS_SEARCH_FP32_TIECHECK ? prune_threshold(ms, m.delta) : -INFINITY;
        a.meta[s] = m;
    }
    if (a.mode == TS_SEARCH_FP64) {
        double *hd = (double *)a.head + (int64_t)s * Lp;
        double *tl = (double *)a.tail + (int64_t)s * Lp;
        const double pL = P[L - 1], qL = Q[L - 1];
        for (int t = threadIdx.x; t < Lp; t += blockDim.x) {
            double h = -INFINITY, g = -INFINITY;
            if (t <= L - 2) {
                h = cls64(P[t], Q[t], c.q, c.sgn, c.hmax);
                g = cls64(pL - P[t], qL - Q[t], c.q, c.sgn, c.hmax);
            }
            hd[t] = h;
            tl[t] = g;
        }
    }
}

// ---------------------------------------------------------------- k = 3 rows

__global__ void __launch_bounds__(256) k_pairs64(Args a)
{
    const int s = blockIdx.x / (a.L - 3);
    const int t2 = 1 + blockIdx.x % (a.L - 3);
    const int L = a.L, Lp = a.Lp;
    const QConst &c = a.qc[s / a.nseg];
    const double *P = a.P + (int64_t)(s % a.nseg) * L;
    const double *Q = a.Q + (int64_t)s * L;
    const double *hd = (const double *)a.head + (int64_t)s * Lp;
    const double *tl = (const double *)a.tail + (int64_t)s * Lp;
    double *Ar = (double *)a.A + ((int64_t)s * L + t2) * Lp;
    double *Rr = (double *)a.R + ((int64_t)s * L + t2) * Lp;
    const double p2 = P[t2], q2 = Q[t2];
    for (int t = threadIdx.x; t < Lp; t += blockDim.x) {
        double av = -INFINITY, rv = -INFINITY;
        if (t < t2)
            av = hd[t] + cls64(p2 - P[t], q2 - Q[t], c.q, c.sgn, c.hmax);
        else if (t <= L - 2 && t > t2)
            rv = cls64(P[t] - p2, Q[t] - q2, c.q, c.sgn, c.hmax) + tl[t];
        Ar[t] = av;
        Rr[t] = rv;
    }
}

// ---------------------------------------------------------------- tiles

// Tile geometry.  k = 1: column block b.  k = 2: column block b of t2 and row
// group c of t1 (T1 rows).  k = 3: row t2 (heaviest first) and column block b
// of t3.  The wavefront index comes from readfirstlane so that every tile
// quantity lives in scalar registers.
struct Tile {
    int s, tile, b, c, valid;
};

__device__ __forceinline__ Tile tile_of(const Args &a)
{
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
    Tile t;
    t.valid = g < (int64_t)a.nprob * a.tiles;
    t.s = (int)(g / a.tiles);
    t.tile = (int)(g % a.tiles);
    t.b = t.tile % a.NB;
    t.c = t.tile / a.NB;
    return t;
}

struct Cand {
    double r, l; // rank, FP64 signed Lambda
    long long c; // lexicographic code
};

// Everything a tile body reads for one problem.
struct TileCtx {
    const double *P, *Q; // prefix sums of the problem
    const float *hd, *tr; // head / tail rows (LDS or global)
    const float4 *hl;     // split prefixes (LDS or global)
    const float *A, *R;   // k = 3 rows of the problem (global)
    const unsigned long long *prune; // k = 2: rows skipped in phase 1, [NB][Lp / 64] bit words (or null)
    int L, Lp, mode, CW, T1;
    double q, sgn, hmax;
    float mq, gmax, cw;
};

__device__ __forceinline__ TileCtx make_ctx(const Args &a, int s, const float *hd, const float *tr,
                                            const float4 *hl)
{
    TileCtx x;
    x.hl = hl;
    const QConst &c = a.qc[s / a.nseg];
    x.P = a.P + (int64_t)(s % a.nseg) * a.L;
    x.Q = a.Q + (int64_t)s * a.L;
    x.hd = hd;
    x.tr = tr;
    x.A = (const float *)a.A + (int64_t)s * a.L * a.Lp;
    x.R = (const float *)a.R + (int64_t)s * a.L * a.Lp;
    x.L = a.L;
    x.Lp = a.Lp;
    x.mode = a.mode;
    x.CW = a.CW;
    x.T1 = a.T1;
    x.q = c.q;
    x.sgn = c.sgn;
    x.hmax = c.hmax;
    x.mq = c.mq;
    x.gmax = c.gmax;
    x.cw = c.cw;
    x.prune = nullptr;
    return x;
}

// Whether phase 2 re-checks a tuple: its indices form a tuple (the padded
// slots past L - 2 and the masked triangle do not) and its FP32 key is not
// below thr.  Written as !(key < thr) so that thr = -inf (an infinite error
// bound) selects every tuple whatever its FP32 key.
__device__ __forceinline__ bool rechecked(bool is_tuple, float key, float thr)
{
    return is_tuple && !(key < thr);
}

// Phase 1 folds every key into acc; phase 2 evaluates every re-checked tuple
// in FP64 and keeps the best (rank, then first tuple).  is_tuple: t1 < t2 < t3
// all within [0, L - 2].
template <int PHASE, int K>
__device__ __forceinline__ void take(const TileCtx &x, float key, float thr, float &acc, Cand &b, int t1, int t2,
                                     int t3, bool is_tuple)
{
    if (PHASE == 1) {
        acc = fmaxf(acc, key);
    } else if (rechecked(is_tuple, key, thr)) {
        const int t[3] = {t1, t2, t3};
        const double lam = lambda64_k<K>(x.P, x.Q, x.L, t, x.q, x.sgn, x.hmax);
        const double rank = x.mode == TS_SEARCH_FP32_ONLY ? (double)key : lam;
        const long long code = make_code(K, t);
        if (better(rank, code, b.r, b.c)) {
            b.r = rank;
            b.l = lam;
            b.c = code;
        }
    }
}

// Phase 2, one row: FP64 evaluation of the re-checked columns (bits of
// `valid` mark the columns that hold a tuple: every index within [0, L - 2]
// and ascending).  Candidates are
// rare, so the FP64 objective appears once, in a loop over the set bits,
// rather than once per unrolled tuple: the phase-2 code stays small and its
// first execution in each workgroup fetches little from the L2.
template <int K, int COLS>
__device__ __forceinline__ void take_cols(const TileCtx &x, const float (&key)[COLS], const int (&tv)[COLS],
                                          unsigned valid, float thr, Cand &b, int t1, int t2)
{
    unsigned m = 0;
#pragma unroll
    for (int v = 0; v < COLS; ++v)
        m |= rechecked((valid >> v) & 1u, key[v], thr) ? (1u << v) : 0u;
    while (m) {
        const int v = __builtin_ctz(m);
        m &= m - 1;
        int tl = tv[0];
        float kv = key[0];
#pragma unroll
        for (int w = 1; w < COLS; ++w)
            if (v == w) {
                tl = tv[w];
                kv = key[w];
            }
        const int t[3] = {t1, K == 2 ? tl : t2, tl};
        const double lam = lambda64_k<K>(x.P, x.Q, x.L, t, x.q, x.sgn, x.hmax);
        const double rank = x.mode == TS_SEARCH_FP32_ONLY ? (double)kv : lam;
        const long long code = make_code(K, t);
        if (better(rank, code, b.r, b.c)) {
            b.r = rank;
            b.l = lam;
            b.c = code;
        }
    }
}

template <int COLS, int PHASE>
__device__ __forceinline__ void tile_k1(const TileCtx &x, int b, float thr, float &acc, Cand &best)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < COLS; ++v) {
        const int t = b * x.CW + v * 64 + lane; // t < Lp: entries past L-2 are -inf
        take<PHASE, 1>(x, x.hd[t] + x.tr[t], thr, acc, best, t, 0, 0, t <= x.L - 2);
    }
}

// Rows [t1b, t1e) of a k = 2 tile; MASK keeps only t1 < t2.  Four rows are
// loaded together so the scalar loads and the transcendental latencies of
// consecutive rows overlap.
// Rows [t1b, t1e) of a k = 2 tile; MASK keeps only t1 < t2.  Rows go in
// groups of R: the group's row operands are all loaded before any of its
// tuples is evaluated, so one load latency covers R x COLS class terms.
// Columns [V0, COLS) only: column blocks below V0 hold no t2 > t1 for these rows.
template <int SGN, int COLS, int PHASE, bool MASK, int R, int V0 = 0>
__device__ __forceinline__ void rows_k2_group(const TileCtx &x, int t1, const float4 (&hc)[COLS],
                                              const float (&tc)[COLS], const int (&t2v)[COLS], float thr, float &acc,
                                              Cand &best)
{
    float4 hr[R];
    float hdr[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        hr[u] = x.hl[t1 + u];
        hdr[u] = x.hd[t1 + u];
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
#pragma unroll
        for (int v = V0; v < COLS; ++v) {
            const float key = (hdr[u] + cls32<SGN>(hc[v], hr[u], x.mq, x.gmax)) + tc[v];
            if (!MASK || t1 + u < t2v[v])
                take<PHASE, 2>(x, key, thr, acc, best, t1 + u, t2v[v], 0, t2v[v] <= x.L - 2);
        }
    }
}

// Whether every row of [t1, t1 + R) is marked in a column block's prune
// words pw (null: no row is).  The words are the same in every lane.
template <int R>
__device__ __forceinline__ bool rows_marked(const unsigned long long *pw, int t1)
{
    if (!pw)
        return false;
    const int o = t1 & 63, wi = t1 >> 6;
    unsigned long long m = pw[wi] >> o;
    if (o + R > 64)
        m |= pw[wi + 1] << (64 - o);
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)m);
    constexpr unsigned long long want = (1ull << R) - 1ull;
    if (R <= 32)
        return (lo & (unsigned int)want) == (unsigned int)want;
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)(m >> 32));
    return ((((unsigned long long)hi << 32) | lo) & want) == want;
}

// pw: the column block's prune words (phase 1), or null.
template <int SGN, int COLS, int PHASE, bool MASK, int V0 = 0>
__device__ __forceinline__ void rows_k2(const TileCtx &x, int t1b, int t1e, const float4 (&hc)[COLS],
                                        const float (&tc)[COLS], const int (&t2v)[COLS], float thr, float &acc,
                                        Cand &best, const unsigned long long *pw)
{
    int t1 = t1b;
    for (; t1 + 8 <= t1e; t1 += 8)
        if (!rows_marked<8>(pw, t1))
            rows_k2_group<SGN, COLS, PHASE, MASK, 8, V0>(x, t1, hc, tc, t2v, thr, acc, best);
    if (t1 + 4 <= t1e) {
        if (!rows_marked<4>(pw, t1))
            rows_k2_group<SGN, COLS, PHASE, MASK, 4, V0>(x, t1, hc, tc, t2v, thr, acc, best);
        t1 += 4;
    }
    for (; t1 < t1e; ++t1)
        if (!rows_marked<1>(pw, t1))
            rows_k2_group<SGN, COLS, PHASE, MASK, 1, V0>(x, t1, hc, tc, t2v, thr, acc, best);
}

// Rows [rb, re) on the diagonal of a tile whose columns start at cbase: rows
// in [cbase + 64 V, cbase + 64 (V + 1)) evaluate column blocks V..COLS-1 only
// (block v < V has every t2 <= t1).
template <int SGN, int COLS, int PHASE, int V = 0>
__device__ __forceinline__ void rows_k2_diag(const TileCtx &x, int rb, int re, int cbase, const float4 (&hc)[COLS],
                                             const float (&tc)[COLS], const int (&t2v)[COLS], float thr,
                                             float &acc, Cand &best, const unsigned long long *pw)
{
    if constexpr (V < COLS) {
        const int lo = max(rb, cbase + 64 * V), hi = min(re, cbase + 64 * (V + 1));
        if (lo < hi)
            rows_k2<SGN, COLS, PHASE, true, V>(x, lo, hi, hc, tc, t2v, thr, acc, best, pw);
        rows_k2_diag<SGN, COLS, PHASE, V + 1>(x, rb, re, cbase, hc, tc, t2v, thr, acc, best, pw);
    }
}

// Rows of part `part` of `nparts` of the tile (every row when nparts = 1).
template <int SGN, int COLS, int PHASE>
__device__ __forceinline__ void tile_k2(const TileCtx &x, int b, int c, float thr, float &acc, Cand &best,
                                        int part = 0, int nparts = 1)
{
    const int lane = threadIdx.x & 63;
    const int L = x.L;
    const int cbase = b * x.CW;
    const int rs = (x.T1 + nparts - 1) / nparts;
    const int r0 = c * x.T1 + part * rs;
    const int r1 = min(min(c * x.T1 + x.T1, r0 + rs), min(L - 2, cbase + x.CW - 1));
    if (r0 >= r1)
        return;
    float4 hc[COLS];
    float tc[COLS];
    int t2v[COLS];
#pragma unroll
    for (int v = 0; v < COLS; ++v) {
        const int t2 = cbase + v * 64 + lane;
        t2v[v] = t2;
        hc[v] = x.hl[min(t2, L - 1)];
        tc[v] = x.tr[t2]; // -inf past L-2
    }
    if (PHASE == 2) { // rows one at a time, keys as in phase 1
#pragma unroll 1
        for (int t1 = r0; t1 < r1; ++t1) {
            const float4 hr = x.hl[t1];
            const float hdr = x.hd[t1];
            float key[COLS];
            unsigned valid = 0;
#pragma unroll
            for (int v = 0; v < COLS; ++v) {
                key[v] = (hdr + cls32<SGN>(hc[v], hr, x.mq, x.gmax)) + tc[v];
                valid |= (t1 < t2v[v] && t2v[v] <= L - 2) ? (1u << v) : 0u;
            }
            take_cols<2, COLS>(x, key, t2v, valid, thr, best, t1, 0);
        }
        return;
    }
    const int ra = min(r1, cbase);
    const unsigned long long *pw = x.prune ? x.prune + b * (x.Lp >> 6) : nullptr;
    rows_k2<SGN, COLS, PHASE, false>(x, r0, ra, hc, tc, t2v, thr, acc, best, pw); // every t2 > t1
    rows_k2_diag<SGN, COLS, PHASE>(x, max(r0, cbase), r1, cbase, hc, tc, t2v, thr, acc, best, pw);
}

template <int SGN, int COLS, int PHASE, int K>
__device__ __forceinline__ void tile_body(const TileCtx &x, int b, int c, float thr, float &acc, Cand &best)
{
    if (K == 1)
        tile_k1<COLS, PHASE>(x, b, thr, acc, best);
    else
        tile_k2<SGN, COLS, PHASE>(x, b, c, thr, acc, best);
}

__device__ __forceinline__ float phase2_threshold(float M, float delta)
{
    const double t64 = (double)M - 2.0 * (double)delta;
    float t = (float)t64;
    if ((double)t > t64)
        t = nextafterf(t, -INFINITY);
    return t;
}

// Multi-launch path, one tile per wavefront.  PHASE 1 writes the tile max and
// the problem max; PHASE 2 re-checks tiles whose max reaches the threshold.
template <int SGN, int COLS, int PHASE, int K>
__device__ __forceinline__ void tiles32_wave(const Args &a, const Tile &tl)
{
    const int lane = threadIdx.x & 63;
    const int s = tl.s;
    const int64_t tid = (int64_t)s * a.tiles + tl.tile;
    const TileCtx x = make_ctx(a, s, (const float *)a.head + (int64_t)s * a.Lp, (const float *)a.tail + (int64_t)s * a.Lp,
                               a.hl + (int64_t)s * a.Lp);
    float thr = -INFINITY;
    if (PHASE == 2) {
        const Meta m = a.meta[s];
        const float M = ordered_to_float(m.menc);
        const float tm = a.tmax[tid];
        thr = phase2_threshold(M, m.delta);
        if (!(tm > -INFINITY) || M == -INFINITY || tm < thr) {
            if (lane == 0)
                a.best[tid] = Best{-INFINITY, -INFINITY, 0x7fffffffffffffffLL, 0};
            return;
        }
    }
    float acc = -INFINITY;
    Cand best = {-INFINITY, -INFINITY, 0x7fffffffffffffffLL};
    tile_body<SGN, COLS, PHASE, K>(x, tl.b, tl.c, thr, acc, best);
    if (PHASE == 1) {
        acc = wave_max(acc);
        if (lane == 0) {
            a.tmax[tid] = acc;
            if (acc > -INFINITY)
                atomicMax(&a.meta[s].menc, float_to_ordered(acc));
        }
    } else {
        wave_best(best.r, best.l, best.c);
        if (lane == 0)
            a.best[tid] = Best{best.r, best.l, best.c, 0};
    }
}

// The sign of 1 - q is uniform over a tile's wavefront.
template <int COLS, int PHASE, int K>
__global__ void __launch_bounds__(256) k_tiles32(Args a)
{
    const Tile tl = tile_of(a);
    if (!tl.valid)
        return;
    const double sgn = a.qc[tl.s / a.nseg].sgn;
    if (sgn > 0)
        tiles32_wave<1, COLS, PHASE, K>(a, tl);
    else if (sgn < 0)
        tiles32_wave<-1, COLS, PHASE, K>(a, tl);
    else
        tiles32_wave<0, COLS, PHASE, K>(a, tl);
}

// k = 3, one workgroup per (problem, row t2, chunk of 1024 columns).  The A
// row head(t1) + g(t1, t2), t1 < t2, is built in LDS; lane columns are
// t3 = t2 + 1 + c for c in the chunk, each holding R(t3) = g(t2, t3) + tail(t3)
// in a register.  Every tuple's key is A[t1] + R[t3]: one add, and one max3 per
// two tuples.  Tiles are (row, chunk, wavefront); rows are visited from the
// middle outwards so the heaviest rows (t2 (L - t2) tuples) start first.

__device__ __forceinline__ int k3_row(int r, int L)
{
    const int lo = 1, hi = L - 3, mid = (lo + hi) / 2;
    const int off = (r + 1) / 2;
    const int t2 = (r & 1) ? mid + off : mid - off;
    return t2; // r in [0, L-3) visits every row in [1, L-3] once
}

// Rows t1 in [g0, g1) of one wavefront: key = A[t1] + R[t3] (g0, g1 multiples
// of 8; A is -inf from t2 up to the padded end).
template <int COLS, int PHASE>
__device__ __forceinline__ void rows3_loop(const TileCtx &x, const float *Arow, int g0, int g1,
                                           const float (&r)[K3_COLS], int t2, const int (&t3v)[K3_COLS], float thr,
                                           float &acc, Cand &best)
{
    const float4 *A4 = reinterpret_cast<const float4 *>(Arow);
    float acc0 = -INFINITY, acc1 = -INFINITY;
    for (int t1 = g0; t1 < g1; t1 += 8) {
        const float4 u0 = A4[t1 >> 2], u1 = A4[(t1 >> 2) + 1];
        const float av[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        if (PHASE == 1) {
#pragma unroll
            for (int v = 0; v < COLS; ++v) {
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    const float m = __builtin_fmaxf(av[u] + r[v], av[u + 1] + r[v]);
                    if (v & 1)
                        acc1 = __builtin_fmaxf(acc1, m);
                    else
                        acc0 = __builtin_fmaxf(acc0, m);
                }
            }
        } else {
#pragma unroll 1
            for (int u = 0; u < 8; ++u) {
                const float a = Arow[t1 + u];
                float key[COLS];
                int tv[COLS];
                unsigned valid = 0;
#pragma unroll
                for (int v = 0; v < COLS; ++v) {
                    key[v] = a + r[v]; // -inf for columns past the row end
                    tv[v] = t3v[v];
                    // rows t1 >= t2 (A is -inf there) and columns past L - 2 hold no tuple
                    valid |= (t1 + u < t2 && t3v[v] <= x.L - 2) ? (1u << v) : 0u;
                }
                take_cols<3, COLS>(x, key, tv, valid, thr, best, t1 + u, t2);
            }
        }
    }
    acc = fmaxf(acc, fmaxf(acc0, acc1));
}

// k = 3, one workgroup per (problem, row t2, chunk of 1024 columns).  The A
// row head(t1) + g(t1, t2), t1 < t2, is built in LDS; column c of the chunk is
// t3 = t2 + 1 + c, held by lane c % 64 of wavefront (c / 64) % 4 as
// R(t3) = g(t2, t3) + tail(t3) in a register, so the valid columns of a short
// row are spread over all four wavefronts (and SIMDs).  Every tuple's key is
// A[t1] + R[t3]: one add, and one max3 per two tuples.  Phase 1 records the
// wavefront max of every group of K3_GROUP rows; phase 2 re-checks only groups
// whose max reaches the threshold.  Rows are visited from the middle
// outwards so the heaviest rows (t2 (L - t2) tuples) start first.
template <int SGN, int PHASE>
__device__ __forceinline__ void rows3_body(const Args &a, float *Arow, float *wm)
{
    const int L = a.L;
    const int nrow = L - 3, nch = a.NC; // NC = column chunks per row
    const int ng = a.T1;                // row groups per wavefront tile
    const int64_t bid = blockIdx.x;
    const int s = (int)(bid / ((int64_t)nrow * nch));
    const int rem = (int)(bid % ((int64_t)nrow * nch));
    const int t2 = k3_row(rem / nch, L);
    const int chunk = rem % nch;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t tid0 = (((int64_t)s * nrow + (t2 - 1)) * nch + chunk) * (K3_THREADS / 64);
    const int ncols = L - 2 - t2;
    const int c0 = chunk * K3_CHUNK;
    const int n1 = (t2 + 7) & ~7;
    const int ngr = (n1 + K3_GROUP - 1) / K3_GROUP; // groups used by this row
    const TileCtx x = make_ctx(a, s, (const float *)a.head + (int64_t)s * a.Lp, (const float *)a.tail + (int64_t)s * a.Lp,
                               a.hl + (int64_t)s * a.Lp);
    const Best none = {-INFINITY, -INFINITY, 0x7fffffffffffffffLL, 0};
    float *gmax_w = a.tmax + (tid0 + w) * ng; // this wavefront's group maxima
    if (c0 >= ncols) { // empty chunk (whole workgroup)
        if (PHASE == 1) {
            for (int i = threadIdx.x; i < (K3_THREADS / 64) * ng; i += K3_THREADS)
                a.tmax[tid0 * ng + i] = -INFINITY;
        } else if (threadIdx.x < K3_THREADS / 64) {
            a.best[tid0 + threadIdx.x] = none;
        }
        return;
    }
    float thr = -INFINITY;
    if (PHASE == 2) {
        const Meta m = a.meta[s];
        const float M = ordered_to_float(m.menc);
        thr = phase2_threshold(M, m.delta);
        bool any = false;
        for (int i = threadIdx.x; i < (K3_THREADS / 64) * ng; i += K3_THREADS) {
            const float tm = a.tmax[tid0 * ng + i];
            any = any || (tm > -INFINITY && tm >= thr);
        }
        any = __syncthreads_or(any) && M > -INFINITY;
        if (!any) {
            if (threadIdx.x < K3_THREADS / 64)
                a.best[tid0 + threadIdx.x] = none;
            return;
        }
    }
    const float4 h2 = x.hl[t2];
    for (int t1 = threadIdx.x; t1 < n1; t1 += K3_THREADS)
        Arow[t1] = t1 < t2 ? x.hd[t1] + cls32<SGN>(h2, x.hl[t1], x.mq, x.gmax) : -INFINITY;
    float r[K3_COLS];
    int t3v[K3_COLS];
    int nv = 0; // column blocks of this wavefront holding a valid column
#pragma unroll
    for (int v = 0; v < K3_COLS; ++v) {
        const int cb = c0 + v * K3_THREADS + w * 64;
        const int c = cb + lane;
        const int t3 = t2 + 1 + c;
        t3v[v] = t3;
        r[v] = c < ncols ? cls32<SGN>(x.hl[t3], h2, x.mq, x.gmax) + x.tr[t3] : -INFINITY;
        nv += cb < ncols ? 1 : 0;
    }
    __syncthreads();
    Cand best = {-INFINITY, -INFINITY, 0x7fffffffffffffffLL};
    float wmax = -INFINITY;
    // phase 1 skips a group when the largest A of its rows plus the largest
    // column term of this wavefront is below the seeds' threshold: that sum
    // bounds every FP32 key of the block (rounded addition is monotone), and
    // no tuple of it is the arg max or ties with it (the argument of the k = 2
    // row pruning, k_setup)
    float pthr = -INFINITY, rmx = -INFINITY;
    if (PHASE == 1) {
        pthr = a.meta[s].pthr;
#pragma unroll
        for (int v = 0; v < K3_COLS; ++v)
            rmx = fmaxf(rmx, r[v]);
        rmx = wave_max(rmx);
    }
    for (int g = 0; g < ngr; ++g) {
        const int g0 = g * K3_GROUP, g1 = min(n1, g0 + K3_GROUP);
        if (PHASE == 2 && !(gmax_w[g] >= thr))
            continue;
        if (PHASE == 1 && pthr > -INFINITY) {
            const float ga = wave_max(lane < K3_GROUP && g0 + lane < g1 ? Arow[g0 + lane] : -INFINITY);
            if (ga + rmx < pthr) {
                if (lane == 0)
                    gmax_w[g] = -INFINITY;
                continue;
            }
        }
        float acc = -INFINITY;
        if (nv > 2)
            rows3_loop<4, PHASE>(x, Arow, g0, g1, r, t2, t3v, thr, acc, best);
        else if (nv == 2)
            rows3_loop<2, PHASE>(x, Arow, g0, g1, r, t2, t3v, thr, acc, best);
        else if (nv == 1)
            rows3_loop<1, PHASE>(x, Arow, g0, g1, r, t2, t3v, thr, acc, best);
        if (PHASE == 1) {
            acc = wave_max(acc);
            if (lane == 0)
                gmax_w[g] = acc;
            wmax = fmaxf(wmax, acc);
        }
    }
    if (PHASE == 1) {
        for (int g = ngr + lane; g < ng; g += 64)
            gmax_w[g] = -INFINITY;
        // one atomic per workgroup for the problem max
        if (lane == 0)
            wm[w] = wmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = wm[0];
            for (int i = 1; i < K3_THREADS / 64; ++i)
                m = fmaxf(m, wm[i]);
            if (m > -INFINITY)
                atomicMax(&a.meta[s].menc, float_to_ordered(m));
        }
    } else {
        wave_best(best.r, best.l, best.c);
        if (lane == 0)
            a.best[tid0 + w] = Best{best.r, best.l, best.c, 0};
    }
}

template <int PHASE>
__global__ void __launch_bounds__(K3_THREADS) k_rows3(Args a)
{
    extern __shared__ float4 arow_dyn[]; // Lp floats: the A row up to t2 (rounded up to 8)
    float *Arow = reinterpret_cast<float *>(arow_dyn);
    __shared__ float wm[K3_THREADS / 64];
    const int s = (int)((int64_t)blockIdx.x / ((int64_t)(a.L - 3) * a.NC));
    const double sgn = a.qc[s / a.nseg].sgn;
    if (sgn > 0)
        rows3_body<1, PHASE>(a, Arow, wm);
    else if (sgn < 0)
        rows3_body<-1, PHASE>(a, Arow, wm);
    else
        rows3_body<0, PHASE>(a, Arow, wm);
}

// Write problem s's result from its best candidate (plast = P(L-1) of the
// problem: 1, or 0 when it holds no voxel).
__device__ __forceinline__ void write_result(const Cand &b, const Args &a, int s, double plast, int32_t *thr,
                                             double *obj, int32_t *status)
{
    const int k = a.k;
    const QConst &qc = a.qc[s / a.nseg];
    const double q = qc.q, sgn = qc.sgn;
    if (b.r == -INFINITY) {
        for (int j = 0; j < k; ++j)
            thr[(int64_t)s * k + j] = -1;
        obj[s] = NAN;
        status[s] = plast > 0.0 ? TS_PROBLEM_DEGENERATE : TS_PROBLEM_EMPTY;
    } else {
        long long c = b.c;
        for (int j = k - 1; j >= 0; --j) {
            thr[(int64_t)s * k + j] = (int32_t)(c & 4095);
            c >>= 12;
        }
        // Shannon: S = sum of S_j; the sum-product variant ranks by S itself
        obj[s] = (sgn == 0.0 || a.mode == TS_SEARCH_SUMPROD) ? b.l : expm1(sgn * b.l) / (1.0 - q);
        status[s] = TS_PROBLEM_OK;
    }
}

// Single-launch path: one workgroup per problem does the setup, phase 1,
// phase 2 and the final reduction; head/tail rows and tile maxima stay in LDS.

// LDS of the one-workgroup path: the split prefixes hls [Lp] and FP64 copies
// of P, Q [Lp] (k = 2; phase 2 reads them), the rows hd, tr [Lp] and the tile
// maxima tmax [tiles] are carved from dynamic LDS sized for the launch
// (fused_lds_bytes); the rest is static.
constexpr int PRUNE_WORDS = 16 * 16; // k = 2: column blocks (<= 16) x Lp / 64 (<= 16)

struct FusedLds {
    float *hd, *tr, *tmax;
    float4 *hls;
    double *pd, *qd;
    double red[2 * (FUSED_THREADS / 64)];
    float wmax[FUSED_THREADS / 64];
    float wseed[FUSED_THREADS / 64];
    unsigned long long prune[PRUNE_WORDS];
    double wr[FUSED_THREADS / 64], wl[FUSED_THREADS / 64];
    long long wc[FUSED_THREADS / 64];
    float sdelta;
    int next;       // next tile to hand out in phase 1
    long long code; // the result's tuple code (-1: none)
};

static size_t fused_lds_bytes(int Lp, int k, int tiles)
{
    return (size_t)Lp * (2 * sizeof(float) + (k == 2 ? sizeof(float4) + 2 * sizeof(double) : 0)) +
           (size_t)tiles * sizeof(float);
}

// k = 2, rows of phase 1 that cannot hold the arg max.  For a row t1 and a
// column block [c0, c1] (c1 <= L - 2) every tuple (t1, t2) of the block has
//   key <= head(t1) + gb + max over the block of tail(t2),
// where gb bounds the middle class term g(t1, t2) (Tsallis-entropy section:
// the class terms of the objective).  A class of n bins has, by the power
// mean inequality, sum p^q <= n^(1-q) (sum p)^q for q < 1 and >= for q > 1,
// so g <= |1-q| log2 n (q = 1: the class entropy, <= log2 n); for t1 < c0
// its masses also lie between those of (t1, c0] and (t1, c1], so g <=
// log2 dQ(t1, c1) - q log2 dP(t1, c0) for q < 1 and q log2 dP(t1, c1) -
// log2 dQ(t1, c0) for q > 1.  The bound U is formed in FP32 like the keys;
// with E = delta / 2 the per-key error bound, U is within E of its FP64 value.
//
// Given the largest FP32 key Ms of some tuples sigma, a row with U < Ms -
// 3 delta has every FP64 key below key64(sigma) - delta: none of its tuples
// is the arg max or ties with it, while the row of sigma is kept.  Phase 1
// then skips groups of rows that are all marked; phase 2 is unchanged (its
// threshold comes from the keys phase 1 did evaluate, and the arg max is
// among them).  The seeds sigma are a coarse grid of tuples, one per thread.
template <int SGN>
__device__ __forceinline__ float seed_key(const TileCtx &x)
{
    int G = 1;
    while ((G + 1) * (G + 1) <= (int)blockDim.x)
        ++G;
    const int S = (x.L - 1 + G - 1) / G; // G positions over [0, L - 2]
    const int i = threadIdx.x / G, j = threadIdx.x % G;
    const int t1 = min(i * S + S / 2, x.L - 2), t2 = min(j * S + S / 2, x.L - 2);
    if (i >= G || !(t1 < t2))
        return -INFINITY;
    return (x.hd[t1] + cls32<SGN>(x.hl[t2], x.hl[t1], x.mq, x.gmax)) + x.tr[t2]; // as in phase 1
}


// Bit t1 % 64 of words[b * (Lp / 64) + t1 / 64] set: row t1 of column block b
// is skipped (rows without a tuple in the block are marked too).  One
// wavefront per word, lanes over rows.
template <int SGN>
__device__ __forceinline__ void prune_rows(const TileCtx &x, int NB, float pthr, unsigned long long *words)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int PW = x.Lp >> 6, L = x.L;
    for (int idx = w; idx < NB * PW; idx += nw) {
        const int b = idx / PW, t1 = (idx % PW) * 64 + lane;
        const int c0 = b * x.CW, c1 = min(c0 + x.CW - 1, L - 2);
        float tm = -INFINITY;
        for (int t2 = c0 + lane; t2 <= c1; t2 += 64)
            tm = fmaxf(tm, x.tr[t2]);
        tm = wave_max(tm);
        bool skip = true;
        if (t1 < c1) {
            float gb = x.cw * __builtin_amdgcn_logf((float)(c1 - t1)); // the widest class (t1, c1]
            if (SGN != 0 && t1 < c0) {
                const float4 hr = x.hl[t1], h0 = x.hl[c0], h1 = x.hl[c1];
                const float4 hp = SGN > 0 ? h0 : h1, hq = SGN > 0 ? h1 : h0;
                const float dp = (hp.x - hr.x) + (hp.y - hr.y);
                const float dq = (hq.z - hr.z) + (hq.w - hr.w);
                const float lx = __builtin_amdgcn_logf(dq), ly = __builtin_amdgcn_logf(dp);
                gb = fminf(gb, fmaf(x.mq, ly, SGN > 0 ? lx : -lx)); // NaN (empty classes) keeps gb
            }
            gb = __builtin_amdgcn_fmed3f(gb, 0.0f, x.gmax);
            skip = (x.hd[t1] + gb) + tm < pthr;
        }
        const unsigned long long m = __ballot(skip);
        if (lane == 0)
            words[idx] = m;
    }
}

// The whole search of problem s by the calling workgroup, from its prefix
// sums P, Q [L] (global memory, or LDS); stage: copy them to LDS for phase 2
// (k = 2 from global memory).  Writes the result and returns its tuple code
// (-1: no valid tuple) in every thread.
template <int SGN, int COLS, int K>
__device__ __forceinline__ long long fused_body(const Args &a, FusedLds &sh, int s, const double *P, const double *Q,
                                                bool stage, int32_t *__restrict__ thr_out, double *__restrict__ obj,
                                                int32_t *__restrict__ status)
{
    float *hd = sh.hd, *tr = sh.tr, *tmax = sh.tmax, *wmax = sh.wmax;
    float4 *hls = sh.hls;
    const QConst &qc = a.qc[s / a.nseg];
    // k = 2: split prefixes (and FP64 prefixes, when staged) in LDS
    const Steps stp = head_tail32<SGN>(a, qc, P, Q, hd, tr, K == 2 ? hls : nullptr, sh.red,
                                       K == 2 && stage ? sh.pd : nullptr, K == 2 && stage ? sh.qd : nullptr);
    TileCtx x = make_ctx(a, s, hd, tr, hls);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nw = blockDim.x >> 6;
    const bool prune = K == 2 && a.mode == TS_SEARCH_FP32_TIECHECK && a.NB * (a.Lp >> 6) <= PRUNE_WORDS;
    if (prune) { // the rows are in LDS (head_tail32 ends with a barrier)
        const float sk = wave_max(seed_key<SGN>(x));
        if (lane == 0)
            sh.wseed[w] = sk;
    }
    if (threadIdx.x == 0) {
        sh.sdelta = problem_delta(a, qc, stp, Q[a.L - 1]);
        sh.next = 0;
    }
    __syncthreads();
    if (prune) {
        float ms = -INFINITY;
        for (int i = 0; i < nw; ++i)
            ms = fmaxf(ms, sh.wseed[i]);
        const float pthr = prune_threshold(ms, sh.sdelta); // the same in every thread
        if (pthr > -INFINITY) {
            prune_rows<SGN>(x, a.NB, pthr, sh.prune);
            __syncthreads();
            x.prune = sh.prune;
        }
    }
    x.P = P;
    x.Q = Q;
    if (K == 2 && stage) { // phase 2 reads the prefixes from LDS
        x.P = sh.pd;
        x.Q = sh.qd;
    }
    Cand best = {-INFINITY, -INFINITY, 0x7fffffffffffffffLL};
    float wm = -INFINITY;
    // tiles are handed out one at a time from an LDS counter, heaviest first
    // (the last column block holds the longest t1 rows), so the wavefronts
    // finish phase 1 together
    for (;;) {
        int t = 0;
        if (lane == 0)
            t = atomicAdd(&sh.next, 1);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= a.tiles)
            break;
        const int b = a.NB - 1 - t / a.NC, c = t % a.NC;
        const int tile = c * a.NB + b;
        float acc = -INFINITY;
        tile_body<SGN, COLS, 1, K>(x, b, c, 0.0f, acc, best);
        acc = wave_max(acc);
        if (lane == 0)
            tmax[tile] = acc;
        wm = fmaxf(wm, acc);
    }
    if (lane == 0)
        wmax[w] = wm;
    __syncthreads();
    float M = -INFINITY;
    for (int i = 0; i < nw; ++i)
        M = fmaxf(M, wmax[i]);
    if (M > -INFINITY) {
        const float thr = phase2_threshold(M, sh.sdelta);
        // qualifying tiles found 64 at a time with a ballot (few qualify,
        // typically one); k = 1: the i-th goes to wavefront i mod nw; k = 2:
        // every wavefront takes a share of the rows of each of them
        int nth = 0;
        for (int base = 0; base < a.tiles; base += 64) {
            const int t = base + lane;
            unsigned long long m = __ballot(t < a.tiles && tmax[t] >= thr);
            while (m) {
                const int tile = base + __builtin_ctzll(m);
                m &= m - 1;
                float acc = -INFINITY;
                if (K == 1) {
                    if (nth++ % nw == w)
                        tile_body<SGN, COLS, 2, K>(x, tile % a.NB, tile / a.NB, thr, acc, best);
                } else {
                    tile_k2<SGN, COLS, 2>(x, tile % a.NB, tile / a.NB, thr, acc, best, w, nw);
                }
            }
        }
    }
    wave_best(best.r, best.l, best.c);
    if (lane == 0) {
        sh.wr[w] = best.r;
        sh.wl[w] = best.l;
        sh.wc[w] = best.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < nw; ++i)
            if (better(sh.wr[i], sh.wc[i], best.r, best.c)) {
                best.r = sh.wr[i];
                best.l = sh.wl[i];
                best.c = sh.wc[i];
            }
        write_result(best, a, s, P[a.L - 1], thr_out, obj, status);
        sh.code = best.r == -INFINITY ? -1LL : best.c;
    }
    lds_barrier(); // the result's global stores need not land before the workgroup goes on
    return sh.code;
}

template <int COLS, int K>
__global__ void __launch_bounds__(FUSED_THREADS) k_fused(Args a, int32_t *__restrict__ thr_out,
                                                         double *__restrict__ obj, int32_t *__restrict__ status)
{
    __shared__ FusedLds sh;
    extern __shared__ float4 dyn[]; // fused_lds_bytes(Lp, K, tiles)
    sh.hls = dyn;                   // 16-byte aligned: Lp is a multiple of 256
    sh.pd = reinterpret_cast<double *>(dyn + (K == 2 ? a.Lp : 0));
    sh.qd = sh.pd + (K == 2 ? a.Lp : 0);
    sh.hd = reinterpret_cast<float *>(sh.qd + (K == 2 ? a.Lp : 0));
    sh.tr = sh.hd + a.Lp;
    sh.tmax = sh.tr + a.Lp;
    const int s = blockIdx.x;
    const double sgn = a.qc[s / a.nseg].sgn;
    const double *P = a.P + (int64_t)(s % a.nseg) * a.L;
    const double *Q = a.Q + (int64_t)s * a.L;
    if (sgn > 0)
        fused_body<1, COLS, K>(a, sh, s, P, Q, true, thr_out, obj, status);
    else if (sgn < 0)
        fused_body<-1, COLS, K>(a, sh, s, P, Q, true, thr_out, obj, status);
    else
        fused_body<0, COLS, K>(a, sh, s, P, Q, true, thr_out, obj, status);
}

// FP64 mode: exhaustive FP64 keys with the lexicographic tie rule.
template <int COLS>
__global__ void __launch_bounds__(256) k_tiles64(Args a)
{
    const Tile tl = tile_of(a);
    if (!tl.valid)
        return;
    const int lane = threadIdx.x & 63;
    const int L = a.L, Lp = a.Lp, k = a.k;
    const int s = tl.s;
    const int64_t tid = (int64_t)s * a.tiles + tl.tile;
    const QConst &c = a.qc[s / a.nseg];
    const double *P = a.P + (int64_t)(s % a.nseg) * L;
    const double *Q = a.Q + (int64_t)s * L;
    const double *hd = (const double *)a.head + (int64_t)s * Lp;
    const double *tr = (const double *)a.tail + (int64_t)s * Lp;
    double br = -INFINITY;
    long long bc = 0x7fffffffffffffffLL;
    auto offer = [&](double key, long long code) {
        if (better(key, code, br, bc)) {
            br = key;
            bc = code;
        }
    };
    if (k == 1) {
        for (int v = 0; v < COLS; ++v) {
            const int t = tl.b * a.CW + v * 64 + lane;
            offer(hd[t] + tr[t], t);
        }
    } else if (k == 2) {
        const int cbase = tl.b * a.CW;
        const int r0 = tl.c * a.T1;
        const int r1 = min(r0 + a.T1, min(L - 2, cbase + a.CW - 1));
        for (int t1 = r0; t1 < r1; ++t1) {
            const double pr = P[t1], qr = Q[t1], hr = hd[t1];
            for (int v = 0; v < COLS; ++v) {
                const int t2 = cbase + v * 64 + lane;
                if (t1 < t2) {
                    const int ti = min(t2, L - 1);
                    const double key = (hr + cls64(P[ti] - pr, Q[ti] - qr, c.q, c.sgn, c.hmax)) + tr[t2];
                    offer(key, ((long long)t1 << 12) | t2);
                }
            }
        }
    } else {
        const int t2 = L - 3 - tl.c;
        const int cbase = tl.b * a.CW;
        if (cbase + a.CW - 1 > t2 && cbase <= L - 2) {
            const double *Ar = (const double *)a.A + ((int64_t)s * L + t2) * Lp;
            const double *Rr = (const double *)a.R + ((int64_t)s * L + t2) * Lp;
            for (int v = 0; v < COLS; ++v) {
                const int t3 = cbase + v * 64 + lane;
                const double rc = Rr[t3];
                double vb = -INFINITY;
                int vt = 0;
                for (int t1 = 0; t1 < t2; ++t1) { // t1 ascending: strict > keeps the first
                    const double key = Ar[t1] + rc;
                    if (key > vb) {
                        vb = key;
                        vt = t1;
                    }
                }
                offer(vb, ((long long)vt << 24) | ((long long)t2 << 12) | t3);
            }
        }
    }
    double bl = br;
    wave_best(br, bl, bc);
    if (lane == 0)
        a.best[tid] = Best{br, br, bc, 0};
}

// ---------------------------------------------------------------- final

__global__ void __launch_bounds__(1024) k_final(Args a, const Best *__restrict__ best, int per,
                                                int32_t *__restrict__ thr, double *__restrict__ obj,
                                                int32_t *__restrict__ status, int s_base)
{
    const int s = s_base + blockIdx.x;
    const Best *b = best + (int64_t)blockIdx.x * per;
    double br = -INFINITY, bl = -INFINITY;
    long long bc = 0x7fffffffffffffffLL;
    int i = threadIdx.x;
    const int st = blockDim.x;
    for (; i + 3 * st < per; i += 4 * st) { // four loads in flight per thread
        Best x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            x[u] = b[i + u * st];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (better(x[u].rank, x[u].code, br, bc)) {
                br = x[u].rank;
                bl = x[u].lam;
                bc = x[u].code;
            }
    }
    for (; i < per; i += st) {
        const Best x = b[i];
        if (better(x.rank, x.code, br, bc)) {
            br = x.rank;
            bl = x.lam;
            bc = x.code;
        }
    }
    wave_best(br, bl, bc);
    __shared__ double sr[16], sl[16];
    __shared__ long long sc[16];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[w] = br;
        sl[w] = bl;
        sc[w] = bc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 1; j < (int)(blockDim.x >> 6); ++j)
            if (better(sr[j], sc[j], br, bc)) {
                br = sr[j];
                bl = sl[j];
                bc = sc[j];
            }
        write_result(Cand{br, bl, bc}, a, s, a.P[(int64_t)(s % a.nseg) * a.L + a.L - 1], thr, obj, status);
    }
}

// ---------------------------------------------------------------- plain

__device__ __forceinline__ int64_t binom(int64_t x, int r)
{
    if (x < r)
        return 0;
    if (r == 1)
        return x;
    if (r == 2)
        return x * (x - 1) / 2;
    return x * (x - 1) * (x - 2) / 6;
}

// largest x with binom(x, r) <= v
__device__ __forceinline__ int64_t inv_binom(int64_t v, int r)
{
    double est;
    if (r == 1)
        return v;
    if (r == 2)
        est = floor(sqrt(2.0 * (double)v)) + 1.0;
    else
        est = floor(cbrt(6.0 * (double)v)) + 2.0;
    int64_t x = (int64_t)est;
    while (binom(x, r) > v)
        --x;
    while (binom(x + 1, r) <= v)
        ++x;
    return x;
}

__global__ void __launch_bounds__(256) k_plain(const double *__restrict__ P, const double *__restrict__ Q, int L,
                                               int k, int64_t ntup, double q, double sgn, double hmax,
                                               Best *__restrict__ out)
{
    double br = -INFINITY, bl = -INFINITY;
    long long bc = 0x7fffffffffffffffLL;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ntup;
         r += (int64_t)gridDim.x * blockDim.x) {
        // combinatorial number system: r = C(t_k, k) + ... + C(t_1, 1)
        int t[3];
        int64_t v = r;
        for (int j = k; j >= 1; --j) {
            const int64_t x = inv_binom(v, j);
            t[j - 1] = (int)x;
            v -= binom(x, j);
        }
        const double lam = lambda64(P, Q, L, k, t, q, sgn, hmax);
        const long long code = make_code(k, t);
        if (better(lam, code, br, bc)) {
            br = lam;
            bl = lam;
            bc = code;
        }
    }
    wave_best(br, bl, bc);
    __shared__ double sr[4];
    __shared__ long long sc[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[w] = br;
        sc[w] = bc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
            if (better(sr[i], sc[i], br, bc)) {
                br = sr[i];
                bc = sc[i];
            }
        out[blockIdx.x] = Best{br, br, bc, 0};
    }
}

// The plain GPU form in single precision: one thread per tuple (unranked as
// in k_plain), every class term evaluated directly in FP32 from the prefix
// sums split into two floats (cls32, the keys of the FP32 modes); the first
// tuple with the largest key, and its FP64 Lambda beside it for the result.
template <int SGN>
__global__ void __launch_bounds__(256) k_plain32(const double *__restrict__ P, const double *__restrict__ Q, int L,
                                                 int k, int64_t ntup, QConst c, Best *__restrict__ out)
{
    float bk = -INFINITY;
    long long bc = 0x7fffffffffffffffLL;
    int bt[3] = {0, 0, 0};
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ntup;
         r += (int64_t)gridDim.x * blockDim.x) {
        int t[3] = {0, 0, 0};
        int64_t v = r;
        for (int j = k; j >= 1; --j) {
            const int64_t x = inv_binom(v, j);
            t[j - 1] = (int)x;
            v -= binom(x, j);
        }
        float key = 0.0f;
        float4 ha = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int j = 0; j <= k; ++j) {
            const int b = j == k ? L - 1 : t[j];
            const float4 hb = split_hl(P[b], Q[b]);
            key += cls32<SGN>(hb, ha, c.mq, c.gmax);
            ha = hb;
        }
        const long long code = make_code(k, t);
        if (key > bk || (key == bk && code < bc)) {
            bk = key;
            bc = code;
            bt[0] = t[0];
            bt[1] = t[1];
            bt[2] = t[2];
        }
    }
    double rank = (double)bk, lam = -INFINITY;
    if (bk > -INFINITY)
        lam = lambda64(P, Q, L, k, bt, c.q, c.sgn, c.hmax);
    wave_best(rank, lam, bc);
    __shared__ double sr[4], sl[4];
    __shared__ long long sc[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[w] = rank;
        sl[w] = lam;
        sc[w] = bc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
            if (better(sr[i], sc[i], rank, bc)) {
                rank = sr[i];
                lam = sl[i];
                bc = sc[i];
            }
        out[blockIdx.x] = Best{rank, lam, bc, 0};
    }
}

// ---------------------------------------------------------------- sum-product variant

// The multilevel variant sum_j S_j + (1-q) prod_j S_j of one tuple in FP64
// from the prefix sums, each class entropy S_j = (1 - Q_j / w_j^q) / (q - 1)
// = -expm1(ln Q_j - q ln w_j) / (q - 1) (for q = 1 the Shannon entropy
// ln w_j - E_j / w_j, composed by the plain sum); -inf when a class is empty.
__device__ __forceinline__ double sumprod64(const double *P, const double *Q, int L, int k, const int *t, double q,
                                            double sgn)
{
    double sum = 0.0, prod = 1.0;
    double pa = 0.0, qa = 0.0;
#pragma unroll 1
    for (int j = 0; j <= k; ++j) {
        const int b = j == k ? L - 1 : t[j];
        const double pb = P[b], qb = Q[b];
        const double dP = pb - pa, dQ = qb - qa;
        if (!(dP > 0.0))
            return -INFINITY;
        const double S = sgn == 0.0 ? log(dP) - dQ / dP : -expm1(log(dQ) - q * log(dP)) / (q - 1.0);
        sum += S;
        prod *= S;
        pa = pb;
        qa = qb;
    }
    return sgn == 0.0 ? sum : sum + (1.0 - q) * prod;
}

// Every tuple of every problem: workgroup blockIdx.x covers one contiguous
// range of tuple ranks of problem blockIdx.x / per (combinatorial number
// system), one tuple per thread at a time; the first best of the range goes
// to out[blockIdx.x] (reduced per problem by k_final).
__global__ void __launch_bounds__(256) k_sumprod(Args a, int64_t ntup, int per, Best *__restrict__ out)
{
    const int s = blockIdx.x / per, part = blockIdx.x % per;
    const QConst &c = a.qc[s / a.nseg];
    const double *P = a.P + (int64_t)(s % a.nseg) * a.L;
    const double *Q = a.Q + (int64_t)s * a.L;
    const int64_t chunk = (ntup + per - 1) / per;
    const int64_t r0 = (int64_t)part * chunk, r1 = min(ntup, r0 + chunk);
    double br = -INFINITY, bl = -INFINITY;
    long long bc = 0x7fffffffffffffffLL;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        int t[3];
        int64_t v = r;
        for (int j = a.k; j >= 1; --j) {
            const int64_t x = inv_binom(v, j);
            t[j - 1] = (int)x;
            v -= binom(x, j);
        }
        const double S = sumprod64(P, Q, a.L, a.k, t, c.q, c.sgn);
        const long long code = make_code(a.k, t);
        if (better(S, code, br, bc)) {
            br = S;
            bl = S;
            bc = code;
        }
    }
    wave_best(br, bl, bc);
    __shared__ double sr[4];
    __shared__ long long sc[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[w] = br;
        sc[w] = bc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
            if (better(sr[i], sc[i], br, bc)) {
                br = sr[i];
                bc = sc[i];
            }
        out[blockIdx.x] = Best{br, br, bc, 0};
    }
}

QConst make_qconst(double q, int L);

// ---------------------------------------------------------------- whole path

// ts_segment: histogram, prefix sums, search and labels of every problem in
// one launch (one workgroup per problem), or in two (P workgroups per problem
// counting parts of it, the last of them to finish doing the prefix sums and
// the search; then the label pass).  The steps are the device code of the
// separate passes (count8_rt, prefix_row with the same bins per thread,
// fused_body, lab8), so every output is bit-identical to theirs.
//
// LDS: area A (the histogram replicas; later the prefix scan's scratch; then
// the search's rows) | counts [Lp] | P [Lp] | Q [nq][Lp].

constexpr int SEG_COLS = 2;            // search columns per lane
constexpr int SEG_MAX_PARTS = 64;      // workgroups per problem
constexpr int SEG_MAX_PART_WG = 1024;  // problems x parts when parts > 1
constexpr size_t SEG_MAX_LDS = 150 * 1024; // dynamic LDS of one workgroup (160 KiB per CU, static part aside)
constexpr int SEG_SEPARATE_BELOW = 1024;   // problems below which a call may take the separate passes

struct SegArgs {
    const int16_t *const *vox;
    const int64_t *offs;
    int nseg, parts, lr, nq, E;
    BinMap bm;
    uint32_t *hist;        // out [nseg][L]
    uint32_t *partial;            // [nseg][parts][L] when parts > 1
    unsigned long long *tickets;  // [nseg] when parts > 1 (any initial contents)
    unsigned int epoch;           // this call's tag of the tickets (never 0)
    LabelSets sets;        // label sets written by this kernel (label = 1)
    int label;
    int areaA; // bytes of LDS area A (a multiple of 16)
};

// The part's ticket for its problem: the word holds (call tag << 32 | parts
// counted so far); a word left by another call, or any other contents, is
// restarted for this call.  Returns 1 for the first part to arrive, parts for
// the last.  Each failed exchange means another part got in, so the loop
// ends after at most parts + 1 rounds.
__device__ __forceinline__ unsigned int take_ticket(unsigned long long *t, unsigned int epoch)
{
    unsigned long long old = __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const unsigned long long nw =
            (unsigned int)(old >> 32) == epoch ? old + 1ull : (((unsigned long long)epoch << 32) | 1ull);
        unsigned long long seen = old;
        if (__hip_atomic_compare_exchange_strong(t, &seen, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return (unsigned int)(nw & 0xffffffffull);
        old = seen;
    }
}

// Count the voxels [i0, i1) of one problem into the LDS replicas: scalar head
// up to the first 16-byte boundary, 16-byte vectors with the next four in
// flight while four are counted, scalar tail.  Ordinary loads: the label
// pass of the same workgroup reads these bytes again.
template <int MAP>
__device__ __forceinline__ void seg_count(uint32_t *lds, int lr, const TS_GLOBAL int16_t *base, int64_t i0, int64_t i1,
                                          const BinMap &bm)
{
    const uint32_t rep = threadIdx.x & ((1u << lr) - 1u);
    int64_t head = (int64_t)(((16u - ((uintptr_t)(base + i0) & 15u)) & 15u) >> 1);
    if (head > i1 - i0)
        head = i1 - i0;
    if (threadIdx.x < head)
        atomicAdd(&lds[(bin_of_t<MAP>(base[i0 + threadIdx.x], bm) << lr) + rep], 1u);
    const int64_t vb = i0 + head;
    const int64_t nvec = (i1 - vb) >> 3;
    const TS_GLOBAL v4i *vp = reinterpret_cast<const TS_GLOBAL v4i *>(base + vb);
    const int64_t st = blockDim.x;
    int64_t j = threadIdx.x;
    bool have = j + 3 * st < nvec;
    v4i a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
    if (have) {
        a0 = vp[j];
        a1 = vp[j + st];
        a2 = vp[j + 2 * st];
        a3 = vp[j + 3 * st];
    }
    while (have) {
        const int64_t jn = j + 4 * st;
        const bool nxt = jn + 3 * st < nvec;
        v4i b0 = a0, b1 = a1, b2 = a2, b3 = a3;
        if (nxt) {
            b0 = vp[jn];
            b1 = vp[jn + st];
            b2 = vp[jn + 2 * st];
            b3 = vp[jn + 3 * st];
        }
        count8_rt<MAP>(lds, a0, bm, lr, rep);
        count8_rt<MAP>(lds, a1, bm, lr, rep);
        count8_rt<MAP>(lds, a2, bm, lr, rep);
        count8_rt<MAP>(lds, a3, bm, lr, rep);
        a0 = b0;
        a1 = b1;
        a2 = b2;
        a3 = b3;
        j = jn;
        have = nxt;
    }
    for (; j < nvec; j += st) {
        const v4i w = vp[j];
        count8_rt<MAP>(lds, w, bm, lr, rep);
    }
    const int64_t tb = vb + (nvec << 3);
    if (threadIdx.x < i1 - tb)
        atomicAdd(&lds[(bin_of_t<MAP>(base[tb + threadIdx.x], bm) << lr) + rep], 1u);
}

// Labels of one whole problem for nq threshold sets (thresholds in LDS), the
// rules of the label pass: 16-byte loads of 8 voxels and 8-byte stores per
// set where the input and outputs share the alignment phase, else voxel by
// voxel.
template <int K>
__device__ __forceinline__ void seg_label(const SegArgs &g, int s, const TS_GLOBAL int16_t *src, int64_t n,
                                          const int (*tsh)[K])
{
    Cuts<K> cu[TS_MAX_LABEL_SETS];
    PCuts<K> pc[TS_MAX_LABEL_SETS];
    TS_GLOBAL uint8_t *dst[TS_MAX_LABEL_SETS];
    int64_t head = (int64_t)(((16u - ((uintptr_t)src & 15u)) & 15u) >> 1);
    if (head > n)
        head = n;
    bool vec = true;
#pragma unroll
    for (int u = 0; u < TS_MAX_LABEL_SETS; ++u) {
        if (u < g.nq) {
            cu[u] = make_cuts<K>(tsh[u], K, g.bm);
            pc[u] = pack_cuts(cu[u]);
            dst[u] = gpw(g.sets.out[u][s]);
            vec = vec && (((uintptr_t)(dst[u] + head)) & 7u) == 0;
        }
    }
    const int64_t bd = blockDim.x;
    if (!vec) {
        for (int64_t i = threadIdx.x; i < n; i += bd) {
            const int v = src[i];
#pragma unroll
            for (int u = 0; u < TS_MAX_LABEL_SETS; ++u)
                if (u < g.nq)
                    dst[u][i] = (uint8_t)lab1(v, cu[u]);
        }
        return;
    }
    if (threadIdx.x < head) {
        const int v = src[threadIdx.x];
#pragma unroll
        for (int u = 0; u < TS_MAX_LABEL_SETS; ++u)
            if (u < g.nq)
                dst[u][threadIdx.x] = (uint8_t)lab1p(v, pc[u]);
    }
    const TS_GLOBAL v4i *vp = reinterpret_cast<const TS_GLOBAL v4i *>(src + head);
    const int64_t nvec = (n - head) >> 3;
    for (int64_t i0 = threadIdx.x; i0 < nvec; i0 += 4 * bd) {
        v4i w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + e * bd;
            w[e] = i < nvec ? __builtin_nontemporal_load(vp + i) : v4i{0, 0, 0, 0};
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + e * bd;
            if (i < nvec) {
#pragma unroll
                for (int u = 0; u < TS_MAX_LABEL_SETS; ++u)
                    if (u < g.nq)
                        __builtin_nontemporal_store(lab8(w[e], pc[u]),
                                                    reinterpret_cast<TS_GLOBAL v2u *>(dst[u] + head) + i);
            }
        }
    }
    const int64_t tb = head + (nvec << 3);
    if (threadIdx.x < n - tb) {
        const int v = src[tb + threadIdx.x];
#pragma unroll
        for (int u = 0; u < TS_MAX_LABEL_SETS; ++u)
            if (u < g.nq)
                dst[u][tb + threadIdx.x] = (uint8_t)lab1p(v, pc[u]);
    }
}

template <int K, int MAP>
__global__ void __launch_bounds__(1024) k_segment(SegArgs g, Args a, int32_t *__restrict__ thr_out,
                                                  double *__restrict__ obj, int32_t *__restrict__ status)
{
    extern __shared__ float4 dyn[];
    __shared__ FusedLds sh;
    __shared__ PrefixLds ps;
    __shared__ unsigned int tk;
    __shared__ int tsh[TS_MAX_LABEL_SETS][K];
    const int L = g.bm.L, Lp = a.Lp;
    char *area = reinterpret_cast<char *>(dyn);
    uint32_t *rl = reinterpret_cast<uint32_t *>(area);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(area + g.areaA);
    double *Pl = reinterpret_cast<double *>(area + g.areaA + (size_t)4 * Lp); // then Q of each q, [Lp] each
    const int s = blockIdx.x / g.parts, part = blockIdx.x % g.parts;
    const int lr = g.lr;

    for (int i = threadIdx.x; i < (L << lr); i += blockDim.x)
        rl[i] = 0u;
    __syncthreads();
    const int64_t o0 = g.offs[s], n = g.offs[s + 1] - o0;
    const TS_GLOBAL int16_t *src = gp(g.vox[s]);
    {
        const int64_t per = ((n + g.parts - 1) / g.parts + 7) & ~(int64_t)7;
        const int64_t i0 = min(n, (int64_t)part * per), i1 = min(n, i0 + per);
        if (i0 < i1)
            seg_count<MAP>(rl, lr, src, i0, i1, g.bm);
    }
    __syncthreads();
    const int R = 1 << lr;
    if (g.parts == 1) {
        for (int b = threadIdx.x; b < L; b += blockDim.x) {
            uint32_t c = 0;
            for (int r = 0; r < R; ++r)
                c += rl[(b << lr) + r];
            cnt[b] = c;
            g.hist[(int64_t)s * L + b] = c;
        }
    } else {
        // the part's counts go out as device-coherent stores; once every
        // store is acknowledged the part takes a ticket, and the part that
        // takes the last one adds all parts up (device-coherent loads) and
        // goes on.  No cache-wide fence is needed: only these stores and
        // loads cross workgroups.
        uint32_t *mine = g.partial + ((int64_t)s * g.parts + part) * L;
        for (int b = threadIdx.x; b < L; b += blockDim.x) {
            uint32_t c = 0;
            for (int r = 0; r < R; ++r)
                c += rl[(b << lr) + r];
            __hip_atomic_store(mine + b, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            tk = take_ticket(g.tickets + s, g.epoch);
        __syncthreads();
        if (tk != (unsigned int)g.parts)
            return;
        const uint32_t *pp = g.partial + (int64_t)s * g.parts * L;
        const int bd = blockDim.x;
        for (int b0 = threadIdx.x; b0 < L; b0 += 4 * bd) {
            uint32_t c[4] = {0u, 0u, 0u, 0u};
            for (int p0 = 0; p0 < g.parts; p0 += 8) { // 32 loads in flight
                uint32_t v[4][8];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int b = b0 + i * bd, p = p0 + u;
                        v[i][u] = (b < L && p < g.parts)
                                      ? __hip_atomic_load(pp + (int64_t)p * L + b, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : 0u;
                    }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        c[i] += v[i][u];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int b = b0 + i * bd;
                if (b < L) {
                    cnt[b] = c[i];
                    g.hist[(int64_t)s * L + b] = c[i];
                }
            }
        }
    }
    __syncthreads();
    // prefix sums and search, one q at a time (P once, Q per q, in LDS)
    double *qs = reinterpret_cast<double *>(area);
    int *lastocc = reinterpret_cast<int *>(area + (size_t)8 * L);
    sh.hls = reinterpret_cast<float4 *>(area);
    sh.pd = nullptr;
    sh.qd = nullptr;
    sh.hd = reinterpret_cast<float *>(area + (K == 2 ? (size_t)16 * Lp : 0));
    sh.tr = sh.hd + Lp;
    sh.tmax = sh.tr + Lp;
    // every q's prefix sums first, then the searches: the scan's constants
    // are then dead before the search starts (a loop over both held them in
    // registers across the search and spilled them to scratch)
    for (int j = 0; j < g.nq; ++j)
        prefix_row([cnt](int b) { return cnt[b]; }, L, g.E, a.qc[j].q, j == 0 ? Pl : nullptr, Pl + (size_t)(1 + j) * Lp,
                   qs, lastocc, ps);
    for (int j = 0; j < g.nq; ++j) {
        const int sj = j * g.nseg + s;
        const double *Ql = Pl + (size_t)(1 + j) * Lp;
        const double sgn = a.qc[j].sgn;
        long long code;
        if (sgn > 0)
            code = fused_body<1, SEG_COLS, K>(a, sh, sj, Pl, Ql, false, thr_out, obj, status);
        else if (sgn < 0)
            code = fused_body<-1, SEG_COLS, K>(a, sh, sj, Pl, Ql, false, thr_out, obj, status);
        else
            code = fused_body<0, SEG_COLS, K>(a, sh, sj, Pl, Ql, false, thr_out, obj, status);
        if (threadIdx.x == 0 && j < TS_MAX_LABEL_SETS) {
            for (int i = K - 1; i >= 0; --i) {
                tsh[j][i] = code < 0 ? -1 : (int)(code & 4095);
                code = code < 0 ? code : code >> 12;
            }
        }
    }
    if (!g.label)
        return;
    __syncthreads();
    seg_label<K>(g, s, src, n, tsh);
}

static size_t seg_areaA(int L, int Lp, int k, int tiles, int lr);

static size_t seg_lds_bytes(int L, int Lp, int k, int tiles, int lr, int nq)
{
    return seg_areaA(L, Lp, k, tiles, lr) + (size_t)Lp * (sizeof(uint32_t) + (size_t)(1 + nq) * sizeof(double));
}

static bool seg_fusable(int L, int k, int mode, int nq, bool labels)
{
    if (mode != TS_SEARCH_FP32_TIECHECK && mode != TS_SEARCH_FP32_ONLY)
        return false;
    if (labels && nq > TS_MAX_LABEL_SETS)
        return false;
    if (!((k == 1 && L <= FUSED_MAX_L) || (k == 2 && L <= FUSED_MAX_L2)))
        return false;
    // the search's tiles (any tuning: the fewest rows per tile) and the LDS
    // with one histogram replica
    const Plan p = make_plan(1, L, k, mode, SEG_COLS, 16);
    return p.tiles <= FUSED_MAX_TILES && seg_lds_bytes(L, p.Lp, k, p.tiles, 0, nq) <= SEG_MAX_LDS;
}

static int seg_log2_replicas(const Tune &t)
{
    int lr = 0;
    while ((1 << lr) < t.hist_replicas)
        ++lr;
    return lr;
}

static size_t seg_areaA(int L, int Lp, int k, int tiles, int lr)
{
    size_t a = ((size_t)L << lr) * sizeof(uint32_t);
    a = std::max(a, (size_t)L * (sizeof(double) + sizeof(int)));
    a = std::max(a, fused_lds_bytes(Lp, k, tiles));
    return (a + 15) & ~(size_t)15;
}

static size_t seg_separate_bytes(int nseg, int L, int k, int nq, int mode)
{
    // P, Q and the search workspace of the separate passes
    return align256((size_t)nseg * L * sizeof(double)) + align256((size_t)nq * nseg * L * sizeof(double)) +
           search_workspace_bytes(nseg * nq, L, k, mode, 4);
}

static size_t small_bytes(int L);
static bool small_path(const ts_batch &b, int L, int k, int nq, int mode, const Tune &t);
static ts_status launch_small(const ts_batch &b, const BinMap &bm, const double *q, uint32_t *hist, int32_t *thr,
                              double *obj, int32_t *status, const LabelSets *sets, void *ws, hipStream_t st);

size_t segment_workspace_bytes(int nseg, int L, int k, int nq, int mode, bool labels)
{
    if (nseg == 1 && k == 1 && nq == 1 && mode == TS_SEARCH_FP32_TIECHECK && L <= FUSED_MAX_L)
        return std::max(small_bytes(L), seg_separate_bytes(nseg, L, k, nq, mode));
    if (!seg_fusable(L, k, mode, nq, labels))
        return seg_separate_bytes(nseg, L, k, nq, mode);
    const size_t fused = align256((size_t)nseg * sizeof(unsigned long long)) +
                         (size_t)L * sizeof(uint32_t) *
                             (size_t)std::min<int64_t>(SEG_MAX_PART_WG, (int64_t)nseg * SEG_MAX_PARTS);
    // below SEG_SEPARATE_BELOW problems the call may take the separate passes
    return nseg < SEG_SEPARATE_BELOW ? std::max(fused, seg_separate_bytes(nseg, L, k, nq, mode)) : fused;
}

// Whether a fusable call takes the fused kernel: with one workgroup per
// problem when the problems fill the chip twice over (fewer problems leave
// compute units idle, and the separate passes, which split every problem
// over many workgroups, are faster there), or as the tuning asks.
static bool seg_use_fused(int nseg, const Tune &t)
{
    if (t.segment_parts)
        return true;
    return nseg >= SEG_SEPARATE_BELOW || nseg >= 2 * device_cu_count();
}

// Workgroups per problem: one unless the tuning asks for more (within what
// the workspace holds).
static int seg_parts(int nseg, const Tune &t)
{
    if (t.segment_parts <= 1)
        return 1;
    return std::max(1, std::min(t.segment_parts, SEG_MAX_PART_WG / std::max(nseg, 1)));
}

template <int K, int MAP>
static void launch_seg_km(dim3 g, dim3 b, size_t lds, hipStream_t st, const SegArgs &sa, const Args &a, int32_t *thr,
                          double *obj, int32_t *status)
{
    allow_dynamic_lds((const void *)k_segment<K, MAP>, lds);
    hipLaunchKernelGGL((k_segment<K, MAP>), g, b, lds, st, sa, a, thr, obj, status);
}

ts_status launch_segment(const ts_batch &b, const BinMap &bm, int k, int nq, const double *q, int mode,
                         uint32_t *hist, int32_t *thr, double *obj, int32_t *status, const LabelSets *sets, void *ws,
                         const Tune &t, hipStream_t st)
{
    const int L = bm.L, nseg = b.nseg;
    char *wb = (char *)ws;
    if (small_path(b, L, k, nq, mode, t))
        return launch_small(b, bm, q, hist, thr, obj, status, sets, ws, st);
    if (!seg_fusable(L, k, mode, nq, sets != nullptr) || !seg_use_fused(nseg, t)) {
        double *P = (double *)wb;
        double *Q = (double *)(wb + align256((size_t)nseg * L * sizeof(double)));
        char *sw = wb + align256((size_t)nseg * L * sizeof(double)) + align256((size_t)nq * nseg * L * sizeof(double));
        ts_status e;
        if ((e = launch_histogram(b, bm, hist, t, st)) != TS_OK)
            return e;
        if ((e = launch_prefix(hist, nseg, L, nq, q, P, Q, st)) != TS_OK)
            return e;
        if ((e = launch_search(P, Q, nseg, L, k, nq, q, mode, sw, search_workspace_bytes(nseg * nq, L, k, mode, 4),
                               thr, obj, status, t, st)) != TS_OK)
            return e;
        return sets ? launch_label(b, bm, *sets, nq, k, t, st) : TS_OK;
    }
    const int parts = seg_parts(nseg, t);
    const Plan p = make_plan(nseg * nq, L, k, mode, SEG_COLS, t.search_rows);
    Args a = {};
    a.P = nullptr;
    a.Q = nullptr;
    a.nseg = nseg;
    a.nprob = nseg * nq;
    a.L = L;
    a.Lp = p.Lp;
    a.k = k;
    a.mode = mode;
    for (int j = 0; j < TS_MAX_Q; ++j)
        a.qc[j] = make_qconst(q[j < nq ? j : 0], L);
    a.CW = p.CW;
    a.NB = p.NB;
    a.NC = p.NC;
    a.T1 = p.T1;
    a.tiles = p.tiles;
    SegArgs sa = {};
    sa.vox = b.vox;
    sa.offs = b.offs;
    sa.nseg = nseg;
    sa.parts = parts;
    sa.lr = seg_log2_replicas(t);
    sa.nq = nq;
    sa.E = prefix_bins_per_thread(L);
    sa.bm = bm;
    sa.hist = hist;
    sa.tickets = (unsigned long long *)wb;
    sa.partial = (uint32_t *)(wb + align256((size_t)nseg * sizeof(unsigned long long)));
    {
        // a tag per call (never 0), starting from a value of this process's
        // clock so that words left in reused memory are unlikely to match
        static std::atomic<unsigned int> seq{(unsigned int)std::chrono::steady_clock::now().time_since_epoch().count()};
        unsigned int e;
        do
            e = ++seq;
        while (e == 0);
        sa.epoch = e;
    }
    sa.label = sets != nullptr && parts == 1;
    if (sets)
        sa.sets = *sets;
    // fewer histogram replicas if the LDS would not hold them (replicas
    // change no result)
    size_t lds;
    for (;;) {
        sa.areaA = (int)seg_areaA(L, p.Lp, k, p.tiles, sa.lr);
        lds = seg_lds_bytes(L, p.Lp, k, p.tiles, sa.lr, nq);
        if (lds <= SEG_MAX_LDS || sa.lr == 0)
            break;
        --sa.lr;
    }
    if (lds > SEG_MAX_LDS)
        return fail(TS_ERR_UNSUPPORTED, "ts_segment: sizes beyond the LDS of one workgroup");
    // the prefix scan needs blockDim * E >= L
    int block = t.segment_block ? t.segment_block : (parts > 1 || L >= 1024 ? 1024 : 512);
    while (block * sa.E < L)
        block *= 2;
    const dim3 g((unsigned)((int64_t)nseg * parts)), blk((unsigned)block);
#define TS_SEG(K)                                                                                                    \
    switch (map_kind(bm)) {                                                                                          \
    case 0: launch_seg_km<K, 0>(g, blk, lds, st, sa, a, thr, obj, status); break;                                   \
    case 1: launch_seg_km<K, 1>(g, blk, lds, st, sa, a, thr, obj, status); break;                                   \
    case 2: launch_seg_km<K, 2>(g, blk, lds, st, sa, a, thr, obj, status); break;                                   \
    default: launch_seg_km<K, 3>(g, blk, lds, st, sa, a, thr, obj, status); break;                                  \
    }
    if (k == 1) {
        TS_SEG(1)
    } else {
        TS_SEG(2)
    }
#undef TS_SEG
    ts_status e = check_launch("ts_segment");
    if (e != TS_OK)
        return e;
    if (sets && parts > 1)
        return launch_label(b, bm, *sets, nq, k, t, st);
    return TS_OK;
}

// ---------------------------------------------------------------- one small problem

// ts_segment for one problem with one threshold (k = 1, one q) and few
// voxels, e.g. one slice at 4096 levels: the per-bin work (p^q of every bin,
// the scans, the objective of every threshold) is spread over many compute
// units instead of one workgroup.  One cooperative launch of G workgroups
// (all resident at once) with three grid barriers:
//   1. each workgroup counts its share of the voxels into LDS and stores its
//      partial histogram;
//   2. virtual wavefront v of the prefix scan (the 64 threads of bins
//      [64 v E, 64 (v + 1) E) in prefix_row's layout, E bins per thread) runs
//      as wavefront 0 of workgroup v: it adds up the partials of its bins,
//      forms p^q (the voxel count N is known up front: every voxel falls in
//      a bin) and the wavefront's part of the scans, and publishes its totals;
//   3. every virtual wavefront takes the exclusive bases from the totals of
//      the ones before it in prefix_row's order (so P and Q are the same bits
//      as the prefix pass), evaluates the FP64 objective of each of its
//      thresholds with the re-check's own function, and publishes its best;
// then every workgroup takes the best of the bests (first threshold among
// equals) and labels its share of the voxels.  The FP64 arg max over every
// threshold is the tuple the FP32 search with its FP64 re-check returns, and
// the objective written is computed from the same Lambda by the same code,
// so every output is bit-identical to the separate passes.  A barrier wait
// gives up after about a quarter of a second (a cooperative launch keeps
// every workgroup resident, so it never should) and the problem's status
// then reports it.

constexpr int SMALL_THREADS = 256;
constexpr int SMALL_MAX_G = 64;                        // workgroups of one launch
constexpr int SMALL_MIN_VOX_PER_WG = 16384;            // voxels per workgroup, at least
constexpr int64_t SMALL_MAX_VOX = (int64_t)SMALL_MAX_G * 65536; // larger problems take the other paths
constexpr int SMALL_REC = 16;                          // 8-byte words per virtual-wavefront record

struct SmallArgs {
    const int16_t *const *vox;    // the batch's table (one problem)
    uint8_t *const *labtab;       // its label table (or null)
    int64_t n;
    BinMap bm;
    int G, E, NWV, lr;
    uint32_t *hist;          // out [L]
    uint32_t *part;          // [G][L] partial histograms
    unsigned long long *rec; // [NWV][SMALL_REC]
    unsigned long long *bar; // barrier word: (call tag << 32) | arrivals
    unsigned int epoch;
};

// Grid barrier number `round` (1, 2, 3) of the launch: every workgroup's
// device-coherent stores are complete before it arrives; returns false if
// the wait gave up.
__device__ __forceinline__ bool small_sync(const SmallArgs &g, int round, int *ok)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        // arrival: one fetch-add on (call tag << 32 | arrivals); before the
        // first barrier a word left by another call (or any contents) is
        // restarted at (tag, 0) by one exchange, which fails harmlessly once
        // some workgroup has restarted it (its tag then matches)
        if (round == 1) {
            unsigned long long v = __hip_atomic_load(g.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((v >> 32) != (unsigned long long)g.epoch)
                (void)__hip_atomic_compare_exchange_strong(g.bar, &v, (unsigned long long)g.epoch << 32,
                                                           __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
        }
        (void)__hip_atomic_fetch_add(g.bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long want = ((unsigned long long)g.epoch << 32) | (unsigned long long)(round * g.G);
        int spins = 0;
        for (;;) {
            const unsigned long long v = __hip_atomic_load(g.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((v >> 32) == (unsigned long long)g.epoch && v >= want)
                break;
            if (++spins > (1 << 22)) {
                *ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    return *ok != 0;
}

__device__ __forceinline__ void small_put(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long small_get(const unsigned long long *p)
{
    return __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Labels of voxels [i0, i1) of the problem (the rules of the label pass).
__device__ __forceinline__ void small_label(const TS_GLOBAL int16_t *src, TS_GLOBAL uint8_t *dst, int64_t i0,
                                            int64_t i1, const PCuts<1> &pc)
{
    int64_t head = (int64_t)(((16u - ((uintptr_t)(src + i0) & 15u)) & 15u) >> 1);
    if (head > i1 - i0)
        head = i1 - i0;
    const bool vec = (((uintptr_t)(dst + i0 + head)) & 7u) == 0;
    if (!vec) {
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
            dst[i] = (uint8_t)lab1p(src[i], pc);
        return;
    }
    if (threadIdx.x < head)
        dst[i0 + threadIdx.x] = (uint8_t)lab1p(src[i0 + threadIdx.x], pc);
    const int64_t vb = i0 + head, nvec = (i1 - vb) >> 3;
    const TS_GLOBAL v4i *vp = reinterpret_cast<const TS_GLOBAL v4i *>(src + vb);
    TS_GLOBAL v2u *op = reinterpret_cast<TS_GLOBAL v2u *>(dst + vb);
    const int64_t bd = blockDim.x;
    for (int64_t i0 = threadIdx.x; i0 < nvec; i0 += 4 * bd) { // four vectors in flight
        v4i x[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            x[e] = i0 + e * bd < nvec ? __builtin_nontemporal_load(vp + i0 + e * bd) : v4i{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (i0 + e * bd < nvec)
                __builtin_nontemporal_store(lab8(x[e], pc), op + i0 + e * bd);
    }
    const int64_t tb = vb + (nvec << 3);
    if (threadIdx.x < i1 - tb)
        dst[tb + threadIdx.x] = (uint8_t)lab1p(src[tb + threadIdx.x], pc);
}

// 64-bit readlane (lane u uniform)
__device__ __forceinline__ unsigned long long small_rl(unsigned long long v, int u)
{
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(v & 0xffffffffull), u);
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(v >> 32), u);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double small_rlf(double v, int u)
{
    return __longlong_as_double((long long)small_rl((unsigned long long)__double_as_longlong(v), u));
}

template <int MAP>
__global__ void __launch_bounds__(SMALL_THREADS) k_small(SmallArgs g, Args a, int32_t *__restrict__ thr_out,
                                                        double *__restrict__ obj, int32_t *__restrict__ status)
{
    // LDS: the histogram replicas; after barrier 1: P, Q [L], then for this
    // virtual wavefront qs, p^q [64 E] and the counts [64 E]
    extern __shared__ double sdyn[];
    __shared__ int ok, tstar;
    __shared__ double wr[SMALL_THREADS / 64], wl[SMALL_THREADS / 64];
    __shared__ long long wc[SMALL_THREADS / 64];
    static_assert(SMALL_THREADS / 64 == PREFIX_MAX_E, "one wavefront per bin slot of a prefix thread");
    const int L = g.bm.L, w = blockIdx.x, lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); // the bin slot e of stages 2 and 3
    if (threadIdx.x == 0)
        ok = 1;
    const TS_GLOBAL int16_t *src = gp(g.vox[0]);
    // ---- 1. partial histogram of this workgroup's voxels
    uint32_t *rl = reinterpret_cast<uint32_t *>(sdyn);
    for (int i = threadIdx.x; i < (L << g.lr); i += blockDim.x)
        rl[i] = 0u;
    __syncthreads();
    const int64_t per = ((g.n + g.G - 1) / g.G + 7) & ~(int64_t)7;
    const int64_t v0 = min(g.n, (int64_t)w * per), v1 = min(g.n, v0 + per);
    if (v0 < v1)
        seg_count<MAP>(rl, g.lr, src, v0, v1, g.bm);
    __syncthreads();
    for (int b = threadIdx.x; b < L; b += blockDim.x) {
        uint32_t c = 0;
        for (int r = 0; r < (1 << g.lr); ++r)
            c += rl[(b << g.lr) + r];
        __hip_atomic_store(g.part + (int64_t)w * L + b, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    small_sync(g, 1, &ok);
    const int E = g.E, wb = w * 64 * E;
    double *Pl = sdyn, *Ql = sdyn + L, *qsl = sdyn + 2 * L, *pql = qsl + 64 * E;
    uint32_t *cl = reinterpret_cast<uint32_t *>(pql + 64 * E);
    const QConst &qc = a.qc[0];
    const double q = qc.q;
    const uint64_t N = (uint64_t)g.n;
    const double Nd = (double)N;
    const bool vw = w < g.NWV;          // workgroup w is virtual wavefront w of the scan (uniform)
    const int b0 = (w * 64 + lane) * E; // this lane's prefix-thread bins [b0, b0 + E)
    uint32_t c[PREFIX_MAX_E];
    double pq[PREFIX_MAX_E];
    uint64_t cincl = 0;
    double qincl = 0.0;
    int oincl = -1;
    if (vw) {
        // ---- 2a. wavefront e adds up the partials of bin b0 + e of every
        // lane (every load in flight at once) and forms its p^q
        if (wv < E) {
            const int b = b0 + wv;
            uint32_t ce = 0;
            if (b < L) {
                for (int p0 = 0; p0 < g.G; p0 += 32) {
                    uint32_t v[32];
#pragma unroll
                    for (int u = 0; u < 32; ++u)
                        v[u] = p0 + u < g.G ? __hip_atomic_load(g.part + (int64_t)(p0 + u) * L + b, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT)
                                            : 0u;
#pragma unroll
                    for (int u = 0; u < 32; ++u)
                        ce += v[u];
                }
                g.hist[b] = ce;
            }
            const double pe = (double)ce / Nd;
            cl[lane * E + wv] = ce;
            pql[lane * E + wv] = ce ? (q == 1.0 ? pe * log(pe) : pow(pe, q)) : 0.0; // q = 1: the Shannon limit
        }
        __syncthreads();
        // ---- 2b. wavefront 0 is the virtual wavefront: the thread totals of
        // prefix_row, the wavefront's part of the scans, its record
        if (wv == 0) {
            uint64_t csum = 0;
            int occ = -1;
            double qloc = 0.0;
#pragma unroll
            for (int e = 0; e < PREFIX_MAX_E; ++e) {
                c[e] = e < E ? cl[lane * E + e] : 0u;
                pq[e] = e < E ? pql[lane * E + e] : 0.0;
                csum += c[e];
                if (c[e])
                    occ = b0 + e;
                qloc += pq[e]; // left to right
            }
            cincl = csum;
            qincl = qloc;
            oincl = occ;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint64_t cv = __shfl_up(cincl, o, 64);
                const double qv = __shfl_up(qincl, o, 64);
                const int ov = __shfl_up(oincl, o, 64);
                if (lane >= o) {
                    cincl = cv + cincl;
                    qincl = qv + qincl;
                    oincl = ov > oincl ? ov : oincl;
                }
            }
            // the record: totals, and what another wavefront needs to rebuild
            // qs at this wavefront's last occupied bin
            const unsigned long long occmask = __ballot(occ >= 0);
            unsigned long long *rv = g.rec + (int64_t)w * SMALL_REC;
            const double qprev = __shfl_up(qincl, 1, 64); // inclusive q of the lane before
            const int jl = occmask ? 63 - __builtin_clzll(occmask) : -1; // lane of the last occupied bin
            if (lane == 63) {
                small_put(rv + 0, cincl);
                small_put(rv + 1, (unsigned long long)__double_as_longlong(qincl));
                small_put(rv + 2, (unsigned long long)(long long)oincl);
            }
            if (lane == jl) {
                double loc = 0.0;
#pragma unroll
                for (int e = 0; e < PREFIX_MAX_E; ++e)
                    if (e < E && b0 + e < L && b0 + e <= occ)
                        loc += pq[e];
                small_put(rv + 3, (unsigned long long)jl);
                small_put(rv + 4, (unsigned long long)__double_as_longlong(qprev));
                small_put(rv + 5, (unsigned long long)__double_as_longlong(loc));
            }
        }
    }
    small_sync(g, 2, &ok);
    if (vw) {
        if (wv == 0) {
            // ---- 3a. bases from the virtual wavefronts before this one (lane
            // u < NWV loads record u; the sequential sums run over readlanes),
            // P and Q of the wavefront's bins
            uint64_t rc = 0, r3 = 0, r4 = 0, r5 = 0;
            long long r2 = -1;
            double rq = 0.0;
            if (lane < g.NWV) {
                const unsigned long long *ru = g.rec + (int64_t)lane * SMALL_REC;
                rc = small_get(ru + 0);
                rq = __longlong_as_double((long long)small_get(ru + 1));
                r2 = (long long)small_get(ru + 2);
                r3 = small_get(ru + 3);
                r4 = small_get(ru + 4);
                r5 = small_get(ru + 5);
            }
            const int om = (int)r2;
            // excl_u = ((0 + t_0) + t_1) + ... + t_(u-1): the scan's sequential order
            double run = 0.0, excl_mine = 0.0;
            uint64_t cbase = 0;
            int obase = -1, lastw = -1;
            for (int u = 0; u < g.NWV; ++u) {
                if (lane == u)
                    excl_mine = run;
                run = run + small_rlf(rq, u);
                const int omu = __builtin_amdgcn_readlane(om, u);
                if (u < w) {
                    cbase += small_rl(rc, u);
                    obase = omu > obase ? omu : obase;
                }
                if (omu >= 0)
                    lastw = u;
            }
            // qs at the last occupied bin of virtual wavefront u (lane u's view)
            const double qs_last_mine =
                ((int)r3 == 0 ? excl_mine : excl_mine + __longlong_as_double((long long)r4)) +
                __longlong_as_double((long long)r5);
            const double qbase_w = small_rlf(excl_mine, w);
            const double qs_before = obase >= 0 ? small_rlf(qs_last_mine, obase / (64 * E)) : 0.0;
            const double qs_end = lastw >= 0 ? small_rlf(qs_last_mine, lastw) : 0.0;
            // exclusive lane prefixes within the wavefront
            const uint64_t cex = __shfl_up(cincl, 1, 64);
            const double qex = __shfl_up(qincl, 1, 64);
            const int oex = __shfl_up(oincl, 1, 64);
            const double qb = lane == 0 ? qbase_w : qbase_w + qex;
            int last = lane == 0 ? obase : (oex > obase ? oex : obase);
            uint64_t C = cbase + (lane == 0 ? 0 : cex);
            double loc = 0.0;
            int lastocc[PREFIX_MAX_E];
#pragma unroll
            for (int e = 0; e < PREFIX_MAX_E; ++e) {
                lastocc[e] = -1;
                if (e < E && b0 + e < L) {
                    const int t = b0 + e;
                    C += c[e];
                    loc += pq[e];
                    if (c[e])
                        last = t;
                    Pl[t] = (double)C / Nd;
                    qsl[t - wb] = qb + loc;
                    lastocc[e] = last;
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
            for (int e = 0; e < PREFIX_MAX_E; ++e) {
                if (e < E && b0 + e < L) { // Q of the last occupied bin at or before t
                    const int t = b0 + e, lt = lastocc[e];
                    Ql[t] = lt < 0 ? 0.0 : (lt >= wb ? qsl[lt - wb] : qs_before);
                }
            }
            if (lane == 0) { // P and Q at L - 1: the whole problem
                Pl[L - 1] = 1.0;
                Ql[L - 1] = qs_end;
            }
        }
        __syncthreads();
        // ---- 3b. wavefront e evaluates threshold b0 + e of every lane with
        // the re-check's FP64 function; the best of the workgroup
        double r = -INFINITY, lm = -INFINITY;
        long long cd = 0x7fffffffffffffffLL;
        const int t = b0 + wv;
        if (wv < E && t <= L - 2) {
            r = lambda64_k<1>(Pl, Ql, L, &t, q, qc.sgn, qc.hmax);
            lm = r;
            cd = t;
        }
        wave_best(r, lm, cd);
        if (lane == 0) {
            wr[wv] = r;
            wl[wv] = lm;
            wc[wv] = cd;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            Cand best = {-INFINITY, -INFINITY, 0x7fffffffffffffffLL};
            for (int i = 0; i < SMALL_THREADS / 64; ++i)
                if (better(wr[i], wc[i], best.r, best.c)) {
                    best.r = wr[i];
                    best.l = wl[i];
                    best.c = wc[i];
                }
            unsigned long long *rv = g.rec + (int64_t)w * SMALL_REC;
            small_put(rv + 6, (unsigned long long)__double_as_longlong(best.r));
            small_put(rv + 7, (unsigned long long)__double_as_longlong(best.l));
            small_put(rv + 8, (unsigned long long)best.c);
        }
    }
    const bool synced = small_sync(g, 3, &ok);
    // ---- the best of the bests (lane u of wavefront 0 loads the best of
    // virtual wavefront u), the result, the labels
    if (threadIdx.x < 64) {
        double r = -INFINITY, l = -INFINITY;
        long long cd = 0x7fffffffffffffffLL;
        if (lane < g.NWV) {
            const unsigned long long *ru = g.rec + (int64_t)lane * SMALL_REC;
            r = __longlong_as_double((long long)small_get(ru + 6));
            l = __longlong_as_double((long long)small_get(ru + 7));
            cd = (long long)small_get(ru + 8);
        }
        wave_best(r, l, cd);
        if (threadIdx.x == 0) {
            const Cand best = {r, l, cd};
            tstar = r == -INFINITY ? -1 : (int)cd;
            if (w == 0) {
                write_result(best, a, 0, 1.0, thr_out, obj, status);
                if (!synced)
                    status[0] = TS_PROBLEM_SYNC_FAILED;
            }
        }
    }
    __syncthreads();
    if (g.labtab && v0 < v1) {
        const int32_t tv[1] = {tstar};
        const PCuts<1> pc = pack_cuts(make_cuts<1>(tv, 1, g.bm));
        small_label(src, gpw(g.labtab[0]), v0, v1, pc);
    }
}

static size_t small_bytes(int L) { return align256((size_t)SMALL_MAX_G * L * sizeof(uint32_t)) + align256((size_t)16 * SMALL_REC * 8) + 256; }

// Whether ts_segment takes the one-problem cooperative path.
static bool small_path(const ts_batch &b, int L, int k, int nq, int mode, const Tune &t)
{
    return b.nseg == 1 && k == 1 && nq == 1 && mode == TS_SEARCH_FP32_TIECHECK && L <= FUSED_MAX_L &&
           b.total > 0 && b.total <= SMALL_MAX_VOX && !t.segment_parts;
}

static ts_status launch_small(const ts_batch &b, const BinMap &bm, const double *q, uint32_t *hist, int32_t *thr,
                              double *obj, int32_t *status, const LabelSets *sets, void *ws, hipStream_t st)
{
    const int L = bm.L;
    SmallArgs g = {};
    g.vox = b.vox;
    g.labtab = sets ? sets->out[0] : nullptr;
    g.n = b.total;
    g.bm = bm;
    g.E = prefix_bins_per_thread(L);
    g.NWV = prefix_threads(L) / 64;
    g.G = (int)std::max<int64_t>(g.NWV, std::min<int64_t>(SMALL_MAX_G, (b.total + SMALL_MIN_VOX_PER_WG - 1) /
                                                                              SMALL_MIN_VOX_PER_WG));
    g.lr = L <= 1024 ? 2 : 0;
    g.hist = hist;
    char *wb = (char *)ws;
    g.part = (uint32_t *)wb;
    g.rec = (unsigned long long *)(wb + align256((size_t)SMALL_MAX_G * L * sizeof(uint32_t)));
    g.bar = g.rec + 16 * SMALL_REC;
    {
        static std::atomic<unsigned int> seq{(unsigned int)std::chrono::steady_clock::now().time_since_epoch().count() ^
                                             0x5a5a5a5au};
        unsigned int e;
        do
            e = ++seq;
        while (e == 0);
        g.epoch = e;
    }
    Args a = {};
    a.nseg = 1;
    a.nprob = 1;
    a.L = L;
    a.Lp = L;
    a.k = 1;
    a.mode = TS_SEARCH_FP32_TIECHECK;
    for (int j = 0; j < TS_MAX_Q; ++j)
        a.qc[j] = make_qconst(q[0], L);
    const size_t lds = std::max((size_t)(L << g.lr) * sizeof(uint32_t),
                                (size_t)(2 * L + 2 * 64 * g.E) * sizeof(double) + (size_t)64 * g.E * sizeof(uint32_t));
    const dim3 grid((unsigned)g.G), blk(SMALL_THREADS);
#define TS_SMALL(M)                                                                                                 \
    allow_dynamic_lds((const void *)k_small<M>, lds);                                                              \
    hipLaunchKernelGGL(k_small<M>, grid, blk, lds, st, g, a, thr, obj, status)
    switch (map_kind(bm)) {
    case 0: TS_SMALL(0); break;
    case 1: TS_SMALL(1); break;
    case 2: TS_SMALL(2); break;
    default: TS_SMALL(3); break;
    }
#undef TS_SMALL
    return check_launch("ts_segment");
}

// ---------------------------------------------------------------- dispatch

template <int COLS>
static void launch_fp32(int fused_block, int k, dim3 g, hipStream_t st, const Args &a, int32_t *thr, double *obj,
                        int32_t *status)
{
    if (fused_block) {
        const dim3 gf((unsigned)a.nprob), bf((unsigned)fused_block);
        const size_t lds = fused_lds_bytes(a.Lp, k, a.tiles);
        if (k == 1)
            hipLaunchKernelGGL((k_fused<COLS, 1>), gf, bf, lds, st, a, thr, obj, status);
        else
            hipLaunchKernelGGL((k_fused<COLS, 2>), gf, bf, lds, st, a, thr, obj, status);
        return;
    }
    if (k == 1) {
        hipLaunchKernelGGL((k_tiles32<COLS, 1, 1>), g, dim3(256), 0, st, a);
        hipLaunchKernelGGL((k_tiles32<COLS, 2, 1>), g, dim3(256), 0, st, a);
    } else { // k = 3 uses k_rows3
        hipLaunchKernelGGL((k_tiles32<COLS, 1, 2>), g, dim3(256), 0, st, a);
        hipLaunchKernelGGL((k_tiles32<COLS, 2, 2>), g, dim3(256), 0, st, a);
    }
}

static void launch_fp32_cols(int cols, int fused, int k, dim3 g, hipStream_t st, const Args &a, int32_t *thr,
                             double *obj, int32_t *status)
{
    if (cols == 1)
        launch_fp32<1>(fused, k, g, st, a, thr, obj, status);
    else if (cols == 2)
        launch_fp32<2>(fused, k, g, st, a, thr, obj, status);
    else
        launch_fp32<4>(fused, k, g, st, a, thr, obj, status);
}

QConst make_qconst(double q, int L)
{
    QConst c;
    c.q = q;
    const bool shannon = q == 1.0; // class entropies at most ln L in either case
    c.sgn = shannon ? 0.0 : (q < 1.0 ? 1.0 : -1.0);
    c.hmax = (shannon ? 1.0 : fabs(1.0 - q)) * log((double)L);
    c.mq = (float)(-c.sgn) * (float)q;
    const double gm = (shannon ? 1.0 : fabs(1.0 - q)) * log2((double)L);
    float g = (float)gm;
    if ((double)g < gm)
        g = nextafterf(g, INFINITY);
    c.gmax = g;
    const double cw = shannon ? 1.0 : fabs(1.0 - q);
    float w = (float)cw;
    if ((double)w < cw)
        w = nextafterf(w, INFINITY);
    c.cw = w;
    return c;
}

// One workgroup per problem (k_fused, nothing in the workspace) when that
// fills the chip or the problem is small, unless the tuning forces a path.
static bool fused_path(const Plan &p, int nprob, const Tune &t)
{
    const bool fp32 = p.mode == TS_SEARCH_FP32_TIECHECK || p.mode == TS_SEARCH_FP32_ONLY;
    const bool can_fuse = fp32 && p.tiles <= FUSED_MAX_TILES && p.Lp <= FUSED_MAX_L &&
                          (p.k == 1 || (p.k == 2 && p.L <= FUSED_MAX_L2));
    return can_fuse && (t.search_path == 1 || (t.search_path == 0 && (p.k == 1 || nprob >= 128)));
}

size_t search_need_bytes(int nprob, int L, int k, int mode, const Tune &t)
{
    const Plan p = make_plan(nprob, L, k, mode, t.search_cols, t.search_rows);
    return fused_path(p, nprob, t) ? 0 : p.bytes;
}

ts_status launch_search(const double *P, const double *Q, int nseg, int L, int k, int nq, const double *q, int mode,
                        void *ws, size_t ws_bytes, int32_t *thr, double *obj, int32_t *status, const Tune &t,
                        hipStream_t st)
{
    (void)ws_bytes;
    const int nprob = nq * nseg;
    const Plan p = make_plan(nprob, L, k, mode, t.search_cols, t.search_rows);
    char *base = (char *)ws;
    Args a;
    a.P = P;
    a.Q = Q;
    a.nseg = nseg;
    a.nprob = nprob;
    a.L = L;
    a.Lp = p.Lp;
    a.k = k;
    a.mode = mode;
    for (int j = 0; j < TS_MAX_Q; ++j)
        a.qc[j] = make_qconst(q[j < nq ? j : 0], L);
    a.CW = p.CW;
    a.NB = p.NB;
    a.NC = p.NC;
    a.T1 = p.T1;
    a.tiles = p.tiles;
    a.meta = (Meta *)(base + p.off_meta);
    a.hl = (float4 *)(base + p.off_hl);
    a.head = base + p.off_head;
    a.tail = base + p.off_tail;
    a.A = base + p.off_A;
    a.R = base + p.off_R;
    a.tmax = (float *)(base + p.off_tmax);
    a.best = (Best *)(base + p.off_best);

    if (mode == TS_SEARCH_SUMPROD) {
        const int per = sumprod_blocks(L, k);
        Best *pb = (Best *)(base + p.off_plain);
        hipLaunchKernelGGL(k_sumprod, dim3((unsigned)((int64_t)nprob * per)), dim3(256), 0, st, a, tuples_of(L, k), per,
                           pb);
        hipLaunchKernelGGL(k_final, dim3((unsigned)nprob), dim3(1024), 0, st, a, pb, per, thr, obj, status, 0);
        return check_launch("ts_threshold_search (sum-product)");
    }
    if (mode == TS_SEARCH_PLAIN_FP32) {
        const int64_t n = L - 1;
        const int64_t ntup = k == 1 ? n : (k == 2 ? n * (n - 1) / 2 : n * (n - 1) * (n - 2) / 6);
        const int blocks = (int)std::min<int64_t>(PLAIN_BLOCKS, std::max<int64_t>(1, (ntup + 255) / 256));
        Best *pb = (Best *)(base + p.off_plain);
        for (int s = 0; s < nprob; ++s) {
            const QConst &c = a.qc[s / nseg];
            const double *Ps = P + (int64_t)(s % nseg) * L, *Qs = Q + (int64_t)s * L;
            if (c.sgn > 0)
                hipLaunchKernelGGL(k_plain32<1>, dim3(blocks), dim3(256), 0, st, Ps, Qs, L, k, ntup, c, pb);
            else if (c.sgn < 0)
                hipLaunchKernelGGL(k_plain32<-1>, dim3(blocks), dim3(256), 0, st, Ps, Qs, L, k, ntup, c, pb);
            else
                hipLaunchKernelGGL(k_plain32<0>, dim3(blocks), dim3(256), 0, st, Ps, Qs, L, k, ntup, c, pb);
            hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, a, pb, blocks, thr, obj, status, s);
        }
        return check_launch("ts_threshold_search (plain FP32)");
    }
    if (mode == TS_SEARCH_PLAIN) {
        const int64_t n = L - 1;
        const int64_t ntup = k == 1 ? n : (k == 2 ? n * (n - 1) / 2 : n * (n - 1) * (n - 2) / 6);
        const int blocks = (int)std::min<int64_t>(PLAIN_BLOCKS, std::max<int64_t>(1, (ntup + 255) / 256));
        Best *pb = (Best *)(base + p.off_plain);
        for (int s = 0; s < nprob; ++s) {
            const QConst &c = a.qc[s / nseg];
            hipLaunchKernelGGL(k_plain, dim3(blocks), dim3(256), 0, st, P + (int64_t)(s % nseg) * L,
                               Q + (int64_t)s * L, L, k, ntup, c.q, c.sgn, c.hmax, pb);
            hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, a, pb, blocks, thr, obj, status, s);
        }
        return check_launch("ts_threshold_search (plain)");
    }

    const bool fp32 = mode == TS_SEARCH_FP32_TIECHECK || mode == TS_SEARCH_FP32_ONLY;
    const bool fused = fused_path(p, nprob, t);
    const int64_t waves = (int64_t)nprob * p.tiles;
    dim3 g((unsigned)((waves + 3) / 4));
    if (fused) {
        launch_fp32_cols(t.search_cols, t.search_block, k, g, st, a, thr, obj, status);
        return check_launch("ts_threshold_search");
    }
    hipLaunchKernelGGL(k_setup, dim3(nprob), dim3(256), 0, st, a);
    if (k == 3 && mode == TS_SEARCH_FP64) {
        dim3 gp((unsigned)((int64_t)(L - 3) * nprob));
        hipLaunchKernelGGL(k_pairs64, gp, dim3(256), 0, st, a);
    }
    if (k == 3 && fp32) {
        dim3 gr((unsigned)((int64_t)(L - 3) * p.NC * nprob));
        const size_t lds = (size_t)p.Lp * sizeof(float);
        hipLaunchKernelGGL(k_rows3<1>, gr, dim3(K3_THREADS), lds, st, a);
        hipLaunchKernelGGL(k_rows3<2>, gr, dim3(K3_THREADS), lds, st, a);
        hipLaunchKernelGGL(k_final, dim3(nprob), dim3(1024), 0, st, a, a.best, p.tiles, thr, obj, status, 0);
        return check_launch("ts_threshold_search");
    }
    if (mode == TS_SEARCH_FP64) {
        if (t.search_cols == 1)
            hipLaunchKernelGGL(k_tiles64<1>, g, dim3(256), 0, st, a);
        else if (t.search_cols == 2)
            hipLaunchKernelGGL(k_tiles64<2>, g, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(k_tiles64<4>, g, dim3(256), 0, st, a);
    } else {
        launch_fp32_cols(t.search_cols, 0, k, g, st, a, thr, obj, status);
    }
    hipLaunchKernelGGL(k_final, dim3(nprob), dim3(1024), 0, st, a, a.best, p.tiles, thr, obj, status, 0);
    return check_launch("ts_threshold_search");
}

} // namespace ts
