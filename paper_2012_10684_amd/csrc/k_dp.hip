// k_dp.hip -- exact multilevel threshold search by dynamic programming over
// the class boundaries, for any k up to TS_DP_MAX_K (Tsallis-entropy section:
// the objective of k thresholds is 1 + (1-q) S = prod_j Q_j / w_j^q, so the
// arg max of S is the arg max of the sum of the class terms
// g(a..b) = sgn(1-q) (ln Q_[a,b] - q ln w_[a,b]), or of the class Shannon
// entropies for q = 1; a sum over consecutive classes is separable).
//
// Completion values, for a threshold at t and m more thresholds after it:
//   V_0(t) = g(t+1 .. L-1)
//   V_m(t) = max over t < u <= L-2 of g(t+1 .. u) + V_{m-1}(u)
// and the maximum M = max over t of g(0 .. t) + V_{k-1}(t).  FP64 addition is
// monotone, so M is exactly the largest of the per-tuple sums formed right
// to left.  The tuple is rebuilt from the left: t_1 is the smallest t whose
// value equals M, then t_j the smallest u > t_{j-1} whose value equals
// V_{k-j+1}(t_{j-1}); values are recomputed by the same expressions, so the
// equalities are exact and the tuple is the first (lexicographically) of
// those reaching M.  A class with zero mass has g = -inf.  Empty bins repeat
// P and Q bit for bit (ts_prefix), so tuples that differ inside a run of
// empty bins tie exactly, as in the exhaustive search.
//
// Work: k (L-1)^2 / 2 class terms (two FP64 logarithms each) per problem,
// against C(L-1, k) tuples for the exhaustive search.
#include <math.h>

#include "common.h"

namespace ts {

constexpr int DP_THREADS = 256;

struct DPQ {
    double q[TS_MAX_Q];
};

struct DPArgs {
    const double *P, *Q;
    int nseg, nprob, L, k;
    DPQ qs;
    double *V; // [k][nprob][L]
};

__device__ __forceinline__ void dp_consts(double q, int L, double &sgn, double &hmax)
{
    sgn = q == 1.0 ? 0.0 : (q < 1.0 ? 1.0 : -1.0);
    hmax = (q == 1.0 ? 1.0 : fabs(1.0 - q)) * log((double)L); // a class holds at most L bins
}

// Class term of the bins a..b (a <= b) from the prefix sums; -inf if the
// class has zero mass; clamped to [0, hmax].
__device__ __forceinline__ double dp_g(const double *P, const double *Q, int a, int b, double q, double sgn,
                                       double hmax)
{
    const double pa = a ? P[a - 1] : 0.0, qa = a ? Q[a - 1] : 0.0;
    const double dP = P[b] - pa, dQ = Q[b] - qa;
    if (!(dP > 0.0))
        return -INFINITY;
    const double h = sgn == 0.0 ? log(dP) - dQ / dP : sgn * (log(dQ) - q * log(dP));
    return fmin(fmax(h, 0.0), hmax);
}

// V_0(t) for every (problem, t): one thread each.
__global__ void __launch_bounds__(DP_THREADS) k_dp_last(DPArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int L = a.L;
    if (i >= (int64_t)a.nprob * L)
        return;
    const int s = (int)(i / L), t = (int)(i % L);
    const double q = a.qs.q[s / a.nseg];
    double sgn, hmax;
    dp_consts(q, L, sgn, hmax);
    const double *P = a.P + (int64_t)(s % a.nseg) * L, *Q = a.Q + (int64_t)s * L;
    a.V[i] = t <= L - 2 ? dp_g(P, Q, t + 1, L - 1, q, sgn, hmax) : -INFINITY;
}

__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// V_m(t) for one (problem, t) per workgroup: the threads split u.
__global__ void __launch_bounds__(DP_THREADS) k_dp_level(DPArgs a, int m)
{
    __shared__ double red[DP_THREADS / 64];
    const int L = a.L;
    const int s = blockIdx.x / (L - 1), t = blockIdx.x % (L - 1);
    const double q = a.qs.q[s / a.nseg];
    double sgn, hmax;
    dp_consts(q, L, sgn, hmax);
    const double *P = a.P + (int64_t)(s % a.nseg) * L, *Q = a.Q + (int64_t)s * L;
    const double *Vp = a.V + ((int64_t)(m - 1) * a.nprob + s) * L;
    double best = -INFINITY;
    for (int u = t + 1 + threadIdx.x; u <= L - 2; u += blockDim.x) {
        const double vu = Vp[u];
        if (vu > -INFINITY)
            best = fmax(best, dp_g(P, Q, t + 1, u, q, sgn, hmax) + vu);
    }
    best = wave_max_d(best);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            best = fmax(best, red[w]);
        a.V[((int64_t)m * a.nprob + s) * L + t] = best;
    }
}

// Smallest index in [lo, hi] whose value equals target (or hi + 1), for the
// wavefront; value(u) is evaluated once per index.
template <typename F>
__device__ __forceinline__ int first_equal(int lo, int hi, double target, F &&value)
{
    int found = 0x7fffffff;
    for (int u = lo + (int)threadIdx.x; u <= hi; u += 64)
        if (u < found && value(u) == target)
            found = u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        found = min(found, __shfl_xor(found, o, 64));
    return found;
}

// One wavefront per problem: the maximum and the first tuple reaching it.
__global__ void __launch_bounds__(64) k_dp_final(DPArgs a, int32_t *__restrict__ thr, double *__restrict__ obj,
                                                 int32_t *__restrict__ status)
{
    const int s = blockIdx.x, L = a.L, k = a.k;
    const double q = a.qs.q[s / a.nseg];
    double sgn, hmax;
    dp_consts(q, L, sgn, hmax);
    const double *P = a.P + (int64_t)(s % a.nseg) * L, *Q = a.Q + (int64_t)s * L;
    auto Vrow = [&](int m) { return a.V + ((int64_t)m * a.nprob + s) * L; };
    // M = max over t of g(0..t) + V_{k-1}(t)
    const double *Vk = Vrow(k - 1);
    auto first = [&](int t) {
        const double v = Vk[t];
        return v > -INFINITY ? dp_g(P, Q, 0, t, q, sgn, hmax) + v : -INFINITY;
    };
    double M = -INFINITY;
    for (int t = threadIdx.x; t <= L - 2; t += 64)
        M = fmax(M, first(t));
    M = wave_max_d(M);
    int32_t *out = thr + (int64_t)s * k;
    if (!(M > -INFINITY)) {
        if (threadIdx.x == 0) {
            for (int j = 0; j < k; ++j)
                out[j] = -1;
            obj[s] = NAN;
            status[s] = P[L - 1] > 0.0 ? TS_PROBLEM_DEGENERATE : TS_PROBLEM_EMPTY;
        }
        return;
    }
    // the recomputed values equal the stored maxima bit for bit, so an index
    // is always found; should one not be, the problem is reported degenerate
    // rather than indexing past the row
    auto lost = [&]() {
        if (threadIdx.x == 0) {
            for (int j = 0; j < k; ++j)
                out[j] = -1;
            obj[s] = NAN;
            status[s] = TS_PROBLEM_DEGENERATE;
        }
    };
    int tj = first_equal(0, L - 2, M, first);
    if (tj > L - 2)
        return lost();
    if (threadIdx.x == 0)
        out[0] = tj;
    double target = Vk[tj];
    for (int j = 1; j < k; ++j) {
        const int m = k - 1 - j; // completions after threshold j+1
        const double *Vm = Vrow(m);
        const int prev = tj;
        auto val = [&](int u) {
            const double v = Vm[u];
            return v > -INFINITY ? dp_g(P, Q, prev + 1, u, q, sgn, hmax) + v : -INFINITY;
        };
        tj = first_equal(prev + 1, L - 2, target, val);
        if (tj > L - 2)
            return lost();
        if (threadIdx.x == 0)
            out[j] = tj;
        target = Vm[tj];
    }
    if (threadIdx.x == 0) {
        obj[s] = sgn == 0.0 ? M : expm1(sgn * M) / (1.0 - q);
        status[s] = TS_PROBLEM_OK;
    }
}

size_t dp_workspace_bytes(int nprob, int L, int k) { return (size_t)k * nprob * L * sizeof(double); }

ts_status launch_dp(const double *P, const double *Q, int nseg, int L, int k, int nq, const double *q, void *ws,
                    int32_t *thr, double *obj, int32_t *status, hipStream_t st)
{
    DPArgs a;
    a.P = P;
    a.Q = Q;
    a.nseg = nseg;
    a.nprob = nseg * nq;
    a.L = L;
    a.k = k;
    for (int j = 0; j < TS_MAX_Q; ++j)
        a.qs.q[j] = q[j < nq ? j : 0];
    a.V = (double *)ws;
    const int64_t n0 = (int64_t)a.nprob * L;
    hipLaunchKernelGGL(k_dp_last, dim3((unsigned)((n0 + DP_THREADS - 1) / DP_THREADS)), dim3(DP_THREADS), 0, st, a);
    for (int m = 1; m < k; ++m)
        hipLaunchKernelGGL(k_dp_level, dim3((unsigned)((int64_t)a.nprob * (L - 1))), dim3(DP_THREADS), 0, st, a, m);
    hipLaunchKernelGGL(k_dp_final, dim3((unsigned)a.nprob), dim3(64), 0, st, a, thr, obj, status);
    return check_launch("ts_threshold_search_dp");
}

} // namespace ts
