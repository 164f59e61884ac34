// k_prefix.hip -- probabilities and prefix sums of one histogram per
// workgroup (Tsallis-entropy section: p_i = c_i / N, class masses
// P(t) = sum_{i<=t} p_i, and Q(t) = sum_{i<=t} p_i^q, whose differences give
// the class sums of p_i^q inside H1 and H2).
//
//  * C(t) is the exact integer count prefix and P(t) = C(t) / N is one IEEE
//    division, so P is exact to half an ulp and P(L-1) = 1;
//  * Q is summed in 256 contiguous chunks: each thread sums its chunk left to
//    right, one thread chains the chunk totals left to right, and
//    Q(t) = base_chunk + local(t).  An empty bin adds +0.0, and a chunk base
//    is computed by the same addition as the last Q of the previous chunk, so
//    Q(t) == Q(t-1) bit for bit whenever bin t is empty.  Tuples that differ
//    only inside a run of empty bins therefore see identical class sums and
//    tie exactly, as they do in exact arithmetic.
#include "common.h"

namespace ts {

constexpr int PREFIX_THREADS = 256;

__global__ void __launch_bounds__(PREFIX_THREADS) k_prefix(const uint32_t *__restrict__ hist, int L, double q,
                                                           double *__restrict__ P, double *__restrict__ Q)
{
    __shared__ double pq[MAX_BINS];
    __shared__ uint64_t csum[PREFIX_THREADS];
    __shared__ double qsum[PREFIX_THREADS];
    __shared__ uint64_t cbase[PREFIX_THREADS];
    __shared__ double qbase[PREFIX_THREADS];
    __shared__ uint64_t total;

    const int s = blockIdx.x;
    const uint32_t *h = hist + (int64_t)s * L;
    double *Ps = P + (int64_t)s * L;
    double *Qs = Q + (int64_t)s * L;
    const int m = (L + PREFIX_THREADS - 1) / PREFIX_THREADS;
    const int b0 = min(L, (int)threadIdx.x * m);
    const int b1 = min(L, b0 + m);

    uint64_t c = 0;
    for (int i = b0; i < b1; ++i)
        c += h[i];
    csum[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int t = 0; t < PREFIX_THREADS; ++t) {
            cbase[t] = run;
            run += csum[t];
        }
        total = run;
    }
    __syncthreads();
    const uint64_t N = total;
    if (N == 0) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) {
            Ps[i] = 0.0;
            Qs[i] = 0.0;
        }
        return;
    }
    const double Nd = (double)N;
    double loc = 0.0;
    for (int i = b0; i < b1; ++i) {
        const uint32_t ci = h[i];
        const double v = ci ? pow((double)ci / Nd, q) : 0.0;
        pq[i] = v;
        loc += v;
    }
    qsum[threadIdx.x] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < PREFIX_THREADS; ++t) {
            qbase[t] = run;
            run = run + qsum[t];
        }
    }
    __syncthreads();
    const double qb = qbase[threadIdx.x];
    uint64_t C = cbase[threadIdx.x];
    loc = 0.0;
    for (int i = b0; i < b1; ++i) {
        C += h[i];
        loc += pq[i];
        Ps[i] = (double)C / Nd;
        Qs[i] = qb + loc;
    }
}

ts_status launch_prefix(const uint32_t *hist, int nseg, int L, double q, double *P, double *Q, hipStream_t st)
{
    hipLaunchKernelGGL(k_prefix, dim3(nseg), dim3(PREFIX_THREADS), 0, st, hist, L, q, P, Q);
    return check_launch("ts_prefix");
}

} // namespace ts
