// k_prefix.hip -- probabilities and prefix sums of one histogram per
// workgroup (Tsallis-entropy section: p_i = c_i / N, class masses
// P(t) = sum_{i<=t} p_i, and Q(t) = sum_{i<=t} p_i^q, whose differences give
// the class sums of p_i^q inside H1 and H2).
//
//  * C(t) is the exact integer count prefix and P(t) = C(t) / N is one IEEE
//    division, so P is exact to half an ulp and P(L-1) = 1;
//  * p_i^q is computed by all threads into LDS; wave 0 then splits the bins
//    into 64 contiguous chunks, one per lane: each lane sums its chunk left
//    to right, the chunk bases are chained left to right in registers
//    (readlane), and Q(t) = base_chunk + local(t).  An empty bin adds +0.0
//    and a chunk base is the same addition as the last Q of the previous
//    chunk, so Q(t) == Q(t-1) bit for bit whenever bin t is empty: tuples
//    that differ only inside a run of empty bins see identical class sums
//    and tie exactly, as in exact arithmetic;
//  * results are staged in LDS and written with coalesced stores;
//  * one workgroup per (q index, histogram): all q of a call in one launch.
//    P does not depend on q and is written by the workgroups of q_0.
#include "common.h"

namespace ts {

constexpr int PREFIX_THREADS = 1024; // upper bound: 256 threads below 1024 bins, 1024 from there

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

struct QList {
    double q[TS_MAX_Q];
};

__global__ void __launch_bounds__(PREFIX_THREADS) k_prefix(const uint32_t *__restrict__ hist, int nseg, int L,
                                                           QList ql, double *__restrict__ P, double *__restrict__ Q)
{
    extern __shared__ double smem[];
    double *pq = smem;                        // [L]: p^q, then Q
    double *sp = smem + L;                    // [L]: P
    uint32_t *cnt = (uint32_t *)(smem + 2 * L); // [L]: counts
    __shared__ uint64_t wsum[PREFIX_THREADS / 64];

    const int s = blockIdx.x % nseg, j = blockIdx.x / nseg;
    const double q = ql.q[j];
    const bool wp = j == 0; // P is written once
    const uint32_t *h = hist + (int64_t)s * L;
    double *Ps = P + (int64_t)s * L;
    double *Qs = Q + (int64_t)blockIdx.x * L;
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;

    uint64_t c = 0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const uint32_t ci = h[i];
        cnt[i] = ci;
        c += ci;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if (lane == 0)
        wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    uint64_t N = 0;
    for (int w = 0; w < nw; ++w)
        N += wsum[w];
    if (N == 0) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) {
            if (wp)
                Ps[i] = 0.0;
            Qs[i] = 0.0;
        }
        return;
    }
    const double Nd = (double)N;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const uint32_t ci = cnt[i];
        pq[i] = ci ? pow((double)ci / Nd, q) : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int m = (L + 63) / 64;
        const int b0 = min(L, lane * m), b1 = min(L, b0 + m);
        uint64_t cs = 0;
        double qs = 0.0;
        for (int i = b0; i < b1; ++i) {
            cs += cnt[i];
            qs += pq[i];
        }
        // exclusive scan of the integer chunk counts (exact in any order)
        uint64_t incl = cs;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t v = __shfl_up(incl, o, 64);
            if (lane >= o)
                incl += v;
        }
        uint64_t C = incl - cs;
        // chunk bases of Q chained left to right
        double run = 0.0, qbase = 0.0;
        for (int j = 0; j < 64; ++j) {
            const double tj = readlane_f64(qs, j);
            if (lane == j)
                qbase = run;
            run = run + tj;
        }
        double loc = 0.0;
        for (int i = b0; i < b1; ++i) {
            C += cnt[i];
            loc += pq[i];
            sp[i] = (double)C / Nd;
            pq[i] = qbase + loc;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        if (wp)
            Ps[i] = sp[i];
        Qs[i] = pq[i];
    }
}

ts_status launch_prefix(const uint32_t *hist, int nseg, int L, int nq, const double *q, double *P, double *Q,
                        hipStream_t st)
{
    QList ql;
    for (int j = 0; j < TS_MAX_Q; ++j)
        ql.q[j] = q[j < nq ? j : 0];
    const size_t lds = (size_t)L * (2 * sizeof(double) + sizeof(uint32_t));
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_prefix, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    // the p^q evaluations (FP64 pow) dominate for large L: more threads there
    const int threads = L >= 1024 ? 1024 : 256;
    hipLaunchKernelGGL(k_prefix, dim3((unsigned)(nseg * nq)), dim3(threads), lds, st, hist, nseg, L, ql, P, Q);
    return check_launch("ts_prefix");
}

} // namespace ts
