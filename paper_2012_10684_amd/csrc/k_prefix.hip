// k_prefix.hip -- probabilities and prefix sums of one histogram per
// workgroup (Tsallis-entropy section: p_i = c_i / N, class masses
// P(t) = sum_{i<=t} p_i, and Q(t) = sum_{i<=t} p_i^q, whose differences give
// the class sums of p_i^q inside H1 and H2; for q = 1, the Shannon limit,
// Q(t) = sum_{i<=t} p_i ln p_i).
//
//  * C(t) is the exact integer count prefix and P(t) = C(t) / N is one IEEE
//    division, so P is exact to half an ulp and P(L-1) = 1;
//  * Q is a block-wide scan in a fixed order: each thread sums E consecutive
//    bins left to right, the thread totals go through a wavefront
//    Hillis-Steele scan and a sequential scan of the wavefront totals, and
//    Q(t) = exclusive base + local prefix;
//  * an empty bin then takes Q of the last occupied bin at or before it (0
//    if none): Q(t) == Q(t-1) bit for bit whenever bin t is empty, as in
//    exact arithmetic, so tuples that differ only inside a run of empty bins
//    see identical class sums and tie exactly.  The last-occupied index is
//    an exact integer max-scan;
//  * one workgroup per (q index, histogram): all q of a call in one launch.
//    P does not depend on q and is written by the workgroups of q_0.
#include "common.h"

namespace ts {

constexpr int PREFIX_THREADS = 1024; // upper bound: 256 threads below 1024 bins, 1024 from there
constexpr int PREFIX_MAX_E = 4;      // bins per thread (L <= 4 * threads)

struct QList {
    double q[TS_MAX_Q];
};

// Exclusive block-wide scans in a fixed order (every thread returns its
// exclusive prefix; *total receives the block total).  ws holds one entry per
// wavefront.
template <typename T, typename Op>
__device__ __forceinline__ T block_excl_scan(T x, T ident, Op op, T *ws, T *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T v = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl = op(v, incl);
    }
    if (lane == 63)
        ws[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) { // sequential over the wavefront totals
        T run = ident;
        for (int i = 0; i < nw; ++i) {
            const T t = ws[i];
            ws[i] = run;
            run = op(run, t);
        }
        ws[nw] = run;
    }
    __syncthreads();
    const T excl_w = ws[w];
    T excl = __shfl_up(incl, 1, 64);
    excl = lane == 0 ? excl_w : op(excl_w, excl);
    *total = ws[nw];
    __syncthreads(); // ws is reused by the next scan
    return excl;
}

__global__ void __launch_bounds__(PREFIX_THREADS) k_prefix(const uint32_t *__restrict__ hist, int nseg, int L,
                                                           QList ql, double *__restrict__ P, double *__restrict__ Q)
{
    extern __shared__ double smem[]; // [L]: Q before the empty-bin fix-up
    __shared__ uint64_t wu[PREFIX_THREADS / 64 + 1];
    __shared__ double wd[PREFIX_THREADS / 64 + 1];
    __shared__ int wi[PREFIX_THREADS / 64 + 1];
    double *qs = smem;
    int *lastocc = reinterpret_cast<int *>(smem + L); // [L]: last occupied bin <= t, or -1

    const int s = blockIdx.x % nseg, j = blockIdx.x / nseg;
    const double q = ql.q[j];
    const bool wp = j == 0; // P is written once
    const uint32_t *h = hist + (int64_t)s * L;
    double *Ps = P + (int64_t)s * L;
    double *Qs = Q + (int64_t)blockIdx.x * L;

    // this thread's bins [b0, b0 + E)
    const int E = (L + blockDim.x - 1) / blockDim.x;
    const int b0 = threadIdx.x * E;
    uint32_t c[PREFIX_MAX_E];
    uint64_t csum = 0;
    int occ = -1;
#pragma unroll
    for (int e = 0; e < PREFIX_MAX_E; ++e) {
        c[e] = (e < E && b0 + e < L) ? h[b0 + e] : 0u;
        csum += c[e];
        if (c[e])
            occ = b0 + e;
    }
    uint64_t N;
    const uint64_t cbase = block_excl_scan<uint64_t>(
        csum, 0, [](uint64_t a, uint64_t b) { return a + b; }, wu, &N);
    if (N == 0) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) {
            if (wp)
                Ps[i] = 0.0;
            Qs[i] = 0.0;
        }
        return;
    }
    const double Nd = (double)N;
    double pq[PREFIX_MAX_E];
    double qloc = 0.0;
#pragma unroll
    for (int e = 0; e < PREFIX_MAX_E; ++e) {
        const double pe = (double)c[e] / Nd;
        pq[e] = c[e] ? (q == 1.0 ? pe * log(pe) : pow(pe, q)) : 0.0; // q = 1: the Shannon limit
        qloc += pq[e]; // left to right
    }
    double qtot;
    const double qbase = block_excl_scan<double>(
        qloc, 0.0, [](double a, double b) { return a + b; }, wd, &qtot);
    int itot;
    const int obase = block_excl_scan<int>(
        occ, -1, [](int a, int b) { return a > b ? a : b; }, wi, &itot);
    uint64_t C = cbase;
    double loc = 0.0;
    int last = obase;
#pragma unroll
    for (int e = 0; e < PREFIX_MAX_E; ++e) {
        if (e < E && b0 + e < L) {
            const int t = b0 + e;
            C += c[e];
            loc += pq[e];
            if (c[e])
                last = t;
            if (wp)
                Ps[t] = (double)C / Nd;
            qs[t] = qbase + loc;
            lastocc[t] = last;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < L; t += blockDim.x) { // coalesced stores
        const int lt = lastocc[t];
        Qs[t] = lt < 0 ? 0.0 : qs[lt];
    }
}

ts_status launch_prefix(const uint32_t *hist, int nseg, int L, int nq, const double *q, double *P, double *Q,
                        hipStream_t st)
{
    QList ql;
    for (int j = 0; j < TS_MAX_Q; ++j)
        ql.q[j] = q[j < nq ? j : 0];
    // L <= 4096 = PREFIX_MAX_E * 1024: 256 threads below 1024 bins (E <= 4)
    const int threads = L >= 1024 ? 1024 : 256;
    const size_t lds = (size_t)L * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(k_prefix, dim3((unsigned)(nseg * nq)), dim3(threads), lds, st, hist, nseg, L, ql, P, Q);
    return check_launch("ts_prefix");
}

} // namespace ts
