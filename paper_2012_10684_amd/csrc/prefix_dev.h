// prefix_dev.h -- the probability set and prefix sums of one histogram,
// computed by one workgroup (Tsallis-entropy section: p_i = c_i / N, class
// masses P(t) = sum_{i<=t} p_i and Q(t) = sum_{i<=t} p_i^q; for q = 1, the
// Shannon limit, Q(t) = sum_{i<=t} p_i ln p_i).  Shared by the prefix pass and
// the fused segmentation kernel, which must produce the same bits.
//
//  * C(t) is the exact integer count prefix and P(t) = C(t) / N is one IEEE
//    division, so P is exact to half an ulp and P(L-1) = 1;
//  * Q is a block-wide scan in a fixed order: each thread sums E consecutive
//    bins left to right, the thread totals go through a wavefront
//    Hillis-Steele scan and a sequential scan of the wavefront totals, and
//    Q(t) = exclusive base + local prefix.  The order depends only on E (a
//    workgroup with more threads than bins / E adds wavefronts of zeros,
//    which change no bit), so E is fixed by L alone;
//  * an empty bin then takes Q of the last occupied bin at or before it (0
//    if none): Q(t) == Q(t-1) bit for bit whenever bin t is empty, as in
//    exact arithmetic, so tuples that differ only inside a run of empty bins
//    see identical class sums and tie exactly.  The last-occupied index is
//    an exact integer max-scan.
#pragma once

#include "common.h"

namespace ts {

constexpr int PREFIX_THREADS = 1024; // largest workgroup the scan supports
constexpr int PREFIX_MAX_E = 4;      // bins per thread (L <= 4 * 1024)

// Threads of the prefix pass for L bins (256 below 1024 bins, else 1024) and
// the bins per thread E that fix the scan's order.
__host__ __device__ inline int prefix_threads(int L) { return L >= 1024 ? 1024 : 256; }
__host__ __device__ inline int prefix_bins_per_thread(int L)
{
    const int T = prefix_threads(L);
    return (L + T - 1) / T;
}

// LDS of one wavefront total per wavefront (plus the block total).
struct PrefixLds {
    uint64_t wu[PREFIX_THREADS / 64 + 1];
    double wd[PREFIX_THREADS / 64 + 1];
    int wi[PREFIX_THREADS / 64 + 1];
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

// Prefix sums of one histogram by the calling workgroup, blockDim.x * E >= L
// (every thread of the workgroup calls it).  cnt(b) is the count of bin b.
// Writes P[t] = C(t) / N (unless P is null) and Q[t] for t < L; with N = 0
// both are 0.  qs [L] doubles and lastocc [L] ints are LDS scratch.  Ends
// with a barrier; returns N.
template <typename Cnt>
__device__ __forceinline__ uint64_t prefix_row(Cnt cnt, int L, int E, double q, double *__restrict__ P,
                                               double *__restrict__ Q, double *qs, int *lastocc, PrefixLds &sh)
{
    // this thread's bins [b0, b0 + E)
    const int b0 = threadIdx.x * E;
    uint32_t c[PREFIX_MAX_E];
    uint64_t csum = 0;
    int occ = -1;
#pragma unroll
    for (int e = 0; e < PREFIX_MAX_E; ++e) {
        c[e] = (e < E && b0 + e < L) ? cnt(b0 + e) : 0u;
        csum += c[e];
        if (c[e])
            occ = b0 + e;
    }
    uint64_t N;
    const uint64_t cbase = block_excl_scan<uint64_t>(
        csum, 0, [](uint64_t a, uint64_t b) { return a + b; }, sh.wu, &N);
    if (N == 0) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) {
            if (P)
                P[i] = 0.0;
            Q[i] = 0.0;
        }
        __syncthreads();
        return 0;
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
        qloc, 0.0, [](double a, double b) { return a + b; }, sh.wd, &qtot);
    int itot;
    const int obase = block_excl_scan<int>(
        occ, -1, [](int a, int b) { return a > b ? a : b; }, sh.wi, &itot);
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
            if (P)
                P[t] = (double)C / Nd;
            qs[t] = qbase + loc;
            lastocc[t] = last;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < L; t += blockDim.x) { // coalesced stores
        const int lt = lastocc[t];
        Q[t] = lt < 0 ? 0.0 : qs[lt];
    }
    __syncthreads();
    return N;
}

} // namespace ts
