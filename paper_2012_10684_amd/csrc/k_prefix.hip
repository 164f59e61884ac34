// k_prefix.hip -- probabilities and prefix sums of one histogram per
// workgroup (Tsallis-entropy section: p_i = c_i / N, class masses
// P(t) = sum_{i<=t} p_i, and Q(t) = sum_{i<=t} p_i^q, whose differences give
// the class sums of p_i^q inside H1 and H2; for q = 1, the Shannon limit,
// Q(t) = sum_{i<=t} p_i ln p_i).  The scan itself (exact integer counts, a
// fixed summation order for Q, empty bins repeating Q bit for bit) is
// prefix_row in prefix_dev.h.  One workgroup per (q index, histogram): all q
// of a call in one launch; P does not depend on q and is written by the
// workgroups of q_0.
#include "common.h"
#include "prefix_dev.h"

namespace ts {

struct QList {
    double q[TS_MAX_Q];
};

__global__ void __launch_bounds__(PREFIX_THREADS) k_prefix(const uint32_t *__restrict__ hist, int nseg, int L,
                                                           QList ql, double *__restrict__ P, double *__restrict__ Q)
{
    extern __shared__ double smem[]; // [L]: Q before the empty-bin fix-up
    __shared__ PrefixLds sh;
    const int s = blockIdx.x % nseg, j = blockIdx.x / nseg;
    const uint32_t *h = hist + (int64_t)s * L;
    prefix_row([h](int b) { return h[b]; }, L, prefix_bins_per_thread(L), ql.q[j],
               j == 0 ? P + (int64_t)s * L : nullptr, // P is written once
               Q + (int64_t)blockIdx.x * L, smem, reinterpret_cast<int *>(smem + L), sh);
}

ts_status launch_prefix(const uint32_t *hist, int nseg, int L, int nq, const double *q, double *P, double *Q,
                        hipStream_t st)
{
    QList ql;
    for (int j = 0; j < TS_MAX_Q; ++j)
        ql.q[j] = q[j < nq ? j : 0];
    const int threads = prefix_threads(L);
    const size_t lds = (size_t)L * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(k_prefix, dim3((unsigned)(nseg * nq)), dim3(threads), lds, st, hist, nseg, L, ql, P, Q);
    return check_launch("ts_prefix");
}

} // namespace ts
