// label_dev.h -- device code of the thresholding kernel function (Algorithm
// 1) generalised to k thresholds, shared by the label pass and the fused
// segmentation kernel: label(v) = #{j : b(v) > t_j} from integer cut values,
// with no bin index materialised.  For the window rule of ts_binning,
// b(v) > t  <=>  v >= cut(t) = lo + ceil((t + 1) * W / L)   (W = hi - lo + 1),
// which also covers values outside the window (below lo: bin 0, never above a
// threshold; above hi: bin L-1, above every threshold since cut(t) <= hi + 1).
#pragma once

#include "common.h"

namespace ts {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// Cut values of one threshold set: label = #{j : v >= c[j]}.  KM = k for k
// <= 3; KM = LABEL_MAX_K holds up to that many, unused cuts are never
// reached.
constexpr int LABEL_MAX_K = TS_DP_MAX_K;

template <int KM>
struct Cuts {
    int c[KM];
};

// Cut values of problem s; a row that is not a strictly ascending tuple in
// [0, L-2] (e.g. the -1 row of a degenerate problem) gives no cuts (all 0).
template <int KM>
__device__ __forceinline__ Cuts<KM> make_cuts(const int32_t *thr, int k, const BinMap &bm)
{
    const int NEVER = 0x7fffffff;
    Cuts<KM> c;
#pragma unroll
    for (int j = 0; j < KM; ++j)
        c.c[j] = NEVER;
    int t[KM];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < KM; ++j) { // static indices: the arrays stay in registers
        t[j] = j < k ? thr[j] : 0;
        if (j < k)
            ok = ok && t[j] >= 0 && t[j] <= bm.L - 2 && (j == 0 || t[j] > t[j > 0 ? j - 1 : 0]);
    }
    if (!ok)
        return c;
    // (t+1) W + L - 1 <= 4095 * 65536 + 4095 < 2^32: exact in uint32
    const uint32_t W = (uint32_t)((int64_t)bm.hi - bm.lo + 1);
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (j < k)
            c.c[j] = bm.lo + (int)(((uint32_t)(t[j] + 1) * W + (uint32_t)bm.L - 1) / (uint32_t)bm.L);
    return c;
}

template <int KM>
__device__ __forceinline__ uint32_t lab1(int v, const Cuts<KM> &c)
{
    uint32_t n = 0; // unused cuts are never reached (0x7fffffff > any int16)
#pragma unroll
    for (int j = 0; j < KM; ++j)
        n += (uint32_t)(v >= c.c[j]);
    return n;
}

typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

// Cut values as int16 for the packed path: label = nk - #{j : v < c[j]},
// where v < c  <=>  the saturated int16 difference v - c is negative (the
// true difference lies in [-65535, 65535] and saturation keeps its sign).
// The cut is clamped to [-32768, 32768] and its low 16 bits kept: a cut
// above 32767 is never reached and becomes 0x8000 = -32768 (v < c never
// holds), left out of nk; a cut at or below -32768 is always reached, -32768
// again, counted in nk.  (No select picks the disabled value: the compiler
// in use dropped such a select when its result fed the packed subtract.)
// base = nk in every byte.
template <int KM>
struct PCuts {
    int c[KM]; // int16 values (int elements stay in registers at every KM)
    uint32_t base;
};

template <int KM>
__device__ __forceinline__ PCuts<KM> pack_cuts(const Cuts<KM> &c)
{
    PCuts<KM> p;
    uint32_t nk = 0;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        p.c[j] = min(max(c.c[j], -32768), 32768);
        nk += c.c[j] <= 32767 ? 1u : 0u;
    }
    p.base = nk * 0x01010101u;
    return p;
}

// Label of one voxel from the packed cuts (the same rule as lab8).
template <int KM>
__device__ __forceinline__ uint32_t lab1p(int v, const PCuts<KM> &p)
{
    const s2 vv = {(short)v, (short)v};
    u2 acc = {0, 0};
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const s2 c = {(short)p.c[j], (short)p.c[j]};
        acc += __builtin_bit_cast(u2, __builtin_elementwise_sub_sat(vv, c)) >> (u2){15, 15};
    }
    return (p.base & 0xffu) - (uint32_t)acc.x;
}

// Labels of 8 int16 voxels (16 bytes) as 8 bytes: two voxels per packed
// 16-bit operation (saturating subtract, sign bit, add), then the 16-bit
// counts are gathered into bytes and subtracted from nk (no borrow: every
// count is <= nk).
template <int KM>
__device__ __forceinline__ v2u lab8(const v4i &w, const PCuts<KM> &p)
{
    uint32_t n[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const s2 v = __builtin_bit_cast(s2, (uint32_t)w[d]);
        u2 acc = {0, 0};
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            const s2 c = {(short)p.c[j], (short)p.c[j]};
            acc += __builtin_bit_cast(u2, __builtin_elementwise_sub_sat(v, c)) >> (u2){15, 15};
        }
        n[d] = __builtin_bit_cast(uint32_t, acc);
    }
    // bytes 0 and 2 of n[0] (voxels 0, 1), then of n[1] (voxels 2, 3)
    v2u r;
    r.x = p.base - __builtin_amdgcn_perm(n[1], n[0], 0x06040200u);
    r.y = p.base - __builtin_amdgcn_perm(n[3], n[2], 0x06040200u);
    return r;
}

} // namespace ts
