// api.hip -- the C ABI of libts: argument checks, tuning defaults, bin-map
// constants and dispatch to the kernels.  See include/ts.h for the contract.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_map>

#include "common.h"

namespace ts {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ts_status fail(ts_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

ts_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(TS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return TS_OK;
}

void allow_dynamic_lds(const void *fn, size_t bytes)
{
    if (bytes <= 64 * 1024)
        return;
    static std::mutex mu;
    static std::unordered_map<uint64_t, size_t> set; // (device, kernel) -> bytes allowed
    int dev = 0;
    (void)hipGetDevice(&dev);
    const uint64_t key = ((uint64_t)(uint32_t)dev << 48) ^ (uint64_t)(uintptr_t)fn;
    std::lock_guard<std::mutex> lk(mu);
    auto it = set.find(key);
    if (it != set.end() && it->second >= bytes)
        return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        set[key] = bytes;
}

int device_cu_count()
{
    static std::mutex mu;
    static std::unordered_map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 256;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end())
        return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    cache[dev] = n;
    return n;
}

static bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

ts_status resolve_tuning(const ts_tuning *t, int nbins, Tune *o)
{
    ts_tuning z;
    memset(&z, 0, sizeof(z));
    if (!t)
        t = &z;
    // histogram: LDS = nbins * replicas * 4 bytes per workgroup; by default
    // 16 KiB of replicas (4096 / nbins copies) in one 1024-thread workgroup
    // per CU, the shapes measured fastest on MI355X for 256..1024 bins
    int rep_default = 32;
    while (rep_default > 1 && nbins * rep_default > 4096)
        rep_default >>= 1;
    o->hist_block = t->hist_block ? t->hist_block : 1024;
    o->hist_replicas = t->hist_replicas ? t->hist_replicas : rep_default;
    o->hist_wg_per_cu = t->hist_wg_per_cu ? t->hist_wg_per_cu : 1;
    o->label_block = t->label_block ? t->label_block : 256;
    o->label_vecs = t->label_vecs ? t->label_vecs : 2;
    o->search_cols = t->search_cols ? t->search_cols : 2;
    o->search_rows = t->search_rows ? t->search_rows : 16;
    o->min_chunk = t->min_chunk ? t->min_chunk : 8192;
    o->search_path = t->search_path;
    o->search_block = t->search_block ? t->search_block : 512;
    o->segment_parts = t->segment_parts;
    o->segment_block = t->segment_block;
    if (o->hist_block < 64 || o->hist_block > 1024 || o->hist_block % 64)
        return fail(TS_ERR_INVALID_ARG, "tuning: hist_block must be a multiple of 64 in [64, 1024]");
    if (!pow2(o->hist_replicas) || o->hist_replicas > 32)
        return fail(TS_ERR_INVALID_ARG, "tuning: hist_replicas must be 1, 2, 4, 8, 16 or 32");
    if ((size_t)nbins * o->hist_replicas * 4 > 160 * 1024)
        return fail(TS_ERR_INVALID_ARG, "tuning: nbins * hist_replicas * 4 exceeds the 160 KiB of LDS");
    if (o->hist_wg_per_cu < 1 || o->hist_wg_per_cu > 16)
        return fail(TS_ERR_INVALID_ARG, "tuning: hist_wg_per_cu must be in [1, 16]");
    if (o->label_block < 64 || o->label_block > 1024 || o->label_block % 64)
        return fail(TS_ERR_INVALID_ARG, "tuning: label_block must be a multiple of 64 in [64, 1024]");
    if (o->label_vecs != 1 && o->label_vecs != 2 && o->label_vecs != 4)
        return fail(TS_ERR_INVALID_ARG, "tuning: label_vecs must be 1, 2 or 4");
    if (o->search_cols != 1 && o->search_cols != 2 && o->search_cols != 4)
        return fail(TS_ERR_INVALID_ARG, "tuning: search_cols must be 1, 2 or 4");
    if (o->search_rows < 16 || o->search_rows > 4096 || o->search_rows % 4)
        return fail(TS_ERR_INVALID_ARG, "tuning: search_rows must be a multiple of 4 in [16, 4096]");
    if (o->min_chunk < 512)
        return fail(TS_ERR_INVALID_ARG, "tuning: min_chunk must be >= 512");
    if (o->search_path < 0 || o->search_path > 2)
        return fail(TS_ERR_INVALID_ARG, "tuning: search_path must be 0, 1 or 2");
    if (o->search_block != 256 && o->search_block != 512 && o->search_block != 1024)
        return fail(TS_ERR_INVALID_ARG, "tuning: search_block must be 256, 512 or 1024");
    if (o->segment_parts < 0 || o->segment_parts > 64)
        return fail(TS_ERR_INVALID_ARG, "tuning: segment_parts must be in [1, 64]");
    if (o->segment_block != 0 && o->segment_block != 256 && o->segment_block != 512 && o->segment_block != 1024)
        return fail(TS_ERR_INVALID_ARG, "tuning: segment_block must be 256, 512 or 1024");
    return TS_OK;
}

// ---------------------------------------------------------------- bin map
// The in-window offset d = v - lo (0 <= d < W) maps to floor(d * L / W).
// Two integer forms are tried and kept only if they reproduce that floor for
// every d in [0, W):
//   narrow multiply: (d * mul) >> shift with mul < 2^24 and d * mul < 2^32;
//   wide multiply:   hi32((d * L) * mul) >> shift.
// Results are cached per (lo, hi, L).
static bool check_map(uint32_t W, uint32_t L, uint64_t mul, uint32_t shift, bool wide)
{
    for (uint32_t d = 0; d < W; ++d) {
        uint64_t want = (uint64_t)d * L / W;
        uint64_t got;
        if (wide)
            got = (((uint64_t)(d * L) * mul) >> 32) >> shift;
        else
            got = ((uint64_t)d * mul) >> shift;
        if (got != want)
            return false;
    }
    return true;
}

ts_status make_binmap(const ts_binning &bin, BinMap *bm)
{
    if (bin.nbins < 2 || bin.nbins > MAX_BINS)
        return fail(TS_ERR_INVALID_ARG, "binning: nbins must be in [2, 4096]");
    if (bin.lo < -32768 || bin.hi > 32767 || bin.lo > bin.hi)
        return fail(TS_ERR_INVALID_ARG, "binning: need -32768 <= lo <= hi <= 32767");
    static std::mutex mu;
    static std::unordered_map<uint64_t, BinMap> cache;
    uint64_t key = ((uint64_t)(uint16_t)bin.lo << 32) | ((uint64_t)(uint16_t)bin.hi << 16) | (uint64_t)bin.nbins;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *bm = it->second;
            return TS_OK;
        }
    }
    const uint32_t W = (uint32_t)(bin.hi - bin.lo + 1), L = (uint32_t)bin.nbins;
    BinMap m;
    m.lo = bin.lo;
    m.hi = bin.hi;
    m.L = bin.nbins;
    m.narrow = W < L ? 1 : 0;
    bool ok = false;
    for (uint32_t s = 0; s < 32 && !ok; ++s) {
        uint64_t num = ((uint64_t)L << s);
        uint64_t mul = (num + W - 1) / W; // ceil(2^s L / W)
        if (mul >= (1u << 24) || (uint64_t)(W - 1) * mul >= (1ull << 32))
            break;
        if (check_map(W, L, mul, s, false)) {
            m.mul = (uint32_t)mul;
            m.shift = s;
            m.wide = 0;
            ok = true;
        }
    }
    for (uint32_t s = 0; s < 32 && !ok; ++s) {
        if ((uint64_t)(W - 1) * L >= (1ull << 32))
            break;
        uint64_t mul = ((1ull << (32 + s)) / W) + 1; // floor(2^(32+s) / W) + 1
        if (mul >= (1ull << 32))
            break;
        if (check_map(W, L, mul, s, true)) {
            m.mul = (uint32_t)mul;
            m.shift = s;
            m.wide = 1;
            ok = true;
        }
    }
    if (!ok)
        return fail(TS_ERR_UNSUPPORTED, "binning: no exact integer bin map found");
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = m;
    *bm = m;
    return TS_OK;
}

static ts_status check_batch(const ts_batch &b)
{
    if (b.nseg < 0 || b.total < 0)
        return fail(TS_ERR_INVALID_ARG, "batch: nseg and total must be >= 0");
    if (b.nseg > 0 && (!b.vox || !b.offs))
        return fail(TS_ERR_INVALID_ARG, "batch: vox and offs must not be null when nseg > 0");
    if (b.nseg == 0 && b.total != 0)
        return fail(TS_ERR_INVALID_ARG, "batch: total must be 0 when nseg == 0");
    return TS_OK;
}

} // namespace ts

using namespace ts;

extern "C" {

int32_t ts_abi_version(void) { return TS_ABI_VERSION; }

const char *ts_last_error(void) { return g_last_error.c_str(); }

ts_status ts_histogram(ts_batch batch, ts_binning bin, uint32_t *hist, const ts_tuning *tune, ts_stream_t stream)
{
    ts_status st = check_batch(batch);
    if (st != TS_OK)
        return st;
    BinMap bm;
    if ((st = make_binmap(bin, &bm)) != TS_OK)
        return st;
    if (batch.nseg > 0 && !hist)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram: hist must not be null");
    Tune t;
    if ((st = resolve_tuning(tune, bin.nbins, &t)) != TS_OK)
        return st;
    if (batch.nseg == 0)
        return TS_OK;
    return launch_histogram(batch, bm, hist, t, (hipStream_t)stream);
}

// Checks nq and the q values of a prefix or search call (fn names the call).
static ts_status check_q(const char *fn, int32_t nq, const double *q, bool search)
{
    if (nq < 1 || nq > TS_MAX_Q)
        return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": nq must be 1.." + std::to_string(TS_MAX_Q));
    if (!q)
        return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": null q array");
    for (int j = 0; j < nq; ++j) {
        if (!(q[j] > 0.0) || !isfinite(q[j]))
            return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": q must be finite and > 0");
    }
    (void)search; // every q > 0 is supported, q = 1 being the Shannon limit
    return TS_OK;
}

ts_status ts_prefix(const uint32_t *hist, int32_t nseg, int32_t nbins, int32_t nq, const double *q, double *P,
                    double *Q, ts_stream_t stream)
{
    if (nseg < 0)
        return fail(TS_ERR_INVALID_ARG, "ts_prefix: nseg must be >= 0");
    if (nbins < 2 || nbins > MAX_BINS)
        return fail(TS_ERR_INVALID_ARG, "ts_prefix: nbins must be in [2, 4096]");
    ts_status st;
    if ((st = check_q("ts_prefix", nq, q, false)) != TS_OK)
        return st;
    if (nseg > 0 && (!hist || !P || !Q))
        return fail(TS_ERR_INVALID_ARG, "ts_prefix: null pointer");
    if (nseg == 0)
        return TS_OK;
    return launch_prefix(hist, nseg, nbins, nq, q, P, Q, (hipStream_t)stream);
}

size_t ts_search_workspace_bytes(int32_t nseg, int32_t nbins, int32_t k, int32_t nq, int32_t mode)
{
    if (nseg < 0 || nbins < 2 || nbins > MAX_BINS || k < 1 || k > 3 || nq < 1 || nq > TS_MAX_Q || mode < 0 ||
        mode > TS_SEARCH_PLAIN_FP32)
        return 0;
    return search_workspace_bytes(nseg * nq, nbins, k, mode, 4);
}

} // extern "C"

namespace ts {

ts_status check_search_args(const char *fn, const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                            int32_t nq, const double *q, int32_t mode, int32_t *thr, double *obj, int32_t *status)
{
    const std::string f(fn);
    if (nseg < 0)
        return fail(TS_ERR_INVALID_ARG, f + ": nseg must be >= 0");
    if (nbins < 2 || nbins > MAX_BINS)
        return fail(TS_ERR_INVALID_ARG, f + ": nbins must be in [2, 4096]");
    if (k < 1 || k > 3)
        return fail(TS_ERR_INVALID_ARG, f + ": k must be 1, 2 or 3");
    if (nbins < k + 1)
        return fail(TS_ERR_INVALID_ARG, f + ": nbins must be >= k + 1");
    if (mode < 0 || mode > TS_SEARCH_PLAIN_FP32)
        return fail(TS_ERR_INVALID_ARG, f + ": unknown mode");
    ts_status st;
    if ((st = check_q(fn, nq, q, true)) != TS_OK)
        return st;
    if ((int64_t)nseg * nq > 0x7fffffff / 2)
        return fail(TS_ERR_INVALID_ARG, f + ": too many problems");
    if (nseg > 0 && (!P || !Q || !thr || !obj || !status))
        return fail(TS_ERR_INVALID_ARG, f + ": null pointer");
    return TS_OK;
}

} // namespace ts

extern "C" {

ts_status ts_threshold_search(const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k, int32_t nq,
                              const double *q, int32_t mode, void *ws, size_t ws_bytes, int32_t *thr, double *obj,
                              int32_t *status, const ts_tuning *tune, ts_stream_t stream)
{
    ts_status st;
    if ((st = check_search_args("ts_threshold_search", P, Q, nseg, nbins, k, nq, q, mode, thr, obj, status)) != TS_OK)
        return st;
    Tune t;
    if ((st = resolve_tuning(tune, nbins, &t)) != TS_OK)
        return st;
    size_t need = search_workspace_bytes(nseg * nq, nbins, k, mode, 4);
    if (nseg > 0 && (ws_bytes < need || (!ws && need > 0)))
        return fail(TS_ERR_WORKSPACE, "ts_threshold_search: workspace too small (need " + std::to_string(need) +
                                          " bytes, got " + std::to_string(ws_bytes) + ")");
    if (nseg == 0)
        return TS_OK;
    return launch_search(P, Q, nseg, nbins, k, nq, q, mode, ws, ws_bytes, thr, obj, status, t, (hipStream_t)stream);
}

} // extern "C"

namespace ts {

// Scratch of ts_threshold_search_noalloc.  Every GPU holds its own copy of
// this array; in host code its name is only a host-side stand-in, so the
// device address is looked up once per device (with that device current)
// and only that address is handed to kernels.
__device__ __align__(256) unsigned char scratch[TS_NOALLOC_SCRATCH_BYTES];

static ts_status scratch_address(void **out)
{
    static std::mutex mu;
    static std::unordered_map<int, void *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(TS_ERR_HIP, std::string("ts_threshold_search_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return TS_OK;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(TS_ERR_HIP, std::string("ts_threshold_search_noalloc: hipGetSymbolAddress: ") +
                                    (e != hipSuccess ? hipGetErrorString(e) : "null address"));
    addr[dev] = p;
    *out = p;
    return TS_OK;
}

} // namespace ts

extern "C" {

ts_status ts_threshold_search_noalloc(const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                                      int32_t nq, const double *q, int32_t mode, int32_t *thr, double *obj,
                                      int32_t *status, const ts_tuning *tune, ts_stream_t stream)
{
    ts_status st;
    if ((st = check_search_args("ts_threshold_search_noalloc", P, Q, nseg, nbins, k, nq, q, mode, thr, obj,
                                status)) != TS_OK)
        return st;
    Tune t;
    if ((st = resolve_tuning(tune, nbins, &t)) != TS_OK)
        return st;
    if (nseg == 0)
        return TS_OK;
    const size_t need = search_need_bytes(nseg * nq, nbins, k, mode, t);
    if (need > TS_NOALLOC_SCRATCH_BYTES)
        return fail(TS_ERR_WORKSPACE, "ts_threshold_search_noalloc: these sizes need " + std::to_string(need) +
                                          " bytes of scratch, more than the fixed " +
                                          std::to_string(TS_NOALLOC_SCRATCH_BYTES));
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != TS_OK)
        return st;
    return launch_search(P, Q, nseg, nbins, k, nq, q, mode, ws, TS_NOALLOC_SCRATCH_BYTES, thr, obj, status, t,
                         (hipStream_t)stream);
}

static ts_status label_common(const char *fn, ts_batch batch, ts_binning bin, int32_t nsets,
                              const int32_t *const *thr, int32_t k, uint8_t *const *const *out, const ts_tuning *tune,
                              ts_stream_t stream)
{
    ts_status st = check_batch(batch);
    if (st != TS_OK)
        return st;
    BinMap bm;
    if ((st = make_binmap(bin, &bm)) != TS_OK)
        return st;
    if (k < 1 || k > TS_DP_MAX_K)
        return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": k must be in 1.." + std::to_string(TS_DP_MAX_K));
    if (nsets < 1 || nsets > TS_MAX_LABEL_SETS)
        return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": nsets must be 1.." + std::to_string(TS_MAX_LABEL_SETS));
    LabelSets sets = {};
    if (batch.nseg > 0) {
        if (!thr || !out)
            return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": null pointer");
        for (int u = 0; u < nsets; ++u) {
            if (!thr[u] || !out[u])
                return fail(TS_ERR_INVALID_ARG, std::string(fn) + ": null pointer");
            sets.thr[u] = thr[u];
            sets.out[u] = out[u];
        }
    }
    Tune t;
    if ((st = resolve_tuning(tune, bin.nbins, &t)) != TS_OK)
        return st;
    if (batch.nseg == 0)
        return TS_OK;
    return launch_label(batch, bm, sets, nsets, k, t, (hipStream_t)stream);
}

ts_status ts_label(ts_batch batch, ts_binning bin, const int32_t *thr, int32_t k, uint8_t *const *out,
                   const ts_tuning *tune, ts_stream_t stream)
{
    return label_common("ts_label", batch, bin, 1, &thr, k, &out, tune, stream);
}

ts_status ts_label_sets(ts_batch batch, ts_binning bin, int32_t nsets, const int32_t *const *thr, int32_t k,
                        uint8_t *const *const *out, const ts_tuning *tune, ts_stream_t stream)
{
    return label_common("ts_label_sets", batch, bin, nsets, thr, k, out, tune, stream);
}

size_t ts_segment_workspace_bytes(int32_t nseg, int32_t nbins, int32_t k, int32_t nq, int32_t mode, int32_t labels)
{
    if (nseg < 0 || nbins < 2 || nbins > MAX_BINS || nbins < k + 1 || k < 1 || k > 3 || nq < 1 || nq > TS_MAX_Q ||
        mode < 0 || mode > TS_SEARCH_PLAIN_FP32 || (labels && nq > TS_MAX_LABEL_SETS))
        return 0;
    return segment_workspace_bytes(nseg, nbins, k, nq, mode, labels != 0);
}

ts_status ts_segment(ts_batch batch, ts_binning bin, int32_t k, int32_t nq, const double *q, int32_t mode,
                     uint32_t *hist, int32_t *thr, double *obj, int32_t *status, uint8_t *const *const *out,
                     void *ws, size_t ws_bytes, const ts_tuning *tune, ts_stream_t stream)
{
    ts_status st = check_batch(batch);
    if (st != TS_OK)
        return st;
    BinMap bm;
    if ((st = make_binmap(bin, &bm)) != TS_OK)
        return st;
    const int32_t nseg = batch.nseg;
    // the search's checks (P and Q stand in for pointers the call makes itself)
    const double *nn = (const double *)1;
    if ((st = check_search_args("ts_segment", nn, nn, nseg, bin.nbins, k, nq, q, mode, thr, obj, status)) != TS_OK)
        return st;
    if (out && nq > TS_MAX_LABEL_SETS)
        return fail(TS_ERR_INVALID_ARG, "ts_segment: labels for at most " + std::to_string(TS_MAX_LABEL_SETS) +
                                            " values of q");
    LabelSets sets = {};
    if (out && nseg > 0) {
        for (int u = 0; u < nq; ++u) {
            if (!out[u])
                return fail(TS_ERR_INVALID_ARG, "ts_segment: null pointer");
            sets.thr[u] = thr + (int64_t)u * nseg * k;
            sets.out[u] = out[u];
        }
    }
    if (nseg > 0 && !hist)
        return fail(TS_ERR_INVALID_ARG, "ts_segment: null pointer");
    Tune t;
    if ((st = resolve_tuning(tune, bin.nbins, &t)) != TS_OK)
        return st;
    const size_t need = segment_workspace_bytes(nseg, bin.nbins, k, nq, mode, out != nullptr);
    if (nseg > 0 && (ws_bytes < need || !ws))
        return fail(TS_ERR_WORKSPACE, "ts_segment: workspace too small (need " + std::to_string(need) +
                                          " bytes, got " + std::to_string(ws_bytes) + ")");
    if (nseg == 0)
        return TS_OK;
    return launch_segment(batch, bm, k, nq, q, mode, hist, thr, obj, status, out ? &sets : nullptr, ws, t,
                          (hipStream_t)stream);
}

ts_status ts_histogram2d(ts_batch batch, int32_t height, int32_t width, ts_binning bin, uint32_t *hist,
                         ts_stream_t stream)
{
    ts_status st = check_batch(batch);
    if (st != TS_OK)
        return st;
    BinMap bm;
    if ((st = make_binmap(bin, &bm)) != TS_OK)
        return st;
    if (bin.nbins > 256)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: nbins must be <= 256");
    if (height < 1 || width < 1 || width > 4096)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: need height >= 1 and 1 <= width <= 4096");
    if (batch.total != (int64_t)batch.nseg * height * width)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: total must be nseg * height * width");
    if (batch.nseg > 0 && !hist)
        return fail(TS_ERR_INVALID_ARG, "ts_histogram2d: hist must not be null");
    if (batch.nseg == 0)
        return TS_OK;
    return launch_hist2d(batch, height, width, bm, hist, (hipStream_t)stream);
}

size_t ts_search2d_workspace_bytes(int32_t nseg, int32_t nbins, int32_t nq)
{
    if (nseg < 0 || nbins < 2 || nbins > 256 || nq < 1 || nq > TS_MAX_Q)
        return 0;
    return search2d_workspace_bytes(nseg, nq, nbins);
}

ts_status ts_threshold_search2d(const uint32_t *hist, int32_t nseg, int32_t nbins, int32_t nq, const double *q,
                                void *ws, size_t ws_bytes, int32_t *thr, double *obj, int32_t *status,
                                ts_stream_t stream)
{
    if (nseg < 0)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search2d: nseg must be >= 0");
    if (nbins < 2 || nbins > 256)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search2d: nbins must be in [2, 256]");
    ts_status st;
    if ((st = check_q("ts_threshold_search2d", nq, q, true)) != TS_OK)
        return st;
    if (nseg > 0 && (!hist || !thr || !obj || !status))
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search2d: null pointer");
    const size_t need = search2d_workspace_bytes(nseg, nq, nbins);
    if (nseg > 0 && (ws_bytes < need || !ws))
        return fail(TS_ERR_WORKSPACE, "ts_threshold_search2d: workspace too small (need " + std::to_string(need) +
                                          " bytes, got " + std::to_string(ws_bytes) + ")");
    if (nseg == 0)
        return TS_OK;
    if ((uintptr_t)ws & 7)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search2d: workspace must be 8-byte aligned");
    return launch_search2d(hist, nseg, nbins, nq, q, ws, thr, obj, status, (hipStream_t)stream);
}

size_t ts_search_dp_workspace_bytes(int32_t nseg, int32_t nbins, int32_t k, int32_t nq)
{
    if (nseg < 0 || nbins < 2 || nbins > MAX_BINS || k < 1 || k > TS_DP_MAX_K || nq < 1 || nq > TS_MAX_Q)
        return 0;
    return dp_workspace_bytes(nseg * nq, nbins, k);
}

ts_status ts_threshold_search_dp(const double *P, const double *Q, int32_t nseg, int32_t nbins, int32_t k,
                                 int32_t nq, const double *q, void *ws, size_t ws_bytes, int32_t *thr, double *obj,
                                 int32_t *status, ts_stream_t stream)
{
    if (nseg < 0)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: nseg must be >= 0");
    if (nbins < 2 || nbins > MAX_BINS)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: nbins must be in [2, 4096]");
    if (k < 1 || k > TS_DP_MAX_K)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: k must be in 1.." + std::to_string(TS_DP_MAX_K));
    if (nbins < k + 1)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: nbins must be >= k + 1");
    ts_status st;
    if ((st = check_q("ts_threshold_search_dp", nq, q, true)) != TS_OK)
        return st;
    if ((int64_t)nseg * nq * (nbins - 1) > 0x7fffffff)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: too many problems");
    if (nseg > 0 && (!P || !Q || !thr || !obj || !status))
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: null pointer");
    const size_t need = dp_workspace_bytes(nseg * nq, nbins, k);
    if (nseg > 0 && (ws_bytes < need || !ws))
        return fail(TS_ERR_WORKSPACE, "ts_threshold_search_dp: workspace too small (need " + std::to_string(need) +
                                          " bytes, got " + std::to_string(ws_bytes) + ")");
    if (nseg == 0)
        return TS_OK;
    if ((uintptr_t)ws & 7)
        return fail(TS_ERR_INVALID_ARG, "ts_threshold_search_dp: workspace must be 8-byte aligned");
    return launch_dp(P, Q, nseg, nbins, k, nq, q, ws, thr, obj, status, (hipStream_t)stream);
}

size_t ts_open2d_workspace_bytes(int32_t nseg, int32_t height, int32_t width)
{
    if (nseg < 0 || height < 1 || width < 1)
        return 0;
    return open2d_workspace_bytes(nseg, height, width);
}

ts_status ts_open2d(ts_batch batch, int32_t height, int32_t width, ts_binning bin, int32_t radius, void *ws,
                    size_t ws_bytes, uint8_t *opened, uint8_t *residue, int16_t *residue16, ts_stream_t stream)
{
    ts_status st = check_batch(batch);
    if (st != TS_OK)
        return st;
    BinMap bm;
    if ((st = make_binmap(bin, &bm)) != TS_OK)
        return st;
    if (bin.nbins > 256)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: nbins must be <= 256 (8-bit gray levels)");
    if (radius < 0 || radius > TS_MORPH_MAX_RADIUS)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: radius must be in 0.." + std::to_string(TS_MORPH_MAX_RADIUS));
    if (height < 1 || width < 1)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: need height >= 1 and width >= 1");
    if ((int64_t)height * width > TS_MORPH_MAX_PIXELS)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: more than " + std::to_string((long long)TS_MORPH_MAX_PIXELS) +
                                            " pixels in one image");
    if (batch.total != (int64_t)batch.nseg * height * width)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: total must be nseg * height * width");
    if (batch.nseg > 0 && !opened && !residue && !residue16)
        return fail(TS_ERR_INVALID_ARG, "ts_open2d: every output is null");
    const size_t need = open2d_workspace_bytes(batch.nseg, height, width);
    if (batch.nseg > 0 && (ws_bytes < need || !ws))
        return fail(TS_ERR_WORKSPACE, "ts_open2d: workspace too small (need " + std::to_string(need) + " bytes, got " +
                                          std::to_string(ws_bytes) + ")");
    if (batch.nseg == 0)
        return TS_OK;
    return launch_open2d(batch, height, width, bm, radius, (uint8_t *)ws, opened, residue, residue16,
                         (hipStream_t)stream);
}

ts_status ts_log2_f32(const float *x, float *y, int64_t n, ts_stream_t stream)
{
    if (n < 0)
        return fail(TS_ERR_INVALID_ARG, "ts_log2_f32: n must be >= 0");
    if (n > 0 && (!x || !y))
        return fail(TS_ERR_INVALID_ARG, "ts_log2_f32: null pointer");
    if (n == 0)
        return TS_OK;
    return launch_log2_f32(x, y, n, (hipStream_t)stream);
}

ts_status ts_issue_rate(int32_t op, int32_t blocks, int32_t iters, float *out, ts_stream_t stream)
{
    if (op < 0 || op > 2)
        return fail(TS_ERR_INVALID_ARG, "ts_issue_rate: op must be 0, 1 or 2");
    if (blocks < 1 || iters < 1)
        return fail(TS_ERR_INVALID_ARG, "ts_issue_rate: blocks and iters must be >= 1");
    if (!out)
        return fail(TS_ERR_INVALID_ARG, "ts_issue_rate: null pointer");
    return launch_issue_rate(op, blocks, iters, out, (hipStream_t)stream);
}

} // extern "C"
