// Host side of the UMI C ABI (include/umi.h): argument checks, the batch
// packer (cost-sorted curve table), per-(device, stream) workspaces, the
// tuning table, and the kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "umi.h"
#include "umi_internal.h"

namespace umi {

hipError_t launch_prepass(const float* flux, const double* time, const CurveDesc* curves,
                          int curve_first, int n_curves, int32_t* segid, int4* segtab,
                          int2* tiles, uint32_t* counter, hipStream_t stream);
hipError_t launch_main(const float* flux, const int32_t* segid, const int4* segtab,
                       const CurveDesc* curves, const int2* tiles, int tile_first, int tile_end,
                       uint32_t* counter, int grid, float alpha, float c, int iters, float* trend,
                       float* median, hipStream_t stream);

namespace {

thread_local std::string t_last_error;
thread_local umi_status t_inject = UMI_OK;

umi_status fail(umi_status s, const std::string& msg)
{
    t_last_error = msg;
    return s;
}

umi_status fail_hip(hipError_t e, const char* where)
{
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(e == hipErrorOutOfMemory ? UMI_ERR_NO_MEMORY : UMI_ERR_DEVICE, m);
}

// ---------------------------------------------------------------------------
// tuning table: W_max -> (tile, groups per CU)

struct TuneRow {
    int w_max;
    int tile;
    int groups_per_cu;
};

std::mutex g_tune_mu;
std::vector<TuneRow> g_tune;  // empty = built-in defaults

// Largest tile whose staged span (tile + W - 1) fits kStageMax.
int max_tile(int W) { return std::max(1, kStageMax - (W - 1)); }

// Built-in default: the largest tile, cut back to a whole number of
// workgroup-wide passes when its last pass would leave most lanes idle.
int default_tile(int W)
{
    const int fill = max_tile(W);
    const int rem = fill % kMainThreads;
    if (fill >= kMainThreads && rem < kMainThreads / 2) return fill - rem;
    return fill;
}
constexpr int kDefaultGroupsPerCU = 4;

void tuned(int W, int* tile, int* gpc)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *tile = default_tile(W);
    *gpc = kDefaultGroupsPerCU;
    for (const TuneRow& r : g_tune) {
        if (W <= r.w_max) {
            if (r.tile > 0) *tile = std::min(r.tile, max_tile(W));
            if (r.groups_per_cu > 0) *gpc = r.groups_per_cu;
            break;
        }
    }
}

// ---------------------------------------------------------------------------
// workspaces, one per (device, stream)

template <class T>
hipError_t grow(T** p, int64_t* cap, int64_t need)
{
    if (need <= *cap) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return e;
    }
    int64_t n = std::max<int64_t>(need + need / 4, 1024);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), (size_t)n * sizeof(T));
    if (e == hipSuccess) *cap = n;
    return e;
}

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    int32_t* segid = nullptr;
    int64_t cap_segid = 0;
    int4* segtab = nullptr;
    int64_t cap_segtab = 0;
    CurveDesc* curves = nullptr;
    int64_t cap_curves = 0;
    int2* tiles = nullptr;
    int64_t cap_tiles = 0;
    uint32_t* counter = nullptr;
    int64_t cap_counter = 0;
    CurveDesc* h_curves = nullptr;  // pinned staging for the curve table
    int64_t cap_h_curves = 0;
    hipEvent_t staged = nullptr;    // last copy out of h_curves
    bool staged_pending = false;

    void free_all()
    {
        if (segid) (void)hipFree(segid);
        if (segtab) (void)hipFree(segtab);
        if (curves) (void)hipFree(curves);
        if (tiles) (void)hipFree(tiles);
        if (counter) (void)hipFree(counter);
        if (h_curves) (void)hipHostFree(h_curves);
        if (staged) (void)hipEventDestroy(staged);
        segid = nullptr;
        segtab = nullptr;
        curves = nullptr;
        tiles = nullptr;
        counter = nullptr;
        h_curves = nullptr;
        staged = nullptr;
        cap_segid = cap_segtab = cap_curves = cap_tiles = cap_counter = cap_h_curves = 0;
        staged_pending = false;
    }

    // Make room; if anything must be reallocated, first wait for work already
    // queued on this stream, which may still read the old buffers.
    hipError_t reserve(int64_t samples, int64_t ncurves, int64_t ntiles)
    {
        const bool need = samples > cap_segid || samples > cap_segtab || ncurves > cap_curves ||
                          ntiles > cap_tiles || cap_counter < 1 || ncurves > cap_h_curves;
        if (!need) return hipSuccess;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if ((e = grow(&segid, &cap_segid, samples)) != hipSuccess) return e;
        if ((e = grow(&segtab, &cap_segtab, samples)) != hipSuccess) return e;
        if ((e = grow(&curves, &cap_curves, ncurves)) != hipSuccess) return e;
        if ((e = grow(&tiles, &cap_tiles, ntiles)) != hipSuccess) return e;
        if ((e = grow(&counter, &cap_counter, 1)) != hipSuccess) return e;
        if (ncurves > cap_h_curves) {
            if (h_curves) (void)hipHostFree(h_curves);
            h_curves = nullptr;
            cap_h_curves = 0;
            const int64_t n = std::max<int64_t>(ncurves + ncurves / 4, 256);
            e = hipHostMalloc(reinterpret_cast<void**>(&h_curves), (size_t)n * sizeof(CurveDesc),
                              hipHostMallocDefault);
            if (e != hipSuccess) return e;
            cap_h_curves = n;
            staged_pending = false;
        }
        if (!staged) {
            e = hipEventCreateWithFlags(&staged, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
std::map<int, int> g_cu_count;

Workspace* workspace_for(int device, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto key = std::make_pair(device, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second;
    Workspace* w = new Workspace();
    w->device = device;
    w->stream = stream;
    g_ws[key] = w;
    return w;
}

int cu_count(int device)
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_cu_count.find(device);
    if (it != g_cu_count.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        n <= 0)
        n = 256;
    g_cu_count[device] = n;
    return n;
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

umi_status check_params(int32_t W, float alpha, float c, int32_t iters)
{
    if (W < 1 || (W % 2) == 0)
        return fail(UMI_ERR_INVALID_ARG, "W must be odd and >= 1 (got " + std::to_string(W) + ")");
    if (W > UMI_MAX_WINDOW)
        return fail(UMI_ERR_UNSUPPORTED,
                    "W=" + std::to_string(W) + " exceeds UMI_MAX_WINDOW=" +
                        std::to_string(UMI_MAX_WINDOW));
    if (!finite_pos(alpha)) return fail(UMI_ERR_INVALID_ARG, "alpha must be finite and > 0");
    if (!finite_pos(c)) return fail(UMI_ERR_INVALID_ARG, "c must be finite and > 0");
    if (iters < 0) return fail(UMI_ERR_INVALID_ARG, "iters must be >= 0");
    return UMI_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

umi_status detrend_batch(const float* flux, const double* time, const int64_t* lengths,
                         int64_t n_curves, const int32_t* W, float alpha, float c, int32_t iters,
                         float* trend, float* median, const umi_launch* launch,
                         hipStream_t stream)
{
    if (t_inject != UMI_OK) {
        umi_status s = t_inject;
        t_inject = UMI_OK;
        return fail(s, "injected error (umi_debug_inject_error)");
    }
    if (n_curves < 0) return fail(UMI_ERR_INVALID_ARG, "n_curves must be >= 0");
    if (n_curves == 0) return UMI_OK;
    if (!lengths || !W) return fail(UMI_ERR_INVALID_ARG, "lengths and W must not be NULL");
    if (n_curves > (int64_t)INT32_MAX) return fail(UMI_ERR_UNSUPPORTED, "too many curves");
    umi_launch opt = {UMI_MODE_PERSISTENT, 0, 0, 0, nullptr, nullptr};
    if (launch) opt = *launch;
    if (opt.reserved != 0) return fail(UMI_ERR_INVALID_ARG, "umi_launch.reserved must be 0");
    if (opt.mode != UMI_MODE_PERSISTENT && opt.mode != UMI_MODE_PER_CURVE)
        return fail(UMI_ERR_INVALID_ARG, "unknown launch mode");
    if (opt.tile < 0 || opt.groups_per_cu < 0)
        return fail(UMI_ERR_INVALID_ARG, "launch tile and groups_per_cu must be >= 0");

    int64_t total = 0;
    for (int64_t b = 0; b < n_curves; ++b) {
        if (lengths[b] < 0) return fail(UMI_ERR_INVALID_ARG, "curve lengths must be >= 0");
        if (lengths[b] > (int64_t)INT32_MAX)
            return fail(UMI_ERR_UNSUPPORTED, "a curve longer than 2^31-1 samples");
        umi_status st = check_params(W[b], alpha, c, iters);
        if (st != UMI_OK) return st;
        total += lengths[b];
    }
    if (total == 0) return UMI_OK;
    if (!flux || !trend) return fail(UMI_ERR_INVALID_ARG, "flux and trend must not be NULL");

    // ---- pack: curve table in decreasing per-tile cost, tile bases ----
    std::vector<int64_t> off((size_t)n_curves);
    {
        int64_t acc = 0;
        for (int64_t b = 0; b < n_curves; ++b) {
            off[(size_t)b] = acc;
            acc += lengths[b];
        }
    }
    std::vector<int> tile_of((size_t)n_curves);
    for (int64_t b = 0; b < n_curves; ++b) {
        int t, g;
        tuned(W[b], &t, &g);
        if (opt.tile > 0) t = std::min(opt.tile, max_tile(W[b]));
        tile_of[(size_t)b] = t;
    }
    std::vector<int32_t> order;
    order.reserve((size_t)n_curves);
    for (int64_t b = 0; b < n_curves; ++b)
        if (lengths[b] > 0) order.push_back((int32_t)b);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int64_t ca = (int64_t)W[a] * tile_of[(size_t)a];
        const int64_t cb = (int64_t)W[b] * tile_of[(size_t)b];
        if (ca != cb) return ca > cb;
        return lengths[a] > lengths[b];
    });
    const int64_t nc = (int64_t)order.size();
    int64_t ntiles = 0;
    std::vector<int64_t> curve_tiles((size_t)nc);
    for (int64_t i = 0; i < nc; ++i) {
        const int32_t b = order[(size_t)i];
        curve_tiles[(size_t)i] = (lengths[b] + tile_of[(size_t)b] - 1) / tile_of[(size_t)b];
        ntiles += curve_tiles[(size_t)i];
    }
    if (ntiles > (int64_t)INT32_MAX) return fail(UMI_ERR_UNSUPPORTED, "too many tiles");
    // persistent grid size: the tuning row of the costliest curve
    int gpc = kDefaultGroupsPerCU;
    if (nc > 0) {
        int t_unused;
        tuned(W[order[0]], &t_unused, &gpc);
    }
    if (opt.groups_per_cu > 0) gpc = opt.groups_per_cu;

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    Workspace* ws = workspace_for(device, stream);
    std::lock_guard<std::mutex> lk(ws->mu);
    e = ws->reserve(total, nc, ntiles);
    if (e != hipSuccess) return fail_hip(e, "workspace allocation");

    // the previous copy out of the staging buffer must be done before reuse
    if (ws->staged_pending) {
        e = hipEventSynchronize(ws->staged);
        if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
        ws->staged_pending = false;
    }
    {
        int64_t base = 0;
        for (int64_t i = 0; i < nc; ++i) {
            const int32_t b = order[(size_t)i];
            CurveDesc& d = ws->h_curves[i];
            d.off = off[(size_t)b];
            d.len = (int32_t)lengths[b];
            d.W = W[b];
            d.tile = tile_of[(size_t)b];
            d.tile_base = (int32_t)base;
            base += curve_tiles[(size_t)i];
        }
    }
    e = hipMemcpyAsync(ws->curves, ws->h_curves, (size_t)nc * sizeof(CurveDesc),
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail_hip(e, "curve table copy");
    e = hipEventRecord(ws->staged, stream);
    if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
    ws->staged_pending = true;

    const int ncu = cu_count(device);
    if (opt.mode == UMI_MODE_PERSISTENT) {
        e = launch_prepass(flux, time, ws->curves, 0, (int)nc, ws->segid, ws->segtab, ws->tiles,
                           ws->counter, stream);
        if (e != hipSuccess) return fail_hip(e, "pre-pass launch");
        const int64_t grid = std::min<int64_t>(ntiles, (int64_t)gpc * ncu);
        if (opt.main_start && (e = hipEventRecord((hipEvent_t)opt.main_start, stream)) != hipSuccess)
            return fail_hip(e, "hipEventRecord(main_start)");
        e = launch_main(flux, ws->segid, ws->segtab, ws->curves, ws->tiles, 0, (int)ntiles,
                        ws->counter, (int)grid, alpha, c, iters, trend, median, stream);
        if (e != hipSuccess) return fail_hip(e, "main kernel launch");
        if (opt.main_stop && (e = hipEventRecord((hipEvent_t)opt.main_stop, stream)) != hipSuccess)
            return fail_hip(e, "hipEventRecord(main_stop)");
    } else {
        if (opt.main_start && (e = hipEventRecord((hipEvent_t)opt.main_start, stream)) != hipSuccess)
            return fail_hip(e, "hipEventRecord(main_start)");
        int64_t tb = 0;
        for (int64_t i = 0; i < nc; ++i) {
            e = launch_prepass(flux, time, ws->curves, (int)i, 1, ws->segid, ws->segtab,
                               ws->tiles, nullptr, stream);
            if (e != hipSuccess) return fail_hip(e, "pre-pass launch");
            const int64_t nt = curve_tiles[(size_t)i];
            e = launch_main(flux, ws->segid, ws->segtab, ws->curves, ws->tiles, (int)tb,
                            (int)(tb + nt), nullptr, (int)nt, alpha, c, iters, trend, median,
                            stream);
            if (e != hipSuccess) return fail_hip(e, "main kernel launch");
            tb += nt;
        }
        if (opt.main_stop && (e = hipEventRecord((hipEvent_t)opt.main_stop, stream)) != hipSuccess)
            return fail_hip(e, "hipEventRecord(main_stop)");
    }
    // curves of length zero produce nothing; everything else was written
    return UMI_OK;
}

}  // namespace umi

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

umi_status umi_detrend(const float* flux, const double* time, int64_t n, int32_t W, float alpha,
                       float c, int32_t iters, float* trend, float* median, void* stream)
{
    if (n < 0) {
        umi::t_last_error = "n must be >= 0";
        return UMI_ERR_INVALID_ARG;
    }
    const int64_t len = n;
    const int32_t w = W;
    return umi::detrend_batch(flux, time, &len, 1, &w, alpha, c, iters, trend, median, nullptr,
                              static_cast<hipStream_t>(stream));
}

umi_status umi_detrend_batch(const float* flux, const double* time, const int64_t* lengths,
                             int64_t n_curves, const int32_t* W, float alpha, float c,
                             int32_t iters, float* trend, float* median, const umi_launch* launch,
                             void* stream)
{
    return umi::detrend_batch(flux, time, lengths, n_curves, W, alpha, c, iters, trend, median,
                              launch, static_cast<hipStream_t>(stream));
}

int32_t umi_window_from_cadence(double cadence_days, double window_days)
{
    if (!(cadence_days > 0.0) || !std::isfinite(cadence_days) || !(window_days > 0.0) ||
        !std::isfinite(window_days))
        return -1;
    const double q = window_days / cadence_days;
    if (!(q < 2.0e9)) return -1;
    const long long r = std::llround(q);  // ties either way give the same W after |1
    return (int32_t)(r | 1LL);
}

umi_status umi_set_tuning(const char* table_text)
{
    std::vector<umi::TuneRow> rows;
    if (table_text) {
        std::istringstream in(table_text);
        std::string line;
        while (std::getline(in, line)) {
            const size_t hash = line.find('#');
            if (hash != std::string::npos) line.resize(hash);
            if (line.find_first_not_of(" \t\r") == std::string::npos) continue;  // blank
            std::istringstream ls(line);
            umi::TuneRow r;
            if (!(ls >> r.w_max >> r.tile >> r.groups_per_cu) || r.w_max < 1 || r.tile < 0 ||
                r.groups_per_cu < 0 || r.groups_per_cu > 64) {
                umi::t_last_error = "malformed tuning line: " + line;
                return UMI_ERR_INVALID_ARG;
            }
            std::string extra;
            if (ls >> extra) {
                umi::t_last_error = "malformed tuning line: " + line;
                return UMI_ERR_INVALID_ARG;
            }
            rows.push_back(r);
        }
        for (size_t i = 1; i < rows.size(); ++i)
            if (rows[i].w_max <= rows[i - 1].w_max) {
                umi::t_last_error = "tuning rows must be sorted by increasing W_max";
                return UMI_ERR_INVALID_ARG;
            }
    }
    std::lock_guard<std::mutex> lk(umi::g_tune_mu);
    umi::g_tune = rows;
    return UMI_OK;
}

const char* umi_last_error(void) { return umi::t_last_error.c_str(); }

void umi_release(void)
{
    std::lock_guard<std::mutex> lk(umi::g_ws_mu);
    for (auto& kv : umi::g_ws) {
        umi::Workspace* w = kv.second;
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(w->device);
        (void)hipDeviceSynchronize();
        w->free_all();
        (void)hipSetDevice(prev);
        delete w;
    }
    umi::g_ws.clear();
}

const char* umi_version(void) { return "umi-mi355x 0.1.0"; }

void umi_debug_inject_error(umi_status s) { umi::t_inject = s; }

}  // extern "C"
