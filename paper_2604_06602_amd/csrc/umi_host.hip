// Host side of the UMI C ABI (include/umi.h): argument checks, the batch
// packer (cost-sorted curve table), per-(device, stream) workspaces, the
// tuning table, the kernel launches, replayable plans (hipGraph), and the
// serving loop's batched host copies (include/umi_serve.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <utility>
#include <vector>
#include <condition_variable>

#include "umi.h"
#include "umi_internal.h"
#include "umi_serve.h"

namespace umi {

hipError_t launch_prepass(const float* flux, const double* time, const BatchHeader* hdr,
                          const CurveDesc* curves, int curve_first, int grid, int32_t* segid,
                          int4* segtab, int2* tiles, uint32_t* counter, hipStream_t stream);
hipError_t launch_main(const float* flux, const int32_t* segid, const int4* segtab,
                       const BatchHeader* hdr, const CurveDesc* curves, const int2* tiles,
                       int tile_first, int tile_count, uint32_t* counter, int grid,
                       float* trend, float* median, hipStream_t stream);

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

bool take_injected(umi_status* s)
{
    if (t_inject == UMI_OK) return false;
    *s = fail(t_inject, "injected error (umi_debug_inject_error)");
    t_inject = UMI_OK;
    return true;
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

// Largest tile: its staged span (tile + W - 1) fits kStageMax, and each lane
// takes at most three of its positions.
int max_tile(int W) { return std::max(1, std::min(kMaxTile, kStageMax - (W - 1))); }

// Built-in default: the largest tile, cut back to a whole number of
// workgroup-wide passes when its last pass would leave most lanes idle.
int default_tile(int W)
{
    const int fill = max_tile(W);
    const int rem = fill % kMainThreads;
    if (fill >= kMainThreads && rem < kMainThreads / 2) return fill - rem;
    return fill;
}
constexpr int kDefaultGroupsPerCU = 4;  // LDS (37.6 KB) allows four 512-thread groups per CU

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
// argument checks

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

umi_status check_window(int32_t W)
{
    if (W < 1 || (W % 2) == 0)
        return fail(UMI_ERR_INVALID_ARG, "W must be odd and >= 1 (got " + std::to_string(W) + ")");
    if (W > UMI_MAX_WINDOW)
        return fail(UMI_ERR_UNSUPPORTED,
                    "W=" + std::to_string(W) + " exceeds UMI_MAX_WINDOW=" +
                        std::to_string(UMI_MAX_WINDOW));
    return UMI_OK;
}

umi_status check_params(float alpha, float c, int32_t iters)
{
    if (!finite_pos(alpha)) return fail(UMI_ERR_INVALID_ARG, "alpha must be finite and > 0");
    if (!finite_pos(c)) return fail(UMI_ERR_INVALID_ARG, "c must be finite and > 0");
    if (iters < 0) return fail(UMI_ERR_INVALID_ARG, "iters must be >= 0");
    return UMI_OK;
}

// The extra options of the _ex calls (NULL = the plain method with the
// call's alpha and c for every curve).
umi_status check_options(const umi_options* o, int64_t n_curves, const double* time,
                         umi_options* out)
{
    *out = umi_options{nullptr, nullptr, UMI_SCALE_UPPER_RMS, 0, nullptr, nullptr};
    if (!o) return UMI_OK;
    *out = *o;
    if (o->reserved != 0) return fail(UMI_ERR_INVALID_ARG, "umi_options.reserved must be 0");
    if (o->scale != UMI_SCALE_UPPER_RMS && o->scale != UMI_SCALE_MAD)
        return fail(UMI_ERR_INVALID_ARG, "unknown umi_options.scale");
    for (int64_t b = 0; b < n_curves; ++b) {
        if (o->alpha && !finite_pos(o->alpha[b]))
            return fail(UMI_ERR_INVALID_ARG, "per-curve alpha must be finite and > 0");
        if (o->c && !finite_pos(o->c[b]))
            return fail(UMI_ERR_INVALID_ARG, "per-curve c must be finite and > 0");
        if (o->window_days) {
            const double L = o->window_days[b];
            if (!std::isfinite(L) || L < 0.0)
                return fail(UMI_ERR_INVALID_ARG, "window_days must be finite and >= 0");
            if (L > 0.0 && !time)
                return fail(UMI_ERR_INVALID_ARG, "time windows need the time array");
        }
    }
    return UMI_OK;
}

// Checks curves at explicit offsets: lengths >= 0, valid windows, ranges
// pairwise disjoint.  `span` gets max(off + len), `total` the sample count.
umi_status check_curves(const int64_t* offsets, const int64_t* lengths, int64_t n,
                        const int32_t* W, int64_t* span, int64_t* total)
{
    *span = 0;
    *total = 0;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    ranges.reserve((size_t)n);
    for (int64_t b = 0; b < n; ++b) {
        if (lengths[b] < 0) return fail(UMI_ERR_INVALID_ARG, "curve lengths must be >= 0");
        if (lengths[b] > (int64_t)INT32_MAX)
            return fail(UMI_ERR_UNSUPPORTED, "a curve longer than 2^31-1 samples");
        if (offsets[b] < 0 || offsets[b] > INT64_MAX - lengths[b])
            return fail(UMI_ERR_INVALID_ARG, "curve offsets must be >= 0");
        umi_status st = check_window(W[b]);
        if (st != UMI_OK) return st;
        if (lengths[b] > 0) ranges.emplace_back(offsets[b], offsets[b] + lengths[b]);
        *span = std::max(*span, offsets[b] + lengths[b]);
        *total += lengths[b];
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second)
            return fail(UMI_ERR_INVALID_ARG, "curves overlap in the sample arrays");
    return UMI_OK;
}

umi_status check_launch(const umi_launch* launch, umi_launch* opt)
{
    *opt = umi_launch{UMI_MODE_PERSISTENT, 0, 0, 0, nullptr, nullptr};
    if (launch) *opt = *launch;
    if (opt->reserved != 0) return fail(UMI_ERR_INVALID_ARG, "umi_launch.reserved must be 0");
    if (opt->mode != UMI_MODE_PERSISTENT && opt->mode != UMI_MODE_PER_CURVE)
        return fail(UMI_ERR_INVALID_ARG, "unknown launch mode");
    if (opt->tile < 0 || opt->groups_per_cu < 0)
        return fail(UMI_ERR_INVALID_ARG, "launch tile and groups_per_cu must be >= 0");
    return UMI_OK;
}

// ---------------------------------------------------------------------------
// packer: the curve table in decreasing per-tile cost

struct Packed {
    std::vector<CurveDesc> curves;      // non-empty curves, cost order
    std::vector<int64_t> curve_tiles;   // tiles per table entry
    int64_t ntiles = 0;
    int gpc = kDefaultGroupsPerCU;      // persistent groups per CU
};

// Tile sizes a batch too small to give every CU a tile falls back to, largest
// first: at 512 each lane of a workgroup takes one window.
constexpr int kSmallBatchTiles[] = {1024, 512};

umi_status pack(const int64_t* offsets, const int64_t* lengths, int64_t n, const int32_t* W,
                float alpha, float c, const umi_options& o, const umi_launch& opt, int n_cu,
                int64_t max_tiles, Packed* out)
{
    std::vector<int> tile_of((size_t)n);
    std::vector<int32_t> order;
    order.reserve((size_t)n);
    for (int64_t b = 0; b < n; ++b) {
        int t, g;
        tuned(W[b], &t, &g);
        if (opt.tile > 0) t = std::min(opt.tile, max_tile(W[b]));
        tile_of[(size_t)b] = t;
        if (lengths[b] > 0) order.push_back((int32_t)b);
    }
    // A batch that the tuned tiles cut into fewer tiles than there are CUs
    // (one curve, a quiet serving step) would leave most of the chip idle:
    // smaller tiles spread its windows over more CUs.  Results do not depend
    // on the tiling.  An explicit launch tile is kept as given.
    auto count_tiles = [&](int cap) {
        int64_t t = 0;
        for (int32_t b : order) {
            const int tb = cap > 0 ? std::min(tile_of[(size_t)b], cap) : tile_of[(size_t)b];
            t += (lengths[b] + tb - 1) / tb;
        }
        return t;
    };
    if (opt.tile == 0 && count_tiles(0) < n_cu) {
        for (int cap : kSmallBatchTiles) {
            if (count_tiles(cap) > max_tiles) break;
            for (int32_t b : order) tile_of[(size_t)b] = std::min(tile_of[(size_t)b], cap);
            if (count_tiles(0) >= n_cu) break;
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int64_t ca = (int64_t)W[a] * tile_of[(size_t)a];
        const int64_t cb = (int64_t)W[b] * tile_of[(size_t)b];
        if (ca != cb) return ca > cb;
        return lengths[a] > lengths[b];
    });
    out->curves.resize(order.size());
    out->curve_tiles.resize(order.size());
    out->ntiles = 0;
    for (size_t i = 0; i < order.size(); ++i) {
        const int32_t b = order[i];
        const int64_t nt = (lengths[b] + tile_of[(size_t)b] - 1) / tile_of[(size_t)b];
        if (out->ntiles + nt > (int64_t)INT32_MAX)
            return fail(UMI_ERR_UNSUPPORTED, "too many tiles in one batch");
        CurveDesc& d = out->curves[i];
        d.off = offsets[b];
        d.len = (int32_t)lengths[b];
        d.W = W[b];
        d.tile = tile_of[(size_t)b];
        d.tile_base = (int32_t)out->ntiles;
        d.alpha = o.alpha ? o.alpha[b] : alpha;
        d.c = o.c ? o.c[b] : c;
        d.window_days = o.window_days ? o.window_days[b] : 0.0;
        out->curve_tiles[i] = nt;
        out->ntiles += nt;
    }
    out->gpc = kDefaultGroupsPerCU;
    if (!order.empty()) {
        int t_unused;
        tuned(W[order[0]], &t_unused, &out->gpc);  // the costliest curve's row
    }
    if (opt.groups_per_cu > 0) out->gpc = opt.groups_per_cu;
    return UMI_OK;
}

size_t block_bytes(int64_t ncurves)
{
    return sizeof(BatchHeader) + (size_t)ncurves * sizeof(CurveDesc);
}

void write_block(uint8_t* dst, const Packed& p, int32_t iters, const umi_options& o,
                 const double* time)
{
    BatchHeader h = {};
    h.n_curves = (int32_t)p.curves.size();
    h.n_tiles = (int32_t)p.ntiles;
    h.iters = iters;
    h.scale = o.scale;
    h.detrended = o.detrended;
    h.time = time;
    std::memcpy(dst, &h, sizeof h);
    if (!p.curves.empty())
        std::memcpy(dst + sizeof h, p.curves.data(), p.curves.size() * sizeof(CurveDesc));
}

// ---------------------------------------------------------------------------
// device buffers of a launch sequence

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

struct DeviceBuffers {
    int32_t* segid = nullptr;   // per sample slot
    int64_t cap_segid = 0;
    int4* segtab = nullptr;     // per sample slot (used per segment)
    int64_t cap_segtab = 0;
    int2* tiles = nullptr;
    int64_t cap_tiles = 0;
    uint32_t* counter = nullptr;
    int64_t cap_counter = 0;

    hipError_t reserve(int64_t span, int64_t ntiles)
    {
        hipError_t e;
        if ((e = grow(&segid, &cap_segid, span)) != hipSuccess) return e;
        if ((e = grow(&segtab, &cap_segtab, span)) != hipSuccess) return e;
        if ((e = grow(&tiles, &cap_tiles, ntiles)) != hipSuccess) return e;
        return grow(&counter, &cap_counter, 1);
    }
    bool fits(int64_t span, int64_t ntiles) const
    {
        return span <= cap_segid && span <= cap_segtab && ntiles <= cap_tiles && cap_counter >= 1;
    }
    void release()
    {
        if (segid) (void)hipFree(segid);
        if (segtab) (void)hipFree(segtab);
        if (tiles) (void)hipFree(tiles);
        if (counter) (void)hipFree(counter);
        *this = DeviceBuffers();
    }
};

// Enqueue the pre-pass and estimate kernels for a staged block (header +
// curve table, at `dblock` on the device by the time the stream reaches them).
hipError_t enqueue_kernels(const float* flux, const double* time, float* trend, float* median,
                           const uint8_t* dblock, const DeviceBuffers& b, int mode,
                           const Packed* p, int prep_grid, int main_grid, hipEvent_t ev0,
                           hipEvent_t ev1, hipStream_t stream)
{
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(dblock);
    const CurveDesc* curves = reinterpret_cast<const CurveDesc*>(dblock + sizeof(BatchHeader));
    hipError_t e;
    if (mode == UMI_MODE_PERSISTENT) {
        if ((e = launch_prepass(flux, time, hdr, curves, 0, prep_grid, b.segid, b.segtab, b.tiles,
                                b.counter, stream)) != hipSuccess)
            return e;
        if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return e;
        if ((e = launch_main(flux, b.segid, b.segtab, hdr, curves, b.tiles, 0, -1, b.counter,
                             main_grid, trend, median, stream)) != hipSuccess)
            return e;
        if (ev1 && (e = hipEventRecord(ev1, stream)) != hipSuccess) return e;
        return hipSuccess;
    }
    // one pre-pass and one estimate launch per curve, one workgroup per tile
    if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return e;
    for (size_t i = 0; i < p->curves.size(); ++i) {
        if ((e = launch_prepass(flux, time, hdr, curves, (int)i, 1, b.segid, b.segtab, b.tiles,
                                nullptr, stream)) != hipSuccess)
            return e;
        const int nt = (int)p->curve_tiles[i];
        if ((e = launch_main(flux, b.segid, b.segtab, hdr, curves, b.tiles,
                             p->curves[i].tile_base, nt, nullptr, nt, trend, median, stream)) !=
            hipSuccess)
            return e;
    }
    if (ev1 && (e = hipEventRecord(ev1, stream)) != hipSuccess) return e;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// workspaces of the direct calls, one per (device, stream)

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    DeviceBuffers buf;
    uint8_t* dblock = nullptr;   // header + curve table on the device
    int64_t cap_dblock = 0;
    uint8_t* hblock = nullptr;   // pinned staging for it
    int64_t cap_hblock = 0;
    hipEvent_t staged = nullptr; // last copy out of hblock
    bool staged_pending = false;

    void free_all()
    {
        buf.release();
        if (dblock) (void)hipFree(dblock);
        if (hblock) (void)hipHostFree(hblock);
        if (staged) (void)hipEventDestroy(staged);
        dblock = hblock = nullptr;
        cap_dblock = cap_hblock = 0;
        staged = nullptr;
        staged_pending = false;
    }

    // Make room; if anything must be reallocated, first wait for work already
    // queued on this stream, which may still read the old buffers.
    hipError_t reserve(int64_t span, int64_t ncurves, int64_t ntiles)
    {
        const int64_t bytes = (int64_t)block_bytes(ncurves);
        if (buf.fits(span, ntiles) && bytes <= cap_dblock && bytes <= cap_hblock && staged)
            return hipSuccess;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        staged_pending = false;
        if ((e = buf.reserve(span, ntiles)) != hipSuccess) return e;
        if ((e = grow(&dblock, &cap_dblock, bytes)) != hipSuccess) return e;
        if (bytes > cap_hblock) {
            if (hblock) (void)hipHostFree(hblock);
            hblock = nullptr;
            cap_hblock = 0;
            const int64_t n = std::max<int64_t>(bytes + bytes / 4, 4096);
            e = hipHostMalloc(reinterpret_cast<void**>(&hblock), (size_t)n, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            cap_hblock = n;
        }
        if (!staged) e = hipEventCreateWithFlags(&staged, hipEventDisableTiming);
        return e;
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

}  // namespace

// ---------------------------------------------------------------------------
// direct calls: curves at explicit offsets

umi_status detrend_gather(const float* flux, const double* time, const int64_t* offsets,
                          const int64_t* lengths, int64_t n_curves, const int32_t* W,
                          float alpha, float c, int32_t iters, float* trend, float* median,
                          const umi_options* options, const umi_launch* launch,
                          hipStream_t stream)
{
    umi_status st;
    if (take_injected(&st)) return st;
    if (n_curves < 0) return fail(UMI_ERR_INVALID_ARG, "n_curves must be >= 0");
    if (n_curves == 0) return UMI_OK;
    if (!offsets || !lengths || !W)
        return fail(UMI_ERR_INVALID_ARG, "offsets, lengths and W must not be NULL");
    if (n_curves > (int64_t)INT32_MAX) return fail(UMI_ERR_UNSUPPORTED, "too many curves");
    umi_launch opt;
    if ((st = check_launch(launch, &opt)) != UMI_OK) return st;
    if ((st = check_params(alpha, c, iters)) != UMI_OK) return st;
    umi_options o;
    if ((st = check_options(options, n_curves, time, &o)) != UMI_OK) return st;
    int64_t span, total;
    if ((st = check_curves(offsets, lengths, n_curves, W, &span, &total)) != UMI_OK) return st;
    if (total == 0) return UMI_OK;
    if (!flux || !trend) return fail(UMI_ERR_INVALID_ARG, "flux and trend must not be NULL");

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    Packed p;
    if ((st = pack(offsets, lengths, n_curves, W, alpha, c, o, opt, cu_count(device),
                   (int64_t)INT32_MAX, &p)) != UMI_OK)
        return st;
    const int64_t nc = (int64_t)p.curves.size();
    Workspace* ws = workspace_for(device, stream);
    std::lock_guard<std::mutex> lk(ws->mu);
    if ((e = ws->reserve(span, nc, p.ntiles)) != hipSuccess)
        return fail_hip(e, "workspace allocation");
    if (ws->staged_pending) {  // the previous copy out of the staging block must be done
        if ((e = hipEventSynchronize(ws->staged)) != hipSuccess)
            return fail_hip(e, "hipEventSynchronize");
        ws->staged_pending = false;
    }
    write_block(ws->hblock, p, iters, o, time);
    if ((e = hipMemcpyAsync(ws->dblock, ws->hblock, block_bytes(nc), hipMemcpyHostToDevice,
                            stream)) != hipSuccess)
        return fail_hip(e, "curve table copy");
    if ((e = hipEventRecord(ws->staged, stream)) != hipSuccess)
        return fail_hip(e, "hipEventRecord");
    ws->staged_pending = true;
    const int grid = (int)std::min<int64_t>(p.ntiles, (int64_t)p.gpc * cu_count(device));
    e = enqueue_kernels(flux, time, trend, median, ws->dblock, ws->buf, opt.mode, &p, (int)nc,
                        grid, (hipEvent_t)opt.main_start, (hipEvent_t)opt.main_stop, stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return UMI_OK;
}


// ---------------------------------------------------------------------------
// batched host copies (umi_host_copy_many)

namespace {

constexpr int64_t kCopyPiece = int64_t(1) << 20;  // bytes per work item

// One call's copies cut into pieces; threads take pieces by an atomic index.
struct CopyJob {
    void* const* dst;
    const void* const* src;
    const int64_t* bytes;
    std::vector<int64_t> first;  // first piece of copy i; first[n] = total pieces
    std::atomic<int64_t> next{0};
    int slots = 0;               // pool threads that may still join

    void work()
    {
        const int64_t total = first.back();
        for (;;) {
            const int64_t p = next.fetch_add(1, std::memory_order_relaxed);
            if (p >= total) return;
            const size_t i = size_t(std::upper_bound(first.begin(), first.end(), p) -
                                    first.begin()) - 1;
            const int64_t off = (p - first[i]) * kCopyPiece;
            const int64_t len = std::min(kCopyPiece, bytes[i] - off);
            std::memcpy(static_cast<char*>(dst[i]) + off,
                        static_cast<const char*>(src[i]) + off, size_t(len));
        }
    }
};

// Pool threads wait for a job, take pieces until none are left, and report
// back; one job runs at a time.  The pool is never destroyed (its threads
// stay blocked on the condition variable until the process exits).
class CopyPool {
  public:
    void run(CopyJob& job, int threads)
    {
        std::lock_guard<std::mutex> one_at_a_time(call_mu_);
        {
            std::lock_guard<std::mutex> lk(mu_);
            try {
                while ((int)workers_ < threads - 1) {
                    std::thread(&CopyPool::worker, this).detach();
                    ++workers_;
                }
            } catch (...) {
                // no more threads: the ones there are (and the caller) do the job
            }
            job.slots = std::min(threads - 1, (int)workers_);
            job_ = &job;
            ++gen_;
        }
        cv_.notify_all();
        job.work();  // the calling thread copies too
        std::unique_lock<std::mutex> lk(mu_);
        job_ = nullptr;  // threads waking from now on skip this job
        done_cv_.wait(lk, [&] { return active_ == 0; });
    }

  private:
    void worker()
    {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            CopyJob* j = job_;
            if (!j || j->slots <= 0) continue;
            --j->slots;
            ++active_;
            lk.unlock();
            j->work();
            lk.lock();
            if (--active_ == 0) done_cv_.notify_all();
        }
    }

    std::mutex call_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    CopyJob* job_ = nullptr;
    uint64_t gen_ = 0;
    int active_ = 0;
    size_t workers_ = 0;
};

CopyPool& copy_pool()
{
    static CopyPool* pool = new CopyPool();  // intentionally never freed
    return *pool;
}

}  // namespace

}  // namespace umi

// ---------------------------------------------------------------------------
// replayable plans

struct umi_plan {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t capacity = 0;
    int64_t max_curves = 0;
    int64_t max_tiles = 0;
    int32_t max_W = 0;
    const float* flux = nullptr;
    const double* time = nullptr;
    float* trend = nullptr;
    float* median = nullptr;
    int main_grid = 0;
    umi::DeviceBuffers buf;
    struct Slot {
        uint8_t* host = nullptr;    // pinned header + curve table
        uint8_t* dev = nullptr;     // its device copy
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t done = nullptr;  // recorded after the slot's last replay
        bool pending = false;
    } slot[2];
    int next = 0;
    std::mutex mu;
};

namespace {

void plan_free(umi_plan* p)
{
    for (auto& s : p->slot) {
        if (s.exec) (void)hipGraphExecDestroy(s.exec);
        if (s.graph) (void)hipGraphDestroy(s.graph);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        s = umi_plan::Slot();
    }
    p->buf.release();
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

umi_status umi_detrend(const float* flux, const double* time, int64_t n, int32_t W, float alpha,
                       float c, int32_t iters, float* trend, float* median, void* stream)
{
    if (n < 0) return umi::fail(UMI_ERR_INVALID_ARG, "n must be >= 0");
    const int64_t off = 0, len = n;
    const int32_t w = W;
    return umi::detrend_gather(flux, time, &off, &len, 1, &w, alpha, c, iters, trend, median,
                               nullptr, nullptr, static_cast<hipStream_t>(stream));
}

umi_status umi_detrend_batch(const float* flux, const double* time, const int64_t* lengths,
                             int64_t n_curves, const int32_t* W, float alpha, float c,
                             int32_t iters, float* trend, float* median, const umi_launch* launch,
                             void* stream)
{
    if (n_curves > 0 && !lengths)
        return umi::fail(UMI_ERR_INVALID_ARG, "lengths must not be NULL");
    std::vector<int64_t> off(n_curves > 0 ? (size_t)n_curves : 0);
    int64_t acc = 0;
    for (int64_t b = 0; b < n_curves; ++b) {
        off[(size_t)b] = acc;
        if (lengths[b] > 0) acc += lengths[b];
    }
    return umi::detrend_gather(flux, time, off.data(), lengths, n_curves, W, alpha, c, iters,
                               trend, median, nullptr, launch, static_cast<hipStream_t>(stream));
}

umi_status umi_detrend_gather(const float* flux, const double* time, const int64_t* offsets,
                              const int64_t* lengths, int64_t n_curves, const int32_t* W,
                              float alpha, float c, int32_t iters, float* trend, float* median,
                              const umi_launch* launch, void* stream)
{
    return umi::detrend_gather(flux, time, offsets, lengths, n_curves, W, alpha, c, iters, trend,
                               median, nullptr, launch, static_cast<hipStream_t>(stream));
}

umi_status umi_detrend_gather_ex(const float* flux, const double* time, const int64_t* offsets,
                                 const int64_t* lengths, int64_t n_curves, const int32_t* W,
                                 float alpha, float c, int32_t iters, float* trend,
                                 float* median, const umi_options* options,
                                 const umi_launch* launch, void* stream)
{
    if (offsets) {
        return umi::detrend_gather(flux, time, offsets, lengths, n_curves, W, alpha, c, iters,
                                   trend, median, options, launch,
                                   static_cast<hipStream_t>(stream));
    }
    if (n_curves > 0 && !lengths)
        return umi::fail(UMI_ERR_INVALID_ARG, "lengths must not be NULL");
    std::vector<int64_t> off(n_curves > 0 ? (size_t)n_curves : 0);
    int64_t acc = 0;
    for (int64_t b = 0; b < n_curves; ++b) {
        off[(size_t)b] = acc;
        if (lengths[b] > 0) acc += lengths[b];
    }
    return umi::detrend_gather(flux, time, off.data(), lengths, n_curves, W, alpha, c, iters,
                               trend, median, options, launch, static_cast<hipStream_t>(stream));
}

umi_status umi_plan_create(umi_plan** out, int64_t capacity, int64_t max_curves, int32_t max_W,
                           const float* flux, const double* time, float* trend, float* median,
                           void* stream)
{
    umi_status st;
    if (umi::take_injected(&st)) return st;
    if (!out) return umi::fail(UMI_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    if (capacity < 1 || max_curves < 1)
        return umi::fail(UMI_ERR_INVALID_ARG, "capacity and max_curves must be >= 1");
    if (max_curves > (1 << 24)) return umi::fail(UMI_ERR_UNSUPPORTED, "max_curves above 2^24");
    if ((st = umi::check_window(max_W)) != UMI_OK) return st;
    if (!flux || !trend) return umi::fail(UMI_ERR_INVALID_ARG, "flux and trend must not be NULL");
    if (!stream)
        return umi::fail(UMI_ERR_INVALID_ARG, "plans need a non-default stream (graph capture)");
    // the smallest tile any W <= max_W may use, with or without tuning
    int64_t min_tile = std::min(umi::max_tile(max_W), umi::default_tile(max_W));
    {
        std::lock_guard<std::mutex> lk(umi::g_tune_mu);
        for (const umi::TuneRow& r : umi::g_tune)
            if (r.tile > 0) min_tile = std::min<int64_t>(min_tile, r.tile);
    }
    const int64_t max_tiles = capacity / std::max<int64_t>(1, min_tile) + max_curves;
    if (max_tiles > (int64_t)INT32_MAX)
        return umi::fail(UMI_ERR_UNSUPPORTED, "plan capacity needs too many tiles");
    umi_plan* p = new umi_plan();
    p->stream = static_cast<hipStream_t>(stream);
    p->capacity = capacity;
    p->max_curves = max_curves;
    p->max_tiles = max_tiles;
    p->max_W = max_W;
    p->flux = flux;
    p->time = time;
    p->trend = trend;
    p->median = median;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = p->buf.reserve(capacity, max_tiles);
    const size_t bytes = umi::block_bytes(max_curves);
    for (auto& s : p->slot) {
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&s.host), bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.dev), bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) std::memset(s.host, 0, bytes);
    }
    if (e != hipSuccess) {
        plan_free(p);
        delete p;
        return umi::fail_hip(e, "plan allocation");
    }
    int t_unused, gpc;
    umi::tuned(max_W, &t_unused, &gpc);
    p->main_grid = gpc * umi::cu_count(p->device);
    *out = p;
    return UMI_OK;
}

umi_status umi_plan_run_ex(umi_plan* p, const int64_t* offsets, const int64_t* lengths,
                           const int32_t* W, int64_t n_curves, float alpha, float c,
                           int32_t iters, const umi_options* options)
{
    umi_status st;
    if (umi::take_injected(&st)) return st;
    if (!p) return umi::fail(UMI_ERR_INVALID_ARG, "plan must not be NULL");
    if (n_curves < 0 || n_curves > p->max_curves)
        return umi::fail(UMI_ERR_INVALID_ARG, "n_curves outside [0, max_curves]");
    if (n_curves > 0 && (!offsets || !lengths || !W))
        return umi::fail(UMI_ERR_INVALID_ARG, "offsets, lengths and W must not be NULL");
    if ((st = umi::check_params(alpha, c, iters)) != UMI_OK) return st;
    umi_options o;
    if ((st = umi::check_options(options, n_curves, p->time, &o)) != UMI_OK) return st;
    int64_t span = 0, total = 0;
    if (n_curves > 0 &&
        (st = umi::check_curves(offsets, lengths, n_curves, W, &span, &total)) != UMI_OK)
        return st;
    if (span > p->capacity)
        return umi::fail(UMI_ERR_INVALID_ARG, "a curve ends beyond the plan capacity");
    for (int64_t b = 0; b < n_curves; ++b)
        if (W[b] > p->max_W) return umi::fail(UMI_ERR_INVALID_ARG, "W above the plan's max_W");
    const umi_launch opt = {UMI_MODE_PERSISTENT, 0, 0, 0, nullptr, nullptr};
    umi::Packed pk;
    if (n_curves > 0 &&
        (st = umi::pack(offsets, lengths, n_curves, W, alpha, c, o, opt,
                        umi::cu_count(p->device), p->max_tiles, &pk)) != UMI_OK)
        return st;
    if (pk.ntiles > p->max_tiles)
        return umi::fail(UMI_ERR_UNSUPPORTED, "batch needs more tiles than the plan holds");

    std::lock_guard<std::mutex> lk(p->mu);
    umi_plan::Slot& s = p->slot[p->next];
    hipError_t e;
    if (s.pending) {  // this slot's previous replay must have consumed its bytes
        if ((e = hipEventSynchronize(s.done)) != hipSuccess)
            return umi::fail_hip(e, "hipEventSynchronize");
        s.pending = false;
    }
    umi::write_block(s.host, pk, iters, o, p->time);
    if (!s.exec) {
        // capture once per slot: copy of the staged block, pre-pass over
        // max_curves (blocks beyond the batch exit), persistent estimate
        if ((e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return umi::fail_hip(e, "hipStreamBeginCapture");
        hipError_t ce = hipMemcpyAsync(s.dev, s.host, umi::block_bytes(p->max_curves),
                                       hipMemcpyHostToDevice, p->stream);
        if (ce == hipSuccess)
            ce = umi::enqueue_kernels(p->flux, p->time, p->trend, p->median, s.dev, p->buf,
                                      UMI_MODE_PERSISTENT, nullptr, (int)p->max_curves,
                                      p->main_grid, nullptr, nullptr, p->stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->stream, &g);
        if (ce != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return umi::fail_hip(ce != hipSuccess ? ce : e, "graph capture");
        }
        s.graph = g;
        if ((e = hipGraphInstantiate(&s.exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            s.exec = nullptr;
            return umi::fail_hip(e, "hipGraphInstantiate");
        }
    }
    if ((e = hipGraphLaunch(s.exec, p->stream)) != hipSuccess)
        return umi::fail_hip(e, "hipGraphLaunch");
    if ((e = hipEventRecord(s.done, p->stream)) != hipSuccess)
        return umi::fail_hip(e, "hipEventRecord");
    s.pending = true;
    p->next ^= 1;
    return UMI_OK;
}

umi_status umi_plan_run(umi_plan* p, const int64_t* offsets, const int64_t* lengths,
                        const int32_t* W, int64_t n_curves, float alpha, float c, int32_t iters)
{
    return umi_plan_run_ex(p, offsets, lengths, W, n_curves, alpha, c, iters, nullptr);
}

umi_status umi_plan_destroy(umi_plan* p)
{
    if (!p) return UMI_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    plan_free(p);
    delete p;
    return e == hipSuccess ? UMI_OK : umi::fail_hip(e, "hipStreamSynchronize");
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
                r.groups_per_cu < 0 || r.groups_per_cu > 64)
                return umi::fail(UMI_ERR_INVALID_ARG, "malformed tuning line: " + line);
            std::string extra;
            if (ls >> extra) return umi::fail(UMI_ERR_INVALID_ARG, "malformed tuning line: " + line);
            rows.push_back(r);
        }
        for (size_t i = 1; i < rows.size(); ++i)
            if (rows[i].w_max <= rows[i - 1].w_max)
                return umi::fail(UMI_ERR_INVALID_ARG,
                                 "tuning rows must be sorted by increasing W_max");
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

const char* umi_version(void) { return "umi-mi355x 0.6.0"; }

void umi_debug_inject_error(umi_status s) { umi::t_inject = s; }

umi_status umi_host_copy_many(void* const* dst, const void* const* src, const int64_t* bytes,
                              int64_t n, int32_t threads)
{
    if (n < 0) return umi::fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: n < 0");
    if (threads < 1 || threads > UMI_HOST_COPY_MAX_THREADS)
        return umi::fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: threads out of range");
    if (n == 0) return UMI_OK;
    if (!dst || !src || !bytes)
        return umi::fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: NULL array");
    umi::CopyJob job;
    job.dst = dst;
    job.src = src;
    job.bytes = bytes;
    job.first.resize(size_t(n) + 1);
    int64_t pieces = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (bytes[i] < 0) return umi::fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: bytes < 0");
        if (bytes[i] > 0 && (!dst[i] || !src[i]))
            return umi::fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: NULL pointer");
        job.first[size_t(i)] = pieces;
        pieces += (bytes[i] + umi::kCopyPiece - 1) / umi::kCopyPiece;
    }
    job.first[size_t(n)] = pieces;
    if (pieces == 0) return UMI_OK;
    const int64_t useful = std::min<int64_t>(threads, pieces);
    if (useful <= 1) {
        job.work();
        return UMI_OK;
    }
    umi::copy_pool().run(job, int(useful));
    return UMI_OK;
}

umi_status umi_copy_async(void* const* dst, const void* const* src, const int64_t* bytes,
                          int64_t n, int32_t kind, void* stream)
{
    if (n < 0) return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: n < 0");
    if (kind != UMI_COPY_H2D && kind != UMI_COPY_D2H)
        return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: unknown kind");
    if (n == 0) return UMI_OK;
    if (!dst || !src || !bytes) return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: NULL array");
    for (int64_t i = 0; i < n; ++i) {
        if (bytes[i] < 0) return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: bytes < 0");
        if (bytes[i] > 0 && (!dst[i] || !src[i]))
            return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: NULL pointer");
    }
    const hipMemcpyKind k = kind == UMI_COPY_H2D ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
    for (int64_t i = 0; i < n; ++i) {
        if (bytes[i] == 0) continue;
        const hipError_t e = hipMemcpyAsync(dst[i], src[i], size_t(bytes[i]), k,
                                            static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return umi::fail_hip(e, "umi_copy_async: hipMemcpyAsync");
    }
    return UMI_OK;
}

}  // extern "C"
