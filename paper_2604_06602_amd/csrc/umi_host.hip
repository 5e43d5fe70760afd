// Host side of the UMI C ABI (include/umi.h): argument checks, the batch
// packer (cost-sorted curve table), per-(device, stream) workspaces, the
// tuning table, the kernel launches, replayable plans (hipGraph), and the
// serving loop's batched host copies (include/umi_serve.h; the serving loop
// itself is in umi_server.hip).
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

hipError_t launch_prepass(const float* flux, const double* time, uint8_t* block,
                          const uint8_t* stage, int curve_one, int grid, int32_t* segid,
                          int2* tiles, Counters* ctr, ChunkRec* recs, bool clear_queue, bool walk,
                          const CurveDesc* one, hipStream_t stream);
hipError_t launch_copy(const CopyBatch& cb, hipStream_t stream);
hipError_t launch_main(const float* flux, const int32_t* segid, const BatchHeader* hdr,
                       const CurveDesc* curves, const int2* tiles, int tile_first,
                       int tile_count, uint32_t* counter, int grid, float* trend, float* median,
                       int feat, hipStream_t stream);

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

// Tuning rows: for windows up to w_max and, when samples_max > 0, batches of
// at most samples_max samples, a tile size and persistent workgroups per CU.
// The table is sorted by w_max, then by samples_max with 0 ("any batch")
// last within a w_max; a window takes the first row that matches.
struct TuneRow {
    int w_max;
    int tile;
    int groups_per_cu;
    int64_t samples_max;  // 0: any batch size
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

// The tile and groups per CU for window W in a batch of `samples` samples
// (< 0: any size).  `sized` tells whether a batch-size row chose them.
void tuned(int W, int64_t samples, int* tile, int* gpc, bool* sized = nullptr)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *tile = default_tile(W);
    *gpc = kDefaultGroupsPerCU;
    if (sized) *sized = false;
    for (const TuneRow& r : g_tune) {
        if (W > r.w_max) continue;
        if (r.samples_max > 0 && (samples < 0 || samples > r.samples_max)) continue;
        if (r.tile > 0) *tile = std::min(r.tile, max_tile(W));
        if (r.groups_per_cu > 0) *gpc = r.groups_per_cu;
        if (sized) *sized = r.samples_max > 0;
        break;
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
        if (lengths[b] >= (int64_t)INT32_MAX)
            return fail(UMI_ERR_UNSUPPORTED, "a curve of 2^31-1 samples or more");
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

// The packed curve table, written into caller-provided arrays of n_curves
// entries (`tile_of` and `order` are scratch of the same length), so that a
// caller can pack into memory it already holds.
struct PackView {
    CurveDesc* curves;        // non-empty curves, cost order
    int64_t* curve_tiles;     // tiles per table entry
    int* tile_of;             // scratch: tile size per input curve
    int32_t* order;           // scratch: input index per table entry
    int64_t ncurves = 0;      // entries written
    int64_t ntiles = 0;
    int64_t nchunks = 0;      // pre-pass chunks
    int gpc = kDefaultGroupsPerCU;  // persistent groups per CU
    int feat = kFeatAll;      // estimate-kernel paths the batch needs (kFeat* bits)
};

// Tile sizes a batch too small to give every CU a tile falls back to, largest
// first: at 512 each lane of a workgroup takes one window, at 256, 128 and 64
// two, four and eight lanes share one.
constexpr int kSmallBatchTiles[] = {1024, 512, 256, 128, 64};

umi_status pack_into(const int64_t* offsets, const int64_t* lengths, int64_t n, const int32_t* W,
                     float alpha, float c, const umi_options& o, const umi_launch& opt, int n_cu,
                     int64_t max_tiles, PackView* out)
{
    int* tile_of = out->tile_of;
    int32_t* order = out->order;
    int64_t nord = 0, samples = 0;
    for (int64_t b = 0; b < n; ++b) samples += std::max<int64_t>(lengths[b], 0);
    bool any_sized = false;
    for (int64_t b = 0; b < n; ++b) {
        int t, g;
        bool sized;
        tuned(W[b], samples, &t, &g, &sized);
        any_sized = any_sized || sized;
        if (opt.tile > 0) t = std::min(opt.tile, max_tile(W[b]));
        tile_of[b] = t;
        if (lengths[b] > 0) order[nord++] = (int32_t)b;
    }
    // A batch that the tuned tiles cut into fewer tiles than there are CUs
    // (one curve, a quiet serving step) would leave most of the chip idle:
    // smaller tiles spread its windows over more CUs, down to tiles that
    // split each window over 2, 4 or 8 lanes.  Tiles above kSplitMaxTile
    // give identical results whatever their size; split tiles agree with them
    // to rounding.  An explicit launch tile, or a tuning row for this batch
    // size, is kept as given.
    auto count_tiles = [&](int cap) {
        int64_t t = 0;
        for (int64_t i = 0; i < nord; ++i) {
            const int32_t b = order[i];
            const int tb = cap > 0 ? std::min(tile_of[b], cap) : tile_of[b];
            t += (lengths[b] + tb - 1) / tb;
        }
        return t;
    };
    if (opt.tile == 0 && !any_sized && count_tiles(0) < n_cu) {
        for (int cap : kSmallBatchTiles) {
            if (count_tiles(cap) > max_tiles) break;
            for (int64_t i = 0; i < nord; ++i) tile_of[order[i]] = std::min(tile_of[order[i]], cap);
            if (count_tiles(0) >= n_cu) break;
        }
    }
    // costliest tiles first; ties by length, then by input position (a total
    // order, so std::sort needs no scratch and the table is deterministic)
    std::sort(order, order + nord, [&](int32_t a, int32_t b) {
        const int64_t ca = (int64_t)W[a] * tile_of[a];
        const int64_t cb = (int64_t)W[b] * tile_of[b];
        if (ca != cb) return ca > cb;
        if (lengths[a] != lengths[b]) return lengths[a] > lengths[b];
        return a < b;
    });
    out->ncurves = nord;
    out->ntiles = 0;
    out->nchunks = 0;
    for (int64_t i = 0; i < nord; ++i) {
        const int32_t b = order[i];
        const int64_t nt = (lengths[b] + tile_of[b] - 1) / tile_of[b];
        const int64_t nch = (lengths[b] + kPrepChunk - 1) / kPrepChunk;
        if (out->ntiles + nt > (int64_t)INT32_MAX)
            return fail(UMI_ERR_UNSUPPORTED, "too many tiles in one batch");
        if (out->nchunks + nch > (int64_t)INT32_MAX)
            return fail(UMI_ERR_UNSUPPORTED, "too many samples in one batch");
        CurveDesc& d = out->curves[i];
        d.off = offsets[b];
        d.len = (int32_t)lengths[b];
        d.W = W[b];
        d.tile = tile_of[b];
        d.tile_base = (int32_t)out->ntiles;
        d.alpha = o.alpha ? o.alpha[b] : alpha;
        d.c = o.c ? o.c[b] : c;
        d.window_days = o.window_days ? o.window_days[b] : 0.0;
        d.chunk_base = (int32_t)out->nchunks;
        d.reserved = 0;
        out->curve_tiles[i] = nt;
        out->ntiles += nt;
        out->nchunks += nch;
    }
    // the estimate-kernel paths this batch needs
    out->feat = o.scale == UMI_SCALE_MAD ? kFeatExtra : 0;
    for (int64_t i = 0; i < nord; ++i) {
        const CurveDesc& d = out->curves[i];
        if (d.W <= kSmallW) out->feat |= kFeatSmall;
        if (d.tile <= kSplitMaxTile) out->feat |= kFeatSplit;
        if (d.window_days > 0.0) out->feat |= kFeatExtra;
    }
    out->gpc = kDefaultGroupsPerCU;
    if (nord > 0) {
        int t_unused;
        tuned(W[order[0]], samples, &t_unused, &out->gpc);  // the costliest curve's row
    }
    if (opt.groups_per_cu > 0) out->gpc = opt.groups_per_cu;
    return UMI_OK;
}

// The allocating calls' packer: the same table in vectors.
struct Packed {
    std::vector<CurveDesc> curves;
    std::vector<int64_t> curve_tiles;
    int64_t ntiles = 0;
    int64_t nchunks = 0;
    int gpc = kDefaultGroupsPerCU;
    int feat = kFeatAll;
};

umi_status pack(const int64_t* offsets, const int64_t* lengths, int64_t n, const int32_t* W,
                float alpha, float c, const umi_options& o, const umi_launch& opt, int n_cu,
                int64_t max_tiles, Packed* out)
{
    std::vector<int> tile_of((size_t)n);
    std::vector<int32_t> order((size_t)n);
    out->curves.resize((size_t)n);
    out->curve_tiles.resize((size_t)n);
    PackView v{out->curves.data(), out->curve_tiles.data(), tile_of.data(), order.data()};
    umi_status st = pack_into(offsets, lengths, n, W, alpha, c, o, opt, n_cu, max_tiles, &v);
    if (st != UMI_OK) return st;
    out->curves.resize((size_t)v.ncurves);
    out->curve_tiles.resize((size_t)v.ncurves);
    out->ntiles = v.ntiles;
    out->nchunks = v.nchunks;
    out->gpc = v.gpc;
    out->feat = v.feat;
    return UMI_OK;
}

size_t block_bytes(int64_t ncurves)
{
    return sizeof(BatchHeader) + (size_t)ncurves * sizeof(CurveDesc);
}

void write_block(uint8_t* dst, const CurveDesc* curves, int64_t ncurves, int64_t ntiles,
                 int64_t nchunks, int32_t iters, const umi_options& o, const double* time)
{
    BatchHeader h = {};
    h.n_curves = (int32_t)ncurves;
    h.n_tiles = (int32_t)ntiles;
    h.n_chunks = (int32_t)nchunks;
    h.iters = iters;
    h.scale = o.scale;
    h.detrended = o.detrended;
    h.time = time;
    std::memcpy(dst, &h, sizeof h);
    if (ncurves > 0) std::memcpy(dst + sizeof h, curves, (size_t)ncurves * sizeof(CurveDesc));
}

// ---------------------------------------------------------------------------
// device buffers of a launch sequence

// Grows `*p` to hold `need` elements.  The direct calls keep a quarter of
// slack so that batches of slowly growing size do not reallocate every call;
// a plan reserves exactly its fixed capacity once (`exact`).
template <class T>
hipError_t grow(T** p, int64_t* cap, int64_t need, bool exact = false, bool* fresh = nullptr)
{
    if (need <= *cap) return hipSuccess;
    if (fresh) *fresh = true;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return e;
    }
    int64_t n = exact ? std::max<int64_t>(need, 1) : std::max<int64_t>(need + need / 4, 1024);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), (size_t)n * sizeof(T));
    if (e == hipSuccess) *cap = n;
    return e;
}

struct DeviceBuffers {
    int32_t* segid = nullptr;   // per sample slot: the segment word of each sample
    int64_t cap_segid = 0;
    int2* tiles = nullptr;
    int64_t cap_tiles = 0;
    ChunkRec* recs = nullptr;   // pre-pass chunk records
    int64_t cap_recs = 0;
    Counters* ctr = nullptr;    // queue, ticket and epoch counters
    int64_t cap_ctr = 0;

    // Zero-filled on allocation (on `stream`, ahead of any kernel there): the
    // counters, and chunk records whose flags must not look like this epoch's.
    hipError_t reserve(int64_t span, int64_t ntiles, int64_t nchunks, hipStream_t stream,
                       bool exact = false)
    {
        hipError_t e;
        if ((e = grow(&segid, &cap_segid, span, exact)) != hipSuccess) return e;
        if ((e = grow(&tiles, &cap_tiles, ntiles, exact)) != hipSuccess) return e;
        bool fresh_recs = false, fresh_ctr = false;
        if ((e = grow(&recs, &cap_recs, nchunks, exact, &fresh_recs)) != hipSuccess) return e;
        if ((e = grow(&ctr, &cap_ctr, 1, true, &fresh_ctr)) != hipSuccess) return e;
        // a fresh counter restarts the epochs: old records must go too
        if ((fresh_recs || fresh_ctr) && cap_recs > 0 &&
            (e = hipMemsetAsync(recs, 0, (size_t)cap_recs * sizeof(ChunkRec), stream)) != hipSuccess)
            return e;
        if (fresh_ctr && (e = hipMemsetAsync(ctr, 0, sizeof(Counters), stream)) != hipSuccess)
            return e;
        return hipSuccess;
    }
    bool fits(int64_t span, int64_t ntiles, int64_t nchunks) const
    {
        return span <= cap_segid && ntiles <= cap_tiles && nchunks <= cap_recs && cap_ctr >= 1;
    }
    // device bytes held
    int64_t bytes() const
    {
        return cap_segid * (int64_t)sizeof(int32_t) + cap_tiles * (int64_t)sizeof(int2) +
               cap_recs * (int64_t)sizeof(ChunkRec) + cap_ctr * (int64_t)sizeof(Counters);
    }
    void release()
    {
        if (segid) (void)hipFree(segid);
        if (tiles) (void)hipFree(tiles);
        if (recs) (void)hipFree(recs);
        if (ctr) (void)hipFree(ctr);
        *this = DeviceBuffers();
    }
};

// The pre-pass of a batch: the curve walker (one workgroup per curve) for
// many curves, else the chunked pre-pass over at most kPrepGroupsPerCU
// workgroups per CU.
struct PrepLaunch {
    bool walk;
    int grid;
};
PrepLaunch prep_launch_for(int64_t ncurves, int64_t nchunks, int n_cu)
{
    if (ncurves >= kPrepWalkMinCurves) return {true, (int)ncurves};
    return {false, (int)std::min<int64_t>(nchunks, (int64_t)kPrepGroupsPerCU * n_cu)};
}

// Enqueue the pre-pass and estimate kernels for a staged block (header +
// curve table).  With `stage` (the device address of the pinned host block
// holding it) the pre-pass reads the block there and copies it to `dblock`
// for the estimate kernel; without, the block is at `dblock` on the device by
// the time the stream reaches the kernels (per-curve mode always).  In
// per-curve mode `table` and `curve_tiles` (host copies of the staged table,
// `ncurves` entries) give each curve's tile range and length.  `staged`, if
// given, is recorded once the pre-pass is done with the staging block.
hipError_t enqueue_kernels(const float* flux, const double* time, float* trend, float* median,
                           uint8_t* dblock, const uint8_t* stage, const DeviceBuffers& b, int mode,
                           const CurveDesc* table, const int64_t* curve_tiles, int ncurves,
                           PrepLaunch prep, int main_grid, int feat, hipEvent_t ev0,
                           hipEvent_t ev1, hipEvent_t staged, hipStream_t stream)
{
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(dblock);
    const CurveDesc* curves = reinterpret_cast<const CurveDesc*>(dblock + sizeof(BatchHeader));
    hipError_t e;
    if (mode == UMI_MODE_PERSISTENT) {
        // a lone curve's descriptor goes to the chunked pre-pass as an argument
        const CurveDesc* one = (table != nullptr && ncurves == 1 && !prep.walk) ? table : nullptr;
        if ((e = launch_prepass(flux, time, dblock, stage, -1, prep.grid, b.segid, b.tiles, b.ctr,
                                b.recs, true, prep.walk, one, stream)) != hipSuccess)
            return e;
        if (staged && (e = hipEventRecord(staged, stream)) != hipSuccess) return e;
        if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return e;
        if ((e = launch_main(flux, b.segid, hdr, curves, b.tiles, 0, -1, &b.ctr->queue, main_grid,
                             trend, median, feat, stream)) != hipSuccess)
            return e;
        if (ev1 && (e = hipEventRecord(ev1, stream)) != hipSuccess) return e;
        return hipSuccess;
    }
    // one pre-pass (the walker, one workgroup) and one estimate launch per
    // curve, one workgroup per tile
    if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return e;
    for (int i = 0; i < ncurves; ++i) {
        if ((e = launch_prepass(flux, time, dblock, nullptr, i, 1, b.segid, b.tiles, b.ctr,
                                b.recs, false, true, nullptr, stream)) != hipSuccess)
            return e;
        const int nt = (int)curve_tiles[i];
        if ((e = launch_main(flux, b.segid, hdr, curves, b.tiles, table[i].tile_base, nt, nullptr,
                             nt, trend, median, feat, stream)) != hipSuccess)
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
    uint8_t* hblock_dev = nullptr;  // hblock's device address
    int64_t cap_hblock = 0;
    hipEvent_t staged = nullptr; // last copy out of hblock
    bool staged_pending = false;

    void free_all()
    {
        buf.release();
        if (dblock) (void)hipFree(dblock);
        if (hblock) (void)hipHostFree(hblock);
        if (staged) (void)hipEventDestroy(staged);
        dblock = hblock = hblock_dev = nullptr;
        cap_dblock = cap_hblock = 0;
        staged = nullptr;
        staged_pending = false;
    }

    // Make room; if anything must be reallocated, first wait for work already
    // queued on this stream, which may still read the old buffers.
    hipError_t reserve(int64_t span, int64_t ncurves, int64_t ntiles, int64_t nchunks)
    {
        const int64_t bytes = (int64_t)block_bytes(ncurves);
        if (buf.fits(span, ntiles, nchunks) && bytes <= cap_dblock && bytes <= cap_hblock &&
            staged)
            return hipSuccess;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        staged_pending = false;
        if ((e = buf.reserve(span, ntiles, nchunks, stream)) != hipSuccess) return e;
        if ((e = grow(&dblock, &cap_dblock, bytes)) != hipSuccess) return e;
        if (bytes > cap_hblock) {
            if (hblock) (void)hipHostFree(hblock);
            hblock = hblock_dev = nullptr;
            cap_hblock = 0;
            const int64_t n = std::max<int64_t>(bytes + bytes / 4, 4096);
            e = hipHostMalloc(reinterpret_cast<void**>(&hblock), (size_t)n, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            cap_hblock = n;
            e = hipHostGetDevicePointer(reinterpret_cast<void**>(&hblock_dev), hblock, 0);
            if (e != hipSuccess) return e;
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

// Sets the calling thread's umi_last_error text (for the other host sources
// of the library) and returns `s`.
umi_status report_error(umi_status s, const std::string& msg) { return fail(s, msg); }

umi_status host_copy_many(int which, void* const* dst, const void* const* src,
                          const int64_t* bytes, int64_t n, int32_t threads);

// The copy kernel over a list of copies whose both ends are device addresses
// (pinned host memory at its device address): lists of at most kCopyMax
// copies, each one launch.  Zero-byte copies are skipped.
hipError_t enqueue_copy_list(uint8_t* const* dst, const uint8_t* const* src, const int64_t* bytes,
                             int64_t n, hipStream_t stream)
{
    CopyBatch cb;
    std::memset(&cb, 0, sizeof cb);
    int64_t pieces = 0;
    for (int64_t i = 0; i <= n; ++i) {
        const bool full = cb.n == kCopyMax ||
                          (i < n && pieces + (bytes[i] + kCopyPieceBytes - 1) / kCopyPieceBytes >
                                        (int64_t)INT32_MAX);
        if ((i == n || full) && cb.n > 0) {
            cb.first[cb.n] = (int32_t)pieces;
            const hipError_t e = launch_copy(cb, stream);
            if (e != hipSuccess) return e;
            std::memset(&cb, 0, sizeof cb);
            pieces = 0;
        }
        if (i == n) break;
        if (bytes[i] == 0) continue;
        cb.first[cb.n] = (int32_t)pieces;
        cb.src[cb.n] = src[i];
        cb.dst[cb.n] = dst[i];
        cb.bytes[cb.n] = bytes[i];
        pieces += (bytes[i] + kCopyPieceBytes - 1) / kCopyPieceBytes;
        ++cb.n;
    }
    return hipSuccess;
}

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
    if ((e = ws->reserve(span, nc, p.ntiles, p.nchunks)) != hipSuccess)
        return fail_hip(e, "workspace allocation");
    if (ws->staged_pending) {  // the previous reads of the staging block must be done
        if ((e = hipEventSynchronize(ws->staged)) != hipSuccess)
            return fail_hip(e, "hipEventSynchronize");
        ws->staged_pending = false;
    }
    write_block(ws->hblock, p.curves.data(), nc, p.ntiles, p.nchunks, iters, o, time);
    // a persistent launch's pre-pass reads the block from pinned memory and
    // copies it to the device itself; per-curve launches take a copy first
    const bool direct = opt.mode == UMI_MODE_PERSISTENT;
    if (!direct) {
        if ((e = hipMemcpyAsync(ws->dblock, ws->hblock, block_bytes(nc), hipMemcpyHostToDevice,
                                stream)) != hipSuccess)
            return fail_hip(e, "curve table copy");
        if ((e = hipEventRecord(ws->staged, stream)) != hipSuccess)
            return fail_hip(e, "hipEventRecord");
    }
    ws->staged_pending = true;
    const int grid = (int)std::min<int64_t>(p.ntiles, (int64_t)p.gpc * cu_count(device));
    e = enqueue_kernels(flux, time, trend, median, ws->dblock, direct ? ws->hblock_dev : nullptr,
                        ws->buf, opt.mode, p.curves.data(), p.curve_tiles.data(), (int)nc,
                        prep_launch_for(nc, p.nchunks, cu_count(device)), grid, p.feat,
                        (hipEvent_t)opt.main_start, (hipEvent_t)opt.main_stop,
                        direct ? ws->staged : nullptr, stream);
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

// Pool 0 serves umi_host_copy_many; pool 1 the serving loop's result copies,
// which run on another thread than its staging copies and must not wait for
// them.
CopyPool& copy_pool(int which = 0)
{
    static CopyPool* pools[2] = {new CopyPool(), new CopyPool()};  // intentionally never freed
    return *pools[which & 1];
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
    int64_t max_chunks = 0;
    int32_t max_W = 0;
    const float* flux = nullptr;
    const double* time = nullptr;
    float* trend = nullptr;
    float* median = nullptr;
    int main_grid = 0;
    umi::DeviceBuffers buf;
    // Two captured graphs per slot: [0] for batches of at most
    // kPrepSmallChunks pre-pass chunks (the chunked pre-pass over that many
    // workgroups), [1] for any batch (the curve walker over max_curves
    // workgroups).  Either pre-pass reads the slot's pinned block and copies
    // it to the slot's device block for the estimate kernel.
    struct Slot {
        uint8_t* host = nullptr;    // pinned header + curve table
        uint8_t* host_dev = nullptr;  // its device address
        uint8_t* dev = nullptr;     // its device copy
        hipGraph_t graph[2] = {nullptr, nullptr};
        hipGraphExec_t exec[2] = {nullptr, nullptr};
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
        for (int k = 0; k < 2; ++k) {
            if (s.exec[k]) (void)hipGraphExecDestroy(s.exec[k]);
            if (s.graph[k]) (void)hipGraphDestroy(s.graph[k]);
        }
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        s = umi_plan::Slot();
    }
    p->buf.release();
}

// Curves the staged table of a graph kind holds, and that kind's pre-pass:
// kind 0 serves batches of at most kPrepSmallChunks chunks with the chunked
// pre-pass over that many workgroups (each curve has a chunk, so the table
// holds at most that many curves); kind 1 any batch, with the curve walker,
// one workgroup per possible curve.
int64_t plan_kind_curves(const umi_plan* p, int kind)
{
    return kind == 0 ? std::min<int64_t>(p->max_curves, umi::kPrepSmallChunks) : p->max_curves;
}

umi::PrepLaunch plan_kind_prep(const umi_plan* p, int kind)
{
    return kind == 0 ? umi::PrepLaunch{false, umi::kPrepSmallChunks}
                     : umi::PrepLaunch{true, (int)p->max_curves};
}

// Capture slot `si`'s graph of `kind`: the pre-pass (which reads the staged
// block from pinned memory and copies it to the device) and the persistent
// estimate kernel.  Nothing runs during capture.
hipError_t plan_capture(umi_plan* p, int si, int kind)
{
    umi_plan::Slot& s = p->slot[si];
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ce = umi::enqueue_kernels(
        p->flux, p->time, p->trend, p->median, s.dev, s.host_dev, p->buf, UMI_MODE_PERSISTENT,
        nullptr, nullptr, (int)plan_kind_curves(p, kind), plan_kind_prep(p, kind), p->main_grid,
        umi::kFeatAll, nullptr, nullptr, nullptr, p->stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->stream, &g);
    if (ce != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ce != hipSuccess ? ce : e;
    }
    s.graph[kind] = g;
    if ((e = hipGraphInstantiate(&s.exec[kind], g, nullptr, nullptr, 0)) != hipSuccess) {
        s.exec[kind] = nullptr;
        return e;
    }
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// The allocation-free batch call (umi_detrend_batch_noalloc): the workspace
// of a batch -- header and curve table, queue counter, tile list, segment
// words -- lives in one file-scope device array, and the host side packs into
// static arrays.  Nothing is allocated per call, on the device or the host.

namespace umi {
namespace noalloc {

constexpr int64_t kMaxSamples = UMI_NOALLOC_MAX_SAMPLES;
constexpr int64_t kMaxCurves = UMI_NOALLOC_MAX_CURVES;
constexpr int64_t kMaxTiles = UMI_NOALLOC_MAX_TILES;
// every curve adds at most one partial chunk
constexpr int64_t kMaxChunks = kMaxSamples / kPrepChunk + kMaxCurves;
constexpr size_t kAlign = 256;
constexpr size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// byte offsets inside the scratch array
constexpr size_t kBlockOff = 0;  // BatchHeader + curve table
constexpr size_t kCounterOff = round_up(sizeof(BatchHeader) + kMaxCurves * sizeof(CurveDesc));
constexpr size_t kRecsOff = kCounterOff + kAlign;
constexpr size_t kTilesOff = round_up(kRecsOff + kMaxChunks * sizeof(ChunkRec));
constexpr size_t kSegidOff = round_up(kTilesOff + kMaxTiles * sizeof(int2));
constexpr size_t kScratchBytes = kSegidOff + kMaxSamples * sizeof(int32_t);
static_assert(kScratchBytes == UMI_NOALLOC_SCRATCH_BYTES, "scratch size in umi.h");

constexpr int kMaxDevices = 64;

}  // namespace noalloc
}  // namespace umi

// Each GPU the library runs on holds its own copy of this array for the life
// of the process.  Its name is a host-side stand-in: host code uses only the
// device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[umi::noalloc::kScratchBytes];

namespace umi {
namespace noalloc {

std::mutex g_mu;                      // guards everything below
uint8_t* g_dev_scratch[kMaxDevices];  // device address of `scratch` per device
// host-side packing arrays (no allocation per call)
int64_t g_off[kMaxCurves];
CurveDesc g_curves[kMaxCurves];
int64_t g_curve_tiles[kMaxCurves];
int g_tile_of[kMaxCurves];
int32_t g_order[kMaxCurves];
alignas(16) uint8_t g_block[kCounterOff];

// The device address of `scratch` on `device` (current), looked up once.
hipError_t scratch_for(int device, uint8_t** out)
{
    if (!g_dev_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_dev_scratch[device] = static_cast<uint8_t*>(ptr);
    }
    *out = g_dev_scratch[device];
    return hipSuccess;
}

umi_status detrend_batch(const float* flux, const double* time, const int64_t* lengths,
                         int64_t n_curves, const int32_t* W, float alpha, float c, int32_t iters,
                         float* trend, float* median, const umi_launch* launch,
                         hipStream_t stream)
{
    umi_status st;
    if (take_injected(&st)) return st;
    if (n_curves < 0) return fail(UMI_ERR_INVALID_ARG, "n_curves must be >= 0");
    if (n_curves == 0) return UMI_OK;
    if (!lengths || !W) return fail(UMI_ERR_INVALID_ARG, "lengths and W must not be NULL");
    if (n_curves > kMaxCurves)
        return fail(UMI_ERR_UNSUPPORTED,
                    "umi_detrend_batch_noalloc: more than UMI_NOALLOC_MAX_CURVES curves");
    umi_launch opt;
    if ((st = check_launch(launch, &opt)) != UMI_OK) return st;
    if ((st = check_params(alpha, c, iters)) != UMI_OK) return st;
    int64_t total = 0;
    for (int64_t b = 0; b < n_curves; ++b) {
        if (lengths[b] < 0) return fail(UMI_ERR_INVALID_ARG, "curve lengths must be >= 0");
        if ((st = check_window(W[b])) != UMI_OK) return st;
        if (lengths[b] > kMaxSamples - total)
            return fail(UMI_ERR_UNSUPPORTED,
                        "umi_detrend_batch_noalloc: more than UMI_NOALLOC_MAX_SAMPLES samples");
        total += lengths[b];
    }
    if (total == 0) return UMI_OK;
    if (!flux || !trend) return fail(UMI_ERR_INVALID_ARG, "flux and trend must not be NULL");

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (device < 0 || device >= kMaxDevices)
        return fail(UMI_ERR_UNSUPPORTED, "umi_detrend_batch_noalloc: device index above 63");
    const int n_cu = cu_count(device);

    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base = nullptr;
    if ((e = scratch_for(device, &base)) != hipSuccess)
        return fail_hip(e, "hipGetSymbolAddress(scratch)");
    int64_t acc = 0;
    for (int64_t b = 0; b < n_curves; ++b) {
        g_off[b] = acc;
        acc += lengths[b];
    }
    const umi_options o{nullptr, nullptr, UMI_SCALE_UPPER_RMS, 0, nullptr, nullptr};
    PackView v{g_curves, g_curve_tiles, g_tile_of, g_order};
    if ((st = pack_into(g_off, lengths, n_curves, W, alpha, c, o, opt, n_cu, kMaxTiles, &v)) !=
        UMI_OK)
        return st;
    if (v.ntiles > kMaxTiles)
        return fail(UMI_ERR_UNSUPPORTED,
                    "umi_detrend_batch_noalloc: the batch needs more than UMI_NOALLOC_MAX_TILES "
                    "tiles (very wide windows cut curves into small tiles)");
    if (v.nchunks > kMaxChunks) return fail(UMI_ERR_UNSUPPORTED, "chunk count above its bound");
    write_block(g_block, g_curves, v.ncurves, v.ntiles, v.nchunks, iters, o, time);
    // from pageable host memory: the source is free again once the call returns
    if ((e = hipMemcpyAsync(base + kBlockOff, g_block, block_bytes(v.ncurves),
                            hipMemcpyHostToDevice, stream)) != hipSuccess)
        return fail_hip(e, "curve table copy");
    DeviceBuffers b;  // a view of the scratch array; never released
    b.segid = reinterpret_cast<int32_t*>(base + kSegidOff);
    b.cap_segid = kMaxSamples;
    b.tiles = reinterpret_cast<int2*>(base + kTilesOff);
    b.cap_tiles = kMaxTiles;
    b.ctr = reinterpret_cast<Counters*>(base + kCounterOff);  // zero from the module load
    b.cap_ctr = 1;
    b.recs = reinterpret_cast<ChunkRec*>(base + kRecsOff);
    b.cap_recs = kMaxChunks;
    const int grid = (int)std::min<int64_t>(v.ntiles, (int64_t)v.gpc * n_cu);
    e = enqueue_kernels(flux, time, trend, median, base + kBlockOff, nullptr, b, opt.mode,
                        g_curves, g_curve_tiles, (int)v.ncurves,
                        prep_launch_for(v.ncurves, v.nchunks, n_cu), grid, v.feat,
                        (hipEvent_t)opt.main_start, (hipEvent_t)opt.main_stop, nullptr, stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return UMI_OK;
}

}  // namespace noalloc
}  // namespace umi

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

umi_status umi_detrend_batch_noalloc(const float* flux, const double* time,
                                     const int64_t* lengths, int64_t n_curves, const int32_t* W,
                                     float alpha, float c, int32_t iters, float* trend,
                                     float* median, const umi_launch* launch, void* stream)
{
    return umi::noalloc::detrend_batch(flux, time, lengths, n_curves, W, alpha, c, iters, trend,
                                       median, launch, static_cast<hipStream_t>(stream));
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
    int device = 0;
    hipError_t de = hipGetDevice(&device);
    if (de != hipSuccess) return umi::fail_hip(de, "hipGetDevice");
    const int64_t n_cu = umi::cu_count(device);
    // Tiles the plan must hold: the whole capacity at the smallest tile any
    // W <= max_W takes for batches of any size; batches at most samples_max
    // long at their batch-size rows' tiles; and the small-batch rule, which
    // only halves tiles while a batch has fewer tiles than CUs, so it never
    // needs more than 2 n_cu + max_curves.  With room for all of these, a run
    // is cut exactly as the direct calls cut the same batch.
    int64_t min_tile = std::min(umi::max_tile(max_W), umi::default_tile(max_W));
    int64_t sized_tiles = 0;
    {
        std::lock_guard<std::mutex> lk(umi::g_tune_mu);
        for (const umi::TuneRow& r : umi::g_tune) {
            if (r.tile <= 0) continue;
            const int64_t t = std::min<int64_t>(r.tile, umi::max_tile(std::min(r.w_max, (int)max_W)));
            if (r.samples_max == 0)
                min_tile = std::min<int64_t>(min_tile, t);
            else
                sized_tiles = std::max(sized_tiles, std::min(r.samples_max, capacity) / t + 1);
        }
    }
    const int64_t max_tiles = std::max(capacity / std::max<int64_t>(1, min_tile),
                                       std::max(sized_tiles, 2 * n_cu)) + max_curves;
    if (max_tiles > (int64_t)INT32_MAX)
        return umi::fail(UMI_ERR_UNSUPPORTED, "plan capacity needs too many tiles");
    // every curve adds at most one partial chunk
    const int64_t max_chunks = capacity / umi::kPrepChunk + max_curves;
    if (max_chunks > (int64_t)INT32_MAX)
        return umi::fail(UMI_ERR_UNSUPPORTED, "plan capacity needs too many pre-pass chunks");
    umi_plan* p = new umi_plan();
    p->device = device;
    p->stream = static_cast<hipStream_t>(stream);
    p->capacity = capacity;
    p->max_curves = max_curves;
    p->max_tiles = max_tiles;
    p->max_chunks = max_chunks;
    p->max_W = max_W;
    p->flux = flux;
    p->time = time;
    p->trend = trend;
    p->median = median;
    hipError_t e = p->buf.reserve(capacity, max_tiles, max_chunks, p->stream, /*exact=*/true);
    const size_t bytes = umi::block_bytes(max_curves);
    for (auto& s : p->slot) {
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&s.host), bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s.host_dev), s.host, 0);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.dev), bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) std::memset(s.host, 0, bytes);
    }
    // the workspace's zero fill is done before anything is captured
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        plan_free(p);
        delete p;
        return umi::fail_hip(e, "plan allocation");
    }
    int t_unused, gpc;
    umi::tuned(max_W, -1, &t_unused, &gpc);
    p->main_grid = gpc * umi::cu_count(p->device);
    // every slot's graphs of both kinds, now rather than on a serving step
    for (int si = 0; si < 2 && e == hipSuccess; ++si)
        for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) e = plan_capture(p, si, kind);
    if (e != hipSuccess) {
        plan_free(p);
        delete p;
        return umi::fail_hip(e, "graph capture");
    }
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
    if (pk.nchunks > p->max_chunks)
        return umi::fail(UMI_ERR_UNSUPPORTED, "batch needs more chunks than the plan holds");

    std::lock_guard<std::mutex> lk(p->mu);
    umi_plan::Slot& s = p->slot[p->next];
    hipError_t e;
    if (s.pending) {  // this slot's previous replay must have consumed its bytes
        if ((e = hipEventSynchronize(s.done)) != hipSuccess)
            return umi::fail_hip(e, "hipEventSynchronize");
        s.pending = false;
    }
    umi::write_block(s.host, pk.curves.data(), (int64_t)pk.curves.size(), pk.ntiles, pk.nchunks,
                     iters, o, p->time);
    // small batches (at most kPrepSmallChunks chunks) replay kind 0
    const int kind = pk.nchunks <= umi::kPrepSmallChunks ? 0 : 1;
    if (!s.exec[kind] && (e = plan_capture(p, p->next, kind)) != hipSuccess)
        return umi::fail_hip(e, "graph capture");
    if ((e = hipGraphLaunch(s.exec[kind], p->stream)) != hipSuccess)
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
            r.samples_max = 0;
            if (!(ls >> r.w_max >> r.tile >> r.groups_per_cu) || r.w_max < 1 || r.tile < 0 ||
                r.groups_per_cu < 0 || r.groups_per_cu > 64)
                return umi::fail(UMI_ERR_INVALID_ARG, "malformed tuning line: " + line);
            std::string extra;
            if (ls >> extra) {  // optional fourth column: batch samples bound
                char* end = nullptr;
                const long long v = std::strtoll(extra.c_str(), &end, 10);
                std::string more;
                if (end == extra.c_str() || *end != '\0' || v < 0 || (ls >> more))
                    return umi::fail(UMI_ERR_INVALID_ARG, "malformed tuning line: " + line);
                r.samples_max = v;
            }
            rows.push_back(r);
        }
        auto after = [](const umi::TuneRow& a, const umi::TuneRow& b) {
            // b may follow a: larger w_max, or the same w_max with a larger
            // batch bound (0, any size, last)
            if (b.w_max != a.w_max) return b.w_max > a.w_max;
            if (a.samples_max == 0) return false;
            return b.samples_max == 0 || b.samples_max > a.samples_max;
        };
        for (size_t i = 1; i < rows.size(); ++i)
            if (!after(rows[i - 1], rows[i]))
                return umi::fail(UMI_ERR_INVALID_ARG,
                                 "tuning rows must be sorted by W_max, then by batch samples "
                                 "(0 = any size, last)");
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

const char* umi_version(void) { return "umi-mi355x 0.8.5"; }

void umi_debug_inject_error(umi_status s) { umi::t_inject = s; }

umi_status umi_host_copy_many(void* const* dst, const void* const* src, const int64_t* bytes,
                              int64_t n, int32_t threads)
{
    return umi::host_copy_many(0, dst, src, bytes, n, threads);
}

}  // extern "C"

namespace umi {

// umi_host_copy_many on copy pool `which` (0 or 1).
umi_status host_copy_many(int which, void* const* dst, const void* const* src,
                          const int64_t* bytes, int64_t n, int32_t threads)
{
    if (n < 0) return fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: n < 0");
    if (threads < 1 || threads > UMI_HOST_COPY_MAX_THREADS)
        return fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: threads out of range");
    if (n == 0) return UMI_OK;
    if (!dst || !src || !bytes)
        return fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: NULL array");
    CopyJob job;
    job.dst = dst;
    job.src = src;
    job.bytes = bytes;
    job.first.resize(size_t(n) + 1);
    int64_t pieces = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (bytes[i] < 0) return fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: bytes < 0");
        if (bytes[i] > 0 && (!dst[i] || !src[i]))
            return fail(UMI_ERR_INVALID_ARG, "umi_host_copy_many: NULL pointer");
        job.first[size_t(i)] = pieces;
        pieces += (bytes[i] + kCopyPiece - 1) / kCopyPiece;
    }
    job.first[size_t(n)] = pieces;
    if (pieces == 0) return UMI_OK;
    const int64_t useful = std::min<int64_t>(threads, pieces);
    if (useful <= 1) {
        job.work();
        return UMI_OK;
    }
    copy_pool(which).run(job, int(useful));
    return UMI_OK;
}

}  // namespace umi

extern "C" {

umi_status umi_copy_async(void* const* dst, const void* const* src, const int64_t* bytes,
                          int64_t n, int32_t kind, void* stream)
{
    if (n < 0) return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: n < 0");
    const bool by_kernel = (kind & UMI_COPY_KERNEL) != 0;
    kind &= ~UMI_COPY_KERNEL;
    if (kind != UMI_COPY_H2D && kind != UMI_COPY_D2H)
        return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: unknown kind");
    if (n == 0) return UMI_OK;
    if (!dst || !src || !bytes) return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: NULL array");
    for (int64_t i = 0; i < n; ++i) {
        if (bytes[i] < 0) return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: bytes < 0");
        if (bytes[i] > 0 && (!dst[i] || !src[i]))
            return umi::fail(UMI_ERR_INVALID_ARG, "umi_copy_async: NULL pointer");
    }
    if (by_kernel) {
        // every host range must be pinned host memory the device can reach:
        // the copy kernel reads and writes it at its device address
        std::vector<void*> hdev((size_t)n, nullptr);
        for (int64_t i = 0; i < n; ++i) {
            if (bytes[i] == 0) continue;
            char* h = static_cast<char*>(kind == UMI_COPY_H2D ? const_cast<void*>(src[i]) : dst[i]);
            for (int end = 0; end < 2; ++end) {
                char* q = end ? h + bytes[i] - 1 : h;
                hipPointerAttribute_t a;
                const hipError_t e = hipPointerGetAttributes(&a, q);
                if (e != hipSuccess) (void)hipGetLastError();  // not sticky for later calls
                if (e != hipSuccess || a.type != hipMemoryTypeHost || !a.devicePointer ||
                    !a.hostPointer)
                    return umi::fail(UMI_ERR_INVALID_ARG,
                                     "umi_copy_async: with UMI_COPY_KERNEL the host side of every "
                                     "copy must be pinned host memory (hipHostMalloc)");
                if (!end)
                    hdev[(size_t)i] = static_cast<char*>(a.devicePointer) +
                                      (q - static_cast<char*>(a.hostPointer));
            }
        }
        // both ends at device addresses, then lists of the copy kernel
        std::vector<uint8_t*> d((size_t)n);
        std::vector<const uint8_t*> sr((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            sr[(size_t)i] = static_cast<const uint8_t*>(kind == UMI_COPY_H2D ? hdev[(size_t)i] : src[i]);
            d[(size_t)i] = static_cast<uint8_t*>(kind == UMI_COPY_D2H ? hdev[(size_t)i] : dst[i]);
        }
        const hipError_t e = umi::enqueue_copy_list(d.data(), sr.data(), bytes, n,
                                                    static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return umi::fail_hip(e, "umi_copy_async: copy kernel");
        return UMI_OK;
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
