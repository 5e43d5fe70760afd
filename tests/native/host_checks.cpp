// Sanitizer driver for the library's host code (test infrastructure).
//
// Built with g++ against the host-only HIP stand-in (tests/native/fake_hip),
// together with the host source itself, and run under AddressSanitizer +
// UndefinedBehaviorSanitizer or ThreadSanitizer.  The kernel launch wrappers
// are replaced by checkers that read what the host staged for the kernels
// (batch header, curve table) and touch every sample, segment word and tile
// slot a launch may touch, so a packer or workspace that under-sizes
// anything, or an offset outside the caller's arrays, is an out-of-bounds
// access the sanitizer reports.  Exercised: argument checks, the tuning
// table, direct batches (packed and gathered, with options and explicit
// launches), plans (create / run / destroy, both graph kinds, whose captured
// launches the stand-in replays), the allocation-free batch call, the host
// copy pool from several threads at once, the native serving loop (requests
// from several threads, oversize requests, a failing step), and
// umi_release.  The stand-in estimate kernel writes flux + W at every output
// position, so results show that each curve's samples and window reached
// the right place.  Prints "host checks ok" and exits 0 on success.  An
// optional argument sets the number of random batches per pass.
#include "umi_host.hip"
#include "umi_server.hip"

#include <random>
#include <thread>

namespace {

std::atomic<int> g_failures{0};
std::atomic<long> g_prepass{0}, g_main{0};
std::atomic<int> g_fail_W{0};  // the estimate kernel fails for curves of this W

#define CHECK(cond)                                                               \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++g_failures;                                                         \
        }                                                                         \
    } while (0)

}  // namespace

namespace umi {

// The pre-pass: chunk g of the launch maps to its curve as in the kernel (the
// last table entry whose first chunk is <= g, or the launch's one curve);
// every chunk reads its flux and time, writes its segment words, its chunk
// record and the tiles that start in it (what the kernel writes), and the
// counters come back to zero with the launch count advanced.
hipError_t prepass_now(const float* flux, const double* time, uint8_t* block,
                       const uint8_t* stage, int curve_one, int grid, int32_t* segid,
                       int2* tiles, Counters* ctr, ChunkRec* recs, bool clear_queue, bool walk)
{
    ++g_prepass;
    // with a staging block, the header and table come from there and are
    // copied to the device block (what the kernels do)
    if (stage) {
        const int nc = reinterpret_cast<const BatchHeader*>(stage)->n_curves;
        CHECK(nc >= 0);
        std::memcpy(block, stage, sizeof(BatchHeader) + (size_t)nc * sizeof(CurveDesc));
    }
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(block);
    const CurveDesc* curves = reinterpret_cast<const CurveDesc*>(block + sizeof(BatchHeader));
    CHECK(grid >= 1);
    if (walk && curve_one < 0) CHECK(grid >= hdr->n_curves);  // a workgroup per curve
    if (walk && curve_one >= 0) CHECK(grid == 1);
    CHECK(hdr->n_curves >= 0 && hdr->n_tiles >= 0 && hdr->n_chunks >= 0);
    CHECK(ctr->tickets == 0u && ctr->done == 0u);
    if (clear_queue) ctr->queue = 0u;
    if (curve_one < 0) {
        int64_t next = 0;
        for (int c = 0; c < hdr->n_curves; ++c) {
            CHECK(curves[c].chunk_base == next);
            next += (curves[c].len + kPrepChunk - 1) / kPrepChunk;
        }
        CHECK(next == hdr->n_chunks);
    } else {
        CHECK(curve_one < hdr->n_curves);
    }
    const int n_chunks = curve_one >= 0 ? (curves[curve_one].len + kPrepChunk - 1) / kPrepChunk
                                        : hdr->n_chunks;
    for (int g = 0; g < n_chunks; ++g) {
        int ci = curve_one;
        if (ci < 0) {
            ci = 0;
            while (ci + 1 < hdr->n_curves && curves[ci + 1].chunk_base <= g) ++ci;
        }
        const CurveDesc& cd = curves[ci];
        CHECK(cd.len > 0 && cd.W >= 1 && (cd.W & 1) == 1 && cd.tile >= 1);
        CHECK(cd.tile <= kMaxTile && cd.tile + cd.W - 1 <= kStageMax);
        const int nt = (cd.len + cd.tile - 1) / cd.tile;
        CHECK(cd.tile_base >= 0 && cd.tile_base + nt <= hdr->n_tiles);
        const int g0 = curve_one >= 0 ? 0 : cd.chunk_base;
        const int lo = (g - g0) * kPrepChunk, hi = std::min(lo + kPrepChunk, cd.len);
        CHECK(lo >= 0 && lo < cd.len);
        for (int i = 0; i < kSegWords; ++i) {
            recs[g].agg[i] = (ctr->epoch + 1) << 32 | (uint32_t)(hi - lo);
            recs[g].inc[i] = (ctr->epoch + 1) << 32 | (uint32_t)hi;
        }
        for (int t = (lo + cd.tile - 1) / cd.tile; t * cd.tile < hi; ++t)
            tiles[cd.tile_base + t] = make_int2(ci, t * cd.tile);
        volatile float fs = 0.0f;
        volatile double ts = 0.0;
        for (int i = lo; i < hi; ++i) {
            fs = fs + flux[cd.off + i];
            if (time) ts = ts + time[cd.off + i];
            segid[cd.off + i] = -1;
        }
        if (hdr->detrended)
            for (int i = lo; i < hi; ++i) hdr->detrended[cd.off + i] = 0.0f;
        if (hdr->time) CHECK(hdr->time == time);
    }
    ctr->epoch += 1;
    return hipSuccess;
}

hipError_t launch_prepass(const float* flux, const double* time, uint8_t* block,
                          const uint8_t* stage, int curve_one, int grid, int32_t* segid,
                          int2* tiles, Counters* ctr, ChunkRec* recs, bool clear_queue, bool walk,
                          const CurveDesc* one, hipStream_t)
{
    if (curve_one >= 0) CHECK(stage == nullptr);  // per-curve launches copy the block first
    if (one != nullptr) {
        // a lone curve's entry, for the chunked form, equal to the staged one
        CHECK(curve_one < 0 && !walk);
        const uint8_t* src = stage ? stage : block;
        CHECK(reinterpret_cast<const BatchHeader*>(src)->n_curves == 1);
        CHECK(std::memcmp(one, src + sizeof(BatchHeader), sizeof(CurveDesc)) == 0);
    }
    return fake_hip::record_or_run([=] {
        return prepass_now(flux, time, block, stage, curve_one, grid, segid, tiles, ctr, recs,
                           clear_queue, walk);
    });
}

// The copy kernel: each copy of the list is done in full, and the pieces
// count matches the sizes.
hipError_t launch_copy(const CopyBatch& cb, hipStream_t)
{
    return fake_hip::record_or_run([cb] {
        CHECK(cb.n >= 1 && cb.n <= kCopyMax);
        for (int i = 0; i < cb.n; ++i) {
            CHECK(cb.first[i + 1] - cb.first[i] ==
                  (cb.bytes[i] + kCopyPieceBytes - 1) / kCopyPieceBytes);
            std::memcpy(cb.dst[i], cb.src[i], (size_t)cb.bytes[i]);
        }
        return hipSuccess;
    });
}

// The estimate kernel: every tile of its range lies in its curve, its
// staged span fits the workgroup, and the outputs of its positions exist.
hipError_t main_now(const float* flux, const int32_t* segid, const BatchHeader* hdr,
                    const CurveDesc* curves, const int2* tiles, int tile_first, int tile_count,
                    uint32_t* counter, int grid, float* trend, float* median, int feat)
{
    ++g_main;
    CHECK(grid >= 1);
    const int end = tile_count < 0 ? hdr->n_tiles : tile_first + tile_count;
    CHECK(end <= hdr->n_tiles);
    if (counter) CHECK(*counter == 0u);
    for (int t = tile_first; t < end; ++t) {
        const int2 td = tiles[t];
        CHECK(td.x >= 0 && td.x < hdr->n_curves);
        const CurveDesc& cd = curves[td.x];
        const int h = (cd.W - 1) / 2;
        const int t0 = td.y, t1 = std::min(t0 + cd.tile, cd.len);
        CHECK(t0 >= 0 && t0 < cd.len && t0 % cd.tile == 0);
        const int s0 = std::max(t0 - h, 0), s1 = std::min(t1 + h, cd.len);
        CHECK(s1 - s0 <= kStageMax);
        // an instance without a path serves no tile that needs it
        if (!(feat & kFeatSmall)) CHECK(cd.W > kSmallW);
        if (!(feat & kFeatSplit)) CHECK(cd.tile > kSplitMaxTile);
        if (!(feat & kFeatExtra)) CHECK(cd.window_days == 0.0 && hdr->scale == UMI_SCALE_UPPER_RMS);
        CHECK(split_lanes(cd.tile) * std::min(cd.tile, kMainThreads) <= kMainThreads ||
              split_lanes(cd.tile) == 1);
        if (cd.W == g_fail_W.load()) return hipErrorLaunchFailure;
        volatile float fs = 0.0f;
        for (int i = s0; i < s1; ++i) fs = fs + flux[cd.off + i] + (float)segid[cd.off + i];
        for (int p = t0; p < t1; ++p) {
            trend[cd.off + p] = flux[cd.off + p] + (float)cd.W;
            if (median) median[cd.off + p] = 1.0f;
        }
    }
    return hipSuccess;
}

hipError_t launch_main(const float* flux, const int32_t* segid, const BatchHeader* hdr,
                       const CurveDesc* curves, const int2* tiles, int tile_first,
                       int tile_count, uint32_t* counter, int grid, float* trend, float* median,
                       int feat, hipStream_t)
{
    return fake_hip::record_or_run([=] {
        return main_now(flux, segid, hdr, curves, tiles, tile_first, tile_count, counter, grid,
                        trend, median, feat);
    });
}

}  // namespace umi

namespace {

std::mt19937_64 rng(2604066020ull);

int64_t uni(int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); }

struct DevArrays {
    float* flux = nullptr;
    double* time = nullptr;
    float* trend = nullptr;
    float* median = nullptr;
    float* det = nullptr;
    explicit DevArrays(int64_t n)
    {
        void* p;
        hipMalloc(&p, sizeof(float) * (size_t)n); flux = (float*)p;
        hipMalloc(&p, sizeof(double) * (size_t)n); time = (double*)p;
        hipMalloc(&p, sizeof(float) * (size_t)n); trend = (float*)p;
        hipMalloc(&p, sizeof(float) * (size_t)n); median = (float*)p;
        hipMalloc(&p, sizeof(float) * (size_t)n); det = (float*)p;
        for (int64_t i = 0; i < n; ++i) {
            flux[i] = 1.0f;
            time[i] = (double)i / 720.0;
        }
    }
    ~DevArrays()
    {
        hipFree(flux); hipFree(time); hipFree(trend); hipFree(median); hipFree(det);
    }
};

int32_t odd_w(int64_t max_w) { return (int32_t)(uni(0, (max_w - 1) / 2) * 2 + 1); }

void check_tuning()
{
    CHECK(umi_set_tuning("31 2000 4\n127 1500 3\n2047 0 0\n") == UMI_OK);
    CHECK(umi_set_tuning("31 64 4 40000\n31 512 4 160000\n31 1536 4\n2047 128 4 9000\n2047 0 4\n") == UMI_OK);
    CHECK(umi_set_tuning("31 10 2\n31 10 2 50") == UMI_ERR_INVALID_ARG);
    CHECK(umi_set_tuning("127 1 2\n31 1 2") == UMI_ERR_INVALID_ARG);
    CHECK(umi_set_tuning("x") == UMI_ERR_INVALID_ARG);
}

int g_rounds = 300;  // batches per pass (the thread-sanitizer run takes fewer)

void check_direct_batches()
{
    for (int round = 0; round < g_rounds; ++round) {
        const int64_t n = uni(0, 40);
        std::vector<int64_t> len((size_t)n), off((size_t)n);
        std::vector<int32_t> W((size_t)n);
        std::vector<float> al((size_t)n), cc((size_t)n);
        std::vector<double> wd((size_t)n);
        int64_t total = 0;
        for (int64_t b = 0; b < n; ++b) {
            const int kind = (int)uni(0, 9);
            len[b] = kind == 0 ? 0 : (kind == 1 ? uni(1, 5) : uni(1, 60000));
            W[b] = odd_w(uni(0, 3) == 0 ? UMI_MAX_WINDOW : 721);
            al[b] = (float)uni(1, 10);
            cc[b] = (float)uni(1, 5);
            wd[b] = uni(0, 3) == 0 ? 0.5 : 0.0;
            total += len[b];
        }
        const bool gather = uni(0, 1) == 1;
        int64_t span = 0;
        for (int64_t b = 0; b < n; ++b) {  // packed, or gathered with gaps in between
            off[b] = span + (gather ? uni(0, 1000) : 0);
            span = off[b] + len[b];
        }
        DevArrays a(std::max<int64_t>(span, 1));
        umi_launch lo = {UMI_MODE_PERSISTENT, 0, 0, 0, nullptr, nullptr};
        const int lk = (int)uni(0, 5);
        if (lk == 1) lo.tile = (int32_t)uni(1, 3000);
        if (lk == 2) lo.mode = UMI_MODE_PER_CURVE;
        if (lk == 3) lo.groups_per_cu = (int32_t)uni(1, 8);
        if (lk == 4) lo.tile = (int32_t)(uni(0, 1) ? 64 : 256);
        umi_options o = {uni(0, 1) ? al.data() : nullptr, uni(0, 1) ? cc.data() : nullptr,
                         (int32_t)uni(0, 1), 0, uni(0, 1) ? a.det : nullptr,
                         uni(0, 1) ? wd.data() : nullptr};
        umi_status st;
        if (gather)
            st = umi_detrend_gather_ex(a.flux, a.time, off.data(), len.data(), n, W.data(), 2.0f,
                                       5.0f, 5, a.trend, uni(0, 1) ? a.median : nullptr, &o, &lo,
                                       nullptr);
        else
            st = umi_detrend_batch(a.flux, uni(0, 3) ? a.time : nullptr, len.data(), n, W.data(),
                                   2.0f, 5.0f, 5, a.trend, a.median, &lo, nullptr);
        CHECK(st == UMI_OK);
        if (st != UMI_OK) std::fprintf(stderr, "  %s\n", umi_last_error());
        // invalid arguments are refused before anything is enqueued
        if (n > 0) {
            std::vector<int32_t> Wbad = W;
            Wbad[0] = 4;
            const long before = g_prepass;
            CHECK(umi_detrend_batch(a.flux, a.time, len.data(), n, Wbad.data(), 2.0f, 5.0f, 5,
                                    a.trend, nullptr, nullptr, nullptr) == UMI_ERR_INVALID_ARG);
            CHECK(g_prepass == before);
        }
        (void)total;
    }
}

void check_plans()
{
    for (int round = 0; round < std::max(2, g_rounds / 15); ++round) {
        const int64_t cap = uni(1000, 400000);
        const int64_t max_curves = uni(1, 100);
        const int32_t max_w = odd_w(721);
        DevArrays a(cap);
        umi_plan* p = nullptr;
        CHECK(umi_plan_create(&p, cap, max_curves, max_w, a.flux, a.time, a.trend, a.median,
                              reinterpret_cast<void*>(uintptr_t(0x1000))) == UMI_OK);
        if (!p) continue;
        for (int run = 0; run < 30; ++run) {
            const int64_t n = uni(0, max_curves);
            std::vector<int64_t> len((size_t)n), off((size_t)n);
            std::vector<int32_t> W((size_t)n);
            int64_t pos = 0;
            bool fits = true;
            for (int64_t b = 0; b < n; ++b) {
                len[b] = uni(0, std::max<int64_t>(1, cap / std::max<int64_t>(n, 1)));
                off[b] = pos + uni(0, 3);
                pos = off[b] + len[b];
                W[b] = odd_w(max_w);
            }
            if (pos > cap) fits = false;
            const umi_status st = umi_plan_run(p, off.data(), len.data(), W.data(), n, 2.0f, 5.0f, 5);
            if (fits) {
                CHECK(st == UMI_OK);
                if (st != UMI_OK) std::fprintf(stderr, "  plan: %s\n", umi_last_error());
                // the replayed graph computed every curve of this batch
                for (int64_t b = 0; b < n && st == UMI_OK; ++b)
                    if (len[b] > 0) {
                        CHECK(a.trend[off[b]] == 1.0f + (float)W[b]);
                        CHECK(a.trend[off[b] + len[b] - 1] == 1.0f + (float)W[b]);
                    }
            } else {
                CHECK(st == UMI_ERR_INVALID_ARG);
            }
        }
        CHECK(umi_plan_destroy(p) == UMI_OK);
    }
}

// The allocation-free call: random batches within its limits run through the
// same checkers on the static workspace; batches beyond them are refused
// before any launch, and no call allocates device memory.
void check_noalloc()
{
    for (int round = 0; round < std::max(2, g_rounds / 10); ++round) {
        const int64_t n = uni(1, 30);
        std::vector<int64_t> len((size_t)n);
        std::vector<int32_t> W((size_t)n);
        int64_t total = 0;
        for (int64_t b = 0; b < n; ++b) {
            len[b] = uni(0, 70000);
            W[b] = odd_w(uni(0, 3) == 0 ? 2047 : 721);
            total += len[b];
        }
        DevArrays a(std::max<int64_t>(total, 1));
        umi_launch lo = {uni(0, 3) == 0 ? UMI_MODE_PER_CURVE : UMI_MODE_PERSISTENT, 0, 0, 0,
                         nullptr, nullptr};
        const long before = g_prepass.load();
        const long mallocs = fake_hip::device_mallocs();
        const umi_status st = umi_detrend_batch_noalloc(a.flux, uni(0, 1) ? a.time : nullptr,
                                                        len.data(), n, W.data(), 2.0f, 5.0f, 5,
                                                        a.trend, a.median, &lo, nullptr);
        CHECK(st == UMI_OK || st == UMI_ERR_UNSUPPORTED);  // tiles of W near 2047
        if (st == UMI_OK && total > 0) CHECK(g_prepass > before);
        CHECK(fake_hip::device_mallocs() == mallocs);
    }
    std::vector<int64_t> big = {UMI_NOALLOC_MAX_SAMPLES, 1};
    std::vector<int32_t> w2 = {25, 25};
    const long before = g_prepass.load();
    CHECK(umi_detrend_batch_noalloc(reinterpret_cast<float*>(16), nullptr, big.data(), 2,
                                    w2.data(), 2.0f, 5.0f, 5, reinterpret_cast<float*>(16),
                                    nullptr, nullptr, nullptr) == UMI_ERR_UNSUPPORTED);
    CHECK(g_prepass == before);
}

// Host/device copy lists through the copy kernel's launcher: lists longer
// than one launch holds, zero sizes mixed in, every byte arrives.
void check_copy_kernel_lists()
{
    for (int round = 0; round < 20; ++round) {
        const int n = (int)uni(0, 200);
        std::vector<std::vector<char>> src((size_t)n), dst((size_t)n);
        std::vector<void*> d((size_t)n);
        std::vector<const void*> sp((size_t)n);
        std::vector<int64_t> bytes((size_t)n);
        for (int i = 0; i < n; ++i) {
            bytes[i] = uni(0, 3) == 0 ? 0 : uni(1, 100000);
            src[i].assign((size_t)bytes[i], (char)(i * 7 + round));
            dst[i].assign((size_t)bytes[i], 0);
            d[i] = dst[i].data();
            sp[i] = src[i].data();
        }
        CHECK(umi_copy_async(d.data(), sp.data(), bytes.data(), n,
                             (int32_t)(uni(0, 1) ? UMI_COPY_H2D : UMI_COPY_D2H) | UMI_COPY_KERNEL,
                             nullptr) == UMI_OK);
        for (int i = 0; i < n; ++i) CHECK(dst[i] == src[i]);
    }
}

void check_copy_pool()
{
    auto worker = [](int seed) {
        std::mt19937_64 r((uint64_t)seed);
        for (int it = 0; it < 20; ++it) {
            const int n = (int)(r() % 12);
            std::vector<std::vector<char>> src((size_t)n), dst((size_t)n);
            std::vector<void*> d((size_t)n);
            std::vector<const void*> s((size_t)n);
            std::vector<int64_t> bytes((size_t)n);
            for (int i = 0; i < n; ++i) {
                bytes[i] = (int64_t)(r() % (3u << 20));
                src[i].assign((size_t)bytes[i], (char)(i + seed));
                dst[i].assign((size_t)bytes[i], 0);
                d[i] = dst[i].data();
                s[i] = src[i].data();
            }
            const int threads = 1 + (int)(r() % 8);
            CHECK(umi_host_copy_many(d.data(), s.data(), bytes.data(), n, threads) == UMI_OK);
            for (int i = 0; i < n; ++i) CHECK(dst[i] == src[i]);
        }
    };
    std::vector<std::thread> ts;
    for (int k = 0; k < 4; ++k) ts.emplace_back(worker, k + 1);
    for (auto& t : ts) t.join();
}

// The native serving loop: requests from three threads (empty ones, ones
// larger than a step, one larger than the staging ring, gaps in time), all
// completing with flux + W in their own output; invalid submissions refused;
// a step whose estimate kernel fails reports its requests as failed and the
// server goes on; shutdown finishes what was queued; nothing leaks.
void check_server()
{
    struct Curve {
        std::vector<float> flux, out;
        std::vector<double> time;
        int32_t W = 1;
        bool with_time = true;
    };
    for (int pass = 0; pass < 2; ++pass) {
        umi_server_config cfg{};
        cfg.capacity = 400000;
        cfg.max_step_samples = 50000;
        cfg.staging_bytes = 3 << 20;  // 262,144 samples: the largest request does not fit
        cfg.max_curves = 8;
        cfg.max_W = 101;
        cfg.max_inflight = pass == 0 ? 2 : 1;
        cfg.copy_threads = 2;
        umi_server* srv = nullptr;
        CHECK(umi_server_create(&cfg, &srv) == UMI_OK);
        if (!srv) return;
        const int per_thread = std::max(8, g_rounds / 10), threads = 3;
        std::vector<Curve> cv((size_t)(per_thread * threads));
        std::mt19937_64 r0(77 + pass);
        for (size_t i = 0; i < cv.size(); ++i) {
            Curve& c = cv[i];
            int64_t n = (int64_t)(r0() % 30000);
            if (i % 17 == 5) n = 0;
            if (i % 23 == 7) n = 60000 + (int64_t)(r0() % 40000);  // beyond one step
            if (i == 11) n = 300000;                                // beyond the staging ring
            c.flux.resize((size_t)n);
            c.time.resize((size_t)n);
            c.out.assign((size_t)n, -1.0f);
            for (int64_t k = 0; k < n; ++k) {
                c.flux[(size_t)k] = (float)(k % 1000) * 0.25f;
                c.time[(size_t)k] = (double)k / 720.0 + (k > n / 2 ? 1.0 : 0.0);
            }
            c.W = (int32_t)(2 * (r0() % 51) + 1);
            c.with_time = (i % 3) != 0;
        }
        // one W whose steps fail, in the second pass
        const int32_t bad_W = pass == 1 ? 99 : 0;
        if (bad_W) cv[4].W = cv[9].W = bad_W;
        g_fail_W.store(bad_W);
        auto submitter = [&](int t) {
            for (int k = 0; k < per_thread; ++k) {
                const size_t i = (size_t)(t * per_thread + k);
                Curve& c = cv[i];
                const umi_status st = umi_server_submit(
                    srv, c.flux.data(), c.with_time ? c.time.data() : nullptr,
                    (int64_t)c.flux.size(), c.W, 2.0f, 5.0f, (int32_t)(3 + (i % 2) * 2), -1.0,
                    c.out.data(), (uint64_t)i);
                CHECK(st == UMI_OK);
            }
        };
        std::vector<std::thread> ts;
        for (int t = 0; t < threads; ++t) ts.emplace_back(submitter, t);
        // invalid submissions are refused and produce no completion
        float dummy = 0.0f;
        CHECK(umi_server_submit(srv, &dummy, nullptr, 1, 2, 2.0f, 5.0f, 5, -1.0, &dummy, 999999) ==
              UMI_ERR_INVALID_ARG);
        CHECK(umi_server_submit(srv, &dummy, nullptr, 1, 103, 2.0f, 5.0f, 5, -1.0, &dummy,
                                999999) == UMI_ERR_INVALID_ARG);
        CHECK(umi_server_submit(srv, &dummy, nullptr, 1, 5, INFINITY, 5.0f, 5, -1.0, &dummy,
                                999999) == UMI_ERR_INVALID_ARG);
        CHECK(umi_server_submit(srv, &dummy, nullptr, 1, 5, 2.0f, 0.0f, 5, -1.0, &dummy, 999999) ==
              UMI_ERR_INVALID_ARG);
        CHECK(umi_server_submit(srv, &dummy, nullptr, cfg.capacity + 1, 5, 2.0f, 5.0f, 5, -1.0,
                                &dummy, 999999) == UMI_ERR_INVALID_ARG);
        CHECK(umi_server_submit(srv, nullptr, nullptr, 1, 5, 2.0f, 5.0f, 5, -1.0, &dummy, 999999) ==
              UMI_ERR_INVALID_ARG);
        for (auto& t : ts) t.join();
        std::vector<int32_t> status(cv.size(), -1);
        size_t got = 0;
        std::vector<umi_server_completion> buf(16);
        for (int spins = 0; got < cv.size() && spins < 20000; ++spins) {
            int32_t k = 0;
            CHECK(umi_server_poll(srv, buf.data(), (int32_t)buf.size(), 0.01, &k) == UMI_OK);
            for (int32_t j = 0; j < k; ++j) {
                const uint64_t tag = buf[(size_t)j].tag;
                CHECK(tag < cv.size());
                if (tag >= cv.size()) continue;
                CHECK(status[tag] == -1);  // reported once
                status[tag] = buf[(size_t)j].status;
                CHECK(buf[(size_t)j].done >= buf[(size_t)j].launched &&
                      buf[(size_t)j].launched >= buf[(size_t)j].admitted);
                ++got;
            }
        }
        CHECK(got == cv.size());
        int64_t ok = 0, bad = 0;
        for (size_t i = 0; i < cv.size(); ++i) {
            const Curve& c = cv[i];
            if (c.W == bad_W && !c.flux.empty()) {
                CHECK(status[i] == UMI_ERR_DEVICE);
                ++bad;
                continue;
            }
            // a request that shared a step with a failing curve fails with it
            if (bad_W != 0 && status[i] == UMI_ERR_DEVICE) {
                ++bad;
                continue;
            }
            CHECK(status[i] == UMI_OK);
            bool same = true;
            for (size_t k = 0; k < c.flux.size(); ++k)
                same = same && c.out[k] == c.flux[k] + (float)c.W;
            CHECK(same);
            ++ok;
        }
        umi_server_stats st{};
        CHECK(umi_server_stats_get(srv, &st) == UMI_OK);
        CHECK(st.submitted == (int64_t)cv.size());
        CHECK(st.completed + st.failed == (int64_t)cv.size());
        CHECK(st.failed == bad && ok > 0 && (bad_W == 0 || bad >= 2));
        CHECK(st.arena_used == 0 && st.arena_high_water <= cfg.capacity);
        CHECK(st.steps > 0 && st.largest_step_samples >= 300000);
        CHECK(st.staging_fallbacks >= 1);  // the request larger than the ring
        CHECK(umi_server_reset_stats(srv) == UMI_OK);
        // requests queued right before shutdown still complete
        std::vector<float> f(1000, 2.0f), o(1000, 0.0f);
        CHECK(umi_server_submit(srv, f.data(), nullptr, 1000, 7, 2.0f, 5.0f, 5, -1.0, o.data(),
                                4242) == UMI_OK);
        CHECK(umi_server_shutdown(srv) == UMI_OK);
        int32_t k = 0;
        CHECK(umi_server_poll(srv, buf.data(), (int32_t)buf.size(), 0.0, &k) == UMI_OK);
        CHECK(k == 1 && buf[0].tag == 4242 && buf[0].status == UMI_OK);
        CHECK(o[0] == 9.0f && o[999] == 9.0f);
        CHECK(umi_server_submit(srv, f.data(), nullptr, 1000, 7, 2.0f, 5.0f, 5, -1.0, o.data(),
                                1) == UMI_ERR_INVALID_ARG);
        CHECK(umi_server_destroy(srv) == UMI_OK);
        g_fail_W.store(0);
    }
    umi_server_config bad{};
    umi_server* none = nullptr;
    CHECK(umi_server_create(&bad, &none) == UMI_ERR_INVALID_ARG && none == nullptr);
    bad.capacity = 1000;
    bad.max_W = 4;
    CHECK(umi_server_create(&bad, &none) == UMI_ERR_INVALID_ARG && none == nullptr);
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc > 1) g_rounds = std::max(1, std::atoi(argv[1]));
    check_tuning();
    check_direct_batches();
    CHECK(umi_set_tuning(nullptr) == UMI_OK);
    check_direct_batches();
    check_plans();
    check_noalloc();
    check_copy_kernel_lists();
    check_copy_pool();
    check_server();
    umi_release();
    CHECK(fake_hip::live_device_blocks() == 0);
    CHECK(fake_hip::live_host_blocks() == 0);
    CHECK(fake_hip::live_events() == 0);
    CHECK(fake_hip::live_graphs() == 0);
    CHECK(fake_hip::live_streams() == 0);
    CHECK(g_prepass > 0 && g_main > 0);
    if (g_failures) {
        std::fprintf(stderr, "%d host checks failed\n", g_failures.load());
        return 1;
    }
    std::printf("host checks ok (%ld pre-pass and %ld estimate launches checked)\n",
                g_prepass.load(), g_main.load());
    return 0;
}
