// HIP kernels of the UMI library for CDNA4 (gfx950).
//
// Two kernels run per batch, both on the caller's stream:
//
//   pre-pass            validity and segmentation (gap handling, minimum
//                       segment length W/3 of Section 4.4): block scans write
//                       a segment word per sample and one record per segment,
//                       and lay out the tile list for the main kernel.  Two
//                       forms: umi_prepass_walk_kernel walks each curve with
//                       one workgroup (batches of many curves);
//                       umi_prepass_chunk_kernel cuts curves into chunks of
//                       2,048 samples taken in ticket order, each joined to
//                       the curve before it by a decoupled look-back (few
//                       curves, so that a lone curve is spread over the chip).
//
//   umi_main_kernel     tiles of consecutive output positions.  A workgroup
//                       stages a tile plus its W-1 halo from HBM once, keeps the
//                       valid samples compacted in LDS, sorts (key, index) pairs
//                       of the staged samples once (bitonic network in LDS), and
//                       builds a wavelet matrix over the sorted ranks.  Every
//                       lane then takes up to three consecutive windows:
//                         Phase 1 (Section 2.1): exact median as the k-th
//                           smallest rank in the window's index range, one
//                           O(log N) wavelet descent -- the sort is shared by
//                           all windows of the tile.  Tiles of full windows
//                           with W <= 31 skip the sort and take their medians
//                           from register networks instead;
//                         Phase 2 (Section 2.2, Eq. 1): upper-RMS scale;
//                         Phase 3 (Section 2.3, Eqs. 2-4): asymmetric bisquare
//                           iterations in the residual form
//                           mu <- mu + sum(w v) / (k sum(w)), v = k (x - mu),
//                           k = A/(c s), A = (1 + alpha)/2: Eq. 4 rewritten
//                           around the current mu, with Eq. 2's two branches
//                           folded into one expression of v.
//                       Windows that share samples and have the same length
//                       are summed in one fused sweep (one LDS read per sample
//                       for all of them).  Launched either persistently (a
//                       grid sized to the chip pops tiles from a device
//                       counter) or one workgroup per tile.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "umi.h"
#include "umi_internal.h"

// Every fused multiply-add below is written out with __builtin_fmaf; the
// compiler may not contract anything else, so the same window gives the same
// bits whichever code path (fused multi-window or single-window) computes it.
#pragma clang fp contract(off)

namespace umi {

// ---------------------------------------------------------------------------
// small wave / block helpers (64-lane wavefronts)

__device__ __forceinline__ int wave_incl_sum(int x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Inclusive "latest" scan over the lanes of a wave: the pair (idx, val) of
// the highest lane so far whose idx is >= 0 (idx grows with the lane where
// set, so the latest is the largest).
__device__ __forceinline__ void wave_incl_latest(int& idx, int& val)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int yi = __shfl_up(idx, d, 64);
        const int yv = __shfl_up(val, d, 64);
        if (lane >= d && yi > idx) {
            idx = yi;
            val = yv;
        }
    }
}

// The same for an (index, time) pair, together with an inclusive sum `cnt`.
template <class T>
__device__ __forceinline__ void wave_incl_latest_sum(int& idx, T& val, int& cnt)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int yi = __shfl_up(idx, d, 64);
        const T yv = __shfl_up(val, d, 64);
        const int yc = __shfl_up(cnt, d, 64);
        if (lane >= d) {
            if (yi > idx) {
                idx = yi;
                val = yv;
            }
            cnt += yc;
        }
    }
}

// ---------------------------------------------------------------------------
// Pre-pass: segments and tiles.
//
// Curves are cut into chunks of kPrepChunk samples (kPrepItems consecutive
// samples per thread); workgroups take chunks in ticket order from a device
// counter and scan each in one pass.  The pre-pass writes one int32 per sample:
//   -1                    the sample is invalid (non-finite flux or time);
//   x >= 0                a valid sample whose segment starts at the valid
//                         sample x (curve-local index), x < this sample;
//   -2 - n  (<= -2)       the first valid sample of a segment of n valid
//                         samples (the segment's record lives in its first
//                         slot, so the workspace is 4 bytes per sample).
// A new segment starts at a valid sample whose predecessor among valid
// samples is more than kGapDays earlier (strictly), and at the first valid
// sample.  The slot of a segment's first sample is written once, by whoever
// sees the segment end (the thread holding the next start, or the workgroup of
// the curve's last chunk), so no slot has two writers.
//
// A chunk's output depends on the curve before it only through a small state
// (SegState: valid count, last valid sample and its time, latest segment
// start).  Each workgroup first scans its chunk alone and publishes the
// chunk's summary; it then finds the state before the chunk by looking back
// over its predecessors' records -- 64 at a time, one per lane -- combining
// summaries until it meets one whose state is final (a decoupled look-back),
// publishes its own final state, and writes its segment words.  Tickets are
// handed out in order, so every chunk a workgroup waits for belongs to a
// workgroup that has already started, and every workgroup publishes its
// summary before it waits for anything: the waits always end.

// The state after run `a` followed by run `b`.  `a_prefix`: `a` starts at the
// curve's first sample, so after an empty `a` the first valid sample of `b`
// starts a segment.  The gap test is the expression the per-sample scan uses.
__device__ __forceinline__ SegState seg_combine(const SegState& a, const SegState& b, bool a_prefix,
                                                bool has_time)
{
    if (b.cnt == 0) return a;
    SegState r = b;
    if (a.cnt == 0) {
        if (a_prefix && b.ls < 0) {
            r.ls = b.fv;
            r.lsb = 0;
        }
        return r;
    }
    r.cnt = a.cnt + b.cnt;
    r.fv = a.fv;
    r.ft = a.ft;
    if (b.ls >= 0) {
        r.lsb = a.cnt + b.lsb;
    } else if (has_time && (b.ft - a.lt) > kGapDays) {
        r.ls = b.fv;
        r.lsb = a.cnt;
    } else {
        r.ls = a.ls;
        r.lsb = a.lsb;
    }
    return r;
}

__device__ __forceinline__ SegState seg_empty()
{
    SegState e;
    e.cnt = 0;
    e.fv = e.lv = e.ls = -1;
    e.lsb = 0;
    e.reserved = 0;
    e.ft = e.lt = 0.0;
    return e;
}

constexpr int kSpinLimit = 1 << 20;  // polls of one record before giving up (never reached)

// Word i of a SegState (see ChunkRec) and the reverse.
__device__ __forceinline__ uint32_t seg_word(const SegState& s, int i)
{
    const uint64_t ft = __double_as_longlong(s.ft), lt = __double_as_longlong(s.lt);
    switch (i) {
    case 0: return (uint32_t)s.cnt;
    case 1: return (uint32_t)s.fv;
    case 2: return (uint32_t)s.lv;
    case 3: return (uint32_t)s.ls;
    case 4: return (uint32_t)s.lsb;
    case 5: return (uint32_t)ft;
    case 6: return (uint32_t)(ft >> 32);
    case 7: return (uint32_t)lt;
    default: return (uint32_t)(lt >> 32);
    }
}

__device__ __forceinline__ SegState seg_from_words(const uint32_t (&v)[kSegWords])
{
    SegState s;
    s.cnt = (int32_t)v[0];
    s.fv = (int32_t)v[1];
    s.lv = (int32_t)v[2];
    s.ls = (int32_t)v[3];
    s.lsb = (int32_t)v[4];
    s.reserved = 0;
    s.ft = __longlong_as_double((long long)(((uint64_t)v[6] << 32) | v[5]));
    s.lt = __longlong_as_double((long long)(((uint64_t)v[8] << 32) | v[7]));
    return s;
}

// Publish a state: lane i < kSegWords of the calling wave stores word i with
// the stamp (relaxed device-scope atomics: no cache flush, no ordering).
__device__ __forceinline__ void seg_publish(uint64_t* words, const SegState& s, uint32_t stamp)
{
    const int lane = __lane_id();
    if (lane < kSegWords)
        __hip_atomic_store(&words[lane], ((uint64_t)stamp << 32) | seg_word(s, lane),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Read a state if every word carries `stamp`.
__device__ __forceinline__ bool seg_read(const uint64_t* words, uint32_t stamp, SegState& out)
{
    uint32_t v[kSegWords];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < kSegWords; ++i) {
        const uint64_t w = __hip_atomic_load(&words[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = ok && (uint32_t)(w >> 32) == stamp;
        v[i] = (uint32_t)w;
    }
    if (ok) out = seg_from_words(v);
    return ok;
}

// The state before chunk g of a curve whose first chunk is g0 (g > g0), from
// the predecessors' records; run by one whole wave.  Lane l examines chunk
// g - 1 - l - 64 k in round k; the nearest chunk with a final state ends the
// walk, and the summaries of the chunks after it are combined in order.  The
// result is returned in every lane.
__device__ SegState lookback(const ChunkRec* __restrict__ recs, int g, int g0, uint32_t stamp,
                             bool has_time, SegState* sh /* [64] */)
{
    const int lane = __lane_id();
    SegState acc = seg_empty();  // the chunks after the current window, in order
    for (int hi = g - 1;; hi -= 64) {
        const int j = hi - lane;
        int status = 2;  // before the curve's first chunk: the empty prefix
        SegState st = seg_empty();
        if (j >= g0) {
            status = 0;
            for (int polls = 0; polls < kSpinLimit && status == 0; ++polls) {
                if (seg_read(recs[j].inc, stamp, st))
                    status = 2;
                else if (seg_read(recs[j].agg, stamp, st))
                    status = 1;
                else
                    __builtin_amdgcn_s_sleep(1);
            }
            if (status == 0) status = 2;  // a timeout reads as final
        }
        sh[lane] = st;
        const uint64_t fin = __ballot(status == 2);
        const int k = fin ? __builtin_ctzll(fin) : 64;  // nearest final state in this window
        // every lane's state is in LDS before lane 0 reads them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane == 0) {
            for (int i = 0; i < k; ++i) acc = seg_combine(sh[i], acc, false, has_time);
            if (k < 64) acc = seg_combine(sh[k], acc, true, has_time);
            sh[0] = acc;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        acc = sh[0];  // every lane
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (k < 64) break;
    }
    return acc;
}

// The batch header and curve table the pre-pass reads sit either in device
// memory already or in the caller's pinned staging block, which the device
// reads over the bus; in the latter case the pre-pass also copies the block
// into device memory (`to`) for the estimate kernel, spread over the grid in
// 8-byte words, so no separate copy precedes it.
__device__ __forceinline__ void stage_block_copy(const uint8_t* __restrict__ src,
                                                 uint8_t* __restrict__ to, int n_curves, int nt)
{
    if (to == nullptr) return;
    const int words = (int)((sizeof(BatchHeader) + (size_t)n_curves * sizeof(CurveDesc)) / 8);
    const uint64_t* s = reinterpret_cast<const uint64_t*>(src);
    uint64_t* d = reinterpret_cast<uint64_t*>(to);
    for (int i = (int)(blockIdx.x * nt + threadIdx.x); i < words; i += (int)gridDim.x * nt)
        d[i] = s[i];
}
static_assert(sizeof(BatchHeader) % 8 == 0 && sizeof(CurveDesc) % 8 == 0, "8-byte words");

template <int NT, int K>
__global__ __launch_bounds__(NT) void umi_prepass_chunk_kernel(
    const float* __restrict__ flux, const double* __restrict__ time,
    const uint8_t* __restrict__ block, uint8_t* __restrict__ block_to, int curve_one,
    int32_t* __restrict__ segid, int2* __restrict__ tiles, Counters* __restrict__ ctr,
    ChunkRec* __restrict__ recs, int clear_queue, CurveDesc one, int one_chunks)
{
    const BatchHeader* __restrict__ hdr = reinterpret_cast<const BatchHeader*>(block);
    const CurveDesc* __restrict__ curves =
        reinterpret_cast<const CurveDesc*>(block + sizeof(BatchHeader));
    constexpr int NW = NT / 64;
    constexpr int kChunk = NT * K;
    __shared__ int sh_vi[NW];      // per wave: latest valid index
    __shared__ double sh_vt[NW];   //           its time
    __shared__ int sh_vc[NW];      //           valid count
    __shared__ int sh_sx[NW];      // per wave: latest segment start
    __shared__ int sh_sz[NW];      //           valid samples before it
    __shared__ int sh_fv;          // the chunk's first valid sample
    __shared__ double sh_ft;       //   its time
    __shared__ int sh_ticket, sh_curve;
    __shared__ SegState sh_carry;  // the curve's state before the chunk
    __shared__ SegState sh_lb[64]; // look-back window

    const int tid = (int)threadIdx.x;
    const int w = tid >> 6;
    const int lane = __lane_id();
    if (clear_queue && blockIdx.x == 0 && tid == 0) ctr->queue = 0u;
    const uint64_t epoch_word = ctr->epoch;
    const uint32_t stamp = (uint32_t)(epoch_word + 1);  // this launch's record stamp
    // one curve (per-curve launches) or the whole batch; a batch of one curve
    // may come with its descriptor and chunk count as arguments, so that no
    // step waits on a read of the table over the bus
    const bool given = one_chunks >= 0;
    const int n_chunks = given ? one_chunks
                               : (curve_one >= 0 ? (curves[curve_one].len + kChunk - 1) / kChunk
                                                 : hdr->n_chunks);
    const int n_curves = given ? 1 : hdr->n_curves;
    stage_block_copy(block, block_to, n_curves, NT);

    for (;;) {
        if (tid == 0) sh_ticket = (int)atomicAdd(&ctr->tickets, 1u);
        __syncthreads();
        const int g = sh_ticket;
        if (g >= n_chunks) break;
        // the chunk's curve: the last table entry whose first chunk is <= g
        // (a 64-way search by wave 0; chunk_base increases along the table)
        if (curve_one >= 0) {
            if (tid == 0) sh_curve = curve_one;
        } else if (w == 0) {
            int lo = 0, hi = n_curves;
            while (hi - lo > 1) {
                const int step = (hi - lo + 63) / 64;
                const int idx = lo + lane * step;
                const bool le = idx < hi && curves[idx].chunk_base <= g;
                const uint64_t m = __ballot(le);
                const int last = 63 - __builtin_clzll(m);  // lane 0 always qualifies
                lo = lo + last * step;
                hi = min(lo + step, hi);
            }
            if (lane == 0) sh_curve = lo;
        }
        __syncthreads();
        const int cidx = sh_curve;
        const CurveDesc cd = given ? one : curves[cidx];
        const int g0 = curve_one >= 0 ? 0 : cd.chunk_base;  // the curve's first chunk
        const int lo = (g - g0) * kChunk;
        const int hi = min(lo + kChunk, cd.len);
        const float* f = flux + cd.off;
        const double* tm = time ? time + cd.off : nullptr;
        const bool has_time = tm != nullptr;
        int32_t* sid = segid + cd.off;

        // the tiles that start in this chunk
        for (int t = (lo + cd.tile - 1) / cd.tile + tid; t * cd.tile < hi; t += NT)
            tiles[cd.tile_base + t] = make_int2(cidx, t * cd.tile);

        float fv[K];
        double tv[K];
        const int e0 = lo + tid * K;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int e = e0 + q;
            fv[q] = e < hi ? f[e] : __builtin_nanf("");
            tv[q] = (has_time && e < hi) ? tm[e] : 0.0;
        }
        uint32_t vmask = 0;  // bit q: item q is valid
        int vi = -1, vc = 0, fi = -1;
        double vt = 0.0, ft = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const bool ok = e0 + q < hi && isfinite(fv[q]) && (!has_time || isfinite(tv[q]));
            vmask |= (ok ? 1u : 0u) << q;
            if (ok) {
                if (fi < 0) {
                    fi = e0 + q;
                    ft = tv[q];
                }
                vi = e0 + q;
                vt = tv[q];
                ++vc;
            }
        }

        // phase 1 (chunk alone): latest valid sample and valid count before
        // this thread's items, the chunk's first and last valid samples
        const int own_vc = vc;
        wave_incl_latest_sum(vi, vt, vc);
        if (lane == 63) {
            sh_vi[w] = vi;
            sh_vt[w] = vt;
            sh_vc[w] = vc;
        }
        int ex_i = __shfl_up(vi, 1, 64);
        double ex_t = __shfl_up(vt, 1, 64);
        int before = vc - own_vc;  // valid samples earlier in this wave
        if (lane == 0) ex_i = -1;
        __syncthreads();
        int tot = 0, blk_i = -1;
        double blk_t = 0.0;
        for (int i = 0; i < NW; ++i) {
            if (i == w && ex_i < 0) {  // nothing valid earlier in this wave
                ex_i = blk_i;
                ex_t = blk_t;
            }
            if (i < w) before += sh_vc[i];
            tot += sh_vc[i];
            if (sh_vi[i] >= 0) {
                blk_i = sh_vi[i];
                blk_t = sh_vt[i];
            }
        }
        if (before == 0 && own_vc > 0) {  // the thread holding the chunk's first valid sample
            sh_fv = fi;
            sh_ft = ft;
        }

        // phase 2 (chunk alone): segment starts that follow a valid sample of
        // the chunk, then the latest such start before this thread's items
        int sx = -1, sz = 0;
        {
            int pi = ex_i;
            double pt = ex_t;
            int v = before;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                if ((vmask >> q) & 1u) {
                    if (pi >= 0 && has_time && (tv[q] - pt) > kGapDays) {
                        sx = e0 + q;
                        sz = v;
                    }
                    pi = e0 + q;
                    pt = tv[q];
                    ++v;
                }
            }
        }
        wave_incl_latest(sx, sz);
        if (lane == 63) {
            sh_sx[w] = sx;
            sh_sz[w] = sz;
        }
        int px = __shfl_up(sx, 1, 64);
        int pz = __shfl_up(sz, 1, 64);
        if (lane == 0) px = -1;
        __syncthreads();
        int bx = -1, bz = 0;
        for (int i = 0; i < NW; ++i) {
            if (i == w && px < 0) {
                px = bx;
                pz = bz;
            }
            if (sh_sx[i] >= 0) {
                bx = sh_sx[i];
                bz = sh_sz[i];
            }
        }

        // publish the chunk's summary, find the state before it, publish the
        // state after it (wave 0)
        if (w == 0) {
            SegState agg = seg_empty();
            if (tot > 0) {
                agg.cnt = tot;
                agg.fv = sh_fv;
                agg.ft = sh_ft;
                agg.lv = blk_i;
                agg.lt = blk_t;
                agg.ls = bx;
                agg.lsb = bz;
            }
            SegState carry = seg_empty();
            if (g > g0) {
                seg_publish(recs[g].agg, agg, stamp);
                carry = lookback(recs, g, g0, stamp, has_time, sh_lb);
            }
            const SegState inc = seg_combine(carry, agg, true, has_time);  // every lane
            seg_publish(recs[g].inc, inc, stamp);
            if (lane == 0) {
                sh_carry = carry;
                // the curve's last segment ends with its last chunk
                if (hi == cd.len && inc.ls >= 0) sid[inc.ls] = -2 - (inc.cnt - inc.lsb);
            }
        }
        __syncthreads();
        const SegState cy = sh_carry;
        const int fv0 = sh_fv;      // the chunk's first valid sample (when tot > 0)
        const double ft0 = sh_ft;

        // writes: segment of each item; a start closes the segment before it.
        // The state entering this thread's items comes from the chunk scan
        // where the chunk holds something before them, else from the carry;
        // it is formed with selects only.
        {
            const bool local_pred = ex_i >= 0;
            int pi = local_pred ? ex_i : cy.lv;
            double pt = local_pred ? ex_t : cy.lt;
            int v = cy.cnt + before;
            // the chunk's first valid sample starts a segment when nothing
            // valid precedes it in the curve or the gap to it is too long
            const bool first_starts =
                tot > 0 && (cy.cnt == 0 || (has_time && (ft0 - cy.lt) > kGapDays));
            const bool local_start = px >= 0;
            const bool use_fv = !local_start && first_starts && fv0 < e0;
            pz = local_start ? pz + cy.cnt : (use_fv ? cy.cnt : cy.lsb);
            px = local_start ? px : (use_fv ? fv0 : cy.ls);
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int e = e0 + q;
                if (e < hi) {
                    if ((vmask >> q) & 1u) {
                        if (pi < 0 || (has_time && (tv[q] - pt) > kGapDays)) {
                            if (px >= 0) sid[px] = -2 - (v - pz);
                            px = e;
                            pz = v;
                        } else {
                            sid[e] = px;
                        }
                        pi = e;
                        pt = tv[q];
                        ++v;
                    } else {
                        sid[e] = -1;
                    }
                }
            }
        }
        __syncthreads();  // LDS of this chunk is reused by the next
    }

    // the last workgroup to finish resets the tickets for the next launch.
    // Every workgroup's final ticket increment has returned its value before
    // the workgroup counts itself done, so once `done` shows all of them no
    // increment is outstanding.
    if (tid == 0) {
        const uint32_t old =
            __hip_atomic_fetch_add(&ctr->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            __hip_atomic_store(&ctr->tickets, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr->epoch, epoch_word + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// The same segment words and tiles from one workgroup per curve, which walks
// the curve's chunks of NT * K samples in order and carries the scan state in
// registers (the next chunk's loads are issued before the current chunk's
// scans).  No tickets, records or look-back: batches of many curves fill the
// chip this way, and every chunk costs one pass.  kTime: a time array is
// given (without one nothing breaks a segment).  Two barriers per chunk:
// each LDS array is written in one phase and read in the next, and a phase's
// writes follow the barrier that ends every wave's reads of the same array in
// the chunk before.
template <int NT, int K, bool kTime>
__global__ __launch_bounds__(NT) void umi_prepass_walk_kernel(
    const float* __restrict__ flux, const double* __restrict__ time,
    const uint8_t* __restrict__ block, uint8_t* __restrict__ block_to, int curve_first,
    int32_t* __restrict__ segid, int2* __restrict__ tiles, uint32_t* __restrict__ counter,
    int32_t* __restrict__ trash)
{
    const BatchHeader* __restrict__ hdr = reinterpret_cast<const BatchHeader*>(block);
    const CurveDesc* __restrict__ curves =
        reinterpret_cast<const CurveDesc*>(block + sizeof(BatchHeader));
    constexpr int NW = NT / 64;
    __shared__ int sh_vi[NW];      // per wave: latest valid index
    __shared__ double sh_vt[NW];   //           its time
    __shared__ int sh_vc[NW];      //           valid count
    __shared__ int sh_sx[NW];      // per wave: latest segment start
    __shared__ int sh_sz[NW];      //           valid samples before it

    if (counter != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
    const int n_curves = hdr->n_curves;
    stage_block_copy(block, block_to, n_curves, NT);
    const int cidx = curve_first + (int)blockIdx.x;
    if (cidx >= n_curves) return;  // fixed-size grids cover fewer curves
    const CurveDesc cd = curves[cidx];

    const int ntiles = cd.len > 0 ? (cd.len + cd.tile - 1) / cd.tile : 0;
    for (int t = threadIdx.x; t < ntiles; t += NT)
        tiles[cd.tile_base + t] = make_int2(cidx, t * cd.tile);

    const float* f = flux + cd.off;
    const double* tm = time + (kTime ? cd.off : 0);  // unused without times
    int32_t* sid = segid + cd.off;

    // carries from earlier chunks (uniform over the block)
    int c_vi = -1;      // latest valid index
    double c_vt = 0.0;  // its time
    int c_vc = 0;       // valid samples so far
    int c_sx = -1;      // latest segment start
    int c_sz = 0;       // valid samples before it

    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    constexpr int kChunk = NT * K;

    // The next chunk's flux and times are loaded while the current one is
    // scanned, so the loads' latency overlaps the scans.  Every step issues
    // the same loads and stores whatever the data (indices past the curve
    // load its last sample and store to `trash`), so the wait for a chunk's
    // loads counts only the memory operations issued after them and never
    // waits for the previous chunk's stores or the next chunk's loads.
    const int last = cd.len - 1;
    float fv[K];
    double tv[K];
    auto load_chunk = [&](int base, float* fo, double* to) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int e = min(base + (int)threadIdx.x * K + q, last);
            fo[q] = f[e];
            to[q] = kTime ? tm[e] : 0.0;
        }
    };
    if (cd.len > 0) load_chunk(0, fv, tv);

    for (int base = 0; base < cd.len; base += kChunk) {
        float nf[K];
        double nt[K];
        load_chunk(base + kChunk, nf, nt);
        const int e0 = base + (int)threadIdx.x * K;
        uint32_t vmask = 0;  // bit q: item q is valid
        int vi = -1, vc = 0;
        double vt = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const bool ok = e0 + q < cd.len && isfinite(fv[q]) && (!kTime || isfinite(tv[q]));
            vmask |= (ok ? 1u : 0u) << q;
            if (ok) {
                vi = e0 + q;
                vt = tv[q];
                ++vc;
            }
        }

        // phase 1: latest valid sample and valid count before this thread's items
        const int own_vc = vc;
        wave_incl_latest_sum(vi, vt, vc);
        if (lane == 63) {
            sh_vi[w] = vi;
            sh_vt[w] = vt;
            sh_vc[w] = vc;
        }
        int ex_i = __shfl_up(vi, 1, 64);
        double ex_t = __shfl_up(vt, 1, 64);
        int before = vc - own_vc;  // valid samples earlier in this wave
        if (lane == 0) ex_i = -1;
        __syncthreads();
        int blk_i = c_vi, tot = 0;
        double blk_t = c_vt;
        for (int i = 0; i < NW; ++i) {
            if (i == w && ex_i < 0) {  // nothing valid earlier in this wave
                ex_i = blk_i;
                ex_t = blk_t;
            }
            if (i < w) before += sh_vc[i];
            tot += sh_vc[i];
            if (sh_vi[i] >= 0) {
                blk_i = sh_vi[i];
                blk_t = sh_vt[i];
            }
        }
        before += c_vc;

        // phase 2: segment starts among this thread's items, then the latest
        // start before them
        int sx = -1, sz = 0;
        {
            int pi = ex_i;
            double pt = ex_t;
            int v = before;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                if ((vmask >> q) & 1u) {
                    if (pi < 0 || (kTime && (tv[q] - pt) > kGapDays)) {
                        sx = e0 + q;
                        sz = v;
                    }
                    pi = e0 + q;
                    pt = tv[q];
                    ++v;
                }
            }
        }
        wave_incl_latest(sx, sz);
        if (lane == 63) {
            sh_sx[w] = sx;
            sh_sz[w] = sz;
        }
        int px = __shfl_up(sx, 1, 64);
        int pz = __shfl_up(sz, 1, 64);
        if (lane == 0) px = -1;
        __syncthreads();
        {
            int bx = c_sx, bz = c_sz;
            for (int i = 0; i < NW; ++i) {
                if (i == w && px < 0) {
                    px = bx;
                    pz = bz;
                }
                if (sh_sx[i] >= 0) {
                    bx = sh_sx[i];
                    bz = sh_sz[i];
                }
            }
            // every wave has read the phase-1 arrays; carries for the next chunk
            if (blk_i >= 0) {
                c_vi = blk_i;
                c_vt = blk_t;
            }
            c_vc += tot;
            c_sx = bx;
            c_sz = bz;
        }

        // writes: segment of each item; a start closes the segment before it.
        // One store per item, its address and value chosen by selects.
        {
            int pi = ex_i;
            double pt = ex_t;
            int v = before;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int e = e0 + q;
                const bool valid = (vmask >> q) & 1u;  // implies e < cd.len
                const bool start = valid && (pi < 0 || (kTime && (tv[q] - pt) > kGapDays));
                int32_t* dst = start ? (px >= 0 ? sid + px : trash) : (e < cd.len ? sid + e : trash);
                const int32_t val = start ? -2 - (v - pz) : (valid ? px : -1);
                *dst = val;
                if (start) {
                    px = e;
                    pz = v;
                }
                if (valid) {
                    pi = e;
                    pt = tv[q];
                    ++v;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            fv[q] = nf[q];
            tv[q] = nt[q];
        }
    }
    if (threadIdx.x == 0 && c_sx >= 0) sid[c_sx] = -2 - (c_vc - c_sz);
}

// ---------------------------------------------------------------------------
// Main kernel.

// IEEE-754 totalOrder of float32 as an unsigned key, and back.
__device__ __forceinline__ uint32_t order_key(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k)
{
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

struct MainSmem {
    uint64_t sortbuf[kStageMax];          // (key << 32 | compacted index)
    float xv[kStageMax];                  // compacted valid samples
    uint16_t seq[2][kStageMax];           // wavelet-matrix level sequences
    uint64_t bits[kStageLog2][kWords];    // wavelet-matrix level bit vectors
    uint32_t pre[kStageLog2][kWords];     // ones before each word
    uint32_t zeros[kStageLog2];           // zeros per level
    uint64_t vbits[kWords];               // staged-sample validity
    uint32_t vpre[kWords];
    uint64_t sbits[kWords];               // staged samples that start a segment
    int tile;
    int nvalid;
};

__device__ __forceinline__ uint32_t rank1(const uint64_t* bits, const uint32_t* pre, uint32_t i)
{
    const uint32_t w = i >> 6;
    const uint64_t m = (1ull << (i & 63u)) - 1ull;
    return pre[w] + (uint32_t)__popcll(bits[w] & m);
}

// Ones-before prefix over `nw` words, computed by wave 0; returns total ones
// in lane 0's view through `total_out` (written to LDS by the caller).
__device__ __forceinline__ void word_prefix(const uint64_t* bits, uint32_t* pre, int nw, uint32_t* total_out)
{
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int c = lane < nw ? __popcll(bits[lane]) : 0;
        const int incl = wave_incl_sum(c);
        if (lane < nw) pre[lane] = (uint32_t)(incl - c);
        if (lane == 63) *total_out = (uint32_t)incl;
    }
}

// k-th smallest (0-based) value of the level-0 sequence within [s, e).
__device__ __forceinline__ uint32_t wavelet_kth(const MainSmem& sm, int levels, uint32_t s, uint32_t e, uint32_t k)
{
    uint32_t r = 0;
    for (int l = 0; l < levels; ++l) {
        const uint32_t os = rank1(sm.bits[l], sm.pre[l], s);
        const uint32_t oe = rank1(sm.bits[l], sm.pre[l], e);
        const uint32_t zs = s - os, ze = e - oe;
        const uint32_t nz = ze - zs;
        if (k < nz) {
            s = zs;
            e = ze;
        } else {
            k -= nz;
            s = sm.zeros[l] + os;
            e = sm.zeros[l] + oe;
            r |= 1u << (levels - 1 - l);
        }
    }
    return r;
}

// Number of level-0 values smaller than v within [s, e).
__device__ __forceinline__ uint32_t wavelet_count_less(const MainSmem& sm, int levels, uint32_t s,
                                                       uint32_t e, uint32_t v)
{
    if (v >> levels) return e - s;  // v beyond every stored value
    uint32_t cnt = 0;
    for (int l = 0; l < levels; ++l) {
        const uint32_t os = rank1(sm.bits[l], sm.pre[l], s);
        const uint32_t oe = rank1(sm.bits[l], sm.pre[l], e);
        if ((v >> (levels - 1 - l)) & 1u) {
            cnt += (e - oe) - (s - os);
            s = sm.zeros[l] + os;
            e = sm.zeros[l] + oe;
        } else {
            s -= os;
            e -= oe;
        }
    }
    return cnt;
}

// Phase 3 (Eqs. 2-4) with the asymmetry folded into one fma.  With
// u = (x - mu)/(c s), A = (1 + alpha)/2 and B = (1 - alpha)/2, the effective
// residual of Eq. 2 is A u + B |u| (u for u >= 0, alpha u for u < 0, any
// alpha > 0).  In the scaled variable v = A u = x*k + b, k = A/(c s), it is
// v + beta |v| with beta = B/A, one fma with an |.| source modifier.  The
// sums are sum(w) and sum(w v); Eq. 4 in residual form is then
// mu + sum(w v) / (k sum(w)).
__device__ __forceinline__ void bisquare_acc(float x, float k, float b, float beta, float& sw,
                                             float& swv)
{
    const float v = __builtin_fmaf(x, k, b);
    const float ue = __builtin_fmaf(__builtin_fabsf(v), beta, v);
    // Eq. 3: (1 - ue^2)^2 on |ue| < 1, else 0.  1 - ue^2 <= 1 always, so
    // clamping to [0, 1] is exactly max(., 0).
    const float t = __builtin_amdgcn_fmed3f(__builtin_fmaf(-ue, ue, 1.0f), 0.0f, 1.0f);
    const float w = t * t;
    sw += w;
    swv = __builtin_fmaf(w, v, swv);
}

// Eq. 4 in residual form: mu + sum(w v) / (k sum(w)), with a correctly
// rounded division.  Every path uses this same expression, so paths that sum
// in the same order agree bit for bit.  (The hardware reciprocal would do
// here too -- the quotient is a correction of the order of the scale -- but
// it changed the register assignment of the estimate loops for the worse.)
__device__ __forceinline__ float mu_update(float mu, float swv, float sw, float k)
{
    return mu + swv / (sw * k);
}

// Eq. 1: s = 0.6745 sqrt(ssq / n+), with the hardware square root and
// reciprocal (1 ulp each): once per window, in place of a correctly rounded
// square root and division that cost some 30 instructions (7 % of the
// estimate kernel's time at W = 25).
__device__ __forceinline__ float upper_scale(float ssq, uint32_t nplus)
{
    return kScaleConst * __builtin_amdgcn_sqrtf(ssq * __builtin_amdgcn_rcpf((float)nplus));
}

// The scaled variable's factor k = A / (c s) (A = (1 + alpha) / 2).
__device__ __forceinline__ float bisquare_k(float kA, float c, float s)
{
    return kA * __builtin_amdgcn_rcpf(c * s);
}

// Phase 3 over the n samples xv[c0], ..., xv[c0 + n - 1] of one window, from
// the median m with the scaled k above.  The samples are summed in index
// order whatever the launch shape, so results do not depend on the tiling.
// `n` may be a per-lane count or a wave-uniform one; with a uniform count
// the loop runs on the scalar unit and only the LDS address stays per lane.
__device__ __forceinline__ float bisquare(const float* __restrict__ xv, int c0, int n, float m,
                                          float k, float beta, int iters)
{
    float mu = m;
    const float* x = xv + c0;
    for (int it = 0; it < iters; ++it) {
        const float b = -mu * k;
        float sw = 0.0f, swv = 0.0f;
#pragma unroll 8
        for (int j = 0; j < n; ++j) bisquare_acc(x[j], k, b, beta, sw, swv);
        if (!(sw > 0.0f)) break;  // no weight left: keep mu
        mu = mu_update(mu, swv, sw, k);
    }
    return mu;
}

// Phase 2 sum of squares above the median over xv[c0 .. c0 + n).
__device__ __forceinline__ float upper_ssq(const float* __restrict__ xv, int c0, int n, float m)
{
    float ssq = 0.0f;
    const float* x = xv + c0;
#pragma unroll 8
    for (int j = 0; j < n; ++j) {
        const float d = __builtin_fmaxf(x[j] - m, 0.0f);
        ssq = __builtin_fmaf(d, d, ssq);
    }
    return ssq;
}

// R windows that start at consecutive compacted samples x[0], x[1], ...,
// x[R-1], each n samples long (n >= R): one LDS read feeds every window that
// contains the sample, and each window still sums its samples in index
// order, so the result equals R single-window sweeps bit for bit.
template <int R>
__device__ __forceinline__ void bisquare_multi(const float* __restrict__ x, int n, const float* k,
                                               float* mu, bool* act, float beta, int iters)
{
    for (int it = 0; it < iters; ++it) {
        float b[R], sw[R], swv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            b[r] = -mu[r] * k[r];
            sw[r] = 0.0f;
            swv[r] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < R - 1; ++j) {  // head: windows 0..j
            const float xj = x[j];
#pragma unroll
            for (int r = 0; r <= j; ++r) bisquare_acc(xj, k[r], b[r], beta, sw[r], swv[r]);
        }
#pragma unroll 8
        for (int j = R - 1; j < n; ++j) {  // every window
            const float xj = x[j];
#pragma unroll
            for (int r = 0; r < R; ++r) bisquare_acc(xj, k[r], b[r], beta, sw[r], swv[r]);
        }
#pragma unroll
        for (int d = 1; d < R; ++d) {  // tail: windows d..R-1 take sample n-1+d
            const float xj = x[n - 1 + d];
#pragma unroll
            for (int r = d; r < R; ++r) bisquare_acc(xj, k[r], b[r], beta, sw[r], swv[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (act[r]) {
                if (sw[r] > 0.0f)
                    mu[r] = mu_update(mu[r], swv[r], sw[r], k[r]);
                else
                    act[r] = false;  // no weight left: keep mu from now on
            }
        }
    }
}

// Phase 2 sums for R consecutive windows (see bisquare_multi).
template <int R>
__device__ __forceinline__ void upper_ssq_multi(const float* __restrict__ x, int n, const float* m,
                                                float* ssq)
{
#pragma unroll
    for (int r = 0; r < R; ++r) ssq[r] = 0.0f;
#pragma unroll
    for (int j = 0; j < R - 1; ++j) {
        const float xj = x[j];
#pragma unroll
        for (int r = 0; r <= j; ++r) {
            const float d = __builtin_fmaxf(xj - m[r], 0.0f);
            ssq[r] = __builtin_fmaf(d, d, ssq[r]);
        }
    }
#pragma unroll 4
    for (int j = R - 1; j < n; ++j) {
        const float xj = x[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float d = __builtin_fmaxf(xj - m[r], 0.0f);
            ssq[r] = __builtin_fmaf(d, d, ssq[r]);
        }
    }
#pragma unroll
    for (int d = 1; d < R; ++d) {
        const float xj = x[n - 1 + d];
#pragma unroll
        for (int r = d; r < R; ++r) {
            const float dd = __builtin_fmaxf(xj - m[r], 0.0f);
            ssq[r] = __builtin_fmaf(dd, dd, ssq[r]);
        }
    }
}

// The j-th smallest value (0-based) of the window held at compacted
// positions [ca, cb), from the wavelet matrix and the sorted tile.
__device__ __forceinline__ float window_value(const MainSmem& sm, int levels, uint32_t ca,
                                              uint32_t cb, uint32_t j)
{
    return key_value((uint32_t)(sm.sortbuf[wavelet_kth(sm, levels, ca, cb, j)] >> 32));
}

// Scale ablation: the standard MAD, the lower median of |x - m| over a window
// of n samples with median m.  With the window sorted (v_0 <= ... <= v_{n-1})
// and m = v_q, q = (n-1)/2, the q+1 smallest deviations belong to a run
// v_lo .. v_{lo+q} with 0 <= lo <= q, so the q-th smallest deviation is the
// minimum over lo of max(m - v_lo, v_{lo+q} - m).  The first term falls and
// the second rises with lo: a binary search finds where they cross.  Float
// subtraction is monotone, so the result is the exact MAD rounded once.
__device__ __forceinline__ float window_mad(const MainSmem& sm, int levels, uint32_t ca,
                                         uint32_t n, float m)
{
    const uint32_t cb = ca + n;
    const uint32_t q = (n - 1) >> 1;
    uint32_t lo = 0, hi = q;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const float below = m - window_value(sm, levels, ca, cb, mid);
        const float above = window_value(sm, levels, ca, cb, mid + q) - m;
        if (below <= above)
            hi = mid;
        else
            lo = mid + 1;
    }
    float mad = window_value(sm, levels, ca, cb, lo + q) - m;
    if (lo > 0) mad = __builtin_fminf(mad, m - window_value(sm, levels, ca, cb, lo - 1));
    return mad;
}


// Sort 32 keys in registers ascending (bitonic network).
__device__ __forceinline__ void sort32(uint32_t (&k)[32])
{
#pragma unroll
    for (int kk = 2; kk <= 32; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const int l = i ^ jj;
                if (l > i) {
                    const uint32_t a = k[i], b = k[l];
                    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    k[i] = (i & kk) == 0 ? lo : hi;
                    k[l] = (i & kk) == 0 ? hi : lo;
                }
            }
        }
    }
}

// Phase 1 for up to three consecutive full windows kp[r .. r + W), r < nwin,
// of W <= kSmallW samples given by their totalOrder keys.  The W - 2 keys the
// three share, kp[2 .. W), are sorted once (padded with the largest key); each
// window is that core plus two keys lo <= hi, and its element of rank
// q = (W-1)/2 is min(A[q], max(A[q-1], lo), max(A[q-2], hi)) for the sorted
// core A (an index below 0 reads as the smallest key): the rank-q element of
// a union of two sorted lists, split over the at most two keys of the second.
// The points strictly above each median are counted on the unsorted keys.
// Keys past kp[lim] are never read.  Same results as the tile-sort path,
// without the tile sort and wavelet matrix.
// kW > 0 fixes W at compile time: the padding and the median rank are then
// constants, and the compiler drops every comparator that only moves padding
// or feeds ranks other than q-2 .. q.
template <int kW>
__device__ __forceinline__ void small_window_medians(const uint32_t* __restrict__ kp, int W_rt,
                                                     int nwin, int lim, float* pm, uint32_t* pn)
{
    const int W = kW > 0 ? kW : W_rt;
    const int q = (W - 1) >> 1;  // <= 15, the same for the whole tile
    uint32_t med[3];
    if (W == 1) {
#pragma unroll
        for (int r = 0; r < 3; ++r) med[r] = kp[min(r, lim)];
    } else {
        uint32_t k[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) k[i] = i < W - 2 ? kp[2 + i] : 0xffffffffu;
        sort32(k);
        uint32_t a0 = k[0], a1 = 0u, a2 = 0u;  // A[q], A[q-1], A[q-2]
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            a0 = q == i ? k[i] : a0;
            a1 = q - 1 == i ? k[i] : a1;
            a2 = q - 2 == i ? k[i] : a2;
        }
        const uint32_t ex[4] = {kp[0], kp[1], kp[min(W, lim)], kp[min(W + 1, lim)]};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const uint32_t lo = min(ex[r], ex[r + 1]), hi = max(ex[r], ex[r + 1]);
            med[r] = min(a0, min(max(a1, lo), max(a2, hi)));
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (r < nwin) {
            const float m = key_value(med[r]);
            // strictly above, numerically: -0 and +0 are equal
            const uint32_t T = m == 0.0f ? order_key(0.0f) : med[r];
            uint32_t cnt = 0;
            for (int j = 0; j < W; ++j) cnt += kp[r + j] > T ? 1u : 0u;
            pm[r] = m;
            pn[r] = cnt;
        }
    }
}

// The window of output position p: its valid samples are the compacted
// positions [ca, ca + n) of the staged tile.  False when p is invalid or in a
// dead segment (a NaN output).
template <int kFeat>
__device__ __forceinline__ bool window_range(const MainSmem& sm, const CurveDesc& cd,
                                             const int32_t* __restrict__ segid,
                                             const double* __restrict__ time, int h, int s0,
                                             int N, int m_min, int p, uint32_t& ca, uint32_t& n)
{
    // p's segment: it starts at the valid sample x and holds cnt valid
    // samples (the record sits in the slot of x)
    const int sidp = segid[cd.off + p];
    int x = -1, cnt = 0;
    if (sidp <= -2) {
        x = p;
        cnt = -2 - sidp;
    } else if (sidp >= 0 && sidp < p) {
        const int rec = segid[cd.off + sidp];
        x = sidp;
        cnt = rec <= -2 ? -2 - rec : 0;
    }
    if (x < 0 || cnt < m_min) return false;
    int a = max(p - h, x);
    // the window ends before the next segment's first sample: the first
    // start bit after p within reach of p + h
    const uint32_t from = (uint32_t)(p + 1 - s0);
    uint32_t lim = (uint32_t)(min(p + h, s0 + N - 1) - s0);
    uint32_t wi = from >> 6;
    uint64_t sb = sm.sbits[wi] & (~0ull << (from & 63u));
    while (sb == 0ull && (wi << 6) + 64u <= lim) sb = sm.sbits[++wi];
    if (sb != 0ull) {
        const uint32_t nx = (wi << 6) + (uint32_t)__builtin_ctzll(sb);
        if (nx <= lim) lim = nx - 1u;
    }
    int b = s0 + (int)lim;
    if ((kFeat & kFeatExtra) && cd.window_days > 0.0) {
        // time window: only the samples within half its length of p count.
        // Times are non-decreasing, so they form a run that two scans in from
        // the index window's ends find (invalid samples inside it are skipped
        // by the ranks).
        const double* tc = time + cd.off;
        const double ti = tc[p];
        const double half = 0.5 * cd.window_days;
        while (a < p && !(__builtin_fabs(tc[a] - ti) <= half)) ++a;
        while (b > p && !(__builtin_fabs(tc[b] - ti) <= half)) --b;
    }
    ca = rank1(sm.vbits, sm.vpre, (uint32_t)(a - s0));
    n = rank1(sm.vbits, sm.vpre, (uint32_t)(b - s0 + 1)) - ca;  // >= 1: p is valid
    return true;
}

// Phase 1 of the window at compacted [ca, ca + n) from the sorted tile and
// the wavelet matrix: the median m, and either n+ (the points strictly
// above m, for Eq. 1) or, with the MAD ablation, the scale itself.
__device__ __forceinline__ void window_phase1(const MainSmem& sm, int levels, int nv, int scale,
                                              uint32_t ca, uint32_t n, float& m, float& sc,
                                              uint32_t& nplus)
{
    const uint32_t cb = ca + n;
    const uint32_t rk = wavelet_kth(sm, levels, ca, cb, (n - 1) >> 1);
    m = key_value((uint32_t)(sm.sortbuf[rk] >> 32));
    if (scale == UMI_SCALE_MAD) {
        sc = window_mad(sm, levels, ca, n, m);
        return;
    }
    // the points strictly above m are the window's elements ranked after
    // the last tile element numerically equal to m (ties and -0/+0 sit next
    // to m in the sorted order); a galloping search: one probe without ties,
    // O(log) with many
    uint32_t rh = rk, hi = rk + 1, step = 1;
    while (hi < (uint32_t)nv && key_value((uint32_t)(sm.sortbuf[hi] >> 32)) == m) {
        rh = hi;
        hi = rh + (step <<= 1);
    }
    if (hi > (uint32_t)nv) hi = (uint32_t)nv;
    while (hi - rh > 1u) {  // last equal in [rh, hi)
        const uint32_t mid = (rh + hi) >> 1;
        if (key_value((uint32_t)(sm.sortbuf[mid] >> 32)) == m)
            rh = mid;
        else
            hi = mid;
    }
    // exactly k + 1 window elements rank at or below rk (rk is the window's
    // k-th); of the tile elements tied with m after rk, count those in the
    // window directly when they are few, else with a wavelet descent
    const uint32_t k = (n - 1) >> 1;
    if (rh - rk <= 16u) {
        uint32_t tied = 0;
        for (uint32_t j = rk + 1; j <= rh; ++j)
            tied += ((uint32_t)(sm.sortbuf[j] & 0xffffffffull) - ca < n) ? 1u : 0u;
        nplus = n - k - 1 - tied;
    } else {
        nplus = n - wavelet_count_less(sm, levels, ca, cb, rh + 1);
    }
}

// The windows of one tile: each lane takes R consecutive output positions.
template <int R, int kFeat>
__device__ __forceinline__ void tile_windows(const MainSmem& sm, int levels, int nv,
                                             const CurveDesc& cd, int h, int s0, int N, int t0,
                                             int t1,
                                             const int32_t* __restrict__ segid, float alpha,
                                             float c, int iters, int scale, bool simple,
                                             const float* pm, const uint32_t* pn,
                                             const double* __restrict__ time,
                                             float* __restrict__ trend,
                                             float* __restrict__ median,
                                             float* __restrict__ detrended)
{
    const int m_min = max(1, cd.W / 3);
    const int pfirst = t0 + (int)threadIdx.x * R;
    uint32_t ca[R], n[R];
    bool live[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = pfirst + r;
        ca[r] = 0;
        n[r] = 0;
        if ((kFeat & kFeatSmall) && simple) {
            // a small-window tile: the whole span is valid and in one live
            // segment, so every window is full and its compacted range is its
            // staged range
            live[r] = p < t1;
            ca[r] = (uint32_t)(p - h - s0);
            n[r] = (uint32_t)cd.W;
        } else {
            live[r] = p < t1 &&
                      window_range<kFeat>(sm, cd, segid, time, h, s0, N, m_min, p, ca[r], n[r]);
        }
    }
    // The common case -- every window of the wave live, of one length, and
    // consecutive -- runs the fused loops with a wave-uniform trip count.
    const uint32_t n_u = __builtin_amdgcn_readfirstlane(n[0]);
    bool mine = live[0] && n[0] == n_u && n_u >= (uint32_t)R;
#pragma unroll
    for (int r = 1; r < R; ++r) mine = mine && live[r] && n[r] == n_u && ca[r] == ca[0] + r;
    const bool uniform = __all(mine);

    // Phase 1 (median) and Phase 2 (Eq. 1, or the MAD ablation) per window
    float m[R], sc[R];
    uint32_t nplus[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        m[r] = 0.0f;
        sc[r] = 0.0f;
        nplus[r] = 0;
        if (live[r] && simple) {
            m[r] = pm[r];  // from the small-window networks
            nplus[r] = pn[r];
        } else if (live[r]) {
            window_phase1(sm, levels, nv, scale, ca[r], n[r], m[r], sc[r], nplus[r]);
        }
    }
    if (scale != UMI_SCALE_MAD) {
        float ssq[R];
        if (uniform) {
            upper_ssq_multi<R>(sm.xv + ca[0], (int)n_u, m, ssq);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                ssq[r] = live[r] ? upper_ssq(sm.xv, (int)ca[r], (int)n[r], m[r]) : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (nplus[r] > 0) sc[r] = upper_scale(ssq[r], nplus[r]);
    }
    float k[R], mu[R];
    bool act[R];
    const float kA = 0.5f * (1.0f + alpha);         // A of the folded residual
    const float beta = (1.0f - alpha) / (1.0f + alpha);  // B / A
#pragma unroll
    for (int r = 0; r < R; ++r) {
        mu[r] = m[r];
        k[r] = 0.0f;
        act[r] = false;
        if (live[r] && sc[r] > 0.0f && iters > 0) {
            const float kk = bisquare_k(kA, c, sc[r]);
            if (isfinite(kk)) {
                k[r] = kk;
                act[r] = true;
            }
        }
    }
    // Phase 3 (Eqs. 2-4)
    if (uniform) {
        bisquare_multi<R>(sm.xv + ca[0], (int)n_u, k, mu, act, beta, iters);
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (act[r]) mu[r] = bisquare(sm.xv, (int)ca[r], (int)n[r], m[r], k[r], beta, iters);
    }
    const float nanf_ = __builtin_nanf("");
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = pfirst + r;
        if (p < t1) {
            trend[cd.off + p] = live[r] ? mu[r] : nanf_;
            if (median) median[cd.off + p] = live[r] ? m[r] : nanf_;
            if (detrended) {
                // normalisation stage: flux / trend (a live sample is valid,
                // so its compacted position is its rank among valid ones)
                float d = nanf_;
                if (live[r]) d = sm.xv[rank1(sm.vbits, sm.vpre, (uint32_t)(p - s0))] / mu[r];
                detrended[cd.off + p] = d;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Split windows: G lanes share one window (tiles of at most kMainThreads / G
// output positions).  Lane l of a group sums the window samples l, l + G,
// l + 2G, ... in order, and a butterfly over the group's G consecutive lanes
// combines the partial sums -- lane xor 1 and xor 2 by DPP quad permutes,
// xor 4 by a ds_swizzle -- in one fixed order.  Every lane of a group ends
// with the same bits (IEEE addition commutes), so the group's lanes iterate
// in step.  The sums are ordered differently from the one-lane-per-window
// path, so the two agree to rounding, not bit for bit; each is deterministic.

__device__ __forceinline__ float dpp_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ float dpp_xor2(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}

__device__ __forceinline__ float swizzle_xor4(float v)
{
    // bitmask mode: and 0x1f, or 0, xor 4 (lanes within 32-lane halves)
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
}

template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(G == 2 || G == 4 || G == 8, "group of 2, 4 or 8 lanes");
    v = v + dpp_xor1(v);
    if (G >= 4) v = v + dpp_xor2(v);
    if (G >= 8) v = v + swizzle_xor4(v);
    return v;
}

// f(x[j]) for j = l, l + G, l + 2G, ... below n, in that order; eight loads
// are issued ahead of their use, so a lane waits on LDS once per eight
// samples rather than once per sample (the order of the sums is unchanged).
template <int G, class F>
__device__ __forceinline__ void strided_sweep(const float* __restrict__ x, int l, int n, F&& f)
{
    int j = l;
    for (; j + 7 * G < n; j += 8 * G) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = x[j + u * G];
#pragma unroll
        for (int u = 0; u < 8; ++u) f(v[u]);
    }
    for (; j < n; j += G) f(x[j]);
}

// Sum over a group of G consecutive lanes (G = 2, 4, 8), integers.
template <int G>
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    if (G >= 4) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    if (G >= 8) v += (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
    return v;
}

// Phase 1 of a split-tile window from the sorted tile alone (no wavelet
// matrix).  The window's G lanes walk the sorted (key, index) pairs from the
// smallest, 8G at a time (lane l takes the 8 consecutive pairs from 8l), and
// count the pairs whose compacted index lies in [ca, ca + n); the pair at
// which the count reaches k + 1 is the window's k-th smallest, the same
// position wavelet_kth gives.  Each lane's counts of a step travel packed 4
// bits per lane through one group sum, so every lane of the group sees them
// all and takes the same decisions.  Padding pairs (~0) lie in no window, and
// a step never reads past npad (a power of two >= 64, so a multiple of 8G).
// The walk takes about nv / 16G steps to a median, against a wavelet build
// of log2(npad) levels of four barriers each for the whole tile.  The median
// and n+ are the same integers as window_phase1's.
template <int G>
__device__ __forceinline__ void window_phase1_scan(const MainSmem& sm, int nv, uint32_t ca,
                                                   uint32_t n, float& m, uint32_t& nplus)
{
    const uint32_t l = threadIdx.x & (G - 1);
    const uint32_t k = (n - 1) >> 1;
    uint32_t need = k + 1;  // window pairs still to pass, the k-th included
    uint32_t rk = 0;
    for (int j0 = 0; j0 < nv; j0 += 8 * G) {
        const int q0 = j0 + 8 * (int)l;
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = sm.sortbuf[q0 + u];
        uint32_t bits = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            bits |= ((uint32_t)(v[u] & 0xffffffffull) - ca < n ? 1u : 0u) << u;
        const uint32_t packed = group_sum_u32<G>((uint32_t)__popc(bits) << (4 * l));
        uint32_t below = 0, lane_hit = G;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t cg = (packed >> (4 * g)) & 15u;
            if (lane_hit == G) {
                if (below + cg >= need)
                    lane_hit = g;
                else
                    below += cg;
            }
        }
        if (lane_hit == G) {  // not in this step
            need -= below;
            continue;
        }
        // the (need - below)-th window pair of lane lane_hit's eight
        uint32_t pos = 0;
        if (l == lane_hit) {
            uint32_t b = bits;
            for (uint32_t r = need - below; r > 1u; --r) b &= b - 1u;
            pos = (uint32_t)q0 + (uint32_t)__builtin_ctz(b);
        }
        rk = group_sum_u32<G>(pos);
        break;
    }
    m = key_value((uint32_t)(sm.sortbuf[rk] >> 32));
    // the points strictly above m: the window pairs after the last tile pair
    // numerically equal to m (ties sit next to m in the sorted order)
    uint32_t rh = rk, hi = rk + 1, step = 1;
    while (hi < (uint32_t)nv && key_value((uint32_t)(sm.sortbuf[hi] >> 32)) == m) {
        rh = hi;
        hi = rh + (step <<= 1);
    }
    if (hi > (uint32_t)nv) hi = (uint32_t)nv;
    while (hi - rh > 1u) {  // last equal in [rh, hi)
        const uint32_t mid = (rh + hi) >> 1;
        if (key_value((uint32_t)(sm.sortbuf[mid] >> 32)) == m)
            rh = mid;
        else
            hi = mid;
    }
    uint32_t tied = 0;
    for (uint32_t j = rk + 1 + l; j <= rh; j += G)
        tied += ((uint32_t)(sm.sortbuf[j] & 0xffffffffull) - ca < n) ? 1u : 0u;
    tied = group_sum_u32<G>(tied);
    nplus = n - k - 1 - tied;
}

template <int G, int kFeat>
__device__ __forceinline__ void tile_windows_split(const MainSmem& sm, int levels, int nv,
                                                   const CurveDesc& cd, int h, int s0, int N,
                                                   int t0, int t1,
                                                   const int32_t* __restrict__ segid,
                                                   float alpha, float c, int iters, int scale,
                                                   const double* __restrict__ time,
                                                   float* __restrict__ trend,
                                                   float* __restrict__ median,
                                                   float* __restrict__ detrended, bool scan)
{
    const int m_min = max(1, cd.W / 3);
    const int l = (int)threadIdx.x & (G - 1);
    const int p = t0 + (int)threadIdx.x / G;
    uint32_t ca = 0, n = 0;
    const bool live =
        p < t1 && window_range<kFeat>(sm, cd, segid, time, h, s0, N, m_min, p, ca, n);
    float m = 0.0f, sc = 0.0f;
    uint32_t nplus = 0;
    if (live) {  // same on every lane
        if (scan)
            window_phase1_scan<G>(sm, nv, ca, n, m, nplus);
        else
            window_phase1(sm, levels, nv, scale, ca, n, m, sc, nplus);
    }
    const float* x = sm.xv + ca;
    if (live && scale != UMI_SCALE_MAD) {
        // Phase 2 (Eq. 1)
        float ssq = 0.0f;
        strided_sweep<G>(x, l, (int)n, [&](float xj) {
            const float d = __builtin_fmaxf(xj - m, 0.0f);
            ssq = __builtin_fmaf(d, d, ssq);
        });
        ssq = group_sum<G>(ssq);
        if (nplus > 0) sc = upper_scale(ssq, nplus);
    }
    // Phase 3 (Eqs. 2-4), as in the one-lane path
    float mu = m;
    const float kA = 0.5f * (1.0f + alpha);
    const float beta = (1.0f - alpha) / (1.0f + alpha);
    const float kk = live && sc > 0.0f ? bisquare_k(kA, c, sc) : 0.0f;
    if (live && sc > 0.0f && iters > 0 && isfinite(kk)) {
        for (int it = 0; it < iters; ++it) {
            const float b = -mu * kk;
            float sw = 0.0f, swv = 0.0f;
            strided_sweep<G>(x, l, (int)n,
                             [&](float xj) { bisquare_acc(xj, kk, b, beta, sw, swv); });
            sw = group_sum<G>(sw);
            swv = group_sum<G>(swv);
            if (!(sw > 0.0f)) break;  // no weight left: keep mu
            mu = mu_update(mu, swv, sw, kk);
        }
    }
    if (p < t1 && l == 0) {
        const float nanf_ = __builtin_nanf("");
        trend[cd.off + p] = live ? mu : nanf_;
        if (median) median[cd.off + p] = live ? m : nanf_;
        if (detrended) {
            float d = nanf_;
            if (live) d = sm.xv[rank1(sm.vbits, sm.vpre, (uint32_t)(p - s0))] / mu;
            detrended[cd.off + p] = d;
        }
    }
}

// kFeat (kFeat* bits) selects the paths an instance carries: the
// small-window networks, split tiles, and the MAD ablation with time windows.
// The host launches the smallest instance that covers the batch; fewer paths
// leave the compiler more registers for the rest, and every instance gives
// the same results on the batches it serves.
template <int kFeat>
__global__ __launch_bounds__(kMainThreads, 8) void umi_main_kernel(
    const float* __restrict__ flux, const int32_t* __restrict__ segid,
    const BatchHeader* __restrict__ hdr,
    const CurveDesc* __restrict__ curves, const int2* __restrict__ tiles, int tile_first,
    int tile_count, uint32_t* __restrict__ counter, float* __restrict__ trend,
    float* __restrict__ median)
{
    __shared__ MainSmem sm;
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wave = tid >> 6;
    const int iters = hdr->iters;
    const int scale = (kFeat & kFeatExtra) ? hdr->scale : (int)UMI_SCALE_UPPER_RMS;
    float* const detrended = hdr->detrended;
    const double* const time = hdr->time;
    // tile range [tile_first, tile_end): a count < 0 means "all tiles of the batch"
    const int tile_end = tile_count < 0 ? hdr->n_tiles : tile_first + tile_count;

    for (int round = 0;; ++round) {
        // Instances with split tiles serve small batches, where a workgroup
        // often has one tile: its first tile is its block index, and the
        // queue counter hands out the tiles after the grid's first round
        // (not touched at all when the first round covers every tile).
        constexpr bool kStaticFirst = (kFeat & kFeatSplit) != 0;
        if (tid == 0) {
            if (counter && !(kStaticFirst && round == 0))
                sm.tile = (kStaticFirst && tile_first + (int)gridDim.x >= tile_end)
                              ? tile_end
                              : tile_first + (kStaticFirst ? (int)gridDim.x : 0) +
                                    (int)atomicAdd(counter, 1u);
            else
                sm.tile = tile_first + (int)blockIdx.x + round * (int)gridDim.x;
        }
        __syncthreads();
        const int tile = sm.tile;
        if (tile >= tile_end) break;

        const int2 td = tiles[tile];
        const CurveDesc cd = curves[td.x];
        const float alpha = cd.alpha;
        const float c = cd.c;
        const int h = (cd.W - 1) >> 1;
        const int t0 = td.y;
        const int t1 = min(t0 + cd.tile, cd.len);
        const int s0 = max(t0 - h, 0);
        const int s1 = min(t1 + h, cd.len);
        const int N = s1 - s0;  // <= kStageMax, guaranteed by the host
        const float* f = flux + cd.off + s0;
        const int32_t* sg = segid + cd.off + s0;

        // --- staged validity bit vector (valid = finite flux and time) ---
        // A tile is "simple" when every one of its windows is full: a small
        // W, no curve end within reach, and the whole span valid and in one
        // segment.  Its medians then come from per-window networks.
        // segment of staged sample i (the start index of its segment, -1 if
        // invalid): a segment's first slot holds its record instead
        const int sg0 = sg[0];
        const int seg0 = sg0 >= 0 ? sg0 : (sg0 == -1 ? -1 : s0);
        bool same = true;
        const int nwv = (N >> 6) + 1;
        for (int i0 = wave * 64; i0 < nwv * 64; i0 += kMainThreads) {
            const int i = i0 + lane;
            const int sgi = i < N ? sg[i] : sg0;
            const bool ok = (i < N) && (sgi != -1);
            if (kFeat & kFeatSmall) {
                const int segi = i < N ? (sgi >= 0 ? sgi : (sgi == -1 ? -1 : s0 + i)) : seg0;
                same = same && segi == seg0;
            }
            const uint64_t bal = __ballot(ok);
            const uint64_t st = __ballot(ok && sgi <= -2);
            if (lane == 0) {
                sm.vbits[i0 >> 6] = bal;
                sm.sbits[i0 >> 6] = st;
            }
        }
        // lanes per window (1: R windows per lane)
        const int G = (kFeat & kFeatSplit) ? split_lanes(cd.tile) : 1;
        bool simple = false;
        if (kFeat & kFeatSmall)
            simple = __syncthreads_and(same) && seg0 >= 0 && cd.W <= kSmallW &&
                     scale != UMI_SCALE_MAD && cd.window_days == 0.0 && t0 >= h &&
                     t1 + h <= cd.len && G == 1;
        else
            __syncthreads();
        word_prefix(sm.vbits, sm.vpre, nwv, reinterpret_cast<uint32_t*>(&sm.nvalid));
        __syncthreads();
        const int nv = sm.nvalid;
        int npad = 64;
        while (npad < nv) npad <<= 1;
        int levels = 6;
        while ((1 << levels) < npad) ++levels;
        const bool scan_tile = (kFeat & kFeatSplit) && G > 1 && scale != UMI_SCALE_MAD;

        if (simple) {
            // every staged sample is valid: values and keys in index order
            uint32_t* keys = reinterpret_cast<uint32_t*>(sm.seq);
            for (int i = tid; i < N; i += kMainThreads) {
                const float x = f[i];
                sm.xv[i] = x;
                keys[i] = order_key(x);
            }
            __syncthreads();
        } else {
        // --- compaction: values in index order, (key, index) for the sort ---
        for (int i0 = wave * 64; i0 < nwv * 64; i0 += kMainThreads) {
            const int i = i0 + lane;
            if (i < N && sg[i] != -1) {
                const float x = f[i];
                const uint32_t ci = rank1(sm.vbits, sm.vpre, (uint32_t)i);
                sm.xv[ci] = x;
                sm.sortbuf[ci] = ((uint64_t)order_key(x) << 32) | ci;
            }
        }
        for (int i = nv + tid; i < npad; i += kMainThreads) sm.sortbuf[i] = ~0ull;
        __syncthreads();

        if ((kFeat & kFeatSplit) && npad <= kMainThreads) {
            // --- a small tile: every element counts the elements below it ---
            // The (key, index) pairs are distinct, so the counts are the
            // ranks the sorting network would give, without a barrier per
            // network stage; padding [nv, npad) already holds ~0.
            uint64_t mine = 0;
            uint32_t rank = 0;
            if (tid < nv) {
                mine = sm.sortbuf[tid];
                // eight loads ahead of their compares; the padding up to the
                // next multiple of eight (within npad) holds ~0 and counts 0
                for (int j0 = 0; j0 < nv; j0 += 8) {
                    uint64_t v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = sm.sortbuf[j0 + u];
#pragma unroll
                    for (int u = 0; u < 8; ++u) rank += v[u] < mine ? 1u : 0u;
                }
            }
            __syncthreads();
            if (tid < nv) sm.sortbuf[rank] = mine;
            __syncthreads();
        } else {
            // --- bitonic sort of sortbuf[0, npad) ascending ---
            for (int kk = 2; kk <= npad; kk <<= 1) {
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int cix = tid; cix < (npad >> 1); cix += kMainThreads) {
                        const int i = 2 * cix - (cix & (jj - 1));
                        const int l = i + jj;
                        const uint64_t a = sm.sortbuf[i], b = sm.sortbuf[l];
                        const bool asc = (i & kk) == 0;
                        if ((a > b) == asc) {
                            sm.sortbuf[i] = b;
                            sm.sortbuf[l] = a;
                        }
                    }
                    __syncthreads();
                }
            }
        }

        // --- wavelet matrix over the sequence rank_of[compacted index]; split
        // tiles take their medians from the sorted tile directly ---
        if (!scan_tile) {
        for (int r = tid; r < npad; r += kMainThreads) {
            if (r < nv)
                sm.seq[0][(uint32_t)(sm.sortbuf[r] & 0xffffffffull)] = (uint16_t)r;
            else
                sm.seq[0][r] = (uint16_t)(npad - 1);
        }
        __syncthreads();
        const int nwl = (npad >> 6) + 1;
        for (int l = 0; l < levels; ++l) {
            const uint16_t* cur = sm.seq[l & 1];
            uint16_t* nxt = sm.seq[(l + 1) & 1];
            const int bit = levels - 1 - l;
            for (int i0 = wave * 64; i0 < nwl * 64; i0 += kMainThreads) {
                const int i = i0 + lane;
                const bool one = (i < npad) && (((cur[i < npad ? i : 0] >> bit) & 1) != 0);
                const uint64_t bal = __ballot(one);
                if (lane == 0) sm.bits[l][i0 >> 6] = bal;
            }
            __syncthreads();
            uint32_t ones_total;
            word_prefix(sm.bits[l], sm.pre[l], nwl, &sm.zeros[l]);
            __syncthreads();
            if (tid == 0) {
                ones_total = sm.zeros[l];
                sm.zeros[l] = (uint32_t)npad - ones_total;
            }
            __syncthreads();
            const uint32_t z = sm.zeros[l];
            for (int i = tid; i < npad; i += kMainThreads) {
                const uint16_t val = cur[i];
                const uint32_t o = rank1(sm.bits[l], sm.pre[l], (uint32_t)i);
                const bool one = ((val >> bit) & 1) != 0;
                nxt[one ? z + o : (uint32_t)i - o] = val;
            }
            __syncthreads();
        }
        }  // wavelet
        }  // not simple

        // --- the tile's windows: G lanes per position, or R consecutive
        // positions per lane ---
        if ((kFeat & kFeatSplit) && G > 1) {
            if (G == 2)
                tile_windows_split<2, kFeat>(sm, levels, nv, cd, h, s0, N, t0, t1, segid, alpha, c, iters,
                                      scale, time, trend, median, detrended, scan_tile);
            else if (G == 4)
                tile_windows_split<4, kFeat>(sm, levels, nv, cd, h, s0, N, t0, t1, segid, alpha, c, iters,
                                      scale, time, trend, median, detrended, scan_tile);
            else
                tile_windows_split<8, kFeat>(sm, levels, nv, cd, h, s0, N, t0, t1, segid, alpha, c, iters,
                                      scale, time, trend, median, detrended, scan_tile);
            __syncthreads();
            continue;
        }
        const int R = (t1 - t0 + kMainThreads - 1) / kMainThreads;  // tile <= kMaxTile -> R <= 3
        // Simple tiles: Phase 1 of this lane's windows from the networks, run
        // here where few registers are live (every window is [p-h, p+h], all
        // of it valid, so its keys start at staged index p - h - s0).
        float pm[3] = {0.0f, 0.0f, 0.0f};
        uint32_t pn[3] = {0u, 0u, 0u};
        if (simple) {
            const uint32_t* keys = reinterpret_cast<const uint32_t*>(sm.seq);
            const int p0 = t0 + tid * R;
            if (p0 < t1) {
                const int b = p0 - h - s0;
                if (cd.W == 25)  // the Kepler long-cadence window
                    small_window_medians<25>(keys + b, 25, min(R, t1 - p0), N - 1 - b, pm, pn);
                else
                    small_window_medians<0>(keys + b, cd.W, min(R, t1 - p0), N - 1 - b, pm, pn);
            }
        }
        if (R == 3)
            tile_windows<3, kFeat>(sm, levels, nv, cd, h, s0, N, t0, t1, segid, alpha, c, iters, scale,
                            simple, pm, pn, time, trend, median, detrended);
        else if (R == 2)
            tile_windows<2, kFeat>(sm, levels, nv, cd, h, s0, N, t0, t1, segid, alpha, c, iters, scale,
                            simple, pm, pn, time, trend, median, detrended);
        else
            tile_windows<1, kFeat>(sm, levels, nv, cd, h, s0, N, t0, t1, segid, alpha, c, iters, scale,
                            simple, pm, pn, time, trend, median, detrended);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Copy kernel (serving helper, not a step of the method): one workgroup per
// piece of a list of copies between device memory and pinned host memory,
// read and written directly over the bus rather than through the runtime's
// copy engines.

__global__ __launch_bounds__(256) void umi_copy_kernel(CopyBatch cb)
{
    __shared__ int sh_copy;
    const int piece = (int)blockIdx.x;
    if (threadIdx.x < 64) {  // the copy this piece belongs to: last i with first[i] <= piece
        const int lane = (int)threadIdx.x;
        const bool le = lane < cb.n && cb.first[lane] <= piece;
        const uint64_t m = __ballot(le);  // lane 0 always qualifies
        if (lane == 0) sh_copy = 63 - __builtin_clzll(m);
    }
    __syncthreads();
    const int i = sh_copy;
    const int64_t off = (int64_t)(piece - cb.first[i]) * kCopyPieceBytes;
    const int64_t len = min((int64_t)kCopyPieceBytes, cb.bytes[i] - off);
    const uint8_t* src = cb.src[i] + off;
    uint8_t* dst = cb.dst[i] + off;
    const uintptr_t align = (uintptr_t)src | (uintptr_t)dst | (uintptr_t)len;
    if ((align & 15u) == 0) {
        const uint4* s4 = reinterpret_cast<const uint4*>(src);
        uint4* d4 = reinterpret_cast<uint4*>(dst);
        for (int64_t k = threadIdx.x; k < len / 16; k += blockDim.x) d4[k] = s4[k];
    } else if ((align & 3u) == 0) {
        const uint32_t* s1 = reinterpret_cast<const uint32_t*>(src);
        uint32_t* d1 = reinterpret_cast<uint32_t*>(dst);
        for (int64_t k = threadIdx.x; k < len / 4; k += blockDim.x) d1[k] = s1[k];
    } else {
        for (int64_t k = threadIdx.x; k < len; k += blockDim.x) dst[k] = src[k];
    }
}

// ---------------------------------------------------------------------------
// Host-side launch wrappers (the host library calls only these).

// `one` (host memory, read before the call returns), for a batch of one curve
// taking the chunked form: that curve's table entry, passed to the kernel by
// value so that it need not read the staged table before its first step.
hipError_t launch_prepass(const float* flux, const double* time, uint8_t* block,
                          const uint8_t* stage, int curve_one, int grid, int32_t* segid,
                          int2* tiles, Counters* ctr, ChunkRec* recs, bool clear_queue, bool walk,
                          const CurveDesc* one, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    // read the header and table from the staging block (and copy them into
    // `block`), or from `block` itself
    const uint8_t* src = stage ? stage : block;
    uint8_t* to = stage ? block : nullptr;
    // one workgroup per curve, from curve_one (or the first) on
    int32_t* trash = reinterpret_cast<int32_t*>(&ctr->trash);
    if (walk && time)
        hipLaunchKernelGGL((umi_prepass_walk_kernel<kPrepThreads, kPrepWalkItems, true>),
                           dim3(grid), dim3(kPrepThreads), 0, stream, flux, time, src, to,
                           curve_one < 0 ? 0 : curve_one, segid, tiles,
                           clear_queue ? &ctr->queue : nullptr, trash);
    else if (walk)
        hipLaunchKernelGGL((umi_prepass_walk_kernel<kPrepThreads, kPrepWalkItems, false>),
                           dim3(grid), dim3(kPrepThreads), 0, stream, flux, time, src, to,
                           curve_one < 0 ? 0 : curve_one, segid, tiles,
                           clear_queue ? &ctr->queue : nullptr, trash);
    else
        hipLaunchKernelGGL((umi_prepass_chunk_kernel<kPrepThreads, kPrepItems>), dim3(grid),
                           dim3(kPrepThreads), 0, stream, flux, time, src, to, curve_one,
                           segid, tiles, ctr, recs, clear_queue ? 1 : 0,
                           one ? *one : CurveDesc{},
                           one ? (one->len + kPrepChunk - 1) / kPrepChunk : -1);
    return hipGetLastError();
}

hipError_t launch_copy(const CopyBatch& cb, hipStream_t stream)
{
    const int pieces = cb.first[cb.n];
    if (pieces <= 0) return hipSuccess;
    hipLaunchKernelGGL(umi_copy_kernel, dim3(pieces), dim3(256), 0, stream, cb);
    return hipGetLastError();
}

hipError_t launch_main(const float* flux, const int32_t* segid, const BatchHeader* hdr,
                       const CurveDesc* curves, const int2* tiles, int tile_first,
                       int tile_count, uint32_t* counter, int grid, float* trend, float* median,
                       int feat, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
#define UMI_LAUNCH_MAIN(F)                                                                      \
    hipLaunchKernelGGL(umi_main_kernel<F>, dim3(grid), dim3(kMainThreads), 0, stream, flux, segid, \
                       hdr, curves, tiles, tile_first, tile_count, counter, trend, median)
    // the instances built: none, small windows, split tiles, everything
    if (feat == 0)
        UMI_LAUNCH_MAIN(0);
    else if (feat == kFeatSmall)
        UMI_LAUNCH_MAIN(kFeatSmall);
    else if (feat == kFeatSplit)
        UMI_LAUNCH_MAIN(kFeatSplit);
    else
        UMI_LAUNCH_MAIN(kFeatAll);
#undef UMI_LAUNCH_MAIN
    return hipGetLastError();
}

}  // namespace umi
