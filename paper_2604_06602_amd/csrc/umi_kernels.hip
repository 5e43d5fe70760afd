// HIP kernels of the UMI library for CDNA4 (gfx950).
//
// Two kernels run per batch, both on the caller's stream:
//
//   umi_prepass_kernel  one workgroup per curve.  Validity and segmentation
//                       (gap handling, minimum segment length W/3 of
//                       Section 4.4): a chunked block scan writes a segment id
//                       per sample and one record per segment, and lays out the
//                       curve's tile list for the main kernel.
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

// Inclusive "latest valid sample" scan: the largest index seen so far (-1 if
// none) together with its time.
__device__ __forceinline__ void wave_incl_latest(int& idx, double& t)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int yi = __shfl_up(idx, d, 64);
        double yt = __shfl_up(t, d, 64);
        if (lane >= d && yi > idx) {
            idx = yi;
            t = yt;
        }
    }
}

// Exclusive block-wide sum over NT threads; `total` gets the sum.
template <int NT>
__device__ __forceinline__ int block_excl_sum(int x, int* sh, int& total)
{
    const int incl = wave_incl_sum(x);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) sh[w] = incl;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        int v = sh[i];
        before += (i < w) ? v : 0;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return before + incl - x;
}

// ---------------------------------------------------------------------------
// Pre-pass: segments and tiles.

template <int NT>
__global__ __launch_bounds__(NT) void umi_prepass_kernel(
    const float* __restrict__ flux, const double* __restrict__ time,
    const BatchHeader* __restrict__ hdr, const CurveDesc* __restrict__ curves, int curve_first,
    int32_t* __restrict__ segid, int4* __restrict__ segtab,
    int2* __restrict__ tiles, uint32_t* __restrict__ counter)
{
    __shared__ int sh_li[NT / 64];
    __shared__ double sh_lt[NT / 64];
    __shared__ int sh_a[NT / 64];
    __shared__ int sh_b[NT / 64];

    if (counter != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
    const int cidx = curve_first + (int)blockIdx.x;
    if (cidx >= hdr->n_curves) return;  // fixed-size grids cover fewer curves
    const CurveDesc cd = curves[cidx];

    const int ntiles = cd.len > 0 ? (cd.len + cd.tile - 1) / cd.tile : 0;
    for (int t = threadIdx.x; t < ntiles; t += NT)
        tiles[cd.tile_base + t] = make_int2(cidx, t * cd.tile);

    const float* f = flux + cd.off;
    const double* tm = time ? time + cd.off : nullptr;
    int32_t* sid = segid + cd.off;
    int* tab = reinterpret_cast<int*>(segtab + cd.off);

    // carries from earlier chunks (uniform over the block)
    int c_idx = -1;    // latest valid index
    double c_t = 0.0;  // its time
    int c_vc = 0;      // valid samples so far
    int c_ns = 0;      // segments so far

    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    constexpr int kChunk = NT * kPrepItems;

    // The next chunk's flux and times are loaded while the current one is
    // scanned, so the loads' latency overlaps the block scans.
    float fv[kPrepItems];
    double tv[kPrepItems];
    auto load_chunk = [&](int base, float* fo, double* to) {
#pragma unroll
        for (int q = 0; q < kPrepItems; ++q) {
            const int e = base + (int)threadIdx.x * kPrepItems + q;
            fo[q] = e < cd.len ? f[e] : __builtin_nanf("");
            to[q] = (tm != nullptr && e < cd.len) ? tm[e] : 0.0;
        }
    };
    load_chunk(0, fv, tv);

    for (int base = 0; base < cd.len; base += kChunk) {
        float nf[kPrepItems];
        double nt[kPrepItems];
        if (base + kChunk < cd.len) load_chunk(base + kChunk, nf, nt);
        const int e0 = base + (int)threadIdx.x * kPrepItems;
        uint32_t vmask = 0;  // bit q: item q is valid
        double t[kPrepItems];
        int a_idx = -1, a_cnt = 0;
        double a_t = 0.0;
#pragma unroll
        for (int q = 0; q < kPrepItems; ++q) {
            const int e = e0 + q;
            const bool ok = e < cd.len && isfinite(fv[q]) && (tm == nullptr || isfinite(tv[q]));
            vmask |= (ok ? 1u : 0u) << q;
            t[q] = tv[q];
            if (ok) {
                a_idx = e;
                a_t = tv[q];
                ++a_cnt;
            }
        }

        // latest valid sample before this thread's items, and valid count
        int li = a_idx;
        double lt = a_t;
        wave_incl_latest(li, lt);
        int ex_i = __shfl_up(li, 1, 64);
        double ex_t = __shfl_up(lt, 1, 64);
        if (lane == 0) {
            ex_i = -1;
            ex_t = 0.0;
        }
        if (lane == 63) {
            sh_li[w] = li;
            sh_lt[w] = lt;
        }
        int tot_cnt;
        const int ex_cnt = block_excl_sum<NT>(a_cnt, sh_a, tot_cnt);  // syncs
        int blk_i = -1;
        double blk_t = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            const int wi = sh_li[i];
            if (wi > blk_i) {
                blk_i = wi;
                blk_t = sh_lt[i];
            }
            if (i + 1 == w && ex_i < 0) {
                // nothing earlier in this wave: take the lower waves' latest
                ex_i = blk_i;
                ex_t = blk_t;
            }
        }
        if (ex_i < 0) {
            ex_i = c_idx;
            ex_t = c_t;
        }

        // segment starts among this thread's items
        uint32_t smask = 0;  // bit q: item q starts a segment
        int n_st = 0;
        {
            int pi = ex_i;
            double pt = ex_t;
#pragma unroll
            for (int q = 0; q < kPrepItems; ++q) {
                if ((vmask >> q) & 1u) {
                    const bool st = (pi < 0) || (tm != nullptr && (t[q] - pt) > kGapDays);
                    smask |= (st ? 1u : 0u) << q;
                    n_st += st ? 1 : 0;
                    pi = e0 + q;
                    pt = t[q];
                }
            }
        }
        int tot_st;
        const int ex_st = block_excl_sum<NT>(n_st, sh_b, tot_st);  // syncs
        {
            int s = c_ns + ex_st - 1;
            int pi = ex_i;               // previous valid index
            int vc = c_vc + ex_cnt;      // valid samples before item q
#pragma unroll
            for (int q = 0; q < kPrepItems; ++q) {
                const int e = e0 + q;
                if (e < cd.len) {
                    if ((vmask >> q) & 1u) {
                        if ((smask >> q) & 1u) {
                            ++s;
                            tab[4 * s + 0] = e;
                            tab[4 * s + 2] = vc;
                            if (s > 0) {
                                tab[4 * (s - 1) + 1] = pi;
                                tab[4 * (s - 1) + 3] = vc;
                            }
                        }
                        sid[e] = s;
                        pi = e;
                        ++vc;
                    } else {
                        sid[e] = -1;
                    }
                }
            }
        }
        if (blk_i >= 0) {
            c_idx = blk_i;
            c_t = blk_t;
        }
        c_vc += tot_cnt;
        c_ns += tot_st;
#pragma unroll
        for (int q = 0; q < kPrepItems; ++q) {
            fv[q] = nf[q];
            tv[q] = nt[q];
        }
        __syncthreads();  // sh_li / sh_lt reused by the next chunk
    }
    if (threadIdx.x == 0 && c_ns > 0) {
        tab[4 * (c_ns - 1) + 1] = c_idx;
        tab[4 * (c_ns - 1) + 3] = c_vc;
    }
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
        mu = mu + swv / (sw * k);
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
                    mu[r] = mu[r] + swv[r] / (sw[r] * k[r]);
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

constexpr int kSmallW = 31;

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

// The windows of one tile: each lane takes R consecutive output positions.
template <int R>
__device__ __forceinline__ void tile_windows(const MainSmem& sm, int levels, int nv,
                                             const CurveDesc& cd, int h, int s0, int t0, int t1,
                                             const int32_t* __restrict__ segid,
                                             const int4* __restrict__ segtab, float alpha,
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
        live[r] = false;
        ca[r] = 0;
        n[r] = 0;
        if (p < t1) {
            const int sidp = segid[cd.off + p];
            if (sidp >= 0) {
                const int4 seg = segtab[cd.off + sidp];
                if (seg.w - seg.z >= m_min) {
                    int a = max(p - h, seg.x);
                    int b = min(p + h, seg.y);
                    if (cd.window_days > 0.0) {
                        // time window: only the samples within half its length
                        // of p count.  Times are non-decreasing, so they form a
                        // run that two scans in from the index window's ends find
                        // (invalid samples inside it are skipped by the ranks).
                        const double* tc = time + cd.off;
                        const double ti = tc[p];
                        const double half = 0.5 * cd.window_days;
                        while (a < p && !(__builtin_fabs(tc[a] - ti) <= half)) ++a;
                        while (b > p && !(__builtin_fabs(tc[b] - ti) <= half)) --b;
                    }
                    ca[r] = rank1(sm.vbits, sm.vpre, (uint32_t)(a - s0));
                    n[r] = rank1(sm.vbits, sm.vpre, (uint32_t)(b - s0 + 1)) - ca[r];  // >= 1: p is valid
                    live[r] = true;
                }
            }
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
            const uint32_t cb = ca[r] + n[r];
            const uint32_t rk = wavelet_kth(sm, levels, ca[r], cb, (n[r] - 1) >> 1);
            m[r] = key_value((uint32_t)(sm.sortbuf[rk] >> 32));
            if (scale == UMI_SCALE_MAD) {
                sc[r] = window_mad(sm, levels, ca[r], n[r], m[r]);
            } else {
                // the points strictly above m are the window's elements ranked
                // after the last tile element numerically equal to m (ties and
                // -0/+0 sit next to m in the sorted order)
                uint32_t rh = rk;
                while (rh + 1 < (uint32_t)nv &&
                       key_value((uint32_t)(sm.sortbuf[rh + 1] >> 32)) == m[r])
                    ++rh;
                nplus[r] = n[r] - wavelet_count_less(sm, levels, ca[r], cb, rh + 1);
            }
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
            if (nplus[r] > 0) sc[r] = kScaleConst * __builtin_sqrtf(ssq[r] / (float)nplus[r]);
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
            const float kk = kA / (c * sc[r]);
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

__global__ __launch_bounds__(kMainThreads, 8) void umi_main_kernel(
    const float* __restrict__ flux, const int32_t* __restrict__ segid,
    const int4* __restrict__ segtab, const BatchHeader* __restrict__ hdr,
    const CurveDesc* __restrict__ curves, const int2* __restrict__ tiles, int tile_first,
    int tile_count, uint32_t* __restrict__ counter, float* __restrict__ trend,
    float* __restrict__ median)
{
    __shared__ MainSmem sm;
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wave = tid >> 6;
    const int iters = hdr->iters;
    const int scale = hdr->scale;
    float* const detrended = hdr->detrended;
    const double* const time = hdr->time;
    // tile range [tile_first, tile_end): a count < 0 means "all tiles of the batch"
    const int tile_end = tile_count < 0 ? hdr->n_tiles : tile_first + tile_count;

    for (int round = 0;; ++round) {
        if (tid == 0)
            sm.tile = counter ? tile_first + (int)atomicAdd(counter, 1u)
                              : tile_first + (int)blockIdx.x + round * (int)gridDim.x;
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
        const int sg0 = sg[0];
        bool same = true;
        const int nwv = (N >> 6) + 1;
        for (int i0 = wave * 64; i0 < nwv * 64; i0 += kMainThreads) {
            const int i = i0 + lane;
            const int sgi = i < N ? sg[i] : sg0;
            const bool ok = (i < N) && (sgi >= 0);
            same = same && sgi == sg0;
            const uint64_t bal = __ballot(ok);
            if (lane == 0) sm.vbits[i0 >> 6] = bal;
        }
        const bool simple = __syncthreads_and(same) && sg0 >= 0 && cd.W <= kSmallW &&
                            scale != UMI_SCALE_MAD && cd.window_days == 0.0 && t0 >= h &&
                            t1 + h <= cd.len;
        word_prefix(sm.vbits, sm.vpre, nwv, reinterpret_cast<uint32_t*>(&sm.nvalid));
        __syncthreads();
        const int nv = sm.nvalid;
        int npad = 64;
        while (npad < nv) npad <<= 1;
        int levels = 6;
        while ((1 << levels) < npad) ++levels;

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
            if (i < N && sg[i] >= 0) {
                const float x = f[i];
                const uint32_t ci = rank1(sm.vbits, sm.vpre, (uint32_t)i);
                sm.xv[ci] = x;
                sm.sortbuf[ci] = ((uint64_t)order_key(x) << 32) | ci;
            }
        }
        for (int i = nv + tid; i < npad; i += kMainThreads) sm.sortbuf[i] = ~0ull;
        __syncthreads();

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

        // --- wavelet matrix over the sequence rank_of[compacted index] ---
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
        }  // not simple

        // --- the tile's windows: R consecutive positions per lane ---
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
            tile_windows<3>(sm, levels, nv, cd, h, s0, t0, t1, segid, segtab, alpha, c, iters, scale,
                            simple, pm, pn, time, trend, median, detrended);
        else if (R == 2)
            tile_windows<2>(sm, levels, nv, cd, h, s0, t0, t1, segid, segtab, alpha, c, iters, scale,
                            simple, pm, pn, time, trend, median, detrended);
        else
            tile_windows<1>(sm, levels, nv, cd, h, s0, t0, t1, segid, segtab, alpha, c, iters, scale,
                            simple, pm, pn, time, trend, median, detrended);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launch wrappers (the host library calls only these).

hipError_t launch_prepass(const float* flux, const double* time, const BatchHeader* hdr,
                          const CurveDesc* curves, int curve_first, int grid, int32_t* segid,
                          int4* segtab, int2* tiles, uint32_t* counter, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    // A launch over few curves walks each curve with a 1024-thread workgroup
    // (a quarter as many chunks in sequence); many curves fill the chip with
    // 256-thread workgroups, one per curve.
    if (grid <= kPrepWideCurves)
        hipLaunchKernelGGL(umi_prepass_kernel<kPrepWideThreads>, dim3(grid),
                           dim3(kPrepWideThreads), 0, stream, flux, time, hdr, curves,
                           curve_first, segid, segtab, tiles, counter);
    else
        hipLaunchKernelGGL(umi_prepass_kernel<kPrepThreads>, dim3(grid), dim3(kPrepThreads), 0,
                           stream, flux, time, hdr, curves, curve_first, segid, segtab, tiles,
                           counter);
    return hipGetLastError();
}

hipError_t launch_main(const float* flux, const int32_t* segid, const int4* segtab,
                       const BatchHeader* hdr, const CurveDesc* curves, const int2* tiles,
                       int tile_first, int tile_count, uint32_t* counter, int grid,
                       float* trend, float* median, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(umi_main_kernel, dim3(grid), dim3(kMainThreads), 0, stream, flux, segid,
                       segtab, hdr, curves, tiles, tile_first, tile_count, counter, trend,
                       median);
    return hipGetLastError();
}

}  // namespace umi
