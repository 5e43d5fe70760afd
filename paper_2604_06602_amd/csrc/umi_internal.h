// Internal layout shared by the host launcher and the HIP kernels of the UMI
// library.  Nothing here is part of the public C ABI (include/umi.h).
#pragma once

#include <stdint.h>

namespace umi {

// Largest staged tile: output positions plus the W-1 halo.  The tile sort and
// the wavelet matrix work on power-of-two padded sizes up to this.
constexpr int kStageMax = 2048;
constexpr int kStageLog2 = 11;
constexpr int kWords = kStageMax / 64 + 1;  // bit-vector words incl. sentinel
constexpr int kMainThreads = 512;            // threads per main-kernel workgroup
constexpr int kMaxTile = 3 * kMainThreads;   // output positions per tile: <= 3 per lane
constexpr int kSplitMaxTile = kMainThreads / 2;  // tiles this small split windows

// Lanes that share one window for a tile of `tile` output positions: 1 above
// kSplitMaxTile (each lane takes up to three windows), else the largest of 2,
// 4, 8 with tile * G <= kMainThreads.
__host__ __device__ constexpr int split_lanes(int tile)
{
    return tile > kSplitMaxTile ? 1 : (tile > kMainThreads / 4 ? 2 : (tile > kMainThreads / 8 ? 4 : 8));
}
constexpr int kPrepThreads = 256;            // threads per pre-pass workgroup
constexpr int kPrepWideThreads = 1024;       // ... when a launch covers few curves
constexpr int kPrepWideCurves = 64;          // "few": at most this many
constexpr int kPrepItems = 4;                // samples per pre-pass thread per chunk
constexpr int kPrepWideItems = 8;            // ... in the 1024-thread workgroups
constexpr float kScaleConst = 0.6745f;       // Section 2.2, after Eq. 1
constexpr double kGapDays = 0.5;             // segment break threshold (days)

// Per-batch parameters, read by the kernels from device memory so that a
// captured launch sequence can be replayed for any batch (only the staged
// bytes change between replays).
struct BatchHeader {
    int32_t n_curves;   // entries in the curve table
    int32_t n_tiles;    // tiles over all curves
    int32_t iters;      // Phase 3 iterations
    int32_t scale;      // umi_scale: Phase 2 estimator
    float* detrended;   // flux / trend output (curve offsets as for trend), or null
    const double* time; // the batch's times (read by the time-window scans), or null
};
static_assert(sizeof(BatchHeader) == 32, "BatchHeader layout");

// One curve of a packed batch, in the (cost-sorted) order tiles are issued.
struct CurveDesc {
    int64_t off;        // first sample in the packed arrays
    int32_t len;        // samples
    int32_t W;          // window (odd)
    int32_t tile;       // output positions per tile
    int32_t tile_base;  // index of this curve's first tile in the tile list
    float alpha;        // asymmetry factor (Eq. 2) of this curve
    float c;            // bisquare tuning constant of this curve
    double window_days; // > 0: time window of this length (W still bounds it)
};
static_assert(sizeof(CurveDesc) == 40, "CurveDesc layout");

// Per-sample segment word written by the pre-pass at segid[curve.off + i]:
//   -1       sample i is invalid;
//   x >= 0   sample i is valid and its segment starts at the valid sample x
//            (curve-local index, x < i);
//   -2 - n   sample i is valid and starts a segment of n valid samples.
// A segment is live when n >= max(1, W / 3).  Curves hold fewer than
// 2^31 - 1 samples, so -2 - n never overflows.

// Tile record written by the pre-pass: x = index into the curve table,
// y = first output position (curve-local).

}  // namespace umi
