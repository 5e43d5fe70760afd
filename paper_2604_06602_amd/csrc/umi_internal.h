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
constexpr int kSmallW = 31;                  // full windows this small take register networks
// Paths of the estimate kernel a batch needs (bits of a kernel instance).
constexpr int kFeatSmall = 1;                // small-window networks (W <= kSmallW)
constexpr int kFeatSplit = 2;                // split tiles (tile <= kSplitMaxTile)
constexpr int kFeatExtra = 4;                // MAD ablation, time windows
constexpr int kFeatAll = kFeatSmall | kFeatSplit | kFeatExtra;

// Lanes that share one window for a tile of `tile` output positions: 1 above
// kSplitMaxTile (each lane takes up to three windows), else the largest of 2,
// 4, 8 with tile * G <= kMainThreads.
__host__ __device__ constexpr int split_lanes(int tile)
{
    return tile > kSplitMaxTile ? 1 : (tile > kMainThreads / 4 ? 2 : (tile > kMainThreads / 8 ? 4 : 8));
}
constexpr int kPrepThreads = 256;            // threads per pre-pass workgroup
constexpr int kPrepItems = 8;                // samples per thread per chunk (chunked pre-pass)
constexpr int kPrepChunk = kPrepThreads * kPrepItems;  // samples per pre-pass chunk
constexpr int kPrepWalkItems = 4;            // samples per thread per step (curve walker)
constexpr int kPrepGroupsPerCU = 8;          // chunked pre-pass workgroups per CU
constexpr int kPrepSmallChunks = 256;        // plan steps of at most this many chunks take
                                             // a chunked pre-pass of this many workgroups
constexpr int kPrepWalkMinCurves = 128;      // batches of this many curves or more take the
                                             // one-workgroup-per-curve walker
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
    int32_t n_chunks;   // pre-pass chunks over all curves
    int32_t reserved;
    float* detrended;   // flux / trend output (curve offsets as for trend), or null
    const double* time; // the batch's times (read by the time-window scans), or null
};
static_assert(sizeof(BatchHeader) == 40, "BatchHeader layout");

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
    int32_t chunk_base; // index of this curve's first pre-pass chunk
    int32_t reserved;
};
static_assert(sizeof(CurveDesc) == 48, "CurveDesc layout");

// Segmentation summary of a run of consecutive samples of one curve, or the
// state after a curve's first samples (a prefix), as the pre-pass scan
// carries it from chunk to chunk.
struct SegState {
    int32_t cnt;        // valid samples
    int32_t fv;         // first valid sample (curve-local), -1 if none
    int32_t lv;         // last valid sample, -1 if none
    int32_t ls;         // latest segment start, -1 if none; in a run that is
                        // not a prefix only starts after fv count (fv's own
                        // status depends on what precedes the run)
    int32_t lsb;        // valid samples of the run (or prefix) before ls
    int32_t reserved;
    double ft;          // time of fv
    double lt;          // time of lv
};
static_assert(sizeof(SegState) == 40, "SegState layout");

// One pre-pass chunk's published scan state: its own summary (`agg`), then
// the state after the curve's samples up to its end (`inc`).  Each holds the
// nine 32-bit words of a SegState (cnt, fv, lv, ls, lsb, then the low and
// high halves of ft and lt), each stored in the low half of a 64-bit word
// whose high half is the launch's stamp: a reader takes a state once all nine
// words carry its launch's stamp, so no word needs ordering against another.
constexpr int kSegWords = 9;
struct ChunkRec {
    uint64_t agg[kSegWords];
    uint64_t inc[kSegWords];
};
static_assert(sizeof(ChunkRec) == 144, "ChunkRec layout");

// Device counters of a workspace (zeroed when it is allocated).
struct Counters {
    uint32_t queue;     // estimate-kernel tile queue (cleared by the pre-pass)
    uint32_t tickets;   // pre-pass chunk tickets (reset by its last workgroup)
    uint32_t done;      // pre-pass workgroups finished (reset likewise)
    uint32_t trash;     // takes the walker pre-pass's stores that have no sample
    uint64_t epoch;     // pre-pass launches completed; stamps use epoch + 1
    uint64_t reserved2;
};
static_assert(sizeof(Counters) == 32, "Counters layout");

// A list of copies for the copy kernel, passed by value as kernel arguments
// (so nothing on either side needs to outlive the launch): copy i moves
// bytes[i] bytes from src[i] to dst[i] and is cut into pieces of kCopyPieceBytes
// bytes, piece p of the launch belonging to the copy i with
// first[i] <= p < first[i + 1].
constexpr int kCopyMax = 64;
constexpr int kCopyPieceBytes = 32768;
struct CopyBatch {
    int32_t n;                   // copies
    int32_t reserved;
    int32_t first[kCopyMax + 1]; // first piece of each copy; first[n] = pieces
    const uint8_t* src[kCopyMax];
    uint8_t* dst[kCopyMax];
    int64_t bytes[kCopyMax];
};
static_assert(sizeof(CopyBatch) <= 2048, "CopyBatch fits the kernel arguments");

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
