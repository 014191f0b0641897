// Limits of one batch of the single-workgroup triangular sweep; the LDS of
// one gfx950 workgroup (160 KiB) holds the batch blob, the results of the
// current and previous batch, the gathered older inputs, the batch's
// right-hand side and fused addend, and one level's products.
#pragma once

namespace rsilu {

constexpr int kSweepThreads = 1024;  // one workgroup
constexpr int kSweepRows = 1024;     // rows per level (one per thread)
constexpr int kSweepPos = 1536;      // rows per batch
constexpr int kSweepExt = 2048;      // distinct older inputs per batch
constexpr int kSweepLevEnt = 1024;   // chunks per level (one per thread; sums staged in LDS)
constexpr int kSweepChunk = 4;       // entries per chunk (a row is cut into chunks)
constexpr int kSweepLevels = 63;     // levels per batch (offsets held in one wavefront's lanes)
constexpr int kSweepZeroSlot = 2 * kSweepPos + kSweepExt;  // LDS slot that always holds 0.0
// The blob gets the rest of the LDS, at most 5 16-byte vectors per thread.
constexpr int kSweepBlobRoom = 163840 - 1024 - (2 * kSweepPos + kSweepExt + 8 + 2 * kSweepPos + kSweepLevEnt) * 8;
constexpr int kSweepBlob = kSweepBlobRoom < 5 * 16 * kSweepThreads ? (kSweepBlobRoom & ~15) : 5 * 16 * kSweepThreads;
constexpr int kSweepHdr = 12;        // int32 header words of a batch blob
// Level schemes of the single-workgroup sweep (one kernel instantiation each).
constexpr int kSchemeTwoPhase = 0;   // one chunk and one row per thread; chunk sums through LDS, two barriers
constexpr int kSchemeSegmented = 1;  // one chunk per thread, a row on one 16-lane group, segmented scan
constexpr int kSchemeRows = 2;       // one row per thread, its chunks loaded kRowsRound at a time
constexpr int kSchemeSegmentedWide = 3;  // segmented, rows of up to 64 chunks (one wavefront)
constexpr int kRowsRound = 2;

// Blocks of the inner products of the CG steps on S~ (and so their per-block partials):
// at most kCgParts; the setup reserves three such partial arrays.
constexpr int kCgParts = 2048;

}  // namespace rsilu
