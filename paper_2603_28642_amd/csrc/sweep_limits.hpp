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
constexpr int kSweepLevEnt = 4096;   // entries per level (products staged in LDS)
constexpr int kSweepBlob =
    163840 - 1024 - (2 * kSweepPos + kSweepExt + 2 * kSweepPos + kSweepLevEnt) * 8;  // 64512 bytes
constexpr int kSweepHdr = 12;        // int32 header words of a batch blob

}  // namespace rsilu
