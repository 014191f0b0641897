// Per-position record of a level-ordered triangular factor, as the batched
// solves read it (built by the host setup, read by the batched kernel).
#pragma once

#include <cstdint>

namespace rsilu {

constexpr int kRecEntries = 4;

// Position p of the level order: the row it solves, its entry range in the
// level-ordered CSR, its first kRecEntries entries (column -1 past the end of
// the row) and the reciprocal of its diagonal (1 for a unit diagonal). One record is read with
// independent loads, so the data of a level's rows arrives in one round trip.
template <class V>
struct alignas(16) LevelRec {
    int32_t row, k0, k1, pad;
    int32_t col[kRecEntries];
    V val[kRecEntries];
    V rdiag;
};

}  // namespace rsilu
