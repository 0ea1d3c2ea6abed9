// Layout of a grouped launch: shared by the plans (grouped.cpp) and the
// allocation-free one-shot entry point (noalloc.hip).
#pragma once

#include <vector>

#include "pk_internal.hpp"

namespace pk {

// The caller's arrays of one grouped call (host arrays of length G).
struct GroupedOperands {
    int32_t G = 0;
    const int64_t *M = nullptr, *N = nullptr, *K = nullptr;
    const void *const *A = nullptr;
    const int64_t *lda = nullptr;
    const void *const *B = nullptr;
    const int64_t *ldb = nullptr;
    void *const *C = nullptr;
    const int64_t *ldc = nullptr;
};

// One persistent launch of a layout: its kernel, its range of descriptors and
// tiles, its grid, and the first tile (relative to first_tile) of each XCD's
// range.
struct GroupedLaunch {
    const KernelEntry *entry = nullptr;
    int64_t first_desc = 0, ndesc = 0;
    int64_t first_tile = 0, total_tiles = 0;
    int64_t grid = 0;
    int64_t bins[pkk::kXcds + 1] = {};
};

// Everything a grouped launch reads, built on the host.
struct GroupedLayout {
    std::vector<GroupedLaunch> launches;
    std::vector<pkk::GroupDesc> descs;
    std::vector<int32_t> tmap;       // per tile of every launch: its descriptor, relative to the launch's first
    std::vector<pk_params> chosen;   // per product, in the caller's order
    // bytes of the descriptors followed by the tile map, as uploaded
    size_t bytes() const { return descs.size() * sizeof(pkk::GroupDesc) + tmap.size() * sizeof(int32_t); }
};

// Checks the operands and builds the layout for `policy` (PK_POLICY_CASE, or
// the given per-product parameters when per_group is non-null).  EXHAUSTIVE
// plans are built in grouped.cpp from the layouts of their candidates.
int grouped_layout(const pk_table *tbl, int dtype, const GroupedOperands &ops, const pk_params *per_group,
                   GroupedLayout *out);

// Queues the layout's launches; `dev` holds its bytes() (descriptors, then
// the tile map) on the device.
int grouped_launch(const GroupedLayout &lay, const void *dev, int accumulate, hipStream_t stream);

}  // namespace pk
