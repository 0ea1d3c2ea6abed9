// Argument block and registry record shared by the kernels and the host
// library.  Plain data only.
#pragma once

#include <stdint.h>

namespace pkk {

// Arguments of every matmul kernel: C (MxN) = [C +] A (MxK) * B (KxN),
// row-major with leading dimensions.  Pointers are device addresses.
struct MmArgs {
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t accumulate;
    int32_t vec;     // MFMA programs: rows aligned for 16-byte loads (else element loads)
    int32_t splits;  // MFMA programs: shares of K (> 1: each adds its sum to C atomically), else 0
    int32_t pad;
};

// Largest workgroup of an MFMA program that runs a product split along K.
constexpr int kSplittableThreads = 512;

// One product of a grouped launch.
struct GroupDesc {
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t vec;         // rows aligned for the wide loads
    int64_t tile_start;  // first global tile index of this product
    int32_t tiles_n;     // tiles along N
    int32_t prog;        // mixed grouped kernels: index into kMixedTile (else 0)
};

// Workgroups are dispatched round-robin over this many XCDs, each with its
// own L2; a grouped launch gives each XCD a range of tiles of its own.
constexpr int kXcds = 8;

// Arguments of a grouped kernel: descriptors, the tile -> product map, and
// the first tile of each XCD's range (bin_first[kXcds] = total_tiles).
struct GroupArgs {
    const GroupDesc *descs;
    const int32_t *tile_group;
    int64_t total_tiles;
    int32_t accumulate;
    int32_t pad;
    int64_t bin_first[kXcds + 1];
};

// Tile programs of the mixed grouped kernels, which run a different output
// tile per product in one launch (GroupDesc::prog indexes this list): BM x BN
// tiles of 2 x 2 wavefronts; K tile 32 (float32) or 64 (bfloat16).
constexpr int kMixedPrograms = 4;
constexpr int kMixedTile[kMixedPrograms][2] = {{64, 64}, {128, 64}, {64, 128}, {128, 128}};
constexpr int kMixedBk[3] = {32, 0, 64};  // by pk_dtype: float32, (int32: none), bfloat16

// One compiled kernel instance, as listed by the generated registry.
struct KernelEntry {
    const char *name;
    const void *fn;     // host stub of the __global__ function
    int family;
    int variant;        // strategy bits applied to the family's fragment
    int dtype;          // pk_dtype
    int bx, by, s, bk;  // VALU parameters (0 when unused)
    int bm, bn, wm, wn; // MFMA parameters (0 when unused)
    int threads;        // workgroup size
    int lds_bytes;      // LDS the kernel allocates
    int tile_m, tile_n; // output tile of one workgroup
    int sy;             // 2-D VALU programs: outputs per work-item along M (0 otherwise)
};

}  // namespace pkk
