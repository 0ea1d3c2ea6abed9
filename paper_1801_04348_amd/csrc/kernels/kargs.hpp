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
    int32_t vec;  // MFMA programs: rows aligned for 16-byte loads (else element loads)
};

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
    int32_t pad;
};

// Arguments of a grouped kernel: descriptors and the tile -> product map.
struct GroupArgs {
    const GroupDesc *descs;
    const int32_t *tile_group;
    int64_t total_tiles;
    int32_t accumulate;
    int32_t pad;
};

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
};

}  // namespace pkk
