// Clearing of an output matrix before a product split along K adds its
// shares' sums into it: a kernel rather than hipMemsetAsync, so that a HIP
// graph capturing the product holds no memset node; 16-byte stores where the
// rows allow them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "pk_internal.hpp"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// C[i][j] = 0 for i < M, j < N; rows of ldc floats.  vec: C and ldc keep
// rows 16-byte aligned, so whole chunks of 4 columns are stored at once.
__global__ void __launch_bounds__(256) pk_fill_zero_f32(float *C, int64_t ldc, int32_t M, int32_t N, int32_t vec) {
    const int64_t cols = vec ? (N + 3) / 4 : N;  // chunks (or elements) per row
    const int64_t total = (int64_t)M * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols, c = i % cols;
        if (vec) {
            float *p = C + r * ldc + 4 * c;
            if (4 * c + 4 <= N) {
                *reinterpret_cast<f32x4 *>(p) = f32x4{0.f, 0.f, 0.f, 0.f};
            } else {
                for (int64_t e = 4 * c; e < N; ++e) C[r * ldc + e] = 0.f;
            }
        } else {
            C[r * ldc + c] = 0.f;
        }
    }
}

}  // namespace

namespace pk {

int zero_matrix(const pk_machine &m, void *C, int64_t ldc, int64_t M, int64_t N, hipStream_t stream) {
    if (M <= 0 || N <= 0) return PK_OK;
    const int vec = ((uintptr_t)C % 16 == 0 && ldc % 4 == 0) ? 1 : 0;
    const int64_t items = M * (vec ? (N + 3) / 4 : N);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, (int64_t)std::max(m.cu_count, 1) * 8));
    hipLaunchKernelGGL(pk_fill_zero_f32, dim3((unsigned)grid), dim3(256), 0, stream, (float *)C, ldc, (int32_t)M,
                       (int32_t)N, vec);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("clearing C: ") + hipGetErrorString(err));
    return PK_OK;
}

}  // namespace pk
