// Measured arithmetic ceilings of the vector ALUs, the roofline of the VALU
// matmul programs: a kernel of independent multiply-add chains (no memory
// traffic inside the timed loop), timed with HIP events.  float32 uses
// v_fma_f32-class instructions, int32 v_mul_lo_u32 + v_add_u32 (wrapping).
#include <hip/hip_runtime.h>

#include <string>

#include "pk_internal.hpp"

namespace pk {

namespace {

constexpr int kChains = 16;   // independent accumulators per work-item
constexpr int kIters = 4096;  // multiply-adds per chain

template <typename T>
__global__ __launch_bounds__(256) void valu_rate(T *__restrict__ out, T a, T b) {
    T acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = (T)(threadIdx.x + c);
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = acc[c] * a + b;
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <>
__global__ __launch_bounds__(256) void valu_rate<int32_t>(int32_t *__restrict__ out, int32_t a, int32_t b) {
    uint32_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = threadIdx.x + c;
    const uint32_t ua = (uint32_t)a, ub = (uint32_t)b;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = acc[c] * ua + ub;
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (int32_t)s;
}

template <typename T>
int measure(int device, const pk_machine &m, double *ops) {
    const int blocks = std::max(1, m.cu_count) * 8;
    T *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return fail(PK_ERR_HIP, "hipSetDevice");
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(T)) != hipSuccess) return fail(PK_ERR_HIP, "allocation failed");
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL(valu_rate<T>, dim3(blocks), dim3(256), 0, 0, out, (T)3, (T)1);
    (void)hipEventRecord(e0, 0);
    const int reps = 5;
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(valu_rate<T>, dim3(blocks), dim3(256), 0, 0, out, (T)3, (T)1);
    (void)hipEventRecord(e1, 0);
    hipError_t err = hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("probe: ") + hipGetErrorString(err));
    // two operations (a multiply and an add) per multiply-add
    *ops = 2.0 * (double)blocks * 256 * kChains * kIters * reps / (ms * 1e-3);
    return PK_OK;
}

}  // namespace

}  // namespace pk

using namespace pk;

extern "C" int pk_probe_valu_rate(const pk_table *tbl, pk_dtype dtype, double *ops_per_second) {
    if (!tbl || !ops_per_second) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "the probe needs a table bound to a device");
    if (dtype == PK_F32) return measure<float>(tbl->device, tbl->machine, ops_per_second);
    if (dtype == PK_I32) return measure<int32_t>(tbl->device, tbl->machine, ops_per_second);
    return fail(PK_ERR_UNSUPPORTED_DTYPE, "probe: f32 or i32");
}
