// pk_matmul_batched_noalloc: the one-shot grouped product without any
// allocation, for callers that cannot allocate device memory.
//
// The descriptors and the tile -> product map of the launch (what a grouped
// plan keeps in memory it allocates) go to `scratch`, a file-scope device
// array of kScratchBytes that every GPU running the library holds until the
// process ends, through a host staging copy of the same size in static
// storage.  Host code never passes the array's name to a kernel or a copy:
// its device address is looked up once per device (noalloc_setup, from
// pk_case_table_build, or from the entry point's first call on the device)
// with that device current, and kept per device.  Calls are serialised by a
// process-wide lock and each returns after its work on the stream is done, so
// one call's layout is never overwritten by the next; work of other processes
// on the same GPU uses those processes' own copies of the array.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "grouped.hpp"
#include "pk_internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

alignas(256) unsigned char g_stage[kScratchBytes];  // host copy of a call's layout
std::mutex g_mu;                                     // one call at a time
void *g_scratch[kMaxDevices] = {};                   // device address of `scratch`, per device

// With g_mu held: the device address of `scratch` on `device`, looked up
// with the device current.
int setup_locked(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return pk::fail(PK_ERR_INVALID_ARG, "device index out of range");
    if (!g_scratch[device]) {
        int cur = -1;
        hipError_t err = hipGetDevice(&cur);
        if (err == hipSuccess && cur != device) err = hipSetDevice(device);
        void *ptr = nullptr;
        if (err == hipSuccess) err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err == hipSuccess && !ptr) err = hipErrorInvalidSymbol;
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        if (err != hipSuccess)
            return pk::fail(PK_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(err));
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return PK_OK;
}

}  // namespace

namespace pk {

int noalloc_setup(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    void *ptr = nullptr;
    return setup_locked(device, &ptr);
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace pk

extern "C" int pk_matmul_batched_noalloc(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M,
                                         const int64_t *N, const int64_t *K, const void *const *A,
                                         const int64_t *lda, const void *const *B, const int64_t *ldb,
                                         void *const *C, const int64_t *ldc, const pk_params *per_group_or_null,
                                         void *hip_stream) {
    using namespace pk;
    if (!tbl || G < 0 || (G > 0 && (!M || !N || !K || !A || !lda || !B || !ldb || !C || !ldc)))
        return fail(PK_ERR_INVALID_ARG, "null argument or negative group count");
    if (dtype != PK_F32 && dtype != PK_BF16) return fail(PK_ERR_UNSUPPORTED_DTYPE, "grouped products: f32 or bf16");
    if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "grouped products need a table bound to a device");
    try {
        std::lock_guard<std::mutex> lock(g_mu);
        void *dev = nullptr;
        int rc = setup_locked(tbl->device, &dev);
        if (rc != PK_OK) return rc;
        GroupedOperands o;
        o.G = G;
        o.M = M, o.N = N, o.K = K, o.A = A, o.lda = lda, o.B = B, o.ldb = ldb, o.C = C, o.ldc = ldc;
        GroupedLayout lay;
        rc = grouped_layout(tbl, (int)dtype, o, per_group_or_null, &lay);
        if (rc != PK_OK) return rc;
        const size_t bytes = lay.bytes();
        if (bytes > kScratchBytes)
            return fail(PK_ERR_INVALID_ARG, "grouped layout of " + std::to_string(bytes) +
                                                " bytes exceeds the allocation-free workspace of " +
                                                std::to_string(kScratchBytes) + " bytes");
        if (lay.launches.empty()) return PK_OK;
        hipStream_t s = (hipStream_t)hip_stream;
        const size_t dbytes = lay.descs.size() * sizeof(pkk::GroupDesc);
        std::memcpy(g_stage, lay.descs.data(), dbytes);
        std::memcpy(g_stage + dbytes, lay.tmap.data(), lay.tmap.size() * sizeof(int32_t));
        hipError_t err = hipSetDevice(tbl->device);
        if (err == hipSuccess) err = hipMemcpyAsync(dev, g_stage, bytes, hipMemcpyHostToDevice, s);
        if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("layout copy: ") + hipGetErrorString(err));
        rc = grouped_launch(lay, dev, 0, s);
        // the staging copy and the array are reused by the next call
        err = hipStreamSynchronize(s);
        if (rc != PK_OK) return rc;
        if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(err));
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}
