// Learned cost model: a 13-64-64-1 ReLU network that predicts the logarithm
// of a candidate's launch time from features of (candidate, M, N, K), trained
// on the device by the kernels below on timings the exhaustive tuner records.
// It replaces the analytic score when selecting among the case table's
// feasible (leaf, E) pairs, with measurement as its fallback.
//
// Network (parameters flat, in this order): W1 (64 x 13, row-major), b1 (64),
// W2 (64 x 64), b2 (64), W3 (1 x 64), b3 (1):
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3.
// Loss: mean squared error over the n rows.  Optimiser: Adam.
//
// Kernels (float32):
//   mlp_rows   one workgroup per 64 rows: forward pass with the activations in
//              LDS, then (training) the backward pass and the workgroup's
//              partial gradient sums, written to its own slot
//   mlp_reduce per parameter, the sum of the slots in slot order (so the
//              gradient does not depend on scheduling)
//   mlp_adam   one Adam step per parameter
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <random>
#include <sstream>
#include <stdexcept>
#include <tuple>

#include "pk_internal.hpp"
#include "select.hpp"

namespace pkcm {

constexpr int IN = PK_NFEATURES;
constexpr int H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H, NP = OFF_B3 + 1;
constexpr int ROWS = 64;
constexpr int NT = 256;
constexpr int HP = H + 1;  // padded row stride in LDS

__global__ __launch_bounds__(NT) void mlp_rows(const float *__restrict__ X, const float *__restrict__ T, int n,
                                               const float *__restrict__ P, float *__restrict__ Y,
                                               float *__restrict__ part_grad, float *__restrict__ part_loss,
                                               int train, float inv_n) {
    __shared__ float sW1[H * IN], sB1[H], sW2[H * HP], sB2[H], sW3[H];
    __shared__ float sX[ROWS * IN];
    __shared__ float sZ1[ROWS * HP], sH1[ROWS * HP], sZ2[ROWS * HP], sH2[ROWS * HP];
    __shared__ float sD[ROWS];
    __shared__ float sRed[NT / 64];
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * ROWS;
    const int nr = min(ROWS, n - row0);

    for (int i = tid; i < H * IN; i += NT) sW1[i] = P[OFF_W1 + i];
    for (int i = tid; i < H * H; i += NT) sW2[(i / H) * HP + i % H] = P[OFF_W2 + i];
    if (tid < H) {
        sB1[tid] = P[OFF_B1 + tid];
        sB2[tid] = P[OFF_B2 + tid];
        sW3[tid] = P[OFF_W3 + tid];
    }
    for (int i = tid; i < ROWS * IN; i += NT) {
        const int r = i / IN;
        sX[i] = r < nr ? X[(int64_t)(row0 + r) * IN + i % IN] : 0.0f;
    }
    __syncthreads();

    const int j = tid & 63, rq = tid >> 6;  // unit j, rows rq + 4 i
    // layer 1
    for (int i = 0; i < ROWS / 4; ++i) {
        const int r = rq + 4 * i;
        float z = sB1[j];
#pragma unroll
        for (int k = 0; k < IN; ++k) z = __builtin_fmaf(sW1[j * IN + k], sX[r * IN + k], z);
        sZ1[r * HP + j] = z;
        sH1[r * HP + j] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    // layer 2
    for (int i = 0; i < ROWS / 4; ++i) {
        const int r = rq + 4 * i;
        float z = sB2[j];
#pragma unroll 8
        for (int k = 0; k < H; ++k) z = __builtin_fmaf(sW2[j * HP + k], sH1[r * HP + k], z);
        sZ2[r * HP + j] = z;
        sH2[r * HP + j] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    // output layer and loss
    float sq = 0.0f;
    if (tid < ROWS) {
        const int r = tid;
        float y = P[OFF_B3];
#pragma unroll 8
        for (int k = 0; k < H; ++k) y = __builtin_fmaf(sW3[k], sH2[r * HP + k], y);
        if (!train) {
            if (r < nr) Y[row0 + r] = y;
        } else {
            const float d = r < nr ? y - T[row0 + r] : 0.0f;
            sq = d * d;
            sD[r] = 2.0f * inv_n * d;  // dL/dy
        }
    }
    if (!train) return;
    // workgroup sum of squared errors (wavefront 0 holds all rows)
    if (tid < 64) {
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
        if (tid == 0) part_loss[blockIdx.x] = sq;
    }
    __syncthreads();
    float *g = part_grad + (int64_t)blockIdx.x * NP;
    // dz2 = dy * W3 * [z2 > 0], kept in sZ2
    for (int i = 0; i < ROWS / 4; ++i) {
        const int r = rq + 4 * i;
        sZ2[r * HP + j] = sZ2[r * HP + j] > 0.0f ? sD[r] * sW3[j] : 0.0f;
    }
    // W3, b3
    if (tid < H) {
        float acc = 0.0f;
        for (int r = 0; r < ROWS; ++r) acc = __builtin_fmaf(sD[r], sH2[r * HP + tid], acc);
        g[OFF_W3 + tid] = acc;
    } else if (tid == H) {
        float acc = 0.0f;
        for (int r = 0; r < ROWS; ++r) acc += sD[r];
        g[OFF_B3] = acc;
    }
    __syncthreads();
    // W2 (j, k) = sum_r dz2[r][j] h1[r][k]; thread handles j and k = rq + 4 i
    for (int i = 0; i < H / 4; ++i) {
        const int k = rq + 4 * i;
        float acc = 0.0f;
        for (int r = 0; r < ROWS; ++r) acc = __builtin_fmaf(sZ2[r * HP + j], sH1[r * HP + k], acc);
        g[OFF_W2 + j * H + k] = acc;
    }
    if (tid < H) {
        float acc = 0.0f;
        for (int r = 0; r < ROWS; ++r) acc += sZ2[r * HP + tid];
        g[OFF_B2 + tid] = acc;
    }
    // dz1[r][k] = (sum_j dz2[r][j] W2[j][k]) [z1 > 0], kept in sZ1 (unit k = j here)
    for (int i = 0; i < ROWS / 4; ++i) {
        const int r = rq + 4 * i;
        float acc = 0.0f;
#pragma unroll 8
        for (int jj = 0; jj < H; ++jj) acc = __builtin_fmaf(sZ2[r * HP + jj], sW2[jj * HP + j], acc);
        sZ1[r * HP + j] = sZ1[r * HP + j] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // W1 (j, k) = sum_r dz1[r][j] x[r][k], b1
    for (int idx = tid; idx < H * IN; idx += NT) {
        const int jj = idx / IN, k = idx % IN;
        float acc = 0.0f;
        for (int r = 0; r < ROWS; ++r) acc = __builtin_fmaf(sZ1[r * HP + jj], sX[r * IN + k], acc);
        g[OFF_W1 + idx] = acc;
    }
    if (tid < H) {
        float acc = 0.0f;
        for (int r = 0; r < ROWS; ++r) acc += sZ1[r * HP + tid];
        g[OFF_B1 + tid] = acc;
    }
}

__global__ void mlp_reduce(const float *__restrict__ part_grad, const float *__restrict__ part_loss, int nblocks,
                           float *__restrict__ grad, float *__restrict__ loss, float inv_n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NP) {
        float s = 0.0f;
        for (int b = 0; b < nblocks; ++b) s += part_grad[(int64_t)b * NP + p];
        grad[p] = s;
    }
    if (p == 0) {
        float s = 0.0f;
        for (int b = 0; b < nblocks; ++b) s += part_loss[b];
        *loss = s * inv_n;
    }
}

// omb1, omb2: 1 - b1 and 1 - b2, rounded once from double on the host
__global__ void mlp_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m,
                         float *__restrict__ v, float lr, float b1, float b2, float omb1, float omb2, float eps,
                         float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + omb1 * g;
    const float vv = b2 * v[p] + omb2 * g * g;
    m[p] = mm;
    v[p] = vv;
    P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ------------------------------------------------------------------ host side
struct DeviceBuffers {
    float *P = nullptr, *X = nullptr, *T = nullptr, *Y = nullptr, *part = nullptr, *ploss = nullptr, *grad = nullptr,
          *loss = nullptr, *m = nullptr, *v = nullptr;
    ~DeviceBuffers() {
        for (float *p : {P, X, T, Y, part, ploss, grad, loss, m, v}) hipFree(p);
    }
};

#define CM_CHECK(x)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) throw std::runtime_error(std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

void forward_backward(hipStream_t s, DeviceBuffers &d, int64_t n, bool train) {
    const int nb = (int)((n + ROWS - 1) / ROWS);
    const float inv_n = 1.0f / (float)n;
    mlp_rows<<<nb, NT, 0, s>>>(d.X, d.T, (int)n, d.P, d.Y, d.part, d.ploss, train ? 1 : 0, inv_n);
    if (train) mlp_reduce<<<(NP + 255) / 256, 256, 0, s>>>(d.part, d.ploss, nb, d.grad, d.loss, inv_n);
    CM_CHECK(hipGetLastError());
}

void alloc(DeviceBuffers &d, int64_t n, bool train) {
    const int nb = (int)((n + ROWS - 1) / ROWS);
    CM_CHECK(hipMalloc(&d.P, NP * sizeof(float)));
    CM_CHECK(hipMalloc(&d.X, std::max<int64_t>(n, 1) * IN * sizeof(float)));
    CM_CHECK(hipMalloc(&d.Y, std::max<int64_t>(n, 1) * sizeof(float)));
    if (train) {
        CM_CHECK(hipMalloc(&d.T, std::max<int64_t>(n, 1) * sizeof(float)));
        CM_CHECK(hipMalloc(&d.part, (size_t)nb * NP * sizeof(float)));
        CM_CHECK(hipMalloc(&d.ploss, nb * sizeof(float)));
        CM_CHECK(hipMalloc(&d.grad, NP * sizeof(float)));
        CM_CHECK(hipMalloc(&d.loss, sizeof(float)));
        CM_CHECK(hipMalloc(&d.m, NP * sizeof(float)));
        CM_CHECK(hipMalloc(&d.v, NP * sizeof(float)));
    }
}

}  // namespace pkcm

struct pk_costmodel {
    std::vector<float> params;            // network parameters (standardized units)
    float xmean[PK_NFEATURES], xstd[PK_NFEATURES];
    float ymean = 0.f, ystd = 1.f;        // of ln(seconds)
    std::string fingerprint;              // machine the timings came from
    int dtype = PK_F32;                   // element type the timings came from
    int epochs = 0;
    float loss = 0.f;
};

namespace pk {

std::string machine_fingerprint(const pk_machine &m) {
    std::ostringstream o;
    o << m.arch << "/cu" << m.cu_count << "/lds" << m.lds_block << "/regs" << m.regs_block << "/thr"
      << m.max_threads_block << "/clk" << m.clock_khz;
    return o.str();
}

// Features of a candidate for C(MxN) = A(MxK) B(KxN):
//   0-2  ln M, ln N, ln K
//   3-4  ln tile_m, ln tile_n         (output tile of a workgroup)
//   5    ln(outputs per work-item)    (coarsening)
//   6    LDS bytes / 65536
//   7    estimated occupancy: resident wavefronts per CU / maximum
//   8    tile padding efficiency: M N / (padded M) (padded N)
//   9    wave quantisation efficiency: workgroups / (rounds * resident slots)
//   10   1 where the operands' rows allow the MFMA programs' 16-byte loads
//        (else the element-load twin runs), 0 otherwise
//   11   ln(shares of K): 0 for a product not split along K
//   12   ln of the analytic estimate of the launch's seconds (estimate_seconds,
//        the CASE policy's ranking)
void features(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K, bool wide,
              int ks, float *f) {
    const int wave = m.wave > 0 ? m.wave : 64;
    const int64_t tm = (M + e.tile_m - 1) / e.tile_m, tn = (N + e.tile_n - 1) / e.tile_n;
    ks = ks > 1 ? ks : 1;
    const int64_t tiles = tm * tn * ks;  // workgroups: a product split along K runs ks per tile
    const int64_t occ = blocks_per_cu(m, e);
    const int64_t slots = (int64_t)m.cu_count * occ;
    const int64_t rounds = std::max<int64_t>(1, (tiles + slots - 1) / slots);
    const double waves_max = std::max(1.0, (double)(m.max_threads_cu > 0 ? m.max_threads_cu : 2048) / wave);
    const double waves = (double)occ * ((e.threads + wave - 1) / wave);
    f[0] = (float)std::log((double)std::max<int64_t>(M, 1));
    f[1] = (float)std::log((double)std::max<int64_t>(N, 1));
    f[2] = (float)std::log((double)std::max<int64_t>(K, 1));
    f[3] = (float)std::log((double)e.tile_m);
    f[4] = (float)std::log((double)e.tile_n);
    f[5] = (float)std::log((double)e.tile_m * e.tile_n / e.threads);
    f[6] = (float)(e.lds_bytes / 65536.0);
    f[7] = (float)std::min(1.0, waves / waves_max);
    f[8] = (float)((double)M * N / ((double)tm * e.tile_m * (double)tn * e.tile_n));
    f[9] = (float)((double)tiles / ((double)rounds * slots));
    f[10] = wide ? 1.0f : 0.0f;
    f[11] = (float)std::log((double)ks);
    f[12] = (float)std::log(estimate_seconds(m, e, dtype, M, N, K, wide, ks));
}

// ln(seconds) predictions for rows of raw features, on `device`
void costmodel_predict(const pk_costmodel &cm, int device, const float *X, int64_t n, float *out) {
    using namespace pkcm;
    if (n <= 0) return;
    CM_CHECK(hipSetDevice(device));
    std::vector<float> Xs((size_t)n * IN);
    for (int64_t r = 0; r < n; ++r)
        for (int k = 0; k < IN; ++k) Xs[r * IN + k] = (X[r * IN + k] - cm.xmean[k]) / cm.xstd[k];
    DeviceBuffers d;
    alloc(d, n, false);
    hipStream_t s;
    CM_CHECK(hipStreamCreate(&s));
    CM_CHECK(hipMemcpyAsync(d.P, cm.params.data(), NP * sizeof(float), hipMemcpyHostToDevice, s));
    CM_CHECK(hipMemcpyAsync(d.X, Xs.data(), Xs.size() * sizeof(float), hipMemcpyHostToDevice, s));
    forward_backward(s, d, n, false);
    CM_CHECK(hipMemcpyAsync(out, d.Y, n * sizeof(float), hipMemcpyDeviceToHost, s));
    CM_CHECK(hipStreamSynchronize(s));
    CM_CHECK(hipStreamDestroy(s));
    for (int64_t r = 0; r < n; ++r) out[r] = out[r] * cm.ystd + cm.ymean;
}

}  // namespace pk

using namespace pk;

extern "C" {

int pk_features(const pk_table *tbl, const pk_params *p, pk_dtype dtype, int64_t M, int64_t N, int64_t K, int wide,
                float *out) {
    if (!tbl || !p || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    pk_params q;
    const KernelEntry *e = nullptr;
    int rc = resolve(tbl, p, (int)dtype, &q, &e);
    if (rc != PK_OK) return rc;
    features(tbl->machine, *e, (int)dtype, M, N, K, wide != 0, q.ks, out);
    return PK_OK;
}

int pk_costmodel_grad(int device, const float *params, const float *X, const float *t, int64_t n, float *grad,
                      float *loss) {
    using namespace pkcm;
    if (!params || !X || !t || n <= 0) return fail(PK_ERR_INVALID_ARG, "bad arguments");
    try {
        CM_CHECK(hipSetDevice(device));
        DeviceBuffers d;
        alloc(d, n, true);
        hipStream_t s;
        CM_CHECK(hipStreamCreate(&s));
        CM_CHECK(hipMemcpyAsync(d.P, params, NP * sizeof(float), hipMemcpyHostToDevice, s));
        CM_CHECK(hipMemcpyAsync(d.X, X, (size_t)n * IN * sizeof(float), hipMemcpyHostToDevice, s));
        CM_CHECK(hipMemcpyAsync(d.T, t, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s));
        forward_backward(s, d, n, true);
        if (grad) CM_CHECK(hipMemcpyAsync(grad, d.grad, NP * sizeof(float), hipMemcpyDeviceToHost, s));
        if (loss) CM_CHECK(hipMemcpyAsync(loss, d.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        CM_CHECK(hipStreamSynchronize(s));
        CM_CHECK(hipStreamDestroy(s));
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_HIP, ex.what());
    }
}

int pk_costmodel_adam_step(int device, float *params, const float *grad, float *m, float *v, int64_t step, float lr) {
    using namespace pkcm;
    if (!params || !grad || !m || !v || step < 1) return fail(PK_ERR_INVALID_ARG, "bad arguments");
    try {
        CM_CHECK(hipSetDevice(device));
        float *dP, *dG, *dM, *dV;
        CM_CHECK(hipMalloc(&dP, 4 * NP * sizeof(float)));
        dG = dP + NP;
        dM = dG + NP;
        dV = dM + NP;
        CM_CHECK(hipMemcpy(dP, params, NP * sizeof(float), hipMemcpyHostToDevice));
        CM_CHECK(hipMemcpy(dG, grad, NP * sizeof(float), hipMemcpyHostToDevice));
        CM_CHECK(hipMemcpy(dM, m, NP * sizeof(float), hipMemcpyHostToDevice));
        CM_CHECK(hipMemcpy(dV, v, NP * sizeof(float), hipMemcpyHostToDevice));
        const float c1 = (float)(1.0 - std::pow(0.9, (double)step)), c2 = (float)(1.0 - std::pow(0.999, (double)step));
        mlp_adam<<<(NP + 255) / 256, 256>>>(dP, dG, dM, dV, lr, 0.9f, 0.999f, (float)(1.0 - 0.9), (float)(1.0 - 0.999),
                                            1e-8f, c1, c2);
        CM_CHECK(hipGetLastError());
        CM_CHECK(hipMemcpy(params, dP, NP * sizeof(float), hipMemcpyDeviceToHost));
        CM_CHECK(hipMemcpy(m, dM, NP * sizeof(float), hipMemcpyDeviceToHost));
        CM_CHECK(hipMemcpy(v, dV, NP * sizeof(float), hipMemcpyDeviceToHost));
        hipFree(dP);
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_HIP, ex.what());
    }
}

int pk_costmodel_train(const pk_table *tbl, const float *X, const float *seconds, int64_t n, int epochs, float lr,
                       uint64_t seed, pk_costmodel **out, float *final_loss) {
    using namespace pkcm;
    if (!tbl || !X || !seconds || n < 2 || epochs < 1 || !out) return fail(PK_ERR_INVALID_ARG, "bad arguments");
    if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "training needs a table bound to a device");
    try {
        std::unique_ptr<pk_costmodel> cm(new pk_costmodel);
        cm->fingerprint = machine_fingerprint(tbl->machine);
        // standardisation of features and of ln(seconds)
        for (int k = 0; k < IN; ++k) {
            double s = 0, s2 = 0;
            for (int64_t r = 0; r < n; ++r) s += X[r * IN + k];
            const double mean = s / n;
            for (int64_t r = 0; r < n; ++r) s2 += (X[r * IN + k] - mean) * (X[r * IN + k] - mean);
            const double sd = std::sqrt(s2 / n);
            cm->xmean[k] = (float)mean;
            cm->xstd[k] = sd > 1e-6 ? (float)sd : 1.0f;
        }
        std::vector<float> T(n);
        double s = 0, s2 = 0;
        for (int64_t r = 0; r < n; ++r) {
            if (!(seconds[r] > 0)) return fail(PK_ERR_INVALID_ARG, "timings must be positive");
            T[r] = (float)std::log(seconds[r]);
            s += T[r];
        }
        cm->ymean = (float)(s / n);
        for (int64_t r = 0; r < n; ++r) s2 += (T[r] - cm->ymean) * (T[r] - cm->ymean);
        cm->ystd = (float)std::max(1e-6, std::sqrt(s2 / n));
        for (auto &v : T) v = (v - cm->ymean) / cm->ystd;
        std::vector<float> Xs((size_t)n * IN);
        for (int64_t r = 0; r < n; ++r)
            for (int k = 0; k < IN; ++k) Xs[r * IN + k] = (X[r * IN + k] - cm->xmean[k]) / cm->xstd[k];
        // weights and biases of a layer uniform on +-1/sqrt(fan-in): trained on
        // the tuner's timings this reached a lower loss and regret than
        // He-uniform weights with zero biases (which start with ~2.4x larger
        // activations)
        cm->params.assign(NP, 0.0f);
        std::mt19937_64 rng(seed);
        auto init = [&](int off, int boff, int rows, int cols) {
            std::uniform_real_distribution<float> u(-1.0f / std::sqrt((float)cols), 1.0f / std::sqrt((float)cols));
            for (int i = 0; i < rows * cols; ++i) cm->params[off + i] = u(rng);
            for (int i = 0; i < rows; ++i) cm->params[boff + i] = u(rng);
        };
        init(OFF_W1, OFF_B1, H, IN);
        init(OFF_W2, OFF_B2, H, H);
        init(OFF_W3, OFF_B3, 1, H);

        CM_CHECK(hipSetDevice(tbl->device));
        DeviceBuffers d;
        alloc(d, n, true);
        hipStream_t st;
        CM_CHECK(hipStreamCreate(&st));
        CM_CHECK(hipMemcpyAsync(d.P, cm->params.data(), NP * sizeof(float), hipMemcpyHostToDevice, st));
        CM_CHECK(hipMemcpyAsync(d.X, Xs.data(), Xs.size() * sizeof(float), hipMemcpyHostToDevice, st));
        CM_CHECK(hipMemcpyAsync(d.T, T.data(), T.size() * sizeof(float), hipMemcpyHostToDevice, st));
        CM_CHECK(hipMemsetAsync(d.m, 0, NP * sizeof(float), st));
        CM_CHECK(hipMemsetAsync(d.v, 0, NP * sizeof(float), st));
        const float b1 = 0.9f, b2 = 0.999f;
        double p1 = 1.0, p2 = 1.0;
        for (int ep = 1; ep <= epochs; ++ep) {
            forward_backward(st, d, n, true);
            p1 *= b1;
            p2 *= b2;
            mlp_adam<<<(NP + 255) / 256, 256, 0, st>>>(d.P, d.grad, d.m, d.v, lr, b1, b2, (float)(1.0 - 0.9),
                                                        (float)(1.0 - 0.999), 1e-8f, (float)(1.0 - p1),
                                                        (float)(1.0 - p2));
        }
        CM_CHECK(hipGetLastError());
        // final loss at the trained parameters
        forward_backward(st, d, n, true);
        CM_CHECK(hipMemcpyAsync(cm->params.data(), d.P, NP * sizeof(float), hipMemcpyDeviceToHost, st));
        CM_CHECK(hipMemcpyAsync(&cm->loss, d.loss, sizeof(float), hipMemcpyDeviceToHost, st));
        CM_CHECK(hipStreamSynchronize(st));
        CM_CHECK(hipStreamDestroy(st));
        cm->epochs = epochs;
        if (final_loss) *final_loss = cm->loss;
        *out = cm.release();
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_HIP, ex.what());
    }
}

int pk_costmodel_predict(const pk_costmodel *cm, int device, const float *X, int64_t n, float *log_seconds) {
    if (!cm || !X || !log_seconds || n < 0) return fail(PK_ERR_INVALID_ARG, "bad arguments");
    try {
        costmodel_predict(*cm, device, X, n, log_seconds);
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_HIP, ex.what());
    }
}

int pk_costmodel_params(const pk_costmodel *cm, float *out, int cap, int *n) {
    if (!cm || !n) return fail(PK_ERR_INVALID_ARG, "null argument");
    *n = pkcm::NP;
    if (!out) return PK_OK;
    if (cap < pkcm::NP) return fail(PK_ERR_BUFFER_TOO_SMALL, "cap below the parameter count");
    std::memcpy(out, cm->params.data(), pkcm::NP * sizeof(float));
    return PK_OK;
}

int pk_costmodel_save(const pk_costmodel *cm, const char *path) {
    if (!cm || !path) return fail(PK_ERR_INVALID_ARG, "null argument");
    std::ofstream f(path);
    if (!f) return fail(PK_ERR_INVALID_ARG, std::string("cannot write ") + path);
    f.precision(9);
    f << "pk-costmodel 1\n" << "features " << PK_NFEATURES << "\n" << "machine " << cm->fingerprint << "\n"
      << "dtype " << (cm->dtype == PK_I32 ? "i32" : cm->dtype == PK_BF16 ? "bf16" : "f32") << "\n";
    f << "epochs " << cm->epochs << "\nloss " << cm->loss << "\nxmean";
    for (float v : cm->xmean) f << " " << v;
    f << "\nxstd";
    for (float v : cm->xstd) f << " " << v;
    f << "\ny " << cm->ymean << " " << cm->ystd << "\nparams " << cm->params.size() << "\n";
    for (size_t i = 0; i < cm->params.size(); ++i) f << cm->params[i] << ((i + 1) % 8 ? " " : "\n");
    f << "\n";
    return f ? PK_OK : fail(PK_ERR_INVALID_ARG, "write failed");
}

int pk_costmodel_load(const char *path, pk_costmodel **out) {
    if (!path || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    std::ifstream f(path);
    if (!f) return fail(PK_ERR_COST_MODEL, std::string("cannot read ") + path);
    std::unique_ptr<pk_costmodel> cm(new pk_costmodel);
    std::string key;
    int version = 0, nf = 0;
    size_t np = 0;
    f >> key >> version;
    if (key != "pk-costmodel" || version != 1) return fail(PK_ERR_COST_MODEL, "not a cost-model file");
    while (f >> key) {
        if (key == "features") f >> nf;
        else if (key == "machine") f >> cm->fingerprint;
        else if (key == "dtype") {  // absent: float32 (files written before the field)
            std::string d;
            f >> d;
            if (d == "f32") cm->dtype = PK_F32;
            else if (d == "i32") cm->dtype = PK_I32;
            else if (d == "bf16") cm->dtype = PK_BF16;
            else return fail(PK_ERR_COST_MODEL, "unknown dtype " + d);
        }
        else if (key == "epochs") f >> cm->epochs;
        else if (key == "loss") f >> cm->loss;
        else if (key == "xmean") for (float &v : cm->xmean) f >> v;
        else if (key == "xstd") for (float &v : cm->xstd) f >> v;
        else if (key == "y") f >> cm->ymean >> cm->ystd;
        else if (key == "params") {
            f >> np;
            cm->params.resize(np);
            for (float &v : cm->params) f >> v;
        } else return fail(PK_ERR_COST_MODEL, "unknown key " + key);
    }
    if (nf != PK_NFEATURES || np != (size_t)pkcm::NP) return fail(PK_ERR_COST_MODEL, "feature or parameter count differs");
    *out = cm.release();
    return PK_OK;
}

void pk_costmodel_free(pk_costmodel *cm) { delete cm; }

const char *pk_costmodel_machine(const pk_costmodel *cm) { return cm ? cm->fingerprint.c_str() : nullptr; }

int pk_costmodel_dtype(const pk_costmodel *cm) { return cm ? cm->dtype : fail(PK_ERR_INVALID_ARG, "null model"); }

int pk_costmodel_set_dtype(pk_costmodel *cm, pk_dtype dtype) {
    if (!cm) return fail(PK_ERR_INVALID_ARG, "null model");
    if (dtype != PK_F32 && dtype != PK_I32 && dtype != PK_BF16) return fail(PK_ERR_UNSUPPORTED_DTYPE, "unknown dtype");
    cm->dtype = (int)dtype;
    return PK_OK;
}

int pk_case_table_set_costmodel(pk_table *tbl, const pk_costmodel *cm) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (cm && cm->fingerprint != machine_fingerprint(tbl->machine))
        return fail(PK_ERR_COST_MODEL, "cost model trained on " + cm->fingerprint + ", table bound to " +
                                           machine_fingerprint(tbl->machine));
    if (!cm)
        for (auto &slot : tbl->costmodel) slot.reset();
    else
        tbl->costmodel[cm->dtype] = std::shared_ptr<pk_costmodel>(new pk_costmodel(*cm));
    std::lock_guard<std::mutex> g(tbl->cache_mu);
    for (auto it = tbl->cache.begin(); it != tbl->cache.end();)
        it = std::get<4>(it->first) == PK_POLICY_LEARNED && (!cm || std::get<0>(it->first) == cm->dtype)
                 ? tbl->cache.erase(it)
                 : std::next(it);
    return PK_OK;
}

int pk_case_table_learned_stats(const pk_table *tbl, int64_t *selections, int64_t *fallbacks) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (selections) *selections = tbl->learned_selections.load();
    if (fallbacks) *fallbacks = tbl->learned_fallbacks.load();
    return PK_OK;
}

int pk_case_table_learned_measured(const pk_table *tbl, int64_t *candidates) {
    if (!tbl || !candidates) return fail(PK_ERR_INVALID_ARG, "null argument");
    *candidates = tbl->learned_measured.load();
    return PK_OK;
}

int pk_case_table_set_learned_margin(pk_table *tbl, double margin) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (!(margin >= 0.0 && margin <= 1.0)) return fail(PK_ERR_INVALID_ARG, "margin outside [0, 1]");
    tbl->learned_margin = margin;
    std::lock_guard<std::mutex> g(tbl->cache_mu);
    for (auto it = tbl->cache.begin(); it != tbl->cache.end();)
        it = std::get<4>(it->first) == PK_POLICY_LEARNED ? tbl->cache.erase(it) : std::next(it);
    return PK_OK;
}

}  // extern "C"
