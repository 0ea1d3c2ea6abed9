// Load-time selection of a leaf and its program parameters.
#pragma once

#include <hip/hip_runtime.h>

#include "pk_internal.hpp"

namespace pk {

// One feasible choice: a leaf of a family's table that holds at the bound
// machine and at the program parameters of the point, with its instance.
struct Candidate {
    int family = 0;
    int point = 0;   // index into the family's point list
    int leaf = -1;
    int variant = 0;
    const KernelEntry *entry = nullptr;
    int ks = 1;             // MFMA programs: shares of K (a launch parameter)
    double estimate = 0.0;  // analytic time estimate, seconds
};

// The feasible set F for (dtype, M, N, K).  When `A` is given, MFMA
// candidates whose alignment conditions fail are left out.
std::vector<Candidate> feasible(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K,
                                const void *A = nullptr, int64_t lda = 0, const void *B = nullptr,
                                int64_t ldb = 0);

// Analytic time of one launch (the CASE score).
// `wide`: the operands' rows are aligned for the MFMA programs' 16-byte loads.
double estimate_seconds(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K,
                        bool wide = true, int ks = 1);

// Shares of K worth trying for an MFMA program at (M, N, K): 2, 4, ... while
// the product has fewer tiles than two per compute unit at the previous
// share count and every share keeps at least two K steps.
std::vector<int> k_splits(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N, int64_t K);

// Compute-unit seconds of a product's tiles under a program when every
// compute unit is kept full of its workgroups (the work a persistent grouped
// launch spends on the product).
double tile_work_seconds(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K);

// Analytic time of one launch of a streaming (HBM-bound) kernel moving
// `bytes`: compulsory bytes over 8 TB/s, scaled by the share one launch can
// sustain -- the filled share of the last round of tiles, the bytes a compute
// unit keeps in flight (about 64 KiB per compute unit covers HBM latency at
// full bandwidth), and the narrowest contiguous segment a wavefront touches
// (below 256 bytes, one wavefront's 64 four-byte lanes, its access is split
// over rows) -- plus launch latency.
double streaming_seconds(const pk_machine &m, const KernelEntry &e, double bytes, int64_t tiles,
                         double inflight_bytes_per_tile, double segment_bytes);

int select_params(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K, int policy, bool cache,
                  pk_params *out, const void *A = nullptr, int64_t lda = 0, const void *B = nullptr,
                  int64_t ldb = 0);

// Operands to time on (device pointers), or scratch buffers when A is null.
struct Operands {
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
};

// Times every candidate (HIP events on a private stream); secs[i] is the
// mean time per launch of candidate i (+inf where its launches or events
// failed).  Returns PK_OK with *best the index of the fastest, or an error
// (PK_ERR_HIP when the timing set-up fails or no candidate could be timed).
int time_candidates(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K,
                    const std::vector<Candidate> &cands, std::vector<double> *secs, const Operands *ops, int *best);

// Queues C[i][j] = 0 (i < M, j < N, rows of ldc floats) on `stream` (fill.hip).
int zero_matrix(const pk_machine &m, void *C, int64_t ldc, int64_t M, int64_t N, hipStream_t stream);

// helpers shared with capi.cpp
int64_t blocks_per_cu(const pk_machine &m, const KernelEntry &e);
int64_t grid_of(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N);
// the same for a launch: residency from the runtime's occupancy calculator
int64_t live_blocks_per_cu(const pk_machine &m, const KernelEntry &e);
int64_t launch_grid(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N);
bool wide_rows(int dtype, const void *A, int64_t lda, const void *B, int64_t ldb);
int launch(const pk_machine &m, const KernelEntry &e, const MmArgs &args, hipStream_t stream);
void fill_params(const pk_table *tbl, const Candidate &c, int dtype, pk_params *out);
int resolve(const pk_table *tbl, const pk_params *pin, int dtype, pk_params *pout, const KernelEntry **entry);

// cost model (costmodel.hip)
std::string machine_fingerprint(const pk_machine &m);
void features(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K, bool wide,
              int ks, float *f);
void costmodel_predict(const pk_costmodel &cm, int device, const float *X, int64_t n, float *out);

}  // namespace pk
