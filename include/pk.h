/*
 * pk.h -- parametric matmul kernels for gfx950 (MI355X), C ABI.
 *
 * A parametric kernel keeps its program parameters (thread-block shape,
 * per-thread coarsening, LDS tile extents) symbolic when it is generated and
 * learns the machine parameters only when it is loaded (Section 1; Section 2,
 * Fig. 4).  A comprehensive parametric kernel is a case discussion: a list of
 * leaves (C_i, S_i) where C_i is a conjunction of polynomial constraints on
 * machine and program parameters and S_i the program optimized under C_i
 * (Definition 3), produced by Algorithms 1 and 2 (Section 3).
 *
 * This library holds
 *   - the symbolic engine of Algorithms 1 and 2 (pk_co_solve),
 *   - the case tables of its kernel families (matmul, and the transposition
 *     and matrix addition of the paper's examples), built once per process
 *     and bound to the machine parameters read from hipDeviceProp_t
 *     (pk_case_table_build),
 *   - load-time selection of a leaf and its program parameters (pk_select),
 *   - the hand-written HIP kernels of every leaf (pk_matmul, and
 *     pk_matmul_batched for many independent products in one launch).
 *
 * Conventions shared by every entry point:
 *   - return value: PK_OK (0) or a negative PK_ERR_* code; nothing throws
 *     across this boundary; pk_last_error() gives a thread-local message;
 *   - matrices are row-major: element (i, j) of X is X[i * ldx + j];
 *   - device pointers are HIP device addresses owned by the caller, which must
 *     keep them alive until the work queued on the given stream completes;
 *   - hip_stream is a hipStream_t (NULL = the default stream); matmul calls
 *     are asynchronous on it;
 *   - every dimension (M, N, K) is at most 2^31 - 2^16 (PK_ERR_INVALID_ARG
 *     beyond): kernels index rows and columns in 32-bit integers.
 */
#ifndef PK_H
#define PK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define PK_OK 0
#define PK_ERR_INVALID_ARG -1         /* null pointer, negative size, ld too small */
#define PK_ERR_NO_FEASIBLE_BRANCH -2  /* no leaf of the case table holds (refuse with no strategy left) */
#define PK_ERR_UNSUPPORTED_DTYPE -3   /* the dtype has no kernel in the requested family */
#define PK_ERR_NOT_INSTANTIATED -4    /* parameters satisfy the constraints but no compiled instance exists */
#define PK_ERR_HIP -5                 /* a HIP runtime call failed; the message holds its code */
#define PK_ERR_COST_MODEL -6          /* no usable cost model (selection fell back, or training failed) */
#define PK_ERR_BUFFER_TOO_SMALL -7    /* an output buffer is too small; *needed holds the size */
#define PK_ERR_PARSE -8               /* a family description given as text could not be parsed */

/* Thread-local message describing the last error returned on this thread. */
const char *pk_last_error(void);

/* ------------------------------------------------------------------ types */
typedef enum {
    PK_F32 = 0,  /* float32 inputs, float32 output, float32 accumulation */
    PK_I32 = 1,  /* int32 inputs and output, arithmetic modulo 2^32 */
    PK_BF16 = 2  /* bfloat16 inputs (raw 16-bit patterns), float32 output and accumulation */
} pk_dtype;

/* Machine parameters (Section 3.2: the resource limits R_i), read from
 * hipDeviceProp_t at load time or given by a caller to model another device. */
typedef struct {
    int32_t wave;              /* W: wavefront width (warpSize) */
    int64_t lds_block;         /* Z: LDS bytes one workgroup may allocate (sharedMemPerBlock) */
    int64_t lds_cu;            /* LDS bytes per compute unit (maxSharedMemoryPerMultiProcessor) */
    int64_t regs_block;        /* V: 32-bit registers one workgroup may allocate (regsPerBlock) */
    int64_t regs_cu;           /* registers per compute unit (regsPerMultiprocessor) */
    int32_t max_threads_block; /* T: work-items per workgroup (maxThreadsPerBlock) */
    int32_t max_threads_cu;    /* resident work-items per compute unit */
    int32_t max_blocks_cu;     /* resident workgroups per compute unit */
    int32_t cu_count;          /* NCU: compute units (multiProcessorCount) */
    int32_t clock_khz;         /* shader clock (clockRate) */
    char arch[64];             /* gcnArchName, e.g. "gfx950:sramecc+:xnack-" */
} pk_machine;

/* Kernel families, i.e. the code fragments S the comprehensive optimization
 * is run on. */
#define PK_FAMILY_VALU 0  /* the blocked kernel of Section 2 (Fig. 3, Fig. 4), f32 and i32 */
#define PK_FAMILY_MFMA 1  /* LDS-tiled matrix-core kernel, f32 and bf16 */
#define PK_FAMILY_TRANSPOSE 2 /* matrix transposition (Section 5.2, Fig. 7), 4-byte elements */
#define PK_FAMILY_MADD 3      /* matrix addition (Section 1, Fig. 1 and Fig. 2), f32 and i32 */
#define PK_FAMILY_JACOBI 4    /* 1D Jacobi time step (Section 5, Fig. 6, Table 2), f32 and i32 */
#define PK_FAMILY_POLYDIV 5   /* polynomial division mod P (Section 5, Fig. 8, Table 4), u32 residues */
#define PK_FAMILY_VALU2 6     /* the kernel of Section 2 with 2-D micro-tiles and a free LDS K extent, f32 and i32 */
#define PK_NUM_FAMILIES 7

/* Strategy bits of the VALU family (a variant is the set of strategies applied):
 * PK_VALU_GRAN  - granularity reduced to one output per thread (decision (3b), Section 5)
 * PK_VALU_NOLDS - operands read straight from global memory, no LDS (decision (4b)) */
#define PK_VALU_GRAN 1
#define PK_VALU_NOLDS 2
/* Strategy bits of the transposition family: PK_VALU_GRAN (one element per
 * work-item) and PK_VALU_NOLDS (no LDS tile), as for the VALU family. */
/* Strategy bits of the MFMA family:
 * PK_MFMA_SINGLE - one LDS stage instead of two (halves the LDS tile footprint)
 * PK_MFMA_GROUPED marks the persistent grouped instances of the same programs
 * (not a strategy of the case table; set only in instance descriptions) */
#define PK_MFMA_SINGLE 1
#define PK_MFMA_GROUPED 2
#define PK_MFMA_ELEMENT 4 /* internal: the twin of a program that reads rows element by element */
#define PK_MFMA_MIXED 8   /* internal: a grouped kernel running a different tile program per product */
#define PK_MFMA_SPLIT 16  /* internal: the form of a program that runs shares of K (pk_params.ks > 1) */

/* A leaf choice together with its program parameters E.
 *   family  - PK_FAMILY_*
 *   leaf    - leaf index in that family's table for the dtype, or -1
 *   variant - strategy bits of the program to run, or -1
 * VALU family: bx = threads along N (the paper's ub1), by = threads along M
 *   (the paper's B0), s = outputs per thread along N (the paper's s), bk =
 *   K extent of an LDS tile (the paper fixes it to B0; 0 means "= by").
 * 2-D VALU family (PK_FAMILY_VALU2; Fig. 4's kernel generalised): bx x by
 *   work-items, each computing s outputs along N (columns tx + w bx) and sy
 *   along M (rows ty + v by), so a workgroup owns a (by sy) x (bx s) tile;
 *   bk is the K extent of its LDS tiles, a parameter of its own (the paper
 *   ties it to B0); LDS bytes e (by sy (bk + 1) + bk bx s); strategy bit
 *   PK_VALU_GRAN (one output per work-item: s = sy = 1).
 * MFMA family: bm x bn output tile per workgroup, bk its K extent, wm x wn
 *   wavefronts of 64 lanes; unused fields are 0.  ks > 1 splits the product
 *   along K into ks shares of about equal numbers of K steps, one workgroup
 *   per tile and share: C is cleared first (unless accumulating) and each
 *   share adds its sum to C with atomic float additions, so the order in
 *   which the shares' sums enter C varies from run to run (the result stays
 *   within the float32 bound; small-integer inputs stay exact).  ks is a
 *   launch parameter, not a point of the case table: it changes no resource
 *   counter (the same program runs every ks, in a split form compiled
 *   beside it).  Programs of more than 512 work-items, and the single-stage
 *   float32 programs of 512, are not split (PK_ERR_INVALID_ARG). 
 * Transposition family: bx = work-items along the columns of A (the paper's
 *   B1), by = work-items along its rows (B0), s = elements per work-item (s);
 *   a workgroup moves a (by * s) x bx tile of A.
 * Matrix-addition family: bx = work-items along a row (Fig. 2's B1), by =
 *   rows per workgroup (B0), s = elements per work-item (2 in Fig. 2's K1);
 *   strategy bit PK_VALU_GRAN (one element per work-item, Fig. 2's K2).
 * 1D Jacobi family: bx = work-items per workgroup (Fig. 6's B), s = points
 *   per work-item (s); by unused (0 or 1); strategy bits as the VALU family
 *   (PK_VALU_GRAN: s = 1, the second case; PK_VALU_NOLDS: no LDS caching,
 *   the third case).  variant PK_JACOBI_FUSED (with leaf = -1) selects this
 *   library's several-steps-per-launch program (bx in {256, 512, 1024}, s in
 *   {1, 2, 4}): a launch advances an odd number of steps, up to 15, in LDS
 *   with a recomputed halo, and the last step runs alone, so both halves end
 *   as the per-step schedule leaves them; not part of the case table (its
 *   resources are checked against the machine when it is chosen).
 * Polynomial-division family: bx = work-items per workgroup (Fig. 8's B),
 *   s = coefficients per work-item; by unused (0 or 1); strategy bits as the
 *   1D Jacobi family.  Its table is stored under PK_I32 (32-bit residues).
 *   variant PK_POLYDIV_FUSED (with leaf = -1) selects this library's
 *   one-launch program instead of the paper's one launch per step: the
 *   quotient first (a short recurrence in one wavefront of every
 *   workgroup), then every remainder coefficient in parallel; it needs
 *   N - M <= 1024 and bx >= 64 and is not part of the case table (its
 *   resources are checked against the machine when it is chosen). */
#define PK_POLYDIV_FUSED 4
#define PK_JACOBI_FUSED 4
#define PK_POLYDIV_WIDE 8 /* internal: the instance holding up to 1024 quotient coefficients */
typedef struct {
    int32_t family;
    int32_t leaf;
    int32_t variant;
    int32_t bx, by, s, bk;
    int32_t bm, bn, wm, wn;
    int32_t ks;  /* MFMA family: shares of K the product is split into (0 or 1: none) */
    int32_t sy;  /* 2-D VALU family: outputs per work-item along M (0 otherwise) */
} pk_params;

/* Selection policies for pk_select. */
#define PK_POLICY_CASE 0        /* first satisfied leaf per E, best analytic score over E */
#define PK_POLICY_LEARNED 1     /* cost-model prediction over the feasible set */
#define PK_POLICY_EXHAUSTIVE 2  /* time every feasible (leaf, E) on the device, keep the fastest */

typedef struct pk_table pk_table; /* opaque; immutable once built */

/* ------------------------------------------------------------------ machine */
/* Fills *out from hipGetDeviceProperties(device).  Errors: PK_ERR_HIP. */
int pk_machine_query(int device, pk_machine *out);

/* ------------------------------------------------------------------ symbolic engine */
/* Runs Algorithms 1 and 2 (Section 3.7) on a code fragment described in text
 * and writes the leaves as JSON into out (cap bytes, NUL-terminated).
 * The description lists symbols, finite domains, counters with their values
 * after given strategy sets, and strategies with sigma (one item per line):
 *     machine R T            program B0 B1          data N
 *     domain R 0 40          (integer interval)     points B0 1 2 4 8 (list)
 *     counter r_R resource R           value r_R gran : 10      value r_R : 14
 *     strategy gran src r_R            (src | ir, then the counters of sigma)
 *     perf_one 100                      (units of a performance measure's 1)
 * A counter's value after a set of applied strategies is the first "value"
 * line of that counter whose strategies are all applied.  Errors:
 * PK_ERR_PARSE, PK_ERR_BUFFER_TOO_SMALL (*needed = bytes required). */
int pk_co_solve(const char *spec, char *out, size_t cap, size_t *needed);

/* ------------------------------------------------------------------ case table */
/* Builds the comprehensive case tables of every family and dtype and binds
 * them to the machine: the parameters of `device` (via pk_machine_query)
 * when override_or_null is NULL, else the given descriptor (no GPU call).
 * `device` is the device later timing (PK_POLICY_EXHAUSTIVE, pk_measure,
 * the LEARNED fallback) and training run on; -1 for none.  The table is
 * owned by the caller and freed with pk_case_table_free.
 * Errors: PK_ERR_HIP, PK_ERR_INVALID_ARG. */
int pk_case_table_build(int device, const pk_machine *override_or_null, pk_table **out);
void pk_case_table_free(pk_table *tbl);

/* JSON description of the table: the machine, every family's leaves (their
 * strategy sets, lambda, constraint systems) and the compiled instances with
 * their resource usage.  Errors: PK_ERR_BUFFER_TOO_SMALL (*needed). */
int pk_case_table_describe(const pk_table *tbl, char *out, size_t cap, size_t *needed);

/* Leaf lookup at fixed program parameters: *leaf_out = index of the first leaf
 * of (family, dtype) whose system holds at the bound machine and at E given
 * in *p (family, bx.. fields), and *variant_out its strategy bits.
 * Errors: PK_ERR_NO_FEASIBLE_BRANCH (no leaf holds), PK_ERR_UNSUPPORTED_DTYPE,
 * PK_ERR_INVALID_ARG (E outside the family's parameter domain). */
int pk_case_table_lookup(const pk_table *tbl, pk_dtype dtype, const pk_params *p,
                         int32_t *leaf_out, int32_t *variant_out);

/* ------------------------------------------------------------------ selection */
/* Chooses a leaf and program parameters for C(MxN) = A(MxK) B(KxN) under a
 * policy and writes them to *out: the load-time step of Section 1, where the
 * case discussion, evaluated at the machine's parameters, fixes which
 * programs may run, and the program parameters the paper leaves to
 * auto-tuning are chosen by an analytic estimate (CASE), a learned cost
 * model (LEARNED) or measurement (EXHAUSTIVE).  Every candidate satisfies its leaf's
 * system at the bound machine.  PK_POLICY_EXHAUSTIVE launches kernels on the
 * table's device on a private stream and synchronizes; its picks are cached
 * per (dtype, M, N, K) for the table's lifetime.  PK_POLICY_LEARNED needs a
 * model for dtype given to the table (pk_case_table_set_costmodel; else
 * PK_ERR_COST_MODEL and *out holds the CASE pick).  Errors: PK_ERR_NO_FEASIBLE_BRANCH, PK_ERR_INVALID_ARG. */
int pk_select(const pk_table *tbl, pk_dtype dtype, int64_t M, int64_t N, int64_t K, int policy,
              pk_params *out);

/* As pk_select, for given operands (device pointers, row-major, as in
 * pk_matmul): MFMA candidates are costed and, under EXHAUSTIVE or the LEARNED
 * fallback, timed as the kernels pk_matmul would run on these operands -- the
 * element-load form where rows are not aligned for 16-byte loads, and a
 * program without one left out.  EXHAUSTIVE and the LEARNED fallback time
 * on A and B with a scratch C they allocate; picks are not cached.  M, N > 0.
 * Errors as pk_select, and PK_ERR_HIP. */
int pk_select_operands(const pk_table *tbl, pk_dtype dtype, const void *A, int64_t lda, const void *B, int64_t ldb,
                       int64_t M, int64_t N, int64_t K, int policy, pk_params *out);

/* Times every feasible (leaf, E) for C(MxN) = A(MxK) B(KxN) on the table's
 * device -- the auto-tuning by which Section 1 fixes program parameters, and
 * the measurement behind PK_POLICY_EXHAUSTIVE, the tuner and the
 * cost model's training data.  A, B, C (device pointers, row-major, as in
 * pk_matmul; C is overwritten) are the operands to time on; with A == NULL
 * the call allocates scratch operands filled with a non-zero byte pattern and
 * frees them.  Candidates are timed in order of their CASE estimate, least
 * first.  Each is launched once between two events (warm-up); if that launch
 * took over 1 ms and twice the best mean so far, its time is that launch's;
 * otherwise it is launched back to back between two events: 3 launches, and,
 * unless their mean is already 1.5x the best so far, more until about 20 ms
 * of work; seconds_out[i] (in the order of params_out) is its mean
 * time per launch (+inf for a candidate whose launches or events failed;
 * PK_ERR_HIP when no candidate could be timed or the timing set-up failed).
 * Runs on a private stream and synchronizes.  *n receives the number
 * of candidates; arrays must hold cap >= *n entries (else
 * PK_ERR_BUFFER_TOO_SMALL).  MFMA candidates are timed on the given
 * operands as they are: rows not aligned for 16-byte loads are read element
 * by element.
 * Errors: PK_ERR_INVALID_ARG, PK_ERR_NO_FEASIBLE_BRANCH, PK_ERR_HIP. */
int pk_measure(const pk_table *tbl, pk_dtype dtype, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
               int64_t ldc, int64_t M, int64_t N, int64_t K, pk_params *params_out, double *seconds_out, int cap,
               int *n);

/* ------------------------------------------------------------------ products */
/* C = A B (accumulate = 0) or C = C + A B (accumulate = 1, the semantics of
 * the kernel of Fig. 4, which loads c, adds the products and stores it back).
 * A is MxK with leading dimension lda, B is KxN (ldb), C is MxN (ldc); for
 * PK_BF16, A and B hold bfloat16 bit patterns and C is float32.
 * params_or_null: NULL selects with PK_POLICY_CASE; otherwise
 *   leaf >= 0           runs that leaf at E (its system must hold),
 *   leaf < 0, variant>=0 runs that variant at E if its resources fit the machine
 *                       (the "forced" mode used to test every program),
 *   both < 0            looks the leaf up at E.
 * M == 0 or N == 0 is a no-op; K == 0 writes zeros (or leaves C unchanged
 * when accumulating).  MFMA programs load 16 bytes at a time along rows that
 * are aligned for it (A and B 16-byte aligned; lda and ldb multiples of 4
 * for f32, of 8 for bf16) and element by element otherwise -- the same
 * arithmetic in the same order, so the result does not depend on the
 * alignment.  One program
 * has no element-load form (the bfloat16 256 x 256 x 64 tile, whose
 * element-load kernel would spill); given it with operands whose rows are not
 * aligned, the call runs the CASE choice for those operands instead.
 * Errors: PK_ERR_INVALID_ARG, PK_ERR_NO_FEASIBLE_BRANCH,
 * PK_ERR_UNSUPPORTED_DTYPE, PK_ERR_NOT_INSTANTIATED, PK_ERR_HIP. */
int pk_matmul(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype,
              const void *A, int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc,
              int64_t M, int64_t N, int64_t K, int accumulate, void *hip_stream);

/* ------------------------------------------------------------------ many products */
/* A plan for G independent products C_g = [C_g +] A_g B_g (f32 or bf16 ->
 * f32), run as persistent launches: the workgroups of a launch stride over
 * the tiles of all its products (the grid-stride loop of the paper's kernel,
 * Section 2, Fig. 4, spanning many products).  Sizes and pointer arrays are
 * host arrays (device pointers inside), all of length G; products with M or
 * N = 0 are skipped, and K = 0 writes zeros (or leaves C with accumulate).
 * Each product runs one MFMA program: a point of the case table whose leaf
 * holds at the bound machine.  A mixed grouped kernel runs a different tile
 * program per product in one launch (64x64, 128x64, 64x128 or 128x128
 * output tiles of 2 x 2 wavefronts, one workgroup size, LDS sized for the
 * largest); a plan is one launch whenever its products' programs are all one
 * program or all programs of the mixed kernel with one LDS-stage count, and
 * one launch per program otherwise.
 * per_group_or_null gives each product's MFMA leaf/parameters (resolved as
 * in pk_matmul).  With NULL, `policy`:
 *   PK_POLICY_CASE        per product, the program of least estimated
 *     compute-unit time at the residency of the kernel it runs in; the
 *     kernel (each uniform program fitting every product, each mixed kernel)
 *     of least summed estimate;
 *   PK_POLICY_EXHAUSTIVE  the auto-tuning of Section 1 at plan level: a plan
 *     of every uniform program and stage count, and of each mixed kernel
 *     under three per-product rules (the CASE estimate, the largest tile
 *     wasting at most 15 % or at most 35 % of its area on padding), each
 *     timed on the device on the plan's own operands (one untimed run, the
 *     median of three); the fastest is kept.  Those runs write C, so it is
 *     refused (PK_ERR_INVALID_ARG) together with accumulate;
 *   PK_POLICY_LEARNED     refused (PK_ERR_INVALID_ARG): the cost model
 *     predicts the time of a single launch, not a product's share of a
 *     persistent one.
 * The tiles of a launch are ordered by estimated cost, most expensive first,
 * and cut into 8 ranges of equal estimated cost, one per XCD.  Rows that are
 * not aligned for the 16-byte loads are read with element loads.  The plan
 * copies its descriptors to the device when created (allocating and
 * synchronizing then); running it allocates nothing and does not
 * synchronize, so it may be captured in a HIP graph.  Pointers must stay
 * valid while the plan is used.  Errors: PK_ERR_INVALID_ARG,
 * PK_ERR_UNSUPPORTED_DTYPE, PK_ERR_NO_FEASIBLE_BRANCH, PK_ERR_NOT_INSTANTIATED,
 * PK_ERR_HIP. */
typedef struct pk_grouped_plan pk_grouped_plan;
int pk_grouped_plan_create(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M, const int64_t *N,
                           const int64_t *K, const void *const *A, const int64_t *lda, const void *const *B,
                           const int64_t *ldb, void *const *C, const int64_t *ldc,
                           const pk_params *per_group_or_null, int policy, int accumulate,
                           pk_grouped_plan **out);
/* Queues the plan's launches on hip_stream. */
int pk_grouped_plan_run(const pk_grouped_plan *plan, void *hip_stream);
/* Captures the plan's launches once into a HIP graph owned by the plan;
 * pk_grouped_plan_replay launches that graph on hip_stream. */
int pk_grouped_plan_capture(pk_grouped_plan *plan);
int pk_grouped_plan_replay(const pk_grouped_plan *plan, void *hip_stream);
/* Launch count, total tiles, and (cap >= G) the choice made per product. */
int pk_grouped_plan_info(const pk_grouped_plan *plan, int32_t *launches, int64_t *total_tiles, pk_params *chosen,
                         int32_t cap);
/* The kernel of launch i (0 <= i < launch count): *name points at a string
 * the library owns (valid for the process).  Errors: PK_ERR_INVALID_ARG. */
int pk_grouped_plan_kernel(const pk_grouped_plan *plan, int32_t i, const char **name);
void pk_grouped_plan_destroy(pk_grouped_plan *plan);

/* One-shot form: creates a plan (CASE choice when per_group_or_null is NULL),
 * runs it on hip_stream, synchronizes the stream and destroys the plan. */
int pk_matmul_batched(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M, const int64_t *N,
                      const int64_t *K, const void *const *A, const int64_t *lda, const void *const *B,
                      const int64_t *ldb, void *const *C, const int64_t *ldc, const pk_params *per_group_or_null,
                      void *hip_stream);

/* pk_matmul_batched for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same products, the same CASE choice (or the given per-product parameters),
 * the same kernels, but the launch's descriptors and tile map go to a
 * workspace that every GPU running the library holds from the table's
 * creation until the process ends, 4 MiB per device (reached through a static
 * host staging copy of the same size), instead of device memory allocated for
 * a plan.  No hipMalloc, hipFree, pinned-memory allocation or allocating
 * library routine is called.  A layout larger than the workspace (about
 * 50000 small products) is refused with PK_ERR_INVALID_ARG before any work
 * is queued.  Every call shares its GPU's workspace: calls in one process are
 * serialised by a lock and each returns after its work on hip_stream is done
 * (it synchronizes the stream), so one call's layout is never overwritten by
 * another's; calls that overlapped on one GPU would race on it.  Errors as
 * pk_matmul_batched. */
int pk_matmul_batched_noalloc(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M, const int64_t *N,
                              const int64_t *K, const void *const *A, const int64_t *lda, const void *const *B,
                              const int64_t *ldb, void *const *C, const int64_t *ldc,
                              const pk_params *per_group_or_null, void *hip_stream);

/* ------------------------------------------------------------------ transposition */
/* C (N x M) = A (M x N) transposed, 4-byte elements copied bit for bit
 * (dtype PK_F32 or PK_I32), row-major with leading dimensions lda >= N,
 * ldc >= M; asynchronous on hip_stream.  params_or_null: family
 * PK_FAMILY_TRANSPOSE, resolved as in pk_matmul (NULL: the CASE choice).
 * Errors: PK_ERR_INVALID_ARG, PK_ERR_NO_FEASIBLE_BRANCH,
 * PK_ERR_UNSUPPORTED_DTYPE, PK_ERR_NOT_INSTANTIATED, PK_ERR_HIP. */
int pk_transpose(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, const void *A, int64_t lda,
                 void *C, int64_t ldc, int64_t M, int64_t N, void *hip_stream);

/* Choice of a transposition leaf and parameters for an M x N matrix:
 * PK_POLICY_CASE (analytic: bytes over bandwidth by program, with wave
 * quantisation) or PK_POLICY_EXHAUSTIVE (every feasible candidate timed on
 * scratch buffers; synchronizes; cached).  Errors as pk_select. */
int pk_select_transpose(const pk_table *tbl, pk_dtype dtype, int64_t M, int64_t N, int policy, pk_params *out);

/* ------------------------------------------------------------------ matrix addition */
/* C = A + B (M x N, row-major, leading dimensions >= N), f32 (one rounding)
 * or i32 (modulo 2^32); asynchronous on hip_stream.  params_or_null: family
 * PK_FAMILY_MADD, resolved as in pk_matmul (NULL: the CASE choice).  The
 * family's counters are registers per workgroup and work-items per workgroup,
 * the two machine parameters of Fig. 2.  Errors as pk_transpose. */
int pk_madd(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, const void *A, int64_t lda,
            const void *B, int64_t ldb, void *C, int64_t ldc, int64_t M, int64_t N, void *hip_stream);
int pk_select_madd(const pk_table *tbl, pk_dtype dtype, int64_t M, int64_t N, int policy, pk_params *out);

/* ------------------------------------------------------------------ 1D Jacobi */
/* `steps` time steps of the three-point stencil of Section 5, Fig. 6, in
 * place on a device array a of 2N elements holding two copies of a length-N
 * vector: step t writes the interior (indices 1 .. N-2) of the second copy
 * from the first when t is even, of the first from the second when t is odd
 * (so the result sits in the second copy after an odd number of steps, in
 * the first after an even number); elements 0, N-1, N and 2N-1 are never
 * written.  Each point becomes (left + centre + right) / 3: i32 sums wrap
 * modulo 2^32 and the quotient truncates toward zero; f32 rounds after each
 * addition (left to right) and after the correctly rounded division.  One
 * kernel launch per step, queued on hip_stream (asynchronous).  N >= 2
 * (N = 2 or steps = 0: nothing to do), steps >= 0.  params_or_null: family
 * PK_FAMILY_JACOBI, resolved as in pk_matmul (NULL: the CASE choice).
 * Errors as pk_transpose. */
int pk_jacobi1d(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, void *a, int64_t N,
                int64_t steps, void *hip_stream);
/* Chooses for `steps` time steps on vectors of N points (CASE or EXHAUSTIVE,
 * among the case table's per-step programs and the several-steps program). */
int pk_select_jacobi1d(const pk_table *tbl, pk_dtype dtype, int64_t N, int64_t steps, int policy, pk_params *out);

/* ------------------------------------------------------------------ polynomial division */
/* Division modulo a prime (Section 5, Fig. 8), in place on device arrays:
 * a holds the N coefficients of the dividend (a[i] multiplies x^i), b the M
 * low coefficients of a monic divisor of degree M, b(x) = x^M + b[M-1]
 * x^(M-1) + ... + b[0].  While the dividend's degree is at least M the
 * leading coefficient q times x^(deg - M) b(x) is subtracted -- one kernel
 * launch per step, N - M steps -- and a[M .. N-1] is cleared at the end, so a
 * returns the remainder in a[0 .. M-1] (N <= M: nothing to do).  Every
 * coefficient must be a residue in [0, P) (not checked: other values give an
 * unspecified result); 2 <= P < 2^31 (PK_ERR_INVALID_ARG otherwise; P need
 * not be prime, as b is monic).  N >= 0, M >= 1.  Asynchronous on
 * hip_stream.  params_or_null: family PK_FAMILY_POLYDIV, resolved as in
 * pk_matmul (NULL: the CASE choice).  Errors as pk_transpose. */
int pk_polydiv(const pk_table *tbl, const pk_params *params_or_null, uint32_t *a, int64_t N, const uint32_t *b,
               int64_t M, uint32_t P, void *hip_stream);
int pk_select_polydiv(const pk_table *tbl, int64_t N, int64_t M, int policy, pk_params *out);

/* The CASE policy's analytic time estimate, in seconds, of one launch of a
 * choice (params resolved as in pk_matmul) for an M x N x K product: the
 * score pk_select's CASE policy minimises over the feasible set.  `wide`: the
 * operands' rows are aligned for the MFMA programs' 16-byte loads (0: they
 * run as their element-load twins, see pk_matmul).  Matmul families only.
 * Errors as pk_launch_shape. */
int pk_estimate(const pk_table *tbl, const pk_params *p, pk_dtype dtype, int64_t M, int64_t N, int64_t K, int wide,
                double *seconds);

/* Measured vector-ALU ceiling of the table's device, in operations per
 * second (a multiply-add counts two): independent multiply-add chains with
 * no memory traffic, f32 (fused multiply-add) or i32 (32-bit multiply and
 * add, wrapping), timed with HIP events; the roofline of the VALU matmul
 * programs.  Synchronous; allocates and frees a small output buffer.
 * Errors: PK_ERR_INVALID_ARG (null, or a table not bound to a device),
 * PK_ERR_UNSUPPORTED_DTYPE, PK_ERR_HIP. */
int pk_probe_valu_rate(const pk_table *tbl, pk_dtype dtype, double *ops_per_second);

/* Analytic launch shape of a choice: grid and block sizes and LDS bytes the
 * kernel of *p uses for an MxN output, by the table's machine model.  A
 * launch on a device sizes the grids of workgroup-stride programs by the HIP
 * runtime's occupancy calculator instead, which can hold more workgroups
 * resident than the model (some runtimes report a block register budget of
 * half the register file).  Errors as pk_matmul (no launch). */
int pk_launch_shape(const pk_table *tbl, const pk_params *p, pk_dtype dtype, int64_t M, int64_t N,
                    int64_t K, int64_t *grid, int32_t *block, int64_t *lds_bytes);

/* Name of the compiled kernel a choice runs (as in profiler traces), or NULL
 * with the reason in pk_last_error(); resolution as in pk_matmul. */
const char *pk_kernel_name(const pk_table *tbl, const pk_params *p, pk_dtype dtype);

/* Number of compiled kernel instances, and the name of instance i. */
int pk_instance_count(void);
const char *pk_instance_name(int i);

/* ------------------------------------------------------------------ cost model */
/* The learned cost model: a 13-64-64-1 ReLU network predicting ln(seconds)
 * of a candidate launch from PK_NFEATURES features, trained on the device by
 * the library's own kernels (forward, backward, Adam) on timings from
 * pk_measure.  Not in the paper: it stands in for the auto-tuning the paper
 * leaves open for the program parameters (Section 1). */
#define PK_NFEATURES 13
typedef struct pk_costmodel pk_costmodel; /* opaque */

/* Features of candidate *p for C(MxN) = A(MxK) B(KxN) on the bound machine:
 * ln M, ln N, ln K, ln tile_m, ln tile_n, ln(outputs per work-item), LDS
 * bytes / 65536, estimated occupancy (resident wavefronts / maximum), tile
 * padding efficiency, wave quantisation efficiency (workgroups: tiles times
 * the shares of K), `wide` (1 when the operands' rows are aligned for the
 * MFMA programs' 16-byte loads, 0 when they run as their element-load twins;
 * see pk_matmul), ln of the shares of K (p->ks; 0 unsplit), and ln of the
 * analytic estimate of the launch's seconds (pk_estimate with the same
 * arguments): the network learns a correction to the estimate the CASE
 * policy ranks by.  out: PK_NFEATURES floats.  Errors as pk_launch_shape. */
int pk_features(const pk_table *tbl, const pk_params *p, pk_dtype dtype, int64_t M, int64_t N, int64_t K, int wide,
                float *out);

/* Trains a model on the table's device: X is n x PK_NFEATURES row-major
 * (host), seconds the n measured launch times (host, > 0).  Features and
 * ln(seconds) are standardised; weights and biases start uniform on
 * +-1/sqrt(fan-in) from `seed`;
 * `epochs` full-batch Adam steps (b1 0.9, b2 0.999, eps 1e-8) at rate lr on
 * the mean squared error.  *out is owned by the caller (pk_costmodel_free);
 * *final_loss (optional) is the loss in standardised units.
 * Errors: PK_ERR_INVALID_ARG, PK_ERR_HIP. */
int pk_costmodel_train(const pk_table *tbl, const float *X, const float *seconds, int64_t n, int epochs, float lr,
                       uint64_t seed, pk_costmodel **out, float *final_loss);

/* ln(seconds) predictions for n raw feature rows (host in, host out), one
 * forward launch on `device`; synchronizes. */
int pk_costmodel_predict(const pk_costmodel *cm, int device, const float *X, int64_t n, float *log_seconds);

/* The network's raw forward/backward on the device: mean squared error of
 * the network with parameters `params` (host, 5121 floats in the order W1
 * (64 x PK_NFEATURES), b1, W2 (64x64), b2, W3 (1x64), b3) on rows X (n x PK_NFEATURES, host) and
 * targets t (host); writes the gradient (5121 floats) and the loss.  Used to
 * check the kernels against a float64 reference. */
int pk_costmodel_grad(int device, const float *params, const float *X, const float *t, int64_t n, float *grad,
                      float *loss);

/* One Adam step of the device kernel on host arrays (params, m, v updated in
 * place; step >= 1 is the step number used for bias correction). */
int pk_costmodel_adam_step(int device, float *params, const float *grad, float *m, float *v, int64_t step, float lr);

/* Parameter export (*n = 5121; out may be NULL to query), text save/load
 * (the file carries the standardisation, the machine and the element type
 * it was trained on; a file without a dtype line is float32), release, and
 * the machine fingerprint string. */
int pk_costmodel_params(const pk_costmodel *cm, float *out, int cap, int *n);
int pk_costmodel_save(const pk_costmodel *cm, const char *path);
int pk_costmodel_load(const char *path, pk_costmodel **out);
void pk_costmodel_free(pk_costmodel *cm);
const char *pk_costmodel_machine(const pk_costmodel *cm);

/* The element type whose timings the model was trained on (a pk_dtype;
 * pk_costmodel_train leaves it PK_F32, the trainer sets it from its data):
 * LEARNED selections use a model only for that type.  Errors:
 * PK_ERR_INVALID_ARG (null), PK_ERR_UNSUPPORTED_DTYPE. */
int pk_costmodel_dtype(const pk_costmodel *cm);
int pk_costmodel_set_dtype(pk_costmodel *cm, pk_dtype dtype);

/* Gives the table a copy of the model for PK_POLICY_LEARNED on the model's
 * element type, replacing the table's model for that type (NULL removes
 * every model).  A model whose machine differs from the table's is refused
 * (PK_ERR_COST_MODEL).  The LEARNED policy orders the feasible candidates by
 * predicted time; when the best two differ by less than the table's margin
 * (5 % unless set with pk_case_table_set_learned_margin), every candidate
 * predicted within that margin of the best is timed (as pk_measure does) and
 * the fastest kept; for a type with no model it returns the CASE pick with
 * PK_ERR_COST_MODEL.  Not to be called while other threads select on the
 * same table. */
int pk_case_table_set_costmodel(pk_table *tbl, const pk_costmodel *cm);

/* The LEARNED policy's measurement margin, a fraction in [0, 1] (default
 * 0.05; 0 never measures: the model's own pick).  Forgets the table's cached
 * LEARNED picks.  Errors: PK_ERR_INVALID_ARG.  Not to be called while other
 * threads select on the same table. */
int pk_case_table_set_learned_margin(pk_table *tbl, double margin);

/* LEARNED selections made on the table and how many fell back to timing. */
int pk_case_table_learned_stats(const pk_table *tbl, int64_t *selections, int64_t *fallbacks);
/* Candidates timed by those fallbacks, in total. */
int pk_case_table_learned_measured(const pk_table *tbl, int64_t *candidates);

/* Library version string. */
const char *pk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PK_H */
