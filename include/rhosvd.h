/*
 * rhosvd.h — C ABI of the MI355X (gfx950) randomized HOSVD library.
 *
 * The library computes a Tucker decomposition [[G; U_1, ..., U_N]] of a dense
 * tensor X with the random-projection HOSVD (Algorithm 6 of Ahmadi-Asl et al.,
 * "Randomized Algorithms for Computation of Tucker Decomposition and Higher
 * Order SVD (HOSVD)") or its sequentially truncated variant R-STHOSVD
 * (Algorithm 8, which applies the basic randomized SVD of Algorithm 1 to the
 * current n-unfolding for each mode in turn).  Inputs follow the problem
 * statement of those algorithms: a tensor, a target multilinear rank
 * (R_1..R_N), an oversampling p and a power-iteration count q (Algorithm 1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Layout.  Tensors are dense and first-index-fastest: element
 *   (i_1, ..., i_N) (0-based) lives at offset i_1 + I_1 (i_2 + I_2 (i_3 + ...)).
 *   With this layout the n-unfolding of Section 2 (column index
 *   j = sum_{k != n} i_k J_k, J_k = prod_{m<k, m!=n} I_m) is a strided view:
 *   element (i_n, j) with j = l + L t sits at l + L (i_n + I_n t), where
 *   L = prod_{m<n} I_m.  Matrices are column-major.
 * - Memory.  `data`, `core`, `factors[n]`, `report`, `workspace` and every
 *   buffer named "device" are device pointers on the context's device; the
 *   caller allocates and owns them.  Arrays named "host" are read during the
 *   call only.  The library never allocates device memory except inside
 *   rhosvd_create (nothing) — all scratch comes from the caller's workspace.
 * - Streams.  `stream` is a hipStream_t passed as void*; NULL is the default
 *   stream.  Every compute call only *enqueues* work and returns; outputs are
 *   valid once the stream has been synchronised.
 * - Errors.  Every argument is validated before anything is enqueued; a
 *   rejected call returns RHOSVD_EINVAL (or RHOSVD_EUNSUPPORTED for a valid
 *   problem outside the implemented limits) and has no side effects.  A HIP
 *   failure returns RHOSVD_EHIP; rhosvd_last_hip_error() gives the code.
 *   Numerical warnings are reported asynchronously in rhosvd_report.flags.
 *   No call throws or aborts.
 * - Omega.  The Gaussian test matrices are generated in the kernels from
 *   Philox4x32-10 (Salmon et al., SC'11): entry (c, k) of the J x K matrix of
 *   mode n has linear index e = k J + c, counter (e>>2 low, e>>2 high, n, tag),
 *   key (seed low, seed high), output word e & 3, uniform
 *   u = ((x >> 9) + 0.5) 2^-23 and Box-Muller on word pairs (0,1), (2,3).
 *   tag = 1 for RP-HOSVD, 2 for R-STHOSVD.  Row c multiplies the unfolding
 *   column whose position in the cyclic order of the other modes
 *   (i_{n+1}, ..., i_N, i_1, ..., i_{n-1}, first fastest) is c: for the
 *   column j = l + L t above (T = J / L), c = t + T l.
 */
#ifndef RHOSVD_H
#define RHOSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RHOSVD_MAX_ORDER 16
#define RHOSVD_MAX_K 128      /* size of the per-mode sigma rows of rhosvd_report */
#define RHOSVD_MAX_SKETCH 64  /* largest sketch width K_n = min(R_n + p, I_n, J_n) the
                                 kernels take; larger problems return RHOSVD_EUNSUPPORTED */

typedef enum {
    RHOSVD_OK = 0,
    RHOSVD_EINVAL = 1,        /* invalid argument; nothing was enqueued */
    RHOSVD_ENOMEM = 2,        /* workspace smaller than rhosvd_workspace_size */
    RHOSVD_EHIP = 3,          /* a HIP runtime call failed */
    RHOSVD_ENUMERIC = 4,      /* reserved */
    RHOSVD_EBUSY = 5,         /* reserved */
    RHOSVD_EUNSUPPORTED = 6,  /* valid problem beyond the implemented limits */
    RHOSVD_ESCRATCH = 7       /* rhosvd_decompose_noalloc: the problem needs more than
                                 RHOSVD_NOALLOC_SCRATCH_BYTES of scratch; nothing enqueued */
} rhosvd_status;

/* Size of the fixed per-device scratch of rhosvd_decompose_noalloc. */
#define RHOSVD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

enum { RHOSVD_F32 = 0, RHOSVD_F64 = 1 };                     /* tensor dtypes */
/* Algorithms: RP-HOSVD (Algorithm 6), R-STHOSVD (Algorithm 8 with Algorithm
 * 1 per mode), RP-HOOI (Algorithm 7: Q_n from the orthonormalised
 * Gaussian start (Omega stream tag 5, mode n, I_n x R_n), then
 * params.power_iters sweeps of S = X x_{p != n} Q_p^T, W = S_(n) Omega
 * (tag 6, counter mode word s N + n), Q_n = QR(W); oversample must be 0;
 * the core X x_n Q_n^T with canonical factor signs) and R-PET (Algorithm 9:
 * the factor sketches Y_n = X_(n) Omega_n of RP-HOSVD (tag 1) with
 * Q_n = QR(Y_n), the core sketch H = X x_1 Omt_1^T ... x_N Omt_N^T with
 * Omt_n Gaussian I_n x S_n, S_n = min(2 K_n + 1, I_n) (tag 3, mode n), the
 * core recovered as H x_n pinv(Omt_n^T Q_n) for every n (eq. Onepass2) and
 * truncated to R_n by a small THOSVD as in RP-HOSVD; power_iters must be 0).
 * R-PET reads X twice (once for all Y_n, once for the first product of H)
 * and, as its core is not X x_n U_n^T, always reports the explicit residual
 * (RHOSVD_FLAG_E_EXPLICIT), one more pass. */
enum { RHOSVD_RP_HOSVD = 0, RHOSVD_R_STHOSVD = 1, RHOSVD_RP_HOOI = 2, RHOSVD_R_PET = 3 };
/* Precision of the streaming contractions (inputs of the matrix cores);
 * accumulation is FP32 (FP64 for RHOSVD_PREC_F64); Gram matrices, Cholesky
 * and eigen-decompositions are always FP64.
 *   RHOSVD_PREC_BF16     sketch on bf16 inputs; power step, projection and
 *                        truncation on split (hi + lo) bf16 operands
 *   RHOSVD_PREC_FP8E4M3  the same, with the sketch of contiguous unfoldings
 *                        on OCP e4m3 inputs (each 32-column block scaled by a
 *                        power of two; strided unfoldings sketch in bf16);
 *                        the split-bf16 power step wins the accuracy back */
enum { RHOSVD_PREC_F64 = 0, RHOSVD_PREC_F32 = 1, RHOSVD_PREC_BF16 = 2, RHOSVD_PREC_FP8E4M3 = 3 };

/* report.flags bits (warnings, set on the device) */
#define RHOSVD_FLAG_K_CAPPED     0x1u  /* some K_n < R_n + p (capped by I_n or J_n) */
#define RHOSVD_FLAG_CQR_SHIFTED  0x2u  /* a Gram matrix needed the shifted Cholesky */
#define RHOSVD_FLAG_EVD_NOCONV   0x4u  /* an eigen-decomposition failed its check: residual
                                          norm(T z - lambda z) > 1e-10 norm(T) or
                                          |z_i^T z_j - delta_ij| > 1e-10 on the tridiagonal T */
#define RHOSVD_FLAG_QR_HOUSEHOLDER 0x8u /* CholeskyQR broke down even with the shift (Y numerically
                                           rank deficient); that basis came from Householder QR */
#define RHOSVD_FLAG_E_EXPLICIT   0x10u /* report.resid2 holds the explicit residual (see
                                          RHOSVD_OPT_EXPLICIT_ERROR) */

/* params.flags bits; a call with any other bit set is rejected (EINVAL) */
#define RHOSVD_OPT_NONE 0u
/* Compute the explicit residual ||X - G x_1 U_1 ... x_N U_N||_F^2 on the GPU
 * (Section 8, eq. Relativeerror) in one more pass over X with FP64
 * accumulation, into report.resid2 (flag RHOSVD_FLAG_E_EXPLICIT).  The pass
 * also runs without this bit whenever the identity-based E of Section 5.1,
 * sqrt(||X||^2 - ||G||^2) / ||X||, comes out below 1e-2: that form cancels
 * catastrophically for small errors (FP64 resolves it only down to ~1e-8).
 * The decision is taken on the device; the workspace always has room. */
#define RHOSVD_OPT_EXPLICIT_ERROR 0x1u
/* Sketch with the structured test matrix of Section 5.1 instead of the dense
 * Gaussian one (the memory-efficient form W = X x_{q != n} Omega_q): the
 * Khatri-Rao form that keeps the width K_n, column k of Omega_n being the
 * Kronecker product of the k-th columns of small Gaussian tables Gamma_q
 * (extent of mode q x K_n, q != n; stream (seed, counter mode word n N + q,
 * tag 4)), i.e. the entry for the other modes' indices i_q is
 * prod_q Gamma_q(i_q, k).  sum_q I_q K_n normals per mode instead of J_n K_n.
 * R-STHOSVD and RP-HOSVD (EINVAL with the other algorithms); also in
 * rhosvd_decompose_adaptive.  RP-HOSVD then sketches mode by mode (the
 * single-pass sketch of every mode generates the Gaussian stream only). */
#define RHOSVD_OPT_KR_SKETCH 0x2u

/* Context options (rhosvd_set_option). */
#define RHOSVD_OPTION_KERNELS 1   /* which streaming-kernel families may run: */
#define RHOSVD_KERNELS_AUTO   0   /*   the fastest that takes each shape (default) */
#define RHOSVD_KERNELS_TILED  1   /*   only the workgroup-tiled FP32/FP64 kernels (the general
                                       fallback; every precision then computes in FP32/FP64) */

typedef struct rhosvd_ctx rhosvd_ctx;

typedef struct {
    int32_t order;            /* N, 2..16 */
    const int64_t* dims;      /* host, N extents, each >= 1 */
    int32_t dtype;            /* RHOSVD_F32 or RHOSVD_F64 */
    const void* data;         /* device, prod(dims) elements, first-index-fastest */
} rhosvd_tensor;

typedef struct {
    int32_t algo;             /* RHOSVD_RP_HOSVD or RHOSVD_R_STHOSVD */
    const int32_t* ranks;     /* host, N target ranks, 1 <= R_n <= I_n */
    int32_t oversample;       /* p >= 0; K_n = min(R_n + p, I_n, J_n) */
    int32_t power_iters;      /* q, 0..8 (RP-HOOI: the number of sweeps) */
    uint64_t seed;            /* Omega key */
    const int32_t* mode_order;/* host permutation of 0..N-1 or NULL (ascending); R-STHOSVD only */
    int32_t precision;        /* RHOSVD_PREC_*; F64 requires F64 data */
    uint32_t flags;           /* RHOSVD_OPT_* bits */
} rhosvd_params;

/* Written by the device at the end of rhosvd_decompose (stream order). */
typedef struct {
    double norm_x2;           /* ||X||_F^2, FP64 accumulation */
    double norm_core2;        /* ||G||_F^2 */
    int32_t order;
    int32_t k_used[RHOSVD_MAX_ORDER];
    uint32_t flags;           /* RHOSVD_FLAG_* */
    double sigma[RHOSVD_MAX_ORDER][RHOSVD_MAX_K]; /* per mode, R_n leading singular values, descending */
    double resid2;            /* ||X - G x_1 U_1 ... x_N U_N||_F^2 when flags has
                                 RHOSVD_FLAG_E_EXPLICIT, else 0 */
} rhosvd_report;

typedef struct {
    void* core;               /* device, R_1 x ... x R_N, first-index-fastest, dtype of X */
    void* const* factors;     /* host array of N device pointers: U_n, I_n x R_n column-major, dtype of X */
    void* report;             /* device, sizeof(rhosvd_report) bytes, or NULL */
} rhosvd_output;

/* Human-readable name of a status code (static string). */
const char* rhosvd_status_string(int32_t status);

/* HIP error code of the most recent RHOSVD_EHIP on this thread (0 if none). */
int32_t rhosvd_last_hip_error(void);

/* Create a context bound to HIP device `device` (records its CU count and
 * limits; allocates no device memory).  EINVAL for a NULL out-pointer or a
 * device index out of range, EHIP if the runtime fails. */
int32_t rhosvd_create(rhosvd_ctx** ctx, int32_t device);
void rhosvd_destroy(rhosvd_ctx* ctx);

/* Set a context option (RHOSVD_OPTION_*) for the calls made with this context
 * afterwards.  EINVAL for a NULL context, an unknown option or a value outside
 * the option's set.  With RHOSVD_KERNELS_TILED a decomposition may need more
 * workspace than rhosvd_workspace_size reports (it then returns ENOMEM). */
int32_t rhosvd_set_option(rhosvd_ctx* ctx, int32_t option, int64_t value);

/* Bytes of device workspace rhosvd_decompose needs for this problem.
 * Pure host computation (no HIP call); EINVAL/EUNSUPPORTED as for decompose. */
int32_t rhosvd_workspace_size(const rhosvd_tensor* x, const rhosvd_params* p, size_t* bytes);

/* Enqueue the whole decomposition on `stream` (Algorithm 6 or 8, every step
 * on the GPU).  X is read only.  Outputs: core, factors, optional report.
 * The workspace must hold at least rhosvd_workspace_size bytes (ENOMEM
 * otherwise) and be 256-byte aligned; it must not be reused by other work
 * until the stream has passed this call. */
int32_t rhosvd_decompose(rhosvd_ctx* ctx, const rhosvd_tensor* x, const rhosvd_params* p,
                         void* workspace, size_t ws_bytes, const rhosvd_output* out,
                         void* stream);

/* rhosvd_decompose without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The call itself allocates nothing (no
 * hipMalloc / hipFree, no host heap): its scratch is a fixed array of
 * RHOSVD_NOALLOC_SCRATCH_BYTES (64 MiB) per device, which the library holds
 * from the first rhosvd_create on that device until the process ends.  A
 * problem whose rhosvd_workspace_size exceeds it returns RHOSVD_ESCRATCH
 * before anything is enqueued.  The caller still provides X, the core, the
 * factors and the report.  Every call on one device shares that device's
 * scratch and nothing in it needs clearing between calls (each call
 * initialises what it reads); calls that may overlap on one device (other
 * streams, other threads, other contexts) race on it and must be ordered by
 * the caller.  Results are identical to rhosvd_decompose's. */
int32_t rhosvd_decompose_noalloc(rhosvd_ctx* ctx, const rhosvd_tensor* x,
                                 const rhosvd_params* p, const rhosvd_output* out,
                                 void* stream);

/* ---- Fixed-precision R-STHOSVD (Section 5.1 with the per-mode split of the
 * tolerance of Algorithm 4; problem DT1 of Section 4) ----
 *
 * The ranks come from a tolerance eps instead of being given.  Modes run in
 * ascending order; mode n sketches the current tensor S with
 * K_n = min(kmax, I_n, J_n) columns (Omega tag 2, as R-STHOSVD), applies q
 * power steps, forms B = Q^T S_(n) and the eigenpairs of B B^T, and keeps the
 * smallest R_n whose residual ||S||^2 - sum_{i <= R_n} sigma_i^2 (the part of
 * S outside span(Q) plus the discarded spectrum of B) is at most
 * eps^2 ||X||^2 / N; when no R <= K_n reaches it, R_n = K_n and the mode is
 * reported unmet.  Then S <- S x_n U_n^T with U_n = Q Ubar[:, :R_n].
 * ||S||^2 is accumulated in FP64 in the sketch pass and the sigma_i come from
 * the FP64 eigen-decomposition of the Gram, so the residual carries the
 * Gram's accumulation error (about 1e-7 ||S||^2 with FP32 inputs, 1e-5 with
 * split-bf16 operands): tolerances well above it are decided reliably.
 *
 * The rank choice reads the eigenvalues on the host: the call synchronises
 * `stream` once per mode and returns when the whole decomposition is done.
 * Capacities: out->factors[n] holds I_n x min(kmax, I_n) elements and
 * out->core prod_n min(kmax, I_n); on return ranks_out[n] (host, N entries)
 * = R_n, U_n is the leading I_n x R_n column-major block of factors[n] and
 * the core the leading R_1 x ... x R_N elements (first-index-fastest).
 * met_out[n] (host, optional) = 1 when mode n met its share.  The report
 * holds sigma[n][0 .. R_n), k_used = K_n and, as rhosvd_decompose, the norms
 * and the explicit residual when requested or when E < 1e-2.
 * Errors as rhosvd_decompose; EINVAL also for eps <= 0 or kmax outside
 * 1..RHOSVD_MAX_SKETCH. */
typedef struct {
    double eps;               /* target relative error, > 0 */
    int32_t kmax;             /* largest sketch width per mode, 1..RHOSVD_MAX_SKETCH */
    int32_t power_iters;      /* q, 0..8 */
    uint64_t seed;            /* Omega key */
    int32_t precision;        /* RHOSVD_PREC_*; F64 requires F64 data */
    uint32_t flags;           /* RHOSVD_OPT_* bits */
} rhosvd_adaptive_params;

/* Workspace bytes of rhosvd_decompose_adaptive (every R_n = K_n bounds it). */
int32_t rhosvd_adaptive_workspace_size(const rhosvd_tensor* x, const rhosvd_adaptive_params* p,
                                       size_t* bytes);
int32_t rhosvd_decompose_adaptive(rhosvd_ctx* ctx, const rhosvd_tensor* x,
                                  const rhosvd_adaptive_params* p, void* workspace,
                                  size_t ws_bytes, const rhosvd_output* out, int32_t* ranks_out,
                                  int32_t* met_out, void* stream);

/* ---- Batched decomposition: many small tensors in one graph launch ----
 *
 * R-STHOSVD (Algorithm 8 with Algorithm 1 per mode) of `count` independent
 * tensors.  Every step of every item runs inside one launch per step for the
 * whole batch (device tables of jobs; the QR and EVD launches are split by
 * the kernel template their K needs), and rhosvd_batch_run captures that
 * sequence into a HIP graph once and replays it.
 * Limits (else RHOSVD_EUNSUPPORTED, nothing allocated): every item
 * RHOSVD_R_STHOSVD in the natural mode order, without
 * RHOSVD_OPT_EXPLICIT_ERROR; one order N and one dtype for the batch; every
 * mode I_n <= 256 and K_n <= RHOSVD_MAX_SKETCH.  Dims, ranks, p, q, seed and
 * precision may differ per item.  Up to 16 workgroups per item and pass
 * (12 on the column and truncation kernels, each with at least 16 column
 * blocks); the items of one kernel instantiation share a launch, the largest
 * first.  The sketch, power
 * step and projection of a bf16-path item (RHOSVD_PREC_BF16, and
 * RHOSVD_PREC_FP8E4M3 with a bf16 sketch) run on the column kernels (32
 * columns per wave), of an RHOSVD_PREC_F32 item on the wave kernels (16
 * columns per wave) when its shape fits them, else, as do FP64 items, on
 * the workgroup-tiled kernels; every truncation runs on the rotated
 * truncation kernel (K_n <= 64, 32 for FP64) or else with the passes.  An
 * item's result depends only on its own problem and on the context's tuned
 * tile parameters, so it is bitwise the same alone (a batch of one) and in
 * any mix.  The reports
 * hold the identity-based E of Section 5.1 only (no explicit residual pass):
 * with FP32 data it cannot resolve errors below about 1e-3.
 *
 * The context's tuner picks the tile width and the tiles per workgroup by
 * timing the candidates on the first batch bound with autotune != 0; the
 * choice is kept in the context for all later batches.
 */
typedef struct rhosvd_batch rhosvd_batch;

/* Validate and plan the batch (host only).  x, p, out: arrays of `count`;
 * the pointers in them (data, core, factors, report) are recorded and must
 * stay valid while the batch is used.  *ws_bytes receives the workspace size. */
int32_t rhosvd_batch_create(rhosvd_ctx* ctx, int32_t count, const rhosvd_tensor* x,
                            const rhosvd_params* p, const rhosvd_output* out,
                            rhosvd_batch** batch, size_t* ws_bytes);

/* Bind the workspace (device, 256-byte aligned, at least *ws_bytes): runs
 * the tuner on `stream` when asked and the context has no choice yet, then
 * uploads the job tables into the workspace (a synchronous copy). */
int32_t rhosvd_batch_bind(rhosvd_batch* batch, void* workspace, size_t ws_bytes,
                          int32_t autotune, void* stream);

/* Enqueue the whole batch on `stream`.  use_graph != 0 and a non-null
 * stream: the first call captures the launch sequence into a HIP graph,
 * every call launches that graph (one launch); the launches of one step that
 * serve different kernel instantiations (disjoint items) are parallel
 * branches of the graph, captured through side streams of default priority
 * that the batch creates on that first call and keeps.  Otherwise the
 * launches are enqueued directly, one after another.  Inputs and outputs are
 * the recorded ones. */
int32_t rhosvd_batch_run(rhosvd_batch* batch, int32_t use_graph, void* stream);

/* Number of kernel launches in one run of the batch (0 before binding). */
int32_t rhosvd_batch_launches(const rhosvd_batch* batch);

void rhosvd_batch_destroy(rhosvd_batch* batch);

/* ---- Serving: a continuous-batching request loop ----
 *
 * Decompositions submitted at any time queue in arrival order; a scheduler
 * thread admits them while one of `max_slots` slots (HIP streams of default
 * priority) is free and the request's workspace (rhosvd_workspace_size) fits
 * in the free part of the caller's device pool (first fit; the oldest
 * `lookahead` = 8 waiting requests are scanned for one that fits), enqueues
 * the whole decomposition on the slot's stream and frees slot and memory as
 * soon as it completes.  Requests that arrive while others run are admitted
 * as slots and memory free up, and their kernels overlap on the device.  A
 * request computes exactly what rhosvd_decompose computes for it alone.
 * Inputs stay on the device: X and the outputs are the caller's buffers,
 * which must stay valid until the request is done. */
typedef struct rhosvd_server rhosvd_server;
enum { RHOSVD_REQ_QUEUED = 0, RHOSVD_REQ_RUNNING = 1, RHOSVD_REQ_DONE = 2 };

/* pool: device, 256-byte aligned, pool_bytes (the HBM budget of the
 * workspaces); 1 <= max_slots <= 64.  Starts the scheduler thread. */
int32_t rhosvd_server_create(rhosvd_ctx* ctx, int32_t device, void* pool, size_t pool_bytes,
                             int32_t max_slots, rhosvd_server** server);

/* Queue one decomposition (descriptors are copied; mode_order must be NULL).
 * Validated at once: EINVAL / EUNSUPPORTED as rhosvd_decompose, ENOMEM when
 * its workspace exceeds the whole pool.  *ticket identifies it. */
int32_t rhosvd_server_submit(rhosvd_server* server, const rhosvd_tensor* x,
                             const rhosvd_params* p, const rhosvd_output* out, uint64_t* ticket);

/* State of a request (RHOSVD_REQ_*); times_ms (optional, 3 doubles): submit,
 * start and completion times on the host's steady clock (ms).  Returns the
 * request's status once it is done (RHOSVD_OK before), EINVAL for an
 * unknown ticket. */
int32_t rhosvd_server_poll(rhosvd_server* server, uint64_t ticket, int32_t* state,
                           double* times_ms);

/* Forget a completed request (its ticket becomes unknown). */
int32_t rhosvd_server_release(rhosvd_server* server, uint64_t ticket);

/* Block until no request is waiting or running. */
int32_t rhosvd_server_drain(rhosvd_server* server);

/* Finish every queued request, stop the thread, free the streams. */
void rhosvd_server_destroy(rhosvd_server* server);

/* Relative error E = ||X - Xhat|| / ||X|| (Section 8, eq. Relativeerror)
 * from a host copy of the report: sqrt(resid2 / ||X||^2) when the explicit
 * residual was computed (RHOSVD_FLAG_E_EXPLICIT), else the orthogonal-
 * projection identity of Section 5.1, sqrt(max(0, ||X||^2 - ||G||^2)) / ||X||.
 * NaN when ||X|| = 0. */
double rhosvd_report_rel_error(const rhosvd_report* r);

/* ---- Step-level entry points (one hot-path step each; used by the per-step
 * parity tests and available to callers that compose their own pipeline).
 * The tensor view (L, I, T) is the n-unfolding of Section 2: element (i, j)
 * with j = l + L t at src[l + L (i + I t)], J = L T columns.  dtype selects
 * float (RHOSVD_F32) or double (RHOSVD_F64) for src and outputs. ---- */

/* Fill out (J x K column-major, dtype) with Omega of (seed, mode, tag), rows
 * in the generator order c.  Test kernel for the in-kernel generator (Algorithm 1 step 1). */
int32_t rhosvd_omega_fill(rhosvd_ctx* ctx, uint64_t seed, int32_t mode, int32_t tag,
                          int64_t J, int32_t K, int32_t dtype, void* out, void* stream);

/* Sketch Y = S_(n) Omega (Algorithm 1 step 2 with q = 0; Algorithm 6 step 3).
 * y: device, I x K column-major, double.  If norm2 != NULL it receives
 * ||S||^2 (device double).  Workspace: rhosvd_step_workspace_size. */
int32_t rhosvd_sketch(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                      int64_t L, int64_t I, int64_t T, int32_t K, uint64_t seed,
                      int32_t mode, int32_t tag, double* y, double* norm2,
                      void* workspace, size_t ws_bytes, void* stream);

/* The same sketch with the structured test matrix of RHOSVD_OPT_KR_SKETCH
 * (Section 5.1): the view's column j = l + L t split in mixed radix over
 * ext[0 .. nq) (fastest first), Omega(j, k) = prod_q tabs[q](i_q, k), each
 * tabs[q] a device ext[q] x K column-major table in src's dtype; prod ext = J
 * (else EINVAL), 1 <= nq <= 15.  Test entry of the structured kernels. */
int32_t rhosvd_sketch_kr(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                         int64_t L, int64_t I, int64_t T, int32_t K, const void* const* tabs,
                         const int64_t* ext, int32_t nq, double* y, double* norm2,
                         void* workspace, size_t ws_bytes, void* stream);

/* Sketch of every mode from one read of X (Algorithm 6 step 3; Section 5.1:
 * no unfolding is formed): Y_n = X_(n) Omega_n for n = 0..N-1, Omega_n the
 * matrix of (seed, mode n, tag) with K[n] columns and cyclic rows (see
 * Omega above).  src: device, prod(dims) elements of dtype, first-index-
 * fastest.  y: device doubles, sum_n dims[n] K[n]; Y_n starts at offset
 * sum_{m<n} dims[m] K[m] and is dims[n] x K[n] column-major.  norm2
 * (optional device double) receives ||X||^2.  Arithmetic in the tensor's
 * dtype (FP32 data: FP32 products and accumulation per workgroup, FP64 sum
 * over workgroups).  EUNSUPPORTED when sum_n dims[n] K[n] does not fit the
 * workgroup's LDS (about 30000 FP32 or 15000 FP64 entries) or a K[n] >
 * RHOSVD_MAX_SKETCH.  Workspace: rhosvd_sketch_all_workspace_size. */
int32_t rhosvd_sketch_all(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t order,
                          const int64_t* dims, const int32_t* K, uint64_t seed, int32_t tag,
                          double* y, double* norm2, void* workspace, size_t ws_bytes,
                          void* stream);

/* Bytes of workspace rhosvd_sketch_all needs (0 if the problem is invalid or
 * unsupported). */
size_t rhosvd_sketch_all_workspace_size(int32_t order, const int64_t* dims, const int32_t* K,
                                        int32_t dtype);

/* One fused power step Y = S_(n) (S_(n)^T Q) (Algorithm 1 step 2, q > 0).
 * q_in: device, I x K column-major, dtype; y: device, I x K double. */
int32_t rhosvd_power(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                     int64_t L, int64_t I, int64_t T, int32_t K, const void* q_in,
                     double* y, void* workspace, size_t ws_bytes, void* stream);

/* Truncation of R-STHOSVD in the rotated layout (Algorithm 8 step 4 as
 * Ubar_R^T B, Section 4.1): out[r J + j] = sum_k M(k, r) B(k, j)
 * for b = B (K x J column-major: the projection's output for one mode) and
 * m = M (K x R column-major), all device, dtype RHOSVD_F32 or RHOSVD_F64,
 * out R x J row-major (the next mode first).  Always on the dedicated
 * truncation kernel (matrix cores in the data's precision), whatever J:
 * the decompositions use it only where it beats the column kernels.
 * K <= 64 (FP32) or 32 (FP64), else EUNSUPPORTED; 1 <= R <= K, J >= 1,
 * else EINVAL.  Stream order; nothing allocated. */
int32_t rhosvd_truncate_rotated(rhosvd_ctx* ctx, int32_t dtype, const void* b, int32_t K, int64_t J,
                                const void* m, int32_t R, void* out, void* stream);

/* Mode-n product out = S x_n M^T with M (I x Kout column-major, dtype;
 * NULL means the identity, which needs Kout == I),
 * written folded: out[l + L (k + Kout t)].  If gram != NULL it also receives
 * the Kout x Kout matrix B B^T of the (Kout x J) unfolding B of out (device
 * double, column-major) — Algorithm 1 step 4 plus the Gram for step 5.
 * If norm2 != NULL it receives ||out||^2 (device double). */
int32_t rhosvd_ttm(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                   int64_t L, int64_t I, int64_t T, int32_t Kout, const void* m,
                   void* out, double* gram, double* norm2,
                   void* workspace, size_t ws_bytes, void* stream);

/* Orthonormal basis of Y (I x K column-major double, I >= K), the Q of
 * Y = QR with diag(R) >= 0 (Algorithm 1 step 3): for I <= 256 and K <= 64,
 * or I <= 512 and K <= 32, by one FP64 Householder QR in a single workgroup
 * (flags untouched); otherwise
 * by CholeskyQR2 with an FP64 Gram/Cholesky and a shifted first pass when the
 * Gram is not numerically positive definite.  q_out: dtype-typed I x K.
 * work: device scratch of 2 I K doubles whose first I K doubles hold the FP64
 * Q on return.  flags (optional device uint32) gets RHOSVD_FLAG_CQR_SHIFTED
 * or-ed in when CholeskyQR2 shifts. */
int32_t rhosvd_orthonormalize(rhosvd_ctx* ctx, const double* y, int64_t I, int32_t K,
                              int32_t dtype, void* q_out, double* work, uint32_t* flags,
                              void* stream);

/* Symmetric eigen-decomposition C = V diag(lambda) V^T of a K x K matrix
 * (device double, column-major), eigenvalues sorted descending (Algorithm 1
 * step 5 through the Gram of B; the EVD variant of Section 4): FP64
 * Householder tridiagonalisation, bisection on Sturm counts and inverse
 * iteration with Gram-Schmidt inside clusters of close eigenvalues.
 * v: K x K double, lambda: K doubles (device).  flags (optional device
 * uint32) gets RHOSVD_FLAG_EVD_NOCONV or-ed in when the eigenpairs fail the
 * residual / orthogonality check.  1 <= K <= RHOSVD_MAX_SKETCH. */
int32_t rhosvd_sym_evd(rhosvd_ctx* ctx, const double* c, int32_t K, double* v,
                       double* lambda, uint32_t* flags, void* stream);

/* Bytes of workspace the step-level calls need for a view (I, K) with at
 * most J columns. */
size_t rhosvd_step_workspace_size(int64_t I, int32_t K, int64_t J);

#ifdef __cplusplus
}
#endif

#endif /* RHOSVD_H */
