/*
 * glass.h -- C-ABI of the MI355X (gfx950) batched small dense linear algebra
 * library: GEMM, GEMV, Cholesky factor / solve, triangular solve and SE(3)
 * compose / inverse at robotics sizes (n <= 64), each with thread-,
 * wavefront- and workgroup-scoped kernels and a measured placement table.
 *
 * Method: GLASS (Sec. III).  Sec. III-A defines the three execution scopes
 * (one problem per thread, per wave -- a 32-lane warp in the paper, a 64-lane
 * wavefront here -- or per block/workgroup), the offline-measured placement
 * table, the bare call that consults it and the advisor that reports it;
 * Sec. III-B lists the operations; Sec. IV-C calls launch packing (problems
 * per workgroup) part of a placement.
 *
 * Common contract of every batched call
 *   - Data: FP32, row-major, batch-contiguous: X[batch][rows][cols], no
 *     leading-dimension argument, no padding between problems.
 *   - Pointers: DEVICE pointers, 4-byte aligned, owned by the caller; the
 *     library allocates nothing and keeps no per-call state.  16-byte aligned
 *     pointers enable wider loads but are not required.
 *   - Sizes: 1 <= n, m, k, nrhs <= 64 (else GLASS_ERR_UNSUPPORTED);
 *     batch == 0 is a no-op returning GLASS_OK; batch < 0 or a required
 *     pointer that is NULL while batch > 0 -> GLASS_ERR_INVALID_VALUE.
 *   - All argument errors are detected on the host before anything is
 *     enqueued: on error nothing runs.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream).  A failed launch returns GLASS_ERR_LAUNCH.
 *   - Numerical failure is never a return code: factorizations report it per
 *     problem in info[] (LAPACK convention, see glass_potrf_batched).
 *   - Placement: `force == NULL` looks the call up in the built-in gfx950
 *     table (the paper's bare call); if the tabulated placement is infeasible
 *     for this exact call (e.g. nrhs or a rectangular GEMM exceeds what that
 *     scope supports) the call takes the first feasible of: the tabulated
 *     scope at pack 1, sub-wave, wavefront, workgroup scope, each at pack 1
 *     (wavefront / pack 1 is feasible for every supported shape).
 *     `force != NULL` runs exactly that
 *     placement (only its `scope` and `pack` fields are read) or returns
 *     GLASS_ERR_INFEASIBLE_PLACEMENT without enqueuing anything.
 *   - Thread safety: stateless apart from a per-process, read-only device
 *     property cache; calls may be made concurrently from several threads.
 *     The one exception is glass_posv_ragged_noalloc, whose calls on one
 *     device share a static workspace and must not overlap in time.
 */
#ifndef GLASS_H_
#define GLASS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GLASS_OK = 0,
    GLASS_ERR_INVALID_VALUE = -1,        /* bad pointer / negative batch / bad enum  */
    GLASS_ERR_UNSUPPORTED = -2,          /* size outside 1..64                       */
    GLASS_ERR_INFEASIBLE_PLACEMENT = -3, /* forced placement cannot run this shape   */
    GLASS_ERR_LAUNCH = -4                /* the HIP runtime rejected the launch      */
} glass_status_t;

typedef enum {
    GLASS_OP_GEMM = 0,
    GLASS_OP_GEMV = 1,
    GLASS_OP_POTRF = 2,
    GLASS_OP_POTRS = 3,
    GLASS_OP_POSV = 4,
    GLASS_OP_TRSV = 5,
    GLASS_OP_SE3_COMPOSE = 6,
    GLASS_OP_SE3_INVERSE = 7,
    GLASS_OP_POSV_ADJOINT = 8
} glass_op_t;

/* Execution scope (Sec. III-A). */
typedef enum {
    GLASS_SCOPE_THREAD = 0,    /* one problem per lane                       */
    GLASS_SCOPE_WAVE = 1,      /* one problem per 64-lane wavefront          */
    GLASS_SCOPE_WORKGROUP = 2, /* one problem per workgroup at a time        */
    GLASS_SCOPE_SUBWAVE = 3    /* 64/SEG problems per wavefront, one per
                                  SEG-lane segment: SEG = 16 for n <= 16,
                                  32 for 16 < n <= 32 (POTRF, POTRS, POSV,
                                  TRSV, the POSV adjoint, the ragged
                                  solve); GEMM and GEMV
                                  with m, n, k <= 16 (SEG = 16, no
                                  transposes)                               */
} glass_scope_t;

/* A placement (Sec. III-A, Sec. IV-C).  `pack` P in {1,2,4,8} counts the
 * scope's unit per workgroup:
 *   thread    : workgroup of 64P lanes, 64P problems per workgroup;
 *   wave      : workgroup of P wavefronts, P problems (one per wavefront);
 *   workgroup : workgroup of T(n) = 64*min(4, ceil(n/16)) lanes that solves
 *               P problems one after the other;
 *   subwave   : workgroup of P wavefronts, P*64/SEG problems.
 * wg_threads and problems_per_wg are outputs (what a launch uses); as input
 * only scope and pack are read. */
typedef struct {
    int32_t scope;
    int32_t pack;
    int32_t wg_threads;
    int32_t problems_per_wg;
} glass_placement_t;

/* C = alpha * A B + beta * C  (Sec. III-B, BLAS L3).
 * A [batch][m][k], B [batch][k][n], C [batch][m][n].  beta == 0: C is not
 * read (NaN in C does not propagate).  C must not overlap A or B.
 * Thread scope requires m == n == k <= 12; sub-wave scope m, n, k <= 16; wave
 * and workgroup scope use FP32 MFMA (v_mfma_f32_16x16x4_f32) when
 * max(m, n, k) >= 16. */
glass_status_t glass_gemm_batched(int m, int n, int k, int batch, float alpha,
                                  const float* A, const float* B, float beta,
                                  float* C, const glass_placement_t* force,
                                  void* stream);

/* C = alpha op(A) op(B) + beta C with op(X) = X (trans 0) or X^T (trans 1),
 * the BLAS form (Sec. III-B, BLAS L3).  op(A) is m x k, op(B) is k x n, C is
 * m x n; A is stored row-major m x k (transa = 0) or k x m (transa = 1), B
 * k x n or n x k.  Same ranges, ownership and errors as glass_gemm_batched
 * (which is this call with both flags 0); a flag other than 0 / 1 is
 * GLASS_ERR_INVALID_VALUE.  Transposed operands run at wavefront or
 * workgroup scope (a forced thread placement is GLASS_ERR_INFEASIBLE_PLACEMENT;
 * a table entry naming thread scope falls back to wavefront scope). */
glass_status_t glass_gemm_batched_ex(int transa, int transb, int m, int n, int k, int batch,
                                     float alpha, const float* A, const float* B, float beta,
                                     float* C, const glass_placement_t* force, void* stream);

/* y = alpha * A x + beta * y  (Sec. III-B, BLAS L2).
 * A [batch][m][n], x [batch][n], y [batch][m]; beta == 0: y is not read.
 * y must not overlap A or x.  Thread scope requires m == n <= 16, sub-wave
 * scope m, n <= 16. */
glass_status_t glass_gemv_batched(int m, int n, int batch, float alpha,
                                  const float* A, const float* x, float beta,
                                  float* y, const glass_placement_t* force,
                                  void* stream);

/* Lower Cholesky factorization A = L L^T, in place  (Sec. III-B).
 * A [batch][n][n]: only the lower triangle (i >= j) is read; on return it
 * holds L and the strict upper triangle holds +0.0.
 * info [batch] (device int32, may be NULL): 0 on success, otherwise j+1 for
 * the first column j whose pivot A_jj - sum_k L_jk^2 is not > 0 (zero,
 * negative or NaN); columns >= j of that problem are then unspecified. */
glass_status_t glass_potrf_batched(int n, int batch, float* A, int32_t* info,
                                   const glass_placement_t* force, void* stream);

/* Solve A X = B with a given Cholesky factor, in place  (Sec. III-B).
 * L [batch][n][n] (lower triangle read, non-unit diagonal),
 * B [batch][n][nrhs]: right-hand sides on entry, X = (L L^T)^{-1} B on exit.
 * B must not overlap L. */
glass_status_t glass_potrs_batched(int n, int nrhs, int batch, const float* L,
                                   float* B, const glass_placement_t* force,
                                   void* stream);

/* Factor and solve in one kernel (POSV; Sec. III-A's example call).
 * A is overwritten by L exactly as glass_potrf_batched does, B by the
 * solution; info as for glass_potrf_batched (may be NULL).  Where
 * info[b] != 0 the contents of B[b] are unspecified. */
glass_status_t glass_posv_batched(int n, int nrhs, int batch, float* A,
                                  float* B, int32_t* info,
                                  const glass_placement_t* force, void* stream);

/* Triangular solve, in place  (Sec. III-B).
 * L [batch][n][n] lower triangle read, non-unit diagonal; x [batch][n] holds
 * b on entry and the solution on exit.  trans = 0: L x = b; trans = 1:
 * L^T x = b; any other value -> GLASS_ERR_INVALID_VALUE. */
glass_status_t glass_trsv_batched(int n, int batch, int trans, const float* L,
                                  float* x, const glass_placement_t* force,
                                  void* stream);

/* SE(3) homogeneous transforms  (Sec. III-B).  Each problem is a 4x4
 * row-major [R t; 0 0 0 1]; row 3 of an input is never read and row 3 of
 * the output is written as exactly (0, 0, 0, 1).
 * op = GLASS_OP_SE3_COMPOSE: Tout = Ta Tb (R = Ra Rb, t = Ra tb + ta);
 * op = GLASS_OP_SE3_INVERSE: Tout = [Ra^T, -Ra^T ta] (closed form for a
 * rigid motion; Tb is ignored and may be NULL).  Tout may be exactly Ta or
 * Tb (every problem is fully read before it is written); partial overlap is
 * undefined. */
glass_status_t glass_se3_batched(glass_op_t op, int batch, const float* Ta,
                                 const float* Tb, float* Tout,
                                 const glass_placement_t* force, void* stream);

/* Reverse mode of the Cholesky solve X = A^{-1} B (the differentiation
 * part; derivatives are validated by finite differences, Sec. III-C).
 * Given the factor L [batch][n][n] (lower triangle read, as returned by
 * glass_posv_batched / glass_potrf_batched), the solution X [batch][n][nrhs]
 * and the upstream gradient G = dl/dX [batch][n][nrhs] of a scalar loss l,
 * writes
 *   dB = A^{-1} G                      [batch][n][nrhs]
 *   dA = -(dB X^T + X dB^T) / 2        [batch][n][n], symmetric
 * dA is the gradient with respect to a symmetric A (the factorization reads
 * A as symmetric).  dB may be G exactly (in place); dA must not overlap any
 * other argument.  Scopes: thread (n <= 16), sub-wave (n <= 32) and wave;
 * the workgroup scope is infeasible.  With force == NULL the placement is the table's POTRS entry
 * for (n, batch) when feasible, else wave / pack 1. */
glass_status_t glass_posv_adjoint_batched(int n, int nrhs, int batch, const float* L,
                                          const float* X, const float* G, float* dB,
                                          float* dA, const glass_placement_t* force,
                                          void* stream);

/* Factor-and-solve of a ragged batch: `count` SPD systems of mixed order and
 * right-hand-side count in one launch sequence (problem packing of Sec. IV-C
 * extended to mixed sizes; no host synchronisation, so the call can be
 * captured in a HIP graph): three small planning kernels and one solve
 * launch with a wavefront per work item (the classes of orders above 24
 * first in the item list).  All arrays are DEVICE arrays:
 *   n[count], nrhs[count]  int32, each in 1..64 (a problem outside that range
 *                          gets info = -1 and is not touched);
 *   offA[count], offB[count] int64 element offsets of problem i's A (n x n,
 *                          row-major) in A and of its B (n x nrhs) in B;
 *   A, B                   packed problems, overwritten by L (strict upper
 *                          +0) and by the solutions, as glass_posv_batched;
 *   info[count]            int32 as for glass_potrf_batched (required);
 *   workspace              caller-owned device scratch of at least
 *                          glass_posv_ragged_workspace_size(count) bytes,
 *                          4-byte aligned; its contents on entry are ignored
 *                          and on exit hold the class-sorted permutation of
 *                          the problems (int32 at byte offset
 *                          glass_posv_ragged_perm_offset(count)).
 * Problems are grouped into eight size classes (orders 8k+1 .. 8k+8) by a
 * deterministic stable counting sort on the device, largest class first;
 * class_scope (HOST int32[8] or NULL) picks each class's scope: thread
 * (class 0 only, 64 problems per wavefront), sub-wave (classes 0 and 1: four
 * problems per wavefront, one per 16-lane row; class 2: two, one per 32-lane
 * half) or wave (one problem per wavefront); a scope a class cannot take is GLASS_ERR_INFEASIBLE_PLACEMENT,
 * another value GLASS_ERR_INVALID_VALUE.  NULL takes the measured per-class
 * choice of the built-in ragged table (glass_ragged_table_provenance()).
 * Concurrent calls must not share a workspace. */
glass_status_t glass_posv_ragged(int count, const int32_t* n, const int32_t* nrhs,
                                 const int64_t* offA, const int64_t* offB, float* A,
                                 float* B, int32_t* info, void* workspace,
                                 size_t workspace_bytes, const int32_t* class_scope,
                                 void* stream);

/* glass_posv_ragged without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results, errors and
 * launches as glass_posv_ragged; the workspace is a static device array of
 * the library (about 4 MiB per device, allocated when the library's code
 * object is loaded and held until the process ends), so the call allocates
 * nothing.  count > glass_posv_ragged_noalloc_max_count() (1,048,576) ->
 * GLASS_ERR_UNSUPPORTED, before anything is enqueued.  The calling thread's
 * current device must be the device of `stream`.  Every call on one device
 * shares that device's array: calls on one stream are ordered and safe, but
 * calls that overlap in time on one device (other streams, other threads)
 * race and give undefined results.  The class-sorted permutation is not
 * returned. */
glass_status_t glass_posv_ragged_noalloc(int count, const int32_t* n, const int32_t* nrhs,
                                         const int64_t* offA, const int64_t* offB, float* A,
                                         float* B, int32_t* info, const int32_t* class_scope,
                                         void* stream);

/* The largest count glass_posv_ragged_noalloc accepts. */
int glass_posv_ragged_noalloc_max_count(void);

/* Provenance of the built-in per-class ragged placement table. */
const char* glass_ragged_table_provenance(void);

/* Workspace bytes glass_posv_ragged needs for `count` problems (0 if
 * count < 0), and the byte offset of the permutation inside it. */
size_t glass_posv_ragged_workspace_size(int count);
size_t glass_posv_ragged_perm_offset(int count);

/* Fused LQR feedback gain K = (R + B^T P B)^{-1} B^T P A, one Riccati step
 * (Sec. III-B: a fused composition of GEMM and solve primitives; Sec. IV-E
 * measures it against the chain of separate launches).  Per problem, all
 * row-major and batch-contiguous: A [nx][nx], B [nx][nu], P [nx][nx]
 * (symmetric, read whole), R [nu][nu] (symmetric positive definite, read
 * whole), K [nu][nx] out; info [batch] (int32, may be NULL) receives the
 * Cholesky info of S = R + B^T P B (0, or the 1-based failing pivot; K is
 * unspecified and not written where it is nonzero).  Device pointers owned
 * by the caller; inputs are not modified.  Sizes: 1 <= nu <= 16,
 * 1 <= nx <= 56, nx + nu <= 64 and nx <= 48 when nu > 8, else
 * GLASS_ERR_UNSUPPORTED.  Three scopes: wavefront (one problem per 64-lane
 * wavefront, every intermediate in VGPRs / LDS; force->pack sets the problems
 * per workgroup); for nx <= 16 and nu <= 8, sub-wave (four problems per
 * wavefront, one per 16-lane row; force->pack wavefronts per workgroup); and,
 * for nx <= 8 and nu <= 4, thread (one problem per lane, every operand and
 * intermediate in VGPRs; force->pack sets 64 * pack lanes per workgroup).
 * With force NULL: thread scope with one wavefront per workgroup where it
 * runs, else wavefront scope.  The workgroup scope, or a scope outside its
 * sizes, is GLASS_ERR_INFEASIBLE_PLACEMENT. */
glass_status_t glass_riccati_gain_batched(int nx, int nu, int batch, const float* A,
                                          const float* B, const float* P, const float* R,
                                          float* K, int32_t* info,
                                          const glass_placement_t* force, void* stream);

/* 1 if the fused LQR gain can run nx, nu with `pack` problems per workgroup
 * within the LDS budget, 0 if not, or a negative status for bad arguments.
 * The wavefront scope's rule of glass_riccati_placement_feasible. */
int glass_riccati_feasible(int nx, int nu, int pack);

/* 1 if glass_riccati_gain_batched accepts force = {scope, pack} for nx, nu,
 * 0 if that placement is infeasible, or a negative status for an invalid
 * scope or pack (GLASS_ERR_INVALID_VALUE) or unsupported sizes
 * (GLASS_ERR_UNSUPPORTED).  Thread scope: nx <= 8 and nu <= 4, any pack;
 * sub-wave scope: nx <= 16 and nu <= 8, any pack; wavefront scope: as
 * glass_riccati_feasible; workgroup scope: 0. */
int glass_riccati_placement_feasible(int nx, int nu, int scope, int pack);

/* Streaming bandwidth probe: the attainable HBM bandwidth of a plain kernel
 * with a given read/write mix, against which the batched kernels' measured
 * bandwidth is read (the evaluation of Sec. IV-A times device kernels on
 * device-resident data; the roofline fractions quote the 8 TB/s spec peak,
 * and these kernels show how much of it each access mix reaches).
 * kind 0: read a (c receives nothing in practice but must hold >= 256
 * floats, so n4 >= 64); 1: write c; 2: copy a -> c; 3: c = a + b (two reads
 * per write, the mix of C = A B).  n4 16-byte elements; a, b, c 16-byte
 * aligned DEVICE pointers (those the kind uses non-NULL); `blocks`
 * workgroups of 1024 lanes (1 .. 2^20), grid-stride.  Bad arguments ->
 * GLASS_ERR_INVALID_VALUE before anything is enqueued. */
glass_status_t glass_stream_probe(int kind, const float* a, const float* b, float* c,
                                  long long n4, int blocks, void* stream);

/* Diagnostics of GLASS_ERR_LAUNCH: the HIP runtime error code of the most
 * recent failed launch made by this library on the calling thread (0 if none;
 * never reset), and the runtime's name for an error code (static string). */
int glass_last_launch_error(void);
const char* glass_hip_error_name(int code);

/* Placement cost model: a 3-layer perceptron d -> 64 -> 64 -> 1 (ReLU) that
 * predicts log run time from placement features, trained by the kernels
 * below (the paper chooses placements by measurement only, Sec. III-A /
 * Sec. IV-A; the model proposes placements for unmeasured shapes and the
 * measured search still decides among its proposals and is the fallback).
 * params: FP32 flat vector of glass_mlp_num_params(d) floats laid out as
 * W1[64][d], b1[64], W2[64][64], b2[64], w3[64], b3.  X [N][d] row-major,
 * y / t [N].  All pointers are DEVICE pointers; 1 <= d <= 32 (else
 * GLASS_ERR_UNSUPPORTED). */
size_t glass_mlp_num_params(int d);

/* y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 per row of X.  H1, H2 [N][64]
 * receive the two hidden activations (needed by the backward pass) or may be
 * NULL. */
glass_status_t glass_mlp_forward(int N, int d, const float* X, const float* params,
                                 float* H1, float* H2, float* y, void* stream);

/* grad = dL/dparams for L = (1/N) sum (y - t)^2, from the forward pass's X,
 * H1, H2, y.  Deterministic: per-block partial sums (in `workspace`, at least
 * glass_mlp_backward_workspace_size(N, d) bytes, 4-byte aligned) are added in
 * a fixed order.  N >= 1. */
size_t glass_mlp_backward_workspace_size(int N, int d);
glass_status_t glass_mlp_backward(int N, int d, const float* X, const float* params,
                                  const float* H1, const float* H2, const float* y,
                                  const float* t, float* grad, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* One Adam step (step >= 1) over P parameters: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, p -= lr (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps). */
glass_status_t glass_mlp_adam(int P, float* params, const float* grad, float* m, float* v,
                              int step, float lr, float beta1, float beta2, float eps,
                              void* stream);

/* The advisor (Sec. III-A): the placement the built-in table gives for
 * (op, n, batch), written to *out (HOST pointer).  Lookup rule: n_key = the
 * smallest tabulated n >= n (n <= 2 maps to the smallest key); batch_key =
 * the tabulated batch nearest in |log2| distance, ties to the smaller; the
 * SE(3) ops ignore n.  n outside 1..64 -> GLASS_ERR_UNSUPPORTED; batch < 1
 * or out == NULL -> GLASS_ERR_INVALID_VALUE.  For GEMM pass n = max(m,n,k). */
glass_status_t glass_query_placement(glass_op_t op, int n, int batch,
                                     glass_placement_t* out);

/* Whether placement (scope, pack) can run a square problem of order n with
 * nrhs right-hand sides (POTRS/POSV; ignored elsewhere).  Returns 1 if
 * feasible, 0 if not, GLASS_ERR_* for bad arguments.  The rule is
 * deterministic and device-independent (a fixed 64 KiB LDS budget per
 * workgroup and per-scope register limits), mirroring Sec. III-A's rule that
 * a body is instantiated only where its size and resources fit. */
int glass_placement_feasible(glass_op_t op, int n, int nrhs, int scope, int pack);

/* Provenance string of the built-in table ("gfx950 / ... / sweep ..."). */
const char* glass_table_provenance(void);

/* Human-readable name of a status code (static storage). */
const char* glass_status_string(glass_status_t s);

#ifdef __cplusplus
}
#endif

#endif /* GLASS_H_ */
