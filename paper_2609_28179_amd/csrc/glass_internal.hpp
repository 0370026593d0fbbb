// glass_internal.hpp -- host-side contract between the C-ABI layer and the
// kernel launchers: placement geometry, LDS budgets and the feasibility rule.
// Both the dispatcher (api.cpp) and the launchers (*.hip) size everything from
// the functions below, so a placement judged feasible is exactly what runs.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/glass.h"

namespace glass {

constexpr int kMaxN = 64;
constexpr int kWave = 64;
constexpr size_t kLdsBudgetBytes = 65536;  // fixed per-workgroup LDS budget
constexpr int kThreadMaxN = 16;            // thread scope: problem in one lane's VGPRs
constexpr int kThreadGemmMaxN = 12;        // thread GEMM holds all of B in VGPRs
constexpr int kStagePassFloats = 8192;     // thread scope: floats staged per LDS pass
constexpr int kSe3Stride = 20;             // thread-scope LDS stride of one 4x4 transform (thread_stride(16))

inline int odd_up(int x) { return x | 1; }

// LDS stride (floats) of one staged thread-scope problem of sz floats.  Odd
// sizes are unpadded: the staging is then a straight 16-byte copy, and lanes
// reading their own problems element by element at an odd stride hit
// distinct banks.  A multiple of 4 gets a stride of 4 x an odd number (sz or
// sz + 4): every problem stays 16-byte aligned, the staging still writes
// whole 16-byte pieces, and lanes reading their problems with 16-byte (or
// 8-byte) accesses hit distinct bank groups.  Other sizes get sz + 1.
constexpr int thread_stride(int sz) {
    return (sz & 1) ? sz : (sz & 3) ? sz + 1 : ((sz >> 2) & 1) ? sz : sz + 4;
}
inline int round4(int x) { return (x + 3) & ~3; }
inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Workgroup size of the workgroup scope: 64 * min(4, ceil(n/16)).
inline int wg_scope_threads(int n) {
    int w = ceil_div(n, 16);
    if (w < 1) w = 1;
    if (w > 4) w = 4;
    return 64 * w;
}

// Problems per LDS staging pass of the thread scope (see thread kernels).
inline int thread_stage_q(int threads, int elems) {
    int s = thread_stride(elems);
    int q = kStagePassFloats / s;
    if (q < 1) q = 1;
    return q < threads ? q : threads;
}

struct Shape {
    glass_op_t op;
    int m, n, k;     // GEMM: C m x n, inner k. GEMV: A m x n. square ops: m=n=k=order
    int nrhs;        // POTRS / POSV
    int trans;       // TRSV: 0 / 1.  GEMM: bit 0 op(A) = A^T, bit 1 op(B) = B^T
};

struct Geometry {
    int scope, pack;
    int threads;           // workgroup size
    int problems_per_wg;
    size_t lds_bytes;      // dynamic LDS per workgroup
    long long grid;        // number of workgroups
};

inline bool gemm_uses_mfma(const Shape& s) {
    int mx = s.m > s.n ? s.m : s.n;
    mx = mx > s.k ? mx : s.k;
    return mx >= 16;
}

// LDS floats of one problem region of the workgroup scope (and of the wave
// scope for GEMV and small-n GEMM): the staged, row-padded problem.
inline size_t region_floats(const Shape& s) {
    const int n = s.n;
    switch (s.op) {
    case GLASS_OP_POTRF:
    case GLASS_OP_TRSV:
        return (size_t)round4(n * odd_up(n)) + kWave;
    case GLASS_OP_POTRS:
    case GLASS_OP_POSV:
        return (size_t)round4(n * odd_up(n)) + (size_t)round4(n * odd_up(s.nrhs)) + kWave;
    case GLASS_OP_GEMV:
        return (size_t)round4(s.m * odd_up(n)) + (size_t)round4(n) + 4 * kWave;  // + partial sums
    case GLASS_OP_GEMM: {
        if (gemm_uses_mfma(s)) return 0;
        // A staged as stored: m x k, or k x m when transposed; B likewise
        const size_t a = (s.trans & 1) ? (size_t)round4(s.k * odd_up(s.m)) : (size_t)round4(s.m * odd_up(s.k));
        const size_t b = (s.trans & 2) ? (size_t)round4(s.n * odd_up(s.k)) : (size_t)round4(s.k * odd_up(s.n));
        return a + b;
    }
    default:
        return 0;
    }
}

inline int bucket8_host(int n) { return ((n + 7) / 8) * 8; }

// LDS floats of one wavefront of the wave scope.  The Cholesky family keeps
// rows in VGPRs and needs only an 8-row chunk buffer for its coalesced
// stores and backward substitution.
constexpr int kGemmStageStride = 68;  // LDS row stride of the staged 16-row output block of the MFMA GEMM

// Orders from kBlkMinN up of POTRF / POSV / POTRS / TRSV run the blocked MFMA
// kernel at wave scope (below, the 16 x 16 tiles would be mostly padding);
// its LDS per wavefront holds one staged 16-row block row of L or four
// 16 x 16 exchange blocks.
constexpr int kBlkMinN = 25;
constexpr int kBlkRegionFloats = 1280;
constexpr int kBlkXS = 20;  // LDS row stride of a 16 x 16 exchange block
// LDS row stride of a staged block row of L: 16 nblk floats and four of padding.
constexpr int blk_row_stride(int nblk) { return 16 * nblk + 4; }
inline int blk_nblk(int n) { return n <= 32 ? 2 : n <= 48 ? 3 : 4; }
// POSV with one right-hand side keeps L_kk^{-1} of every diagonal block but
// the last (16 x 20 floats each) for its backward pass, after the staged
// block row: 896, 1472 and 2048 floats per wavefront for 2, 3 and 4 tiles.
constexpr int blk_posv1_floats(int nblk) { return 16 * blk_row_stride(nblk) + (nblk - 1) * 16 * kBlkXS; }
inline bool blk_posv1_shape(const Shape& s) { return s.op == GLASS_OP_POSV && s.nrhs == 1 && s.n >= kBlkMinN; }
// With one right-hand side (TRSV; POTRS with nrhs = 1) the blocked kernel
// passes only a diagonal block through LDS and reserves 16 x 20 floats per
// wavefront.
constexpr int kBlkSolve1Floats = 320;
inline bool blk_solve1_shape(const Shape& s) {
    return s.n >= kBlkMinN && (s.op == GLASS_OP_TRSV || (s.op == GLASS_OP_POTRS && s.nrhs == 1));
}

// Square GEMV at wave scope keeps A in registers (no LDS) at orders 12 and
// 16 and from 17 up when rows split into whole 16-byte pieces, and at every
// order whose staged regions no longer fit eight wavefronts in the LDS
// budget (from 42 up), so that feasibility stays monotone in the order.
inline bool gemv_uses_dpp(const Shape& s) {
    if (s.op != GLASS_OP_GEMV || s.m != s.n || s.n < 12) return false;
    if (s.n <= 16) return s.n % 4 == 0;
    return s.n % 4 == 0 || 8 * region_floats(s) * sizeof(float) > kLdsBudgetBytes;
}

inline size_t wave_region_floats(const Shape& s) {
    switch (s.op) {
    case GLASS_OP_GEMV:
        return gemv_uses_dpp(s) ? 0 : region_floats(s);
    case GLASS_OP_GEMM:
        // MFMA path: one 16-row block of C staged for full-row stores
        return gemm_uses_mfma(s) ? (size_t)16 * kGemmStageStride : region_floats(s);
    case GLASS_OP_POTRF:
    case GLASS_OP_POTRS:
    case GLASS_OP_POSV:
    case GLASS_OP_TRSV:
        if (blk_solve1_shape(s)) return (size_t)kBlkSolve1Floats;
        if (blk_posv1_shape(s)) return (size_t)blk_posv1_floats(blk_nblk(s.n));
        return s.n >= kBlkMinN ? (size_t)kBlkRegionFloats : (size_t)8 * bucket8_host(s.n);
    case GLASS_OP_POSV_ADJOINT:
        return (size_t)8 * bucket8_host(s.n);
    default:
        return region_floats(s);
    }
}

// Sub-wave scope of the batched Cholesky family (orders <= 32): 64 / SEG
// problems per wavefront, one per SEG-lane segment, SEG = 16 up to order 16
// and 32 above.  Every step of the factorization and the substitutions runs
// once per padded row NB: NB is the order rounded up to a multiple of 4 up
// to 16 and to 24 or 32 above.  LDS per wavefront: one block of L per
// segment, rows padded to NB + 4 floats.
constexpr int kSubwaveMaxN = 32;
constexpr int kSubwaveBlasMaxN = 16;  // GEMM / GEMV at sub-wave scope: m, n, k <= 16, no transposes
inline int subwave_seg(int n) { return n <= 16 ? 16 : 32; }
inline int subwave_nb(int n) { return n <= 16 ? ((n + 3) / 4) * 4 : n <= 24 ? 24 : 32; }
inline size_t subwave_region_floats(int n) {
    const int nb = subwave_nb(n);
    return (size_t)(kWave / subwave_seg(n)) * nb * (nb + 4);
}
inline bool subwave_op(glass_op_t op) {
    return op == GLASS_OP_POTRF || op == GLASS_OP_POSV || op == GLASS_OP_POTRS || op == GLASS_OP_TRSV ||
           op == GLASS_OP_POSV_ADJOINT;
}

// LDS floats of a thread-scope workgroup of `t` lanes.
inline size_t thread_lds_floats(const Shape& s, int t) {
    const int n = s.n;
    const int sz = thread_stride(n * n);
    const size_t pass = (size_t)thread_stage_q(t, n * n) * sz;
    switch (s.op) {
    case GLASS_OP_POTRF:
        return pass;
    case GLASS_OP_POTRS:
    case GLASS_OP_POSV: {
        size_t b = (size_t)t * odd_up(n * s.nrhs);
        return pass > b ? pass : b;
    }
    case GLASS_OP_TRSV: {
        size_t b = (size_t)t * odd_up(n);
        return pass > b ? pass : b;
    }
    case GLASS_OP_GEMV:
        return pass + 2 * (size_t)t * odd_up(n);
    case GLASS_OP_GEMM:
        return (size_t)t * sz;
    case GLASS_OP_SE3_COMPOSE:
        return 2 * (size_t)t * kSe3Stride;
    case GLASS_OP_SE3_INVERSE:
        return (size_t)t * kSe3Stride;
    case GLASS_OP_POSV_ADJOINT:
        return pass + 2 * (size_t)t * odd_up(n * s.nrhs);
    }
    return 0;
}

// The feasibility rule and the launch geometry of a placement.  Returns false
// when the placement cannot run this shape.
inline bool make_geometry(const Shape& s, int scope, int pack, long long batch, Geometry* g) {
    if (pack != 1 && pack != 2 && pack != 4 && pack != 8) return false;
    const bool se3 = s.op == GLASS_OP_SE3_COMPOSE || s.op == GLASS_OP_SE3_INVERSE;
    Geometry out{};
    out.scope = scope;
    out.pack = pack;
    if (scope == GLASS_SCOPE_THREAD) {
        if (!se3) {
            if (s.op == GLASS_OP_GEMM) {
                if (!(s.m == s.n && s.n == s.k) || s.n > kThreadGemmMaxN || s.trans != 0) return false;
            } else if (s.op == GLASS_OP_GEMV) {
                if (s.m != s.n || s.n > kThreadMaxN) return false;
            } else if (s.n > kThreadMaxN) {
                return false;
            }
        }
        out.threads = kWave * pack;
        out.problems_per_wg = out.threads;
        out.lds_bytes = thread_lds_floats(s, out.threads) * sizeof(float);
    } else if (scope == GLASS_SCOPE_WAVE) {
        out.threads = kWave * pack;
        out.problems_per_wg = pack;
        out.lds_bytes = wave_region_floats(s) * pack * sizeof(float);
    } else if (scope == GLASS_SCOPE_SUBWAVE) {
        out.threads = kWave * pack;
        if (s.op == GLASS_OP_GEMM || s.op == GLASS_OP_GEMV) {
            // four problems per wavefront, rows in 16-lane segments
            if (s.m > kSubwaveBlasMaxN || s.n > kSubwaveBlasMaxN || s.k > kSubwaveBlasMaxN || s.trans != 0)
                return false;
            out.problems_per_wg = pack * (kWave / 16);
            out.lds_bytes = 0;
        } else {
            if (!subwave_op(s.op) || s.n > kSubwaveMaxN) return false;
            out.problems_per_wg = pack * (kWave / subwave_seg(s.n));
            out.lds_bytes = subwave_region_floats(s.n) * pack * sizeof(float);
        }
    } else if (scope == GLASS_SCOPE_WORKGROUP) {
        if (s.op == GLASS_OP_POSV_ADJOINT) return false;
        int order = s.n;
        if (s.op == GLASS_OP_GEMM || s.op == GLASS_OP_GEMV) {
            order = s.m > order ? s.m : order;
            if (s.op == GLASS_OP_GEMM) order = s.k > order ? s.k : order;
        }
        out.threads = se3 ? kWave : wg_scope_threads(order);
        out.problems_per_wg = pack;
        out.lds_bytes = region_floats(s) * sizeof(float);
    } else {
        return false;
    }
    if (out.lds_bytes > kLdsBudgetBytes) return false;
    out.grid = batch > 0 ? (batch + out.problems_per_wg - 1) / out.problems_per_wg : 0;
    if (g) *g = out;
    return true;
}

// Kernel launchers (defined in the .hip files).  Each assumes a validated
// shape and a geometry produced by make_geometry for it; returns hipSuccess
// or the launch error as int.
int launch_gemm(const Shape& s, const Geometry& g, int batch, float alpha, const float* A,
                const float* B, float beta, float* C, void* stream);
int launch_gemv(const Shape& s, const Geometry& g, int batch, float alpha, const float* A,
                const float* x, float beta, float* y, void* stream);
int launch_potrf(const Shape& s, const Geometry& g, int batch, float* A, int32_t* info, void* stream);
int launch_potrs(const Shape& s, const Geometry& g, int batch, const float* L, float* B, void* stream);
int launch_posv(const Shape& s, const Geometry& g, int batch, float* A, float* B, int32_t* info,
                void* stream);
int launch_trsv(const Shape& s, const Geometry& g, int batch, const float* L, float* x, void* stream);
// Sub-wave scope of POTRF / POSV / POTRS / TRSV (A is L for the solves; B is
// x for TRSV; info may be NULL), and their blocked wave-scope kernel for
// orders kBlkMinN .. 64 (same arguments).
int launch_chol_blk(const Shape& s, const Geometry& g, int batch, float* A, float* B, int32_t* info,
                    void* stream);
// Sub-wave scope of GEMM (Bx = B, Cy = C) and GEMV (Bx = x, Cy = y).
int launch_blas_subwave(const Shape& s, const Geometry& g, int batch, float alpha, const float* A, const float* Bx,
                        float beta, float* Cy, void* stream);
int launch_chol_subwave(const Shape& s, const Geometry& g, int batch, float* A, float* B, int32_t* info,
                        void* stream);
int launch_se3(const Shape& s, const Geometry& g, int batch, const float* Ta, const float* Tb,
               float* Tout, void* stream);
// Placement (scope) of each of the eight ragged size classes (orders 8k+1 ..
// 8k+8); thread scope is available for class 0 (n <= 8), sub-wave scope
// (GLASS_SCOPE_SUBWAVE: four problems per wavefront for classes 0 and 1, two
// for class 2).
constexpr int kScopeSubwave = GLASS_SCOPE_SUBWAVE;
struct RaggedScopes {
    int32_t s[8];
};
size_t ragged_workspace_bytes(int count);
// No-allocation form of the ragged solve: the largest count it takes, and the
// calling thread's current device's address and size of its static workspace
// (returns hipSuccess or the runtime's error code).
constexpr int kRaggedNoAllocMaxCount = 1 << 20;
int ragged_noalloc_workspace(void** ptr, size_t* bytes);
int launch_posv_ragged(int count, const int32_t* n, const int32_t* nrhs, const int64_t* offA, const int64_t* offB,
                       float* A, float* B, int32_t* info, void* workspace, const RaggedScopes& scopes,
                       void* stream);
// Fused LQR gain (wave scope only): 1 <= nu <= 16, 1 <= nx <= 56, nx + nu <= 64,
// nx <= 48 when nu > 8.  LDS floats of one wavefront.
inline bool riccati_size_ok(int nx, int nu) {
    return nx >= 1 && nu >= 1 && nu <= 16 && nx <= 56 && nx + nu <= 64 && (nu <= 8 || nx <= 48);
}
// The matrix-core form of the fused gain (riccati_mfma) serves nx >=
// kRiccatiMfmaMinNx (measured: the LDS-staged form is faster at nx = 4, the
// matrix-core form from nx = 12 at every batch); its LDS per wavefront is one
// 16 x 20 exchange block.
constexpr int kRiccatiMfmaMinNx = 9;
constexpr int kRiccatiMfmaRegionFloats = 16 * 20;
inline bool riccati_uses_mfma(int nx) { return nx >= kRiccatiMfmaMinNx; }
size_t riccati_region_floats(int nx, int nu);
int launch_riccati(int nx, int nu, int batch, int pack, const float* A, const float* B, const float* P,
                   const float* R, float* K, int32_t* info, void* stream);
const char* hip_error_name(int code);
// Streaming bandwidth probe: kind 0 read a, 1 write c, 2 copy a -> c,
// 3 c = a + b; n4 16-byte elements, `blocks` workgroups of 1024 lanes.
int launch_stream_probe(int kind, const float* a, const float* b, float* c, long long n4, int blocks, void* stream);
size_t mlp_num_params(int d);
size_t mlp_backward_workspace_bytes(int N, int d);
int launch_mlp_forward(int N, int d, const float* X, const float* P, float* H1, float* H2, float* Y, void* stream);
int launch_mlp_backward(int N, int d, const float* X, const float* P, const float* H1, const float* H2,
                        const float* Y, const float* T, float* grad, void* workspace, void* stream);
int launch_mlp_adam(int P, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    float bc1, float bc2, void* stream);
int launch_posv_adjoint(const Shape& s, const Geometry& g, int batch, const float* L, const float* X,
                        const float* G, float* dB, float* dA, void* stream);

}  // namespace glass
