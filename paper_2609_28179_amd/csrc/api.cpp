// api.cpp -- the C-ABI of include/glass.h: host-side argument validation,
// placement resolution (static table, advisor, forced placement) and dispatch
// to the kernel launchers.  Everything before the launch is plain host code
// that touches no HIP API, so every error path runs without a device.
#include <math.h>

#include "glass_internal.hpp"
#include "riccati.hpp"

namespace glass {
namespace {

#include "glass_table_gfx950.inc"
#include "glass_ragged_gfx950.inc"

constexpr int kNumN = sizeof(kTableN) / sizeof(kTableN[0]);
constexpr int kNumB = sizeof(kTableB) / sizeof(kTableB[0]);

inline bool is_se3(glass_op_t op) { return op == GLASS_OP_SE3_COMPOSE || op == GLASS_OP_SE3_INVERSE; }
inline bool size_ok(int v) { return v >= 1 && v <= kMaxN; }

// Smallest tabulated n >= n (n below the first key maps to the first key).
int n_index(int n) {
    for (int i = 0; i < kNumN; ++i)
        if (kTableN[i] >= n) return i;
    return kNumN - 1;
}

// Tabulated batch nearest to `batch` in |log2| distance, ties to the smaller:
// between consecutive keys k1 < b < k2, b is nearer k1 iff b*b <= k1*k2.
int b_index(long long batch) {
    if (batch <= kTableB[0]) return 0;
    for (int i = 0; i + 1 < kNumB; ++i) {
        const long long k1 = kTableB[i], k2 = kTableB[i + 1];
        if (batch == k1) return i;
        if (batch < k2) return batch * batch <= k1 * k2 ? i : i + 1;
    }
    return kNumB - 1;
}

void table_lookup(glass_op_t op, int n, long long batch, int* scope, int* pack) {
    if (op == GLASS_OP_POSV_ADJOINT) op = GLASS_OP_POTRS;  // a POTRS plus an outer-product epilogue
    const int ni = is_se3(op) ? 0 : n_index(n);
    const int bi = b_index(batch);
    *scope = kPlace[(int)op][ni][bi][0];
    *pack = kPlace[(int)op][ni][bi][1];
}

bool valid_force(const glass_placement_t* f) {
    if (!f) return true;
    if (f->scope < GLASS_SCOPE_THREAD || f->scope > GLASS_SCOPE_SUBWAVE) return false;
    return f->pack == 1 || f->pack == 2 || f->pack == 4 || f->pack == 8;
}

// Resolve the placement of a validated call: forced, else the table's
// placement, else (the table is keyed by order and batch only, so nrhs or a
// rectangular GEMM can exceed what its placement supports) the first
// feasible of: the table's scope at pack 1, sub-wave, wavefront, workgroup,
// each at pack 1.  Wavefront / pack 1 runs every supported shape.
glass_status_t resolve(const Shape& s, long long batch, const glass_placement_t* force, Geometry* g) {
    if (force) {
        if (!make_geometry(s, force->scope, force->pack, batch, g)) return GLASS_ERR_INFEASIBLE_PLACEMENT;
        return GLASS_OK;
    }
    int order = s.n;
    if (s.op == GLASS_OP_GEMM || s.op == GLASS_OP_GEMV) {
        order = s.m > order ? s.m : order;
        if (s.op == GLASS_OP_GEMM) order = s.k > order ? s.k : order;
    }
    int scope, pack;
    table_lookup(s.op, order, batch, &scope, &pack);
    if (make_geometry(s, scope, pack, batch, g)) return GLASS_OK;
    if (pack != 1 && make_geometry(s, scope, 1, batch, g)) return GLASS_OK;
    if (make_geometry(s, GLASS_SCOPE_SUBWAVE, 1, batch, g)) return GLASS_OK;
    if (make_geometry(s, GLASS_SCOPE_WAVE, 1, batch, g)) return GLASS_OK;
    if (make_geometry(s, GLASS_SCOPE_WORKGROUP, 1, batch, g)) return GLASS_OK;
    return GLASS_ERR_INFEASIBLE_PLACEMENT;
}

thread_local int t_last_launch_error = 0;

constexpr int kRiccatiDefaultPack = 1;  // problems (wavefronts) per workgroup of the fused LQR gain

inline glass_status_t launched(int err) {
    if (err == 0) return GLASS_OK;
    t_last_launch_error = err;
    return GLASS_ERR_LAUNCH;
}

}  // namespace
}  // namespace glass

using namespace glass;

extern "C" {

glass_status_t glass_gemm_batched(int m, int n, int k, int batch, float alpha, const float* A, const float* B,
                                  float beta, float* C, const glass_placement_t* force, void* stream) {
    return glass_gemm_batched_ex(0, 0, m, n, k, batch, alpha, A, B, beta, C, force, stream);
}

glass_status_t glass_gemm_batched_ex(int transa, int transb, int m, int n, int k, int batch, float alpha,
                                     const float* A, const float* B, float beta, float* C,
                                     const glass_placement_t* force, void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if ((transa != 0 && transa != 1) || (transb != 0 && transb != 1)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(m) || !size_ok(n) || !size_ok(k)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!A || !B || !C) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_GEMM, m, n, k, 1, transa | (transb << 1)};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_gemm(s, g, batch, alpha, A, B, beta, C, stream));
}

glass_status_t glass_gemv_batched(int m, int n, int batch, float alpha, const float* A, const float* x,
                                  float beta, float* y, const glass_placement_t* force, void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(m) || !size_ok(n)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!A || !x || !y) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_GEMV, m, n, n, 1, 0};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_gemv(s, g, batch, alpha, A, x, beta, y, stream));
}

glass_status_t glass_potrf_batched(int n, int batch, float* A, int32_t* info, const glass_placement_t* force,
                                   void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(n)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!A) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_POTRF, n, n, n, 1, 0};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_potrf(s, g, batch, A, info, stream));
}

glass_status_t glass_potrs_batched(int n, int nrhs, int batch, const float* L, float* B,
                                   const glass_placement_t* force, void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(n) || !size_ok(nrhs)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!L || !B) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_POTRS, n, n, n, nrhs, 0};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_potrs(s, g, batch, L, B, stream));
}

glass_status_t glass_posv_batched(int n, int nrhs, int batch, float* A, float* B, int32_t* info,
                                  const glass_placement_t* force, void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(n) || !size_ok(nrhs)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!A || !B) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_POSV, n, n, n, nrhs, 0};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_posv(s, g, batch, A, B, info, stream));
}

glass_status_t glass_trsv_batched(int n, int batch, int trans, const float* L, float* x,
                                  const glass_placement_t* force, void* stream) {
    if (!valid_force(force) || (trans != 0 && trans != 1)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(n)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!L || !x) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_TRSV, n, n, n, 1, trans};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_trsv(s, g, batch, L, x, stream));
}

glass_status_t glass_se3_batched(glass_op_t op, int batch, const float* Ta, const float* Tb, float* Tout,
                                 const glass_placement_t* force, void* stream) {
    if (!valid_force(force) || !is_se3(op)) return GLASS_ERR_INVALID_VALUE;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!Ta || !Tout || (op == GLASS_OP_SE3_COMPOSE && !Tb)) return GLASS_ERR_INVALID_VALUE;
    Shape s{op, 4, 4, 4, 1, 0};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_se3(s, g, batch, Ta, Tb, Tout, stream));
}

glass_status_t glass_posv_adjoint_batched(int n, int nrhs, int batch, const float* L, const float* X,
                                          const float* G, float* dB, float* dA, const glass_placement_t* force,
                                          void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if (!size_ok(n) || !size_ok(nrhs)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!L || !X || !G || !dB || !dA) return GLASS_ERR_INVALID_VALUE;
    Shape s{GLASS_OP_POSV_ADJOINT, n, n, n, nrhs, 0};
    Geometry g;
    glass_status_t st = resolve(s, batch, force, &g);
    if (st != GLASS_OK) return st;
    return launched(launch_posv_adjoint(s, g, batch, L, X, G, dB, dA, stream));
}

size_t glass_posv_ragged_workspace_size(int count) { return count < 0 ? 0 : ragged_workspace_bytes(count); }

size_t glass_posv_ragged_perm_offset(int count) {
    if (count < 0) return 0;
    return ragged_workspace_bytes(count) - sizeof(int32_t) * (size_t)count;
}

glass_status_t glass_posv_ragged(int count, const int32_t* n, const int32_t* nrhs, const int64_t* offA,
                                 const int64_t* offB, float* A, float* B, int32_t* info, void* workspace,
                                 size_t workspace_bytes, const int32_t* class_scope, void* stream) {
    if (count < 0) return GLASS_ERR_INVALID_VALUE;
    RaggedScopes sc{};
    for (int k = 0; k < 8; ++k) {
        const int s = class_scope ? class_scope[k] : kRaggedScope[k];
        if (s != GLASS_SCOPE_THREAD && s != GLASS_SCOPE_WAVE && s != GLASS_SCOPE_SUBWAVE)
            return GLASS_ERR_INVALID_VALUE;
        if ((s == GLASS_SCOPE_THREAD && k > 0) || (s == GLASS_SCOPE_SUBWAVE && k > 2))
            return GLASS_ERR_INFEASIBLE_PLACEMENT;
        sc.s[k] = s;
    }
    if (count == 0) return GLASS_OK;
    if (!n || !nrhs || !offA || !offB || !A || !B || !info || !workspace) return GLASS_ERR_INVALID_VALUE;
    if (workspace_bytes < ragged_workspace_bytes(count) || (reinterpret_cast<uintptr_t>(workspace) & 3))
        return GLASS_ERR_INVALID_VALUE;
    return launched(launch_posv_ragged(count, n, nrhs, offA, offB, A, B, info, workspace, sc, stream));
}

glass_status_t glass_posv_ragged_noalloc(int count, const int32_t* n, const int32_t* nrhs, const int64_t* offA,
                                         const int64_t* offB, float* A, float* B, int32_t* info,
                                         const int32_t* class_scope, void* stream) {
    if (count < 0) return GLASS_ERR_INVALID_VALUE;
    if (count > kRaggedNoAllocMaxCount) return GLASS_ERR_UNSUPPORTED;
    RaggedScopes sc{};
    for (int k = 0; k < 8; ++k) {
        const int s = class_scope ? class_scope[k] : kRaggedScope[k];
        if (s != GLASS_SCOPE_THREAD && s != GLASS_SCOPE_WAVE && s != GLASS_SCOPE_SUBWAVE)
            return GLASS_ERR_INVALID_VALUE;
        if ((s == GLASS_SCOPE_THREAD && k > 0) || (s == GLASS_SCOPE_SUBWAVE && k > 2))
            return GLASS_ERR_INFEASIBLE_PLACEMENT;
        sc.s[k] = s;
    }
    if (count == 0) return GLASS_OK;
    if (!n || !nrhs || !offA || !offB || !A || !B || !info) return GLASS_ERR_INVALID_VALUE;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    const int err = ragged_noalloc_workspace(&ws, &ws_bytes);
    if (err != 0) return launched(err);
    if (ws_bytes < ragged_workspace_bytes(count)) return GLASS_ERR_UNSUPPORTED;
    return launched(launch_posv_ragged(count, n, nrhs, offA, offB, A, B, info, ws, sc, stream));
}

int glass_posv_ragged_noalloc_max_count(void) { return kRaggedNoAllocMaxCount; }

glass_status_t glass_stream_probe(int kind, const float* a, const float* b, float* c, long long n4, int blocks,
                                  void* stream) {
    if (kind < 0 || kind > 3 || n4 < 0 || blocks < 1 || blocks > (1 << 20)) return GLASS_ERR_INVALID_VALUE;
    if (n4 == 0) return GLASS_OK;
    const bool needs_a = kind != 1, needs_b = kind == 3;
    if ((needs_a && !a) || (needs_b && !b) || !c) return GLASS_ERR_INVALID_VALUE;
    const uintptr_t mis = (reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                           reinterpret_cast<uintptr_t>(c)) & 15;
    if (mis) return GLASS_ERR_INVALID_VALUE;
    if (kind == 0 && n4 < 64) return GLASS_ERR_INVALID_VALUE;  // the read kernel's sink is 256 floats of c
    return launched(launch_stream_probe(kind, a, b, c, n4, blocks, stream));
}

glass_status_t glass_riccati_gain_batched(int nx, int nu, int batch, const float* A, const float* B, const float* P,
                                          const float* R, float* K, int32_t* info, const glass_placement_t* force,
                                          void* stream) {
    if (!valid_force(force)) return GLASS_ERR_INVALID_VALUE;
    if (!riccati_size_ok(nx, nu)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 0) return GLASS_ERR_INVALID_VALUE;
    if (batch == 0) return GLASS_OK;
    if (!A || !B || !P || !R || !K) return GLASS_ERR_INVALID_VALUE;
    // without a forced placement, thread scope wherever it runs (measured
    // faster at every batch from 16 to 65,536 at nx, nu = (1, 1), (4, 2),
    // (6, 3), (8, 1) and (8, 4)), one wavefront per workgroup
    if (!force && riccati_thread_ok(nx, nu))
        return launched(launch_riccati_thread(nx, nu, batch, 1, A, B, P, R, K, info, stream));
    int pack = kRiccatiDefaultPack;
    if (force) {
        if (force->scope == GLASS_SCOPE_THREAD) {
            if (!riccati_thread_ok(nx, nu)) return GLASS_ERR_INFEASIBLE_PLACEMENT;
            return launched(launch_riccati_thread(nx, nu, batch, force->pack, A, B, P, R, K, info, stream));
        }
        if (force->scope == GLASS_SCOPE_SUBWAVE) {
            if (!riccati_seg_ok(nx, nu)) return GLASS_ERR_INFEASIBLE_PLACEMENT;
            return launched(launch_riccati_seg(nx, nu, batch, force->pack, A, B, P, R, K, info, stream));
        }
        if (force->scope != GLASS_SCOPE_WAVE) return GLASS_ERR_INFEASIBLE_PLACEMENT;
        pack = force->pack;
    }
    if (riccati_region_floats(nx, nu) * sizeof(float) * pack > kLdsBudgetBytes) {
        if (force) return GLASS_ERR_INFEASIBLE_PLACEMENT;
        pack = 1;
    }
    return launched(launch_riccati(nx, nu, batch, pack, A, B, P, R, K, info, stream));
}

int glass_riccati_feasible(int nx, int nu, int pack) {
    if (!riccati_size_ok(nx, nu)) return GLASS_ERR_UNSUPPORTED;
    if (pack != 1 && pack != 2 && pack != 4 && pack != 8) return GLASS_ERR_INVALID_VALUE;
    return riccati_region_floats(nx, nu) * sizeof(float) * pack <= kLdsBudgetBytes ? 1 : 0;
}

int glass_riccati_placement_feasible(int nx, int nu, int scope, int pack) {
    const glass_placement_t f{scope, pack};
    if (!valid_force(&f)) return GLASS_ERR_INVALID_VALUE;
    if (!riccati_size_ok(nx, nu)) return GLASS_ERR_UNSUPPORTED;
    if (scope == GLASS_SCOPE_THREAD) return riccati_thread_ok(nx, nu) ? 1 : 0;
    if (scope == GLASS_SCOPE_SUBWAVE) return riccati_seg_ok(nx, nu) ? 1 : 0;
    if (scope == GLASS_SCOPE_WAVE) return glass_riccati_feasible(nx, nu, pack);
    return 0;
}

const char* glass_ragged_table_provenance(void) { return kRaggedProvenance; }

int glass_last_launch_error(void) { return t_last_launch_error; }

const char* glass_hip_error_name(int code) { return hip_error_name(code); }

size_t glass_mlp_num_params(int d) { return (d >= 1 && d <= 32) ? mlp_num_params(d) : 0; }

size_t glass_mlp_backward_workspace_size(int N, int d) {
    return (N >= 0 && d >= 1 && d <= 32) ? mlp_backward_workspace_bytes(N, d) : 0;
}

glass_status_t glass_mlp_forward(int N, int d, const float* X, const float* params, float* H1, float* H2, float* y,
                                 void* stream) {
    if (d < 1 || d > 32) return GLASS_ERR_UNSUPPORTED;
    if (N < 0) return GLASS_ERR_INVALID_VALUE;
    if (N == 0) return GLASS_OK;
    if (!X || !params || !y) return GLASS_ERR_INVALID_VALUE;
    return launched(launch_mlp_forward(N, d, X, params, H1, H2, y, stream));
}

glass_status_t glass_mlp_backward(int N, int d, const float* X, const float* params, const float* H1,
                                  const float* H2, const float* y, const float* t, float* grad, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    if (d < 1 || d > 32) return GLASS_ERR_UNSUPPORTED;
    if (N < 1) return GLASS_ERR_INVALID_VALUE;
    if (!X || !params || !H1 || !H2 || !y || !t || !grad || !workspace) return GLASS_ERR_INVALID_VALUE;
    if (workspace_bytes < mlp_backward_workspace_bytes(N, d) || (reinterpret_cast<uintptr_t>(workspace) & 3))
        return GLASS_ERR_INVALID_VALUE;
    return launched(launch_mlp_backward(N, d, X, params, H1, H2, y, t, grad, workspace, stream));
}

glass_status_t glass_mlp_adam(int P, float* params, const float* grad, float* m, float* v, int step, float lr,
                              float beta1, float beta2, float eps, void* stream) {
    if (P < 0 || step < 1) return GLASS_ERR_INVALID_VALUE;
    if (P == 0) return GLASS_OK;
    if (!params || !grad || !m || !v) return GLASS_ERR_INVALID_VALUE;
    const float bc1 = (float)(1.0 - pow((double)beta1, step));
    const float bc2 = (float)(1.0 - pow((double)beta2, step));
    return launched(launch_mlp_adam(P, params, grad, m, v, lr, beta1, beta2, eps, bc1, bc2, stream));
}

glass_status_t glass_query_placement(glass_op_t op, int n, int batch, glass_placement_t* out) {
    if ((int)op < GLASS_OP_GEMM || (int)op > GLASS_OP_POSV_ADJOINT) return GLASS_ERR_INVALID_VALUE;
    if (!is_se3(op) && !size_ok(n)) return GLASS_ERR_UNSUPPORTED;
    if (batch < 1 || !out) return GLASS_ERR_INVALID_VALUE;
    const int order = is_se3(op) ? 4 : n;
    int scope, pack;
    table_lookup(op, order, batch, &scope, &pack);
    Shape s{op, order, order, order, 1, 0};
    Geometry g;
    if (!make_geometry(s, scope, pack, batch, &g)) {
        scope = GLASS_SCOPE_WAVE;
        pack = 1;
        make_geometry(s, scope, pack, batch, &g);
    }
    out->scope = g.scope;
    out->pack = g.pack;
    out->wg_threads = g.threads;
    out->problems_per_wg = g.problems_per_wg;
    return GLASS_OK;
}

int glass_placement_feasible(glass_op_t op, int n, int nrhs, int scope, int pack) {
    if ((int)op < GLASS_OP_GEMM || (int)op > GLASS_OP_POSV_ADJOINT) return GLASS_ERR_INVALID_VALUE;
    if (scope < GLASS_SCOPE_THREAD || scope > GLASS_SCOPE_SUBWAVE) return GLASS_ERR_INVALID_VALUE;
    if (!is_se3(op) && !size_ok(n)) return GLASS_ERR_UNSUPPORTED;
    if (!size_ok(nrhs)) return GLASS_ERR_UNSUPPORTED;
    const int order = is_se3(op) ? 4 : n;
    Shape s{op, order, order, order, nrhs, 0};
    return make_geometry(s, scope, pack, 1, nullptr) ? 1 : 0;
}

const char* glass_table_provenance(void) { return kTableProvenance; }

const char* glass_status_string(glass_status_t s) {
    switch (s) {
    case GLASS_OK: return "GLASS_OK";
    case GLASS_ERR_INVALID_VALUE: return "GLASS_ERR_INVALID_VALUE";
    case GLASS_ERR_UNSUPPORTED: return "GLASS_ERR_UNSUPPORTED";
    case GLASS_ERR_INFEASIBLE_PLACEMENT: return "GLASS_ERR_INFEASIBLE_PLACEMENT";
    case GLASS_ERR_LAUNCH: return "GLASS_ERR_LAUNCH";
    }
    return "GLASS_ERR_UNKNOWN";
}

}  // extern "C"
