// chol.hip -- batched Cholesky factorization (POTRF), Cholesky solve (POTRS),
// fused factor-and-solve (POSV) and triangular solve (TRSV) for gfx950, each
// at the three execution scopes of Sec. III-A:
//
//   thread    one problem per lane.  The workgroup's contiguous span of
//             problems is staged through LDS with coalesced loads (in passes
//             that bound LDS use), each lane then holds its problem's lower
//             triangle in VGPRs at compile-time order N and factors / solves
//             it fully unrolled.
//   wave      one problem per 64-lane wavefront.  Lane i owns row i, loaded
//             straight from global memory (lower triangle only).  POTRF is
//             right-looking in VGPRs: the pivot comes from v_readlane and the
//             scaled column is broadcast with DPP row_newbcast folded into the
//             v_fmac of the update (no LDS).  Forward substitution broadcasts
//             the solved unknown with v_readlane; L leaves through an 8-row
//             LDS chunk as coalesced stores, walked bottom-up so the same
//             chunk also feeds the backward substitution (which needs L by
//             columns).
//   workgroup one problem at a time per workgroup of T(n) lanes, the matrix
//             resident in LDS, cooperative right-looking updates separated
//             by workgroup barriers; P problems back to back.
//
// Arithmetic: FP32 with fused multiply-adds.  A pivot d gives inv = rsq(d)
// (v_rsq_f32) and L_jj = d * inv; divisions by a diagonal entry are multiplies
// by its reciprocal.  The failure test is !(pivot > 0), as in the definition
// of info in glass.h.
#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"

namespace glass {
namespace {

template <int N>
__global__ void __launch_bounds__(512) potrf_thread(int batch, float* __restrict__ A, int* __restrict__ info) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    float* base = A + p0 * (N * N);
    float a[N * (N + 1) / 2];
    float dinv[N];
    thread_load_tri<N>(a, base, lds, cnt, tid, nt);
    const bool active = tid < cnt;
    int inf = 0;
    if (active) inf = tri_potrf<N>(a, dinv);
    if (info && active) info[p0 + tid] = inf;
    thread_store_tri<N>(a, base, lds, cnt, tid, nt);
}

template <int N>
__global__ void __launch_bounds__(512) posv_thread(int nrhs, int batch, float* __restrict__ A, float* __restrict__ B,
                                                   int* __restrict__ info) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    float* base = A + p0 * (N * N);
    float a[N * (N + 1) / 2];
    float dinv[N];
    thread_load_tri<N>(a, base, lds, cnt, tid, nt);
    const bool active = tid < cnt;
    int inf = 0;
    if (active) inf = tri_potrf<N>(a, dinv);
    if (info && active) info[p0 + tid] = inf;
    thread_store_tri<N>(a, base, lds, cnt, tid, nt);
    thread_solve_rhs<N>(a, dinv, B + p0 * N * nrhs, lds, nrhs, cnt, tid, nt, true, true, active && inf == 0);
}

template <int N>
__global__ void __launch_bounds__(512) potrs_thread(int nrhs, int batch, const float* __restrict__ L,
                                                    float* __restrict__ B) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    float a[N * (N + 1) / 2];
    float dinv[N];
    thread_load_tri<N>(a, L + p0 * (N * N), lds, cnt, tid, nt);
#pragma unroll
    for (int i = 0; i < N; ++i) dinv[i] = recip(a[TI(i, i)]);
    thread_solve_rhs<N>(a, dinv, B + p0 * N * nrhs, lds, nrhs, cnt, tid, nt, true, true, tid < cnt);
}

template <int N>
__global__ void __launch_bounds__(512) trsv_thread(int trans, int batch, const float* __restrict__ L,
                                                   float* __restrict__ x) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    float a[N * (N + 1) / 2];
    float dinv[N];
    thread_load_tri<N>(a, L + p0 * (N * N), lds, cnt, tid, nt);
#pragma unroll
    for (int i = 0; i < N; ++i) dinv[i] = recip(a[TI(i, i)]);
    thread_solve_rhs<N>(a, dinv, x + p0 * N, lds, 1, cnt, tid, nt, trans == 0, trans != 0, tid < cnt);
}

// -------------------------------------------------------------- wave scope --
template <int NB>
__global__ void __launch_bounds__(512) potrf_wave(int n, int batch, float* __restrict__ A, int* __restrict__ info,
                                                  int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    float* Ag = A + p * n * n;
    float a[NB];
    rows_load_lower<NB, false>(a, Ag, n, lane);
    float myinv;
    const int inf = wave_potrf<NB>(a, lane, myinv);
    const bool vec = (n & 3) == 0 && aligned16(A);
    wave_chunks_desc<NB>(a, buf, Ag, vec, n, lane, false, 0.f, myinv);
    if (info && lane == 0) info[p] = inf;
}

// MULTI: several right-hand sides are solved in column groups; the nrhs = 1
// instance keeps only the single-column path and its register budget.
template <int NB, bool MULTI>
__global__ void __launch_bounds__(512) posv_wave(int n, int nrhs, int batch, float* __restrict__ A,
                                                 float* __restrict__ B, int* __restrict__ info, int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    float* Ag = A + p * n * n;
    float* Bg = B + p * n * nrhs;
    const float b0 = MULTI ? 0.f : lane_elem(Bg, n, lane);  // issued with the rows
    float a[NB];
    rows_load_lower<NB, false>(a, Ag, n, lane);
    float myinv;
    const int inf = wave_potrf<NB>(a, lane, myinv);
    const bool vec = (n & 3) == 0 && aligned16(A);
    if (inf != 0) {
        wave_chunks_desc<NB>(a, buf, Ag, vec, n, lane, false, 0.f, myinv);
    } else if (MULTI) {
        wave_solve_all<NB>(a, buf, Ag, vec, Bg, n, nrhs, myinv, lane);
    } else {
        float acc = b0;
        acc = wave_fwd<NB>(a, acc, myinv, lane);
        acc = wave_chunks_desc<NB>(a, buf, Ag, vec, n, lane, true, acc, myinv);
        if (lane < n) Bg[lane] = acc;
    }
    if (info && lane == 0) info[p] = inf;
}

template <int NB, bool MULTI>
__global__ void __launch_bounds__(512) potrs_wave(int n, int nrhs, int batch, const float* __restrict__ L,
                                                  float* __restrict__ B, int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    const float* Lg = L + p * n * n;
    float* Bg = B + p * n * nrhs;
    const float dg = diag_load(Lg, n, lane), b0 = MULTI ? 0.f : lane_elem(Bg, n, lane);  // issued with the rows
    float a[NB];
    rows_load_lower<NB, true>(a, Lg, n, lane);
    const float myinv = diag_inv(dg, n, lane);
    if (MULTI) {
        wave_solve_all<NB>(a, buf, nullptr, false, Bg, n, nrhs, myinv, lane);
    } else {
        float acc = b0;
        acc = wave_fwd<NB>(a, acc, myinv, lane);
        acc = wave_chunks_desc<NB>(a, buf, nullptr, false, n, lane, true, acc, myinv);
        if (lane < n) Bg[lane] = acc;
    }
}

template <int NB>
__global__ void __launch_bounds__(512) trsv_wave(int n, int trans, int batch, const float* __restrict__ L,
                                                 float* __restrict__ x, int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    const float* Lg = L + p * n * n;
    const float dg = diag_load(Lg, n, lane);
    float acc = lane_elem(x + p * n, n, lane);  // issued with the rows
    float a[NB];
    rows_load_lower<NB, true>(a, Lg, n, lane);
    const float myinv = diag_inv(dg, n, lane);
    if (trans == 0)
        acc = wave_fwd<NB>(a, acc, myinv, lane);
    else
        acc = wave_chunks_desc<NB>(a, buf, nullptr, false, n, lane, true, acc, myinv);
    if (lane < n) x[p * n + lane] = acc;
}

// --------------------------------------------------------- workgroup scope --
// Right-looking Cholesky of the LDS-resident matrix M (row stride s) by the
// whole workgroup; returns info (identical in every lane).
GLASS_DEV int wg_potrf(float* M, int n, int s, int tid, int nt) {
    const int tr = tid >> 4, tc = tid & 15, rstep = nt >> 4;
    for (int j = 0; j < n; ++j) {
        const float d = M[j * s + j];
        if (!(d > 0.f)) return j + 1;
        const float inv = rsq(d);
        const float l = d * inv;
        __syncthreads();
        for (int i = j + tid; i < n; i += nt) M[i * s + j] = i == j ? l : M[i * s + j] * inv;
        __syncthreads();
        for (int i = j + 1 + tr; i < n; i += rstep) {
            const float lij = M[i * s + j];
            for (int k = j + 1 + tc; k <= i; k += 16) M[i * s + k] = fmaf(-lij, M[k * s + j], M[i * s + k]);
        }
        __syncthreads();
    }
    return 0;
}

// Zero the strict upper triangle of M.
GLASS_DEV void wg_zero_upper(float* M, int n, int s, int tid, int nt) {
    const int tr = tid >> 4, tc = tid & 15, rstep = nt >> 4;
    for (int i = tr; i < n; i += rstep)
        for (int k = i + 1 + tc; k < n; k += 16) M[i * s + k] = 0.f;
}

// Workgroup substitutions on Bm ([n][nrhs], stride sb) with L in M.
GLASS_DEV void wg_solve(const float* M, int s, float* Bm, int sb, int n, int nrhs, int tid, int nt, bool fwd,
                        bool bwd) {
    const FastDiv fr = make_fastdiv(nrhs);
    const int tot = n * nrhs;
    if (fwd) {
        for (int k = 0; k < n; ++k) {
            const float dk = 1.0f / M[k * s + k];
            for (int idx = tid; idx < tot; idx += nt) {
                const int i = (int)fdiv((uint32_t)idx, fr), c = idx - i * nrhs;
                if (i > k) Bm[i * sb + c] = fmaf(-M[i * s + k], Bm[k * sb + c] * dk, Bm[i * sb + c]);
            }
            __syncthreads();
        }
        for (int idx = tid; idx < tot; idx += nt) {
            const int i = (int)fdiv((uint32_t)idx, fr), c = idx - i * nrhs;
            Bm[i * sb + c] *= 1.0f / M[i * s + i];
        }
        __syncthreads();
    }
    if (bwd) {
        for (int k = n - 1; k >= 0; --k) {
            const float dk = 1.0f / M[k * s + k];
            for (int idx = tid; idx < tot; idx += nt) {
                const int i = (int)fdiv((uint32_t)idx, fr), c = idx - i * nrhs;
                if (i < k) Bm[i * sb + c] = fmaf(-M[k * s + i], Bm[k * sb + c] * dk, Bm[i * sb + c]);
            }
            __syncthreads();
        }
        for (int idx = tid; idx < tot; idx += nt) {
            const int i = (int)fdiv((uint32_t)idx, fr), c = idx - i * nrhs;
            Bm[i * sb + c] *= 1.0f / M[i * s + i];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) potrf_wg(int n, int batch, int pack, float* __restrict__ A,
                                                int* __restrict__ info) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const int s = n | 1;
    const FastDiv fd = make_fastdiv(n);
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        float* Ag = A + p * n * n;
        stage_in<4>(lds, Ag, n * n, fd, s, tid, nt);
        __syncthreads();
        const int inf = wg_potrf(lds, n, s, tid, nt);
        wg_zero_upper(lds, n, s, tid, nt);
        __syncthreads();
        stage_out(Ag, lds, n * n, fd, s, tid, nt);
        if (info && tid == 0) info[p] = inf;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) posv_wg(int n, int nrhs, int batch, int pack, float* __restrict__ A,
                                               float* __restrict__ B, int* __restrict__ info) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const int s = n | 1, sb = nrhs | 1;
    float* Bm = lds + ((n * s + 3) & ~3);
    const FastDiv fd = make_fastdiv(n), fdb = make_fastdiv(nrhs);
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        float* Ag = A + p * n * n;
        float* Bg = B + p * n * nrhs;
        stage_in<4>(lds, Ag, n * n, fd, s, tid, nt);
        stage_in<2>(Bm, Bg, n * nrhs, fdb, sb, tid, nt);
        __syncthreads();
        const int inf = wg_potrf(lds, n, s, tid, nt);
        wg_zero_upper(lds, n, s, tid, nt);
        __syncthreads();
        stage_out(Ag, lds, n * n, fd, s, tid, nt);
        if (info && tid == 0) info[p] = inf;
        if (inf == 0) {
            wg_solve(lds, s, Bm, sb, n, nrhs, tid, nt, true, true);
            stage_out(Bg, Bm, n * nrhs, fdb, sb, tid, nt);
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) potrs_wg(int n, int nrhs, int batch, int pack, const float* __restrict__ L,
                                                float* __restrict__ B) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const int s = n | 1, sb = nrhs | 1;
    float* Bm = lds + ((n * s + 3) & ~3);
    const FastDiv fd = make_fastdiv(n), fdb = make_fastdiv(nrhs);
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        float* Bg = B + p * n * nrhs;
        stage_in<4>(lds, L + p * n * n, n * n, fd, s, tid, nt);
        stage_in<2>(Bm, Bg, n * nrhs, fdb, sb, tid, nt);
        __syncthreads();
        wg_solve(lds, s, Bm, sb, n, nrhs, tid, nt, true, true);
        stage_out(Bg, Bm, n * nrhs, fdb, sb, tid, nt);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) trsv_wg(int n, int trans, int batch, int pack, const float* __restrict__ L,
                                               float* __restrict__ x) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const int s = n | 1;
    float* vm = lds + ((n * s + 3) & ~3);
    const FastDiv fd = make_fastdiv(n);
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        stage_in<4>(lds, L + p * n * n, n * n, fd, s, tid, nt);
        for (int i = tid; i < n; i += nt) vm[i] = x[p * n + i];
        __syncthreads();
        wg_solve(lds, s, vm, 1, n, 1, tid, nt, trans == 0, trans != 0);
        for (int i = tid; i < n; i += nt) x[p * n + i] = vm[i];
        __syncthreads();
    }
}

// ----------------------------------------------------------------- launch --
#define GLASS_CASES_1_16(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#define GLASS_BUCKETS(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

inline int bucket8(int n) { return ((n + 7) / 8) * 8; }


inline int finish() { return (int)hipGetLastError(); }

}  // namespace

int launch_potrf(const Shape& sh, const Geometry& g, int batch, float* A, int32_t* info, void* stream) {
    if (g.scope == GLASS_SCOPE_SUBWAVE) return launch_chol_subwave(sh, g, batch, A, nullptr, info, stream);
    if (g.scope == GLASS_SCOPE_WAVE && sh.n >= kBlkMinN) return launch_chol_blk(sh, g, batch, A, nullptr, info, stream);
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD) {
        switch (n) {
#define X(N) \
    case N: hipLaunchKernelGGL(potrf_thread<N>, grid, block, g.lds_bytes, st, batch, A, info); break;
            GLASS_CASES_1_16(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_WAVE) {
        const int region = (int)wave_region_floats(sh);
        switch (bucket8(n)) {
#define X(NB) \
    case NB: hipLaunchKernelGGL(potrf_wave<NB>, grid, block, g.lds_bytes, st, n, batch, A, info, region); break;
            GLASS_BUCKETS(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(potrf_wg, grid, block, g.lds_bytes, st, n, batch, g.pack, A, info);
    }
    return finish();
}

int launch_posv(const Shape& sh, const Geometry& g, int batch, float* A, float* B, int32_t* info, void* stream) {
    if (g.scope == GLASS_SCOPE_SUBWAVE) return launch_chol_subwave(sh, g, batch, A, B, info, stream);
    if (g.scope == GLASS_SCOPE_WAVE && sh.n >= kBlkMinN) return launch_chol_blk(sh, g, batch, A, B, info, stream);
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n, r = sh.nrhs;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD) {
        switch (n) {
#define X(N) \
    case N: hipLaunchKernelGGL(posv_thread<N>, grid, block, g.lds_bytes, st, r, batch, A, B, info); break;
            GLASS_CASES_1_16(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_WAVE) {
        const int region = (int)wave_region_floats(sh);
        switch (bucket8(n)) {
#define X(NB) \
    case NB:                                                                                                  \
        if (r == 1)                                                                                           \
            hipLaunchKernelGGL((posv_wave<NB, false>), grid, block, g.lds_bytes, st, n, r, batch, A, B, info, region); \
        else                                                                                                  \
            hipLaunchKernelGGL((posv_wave<NB, true>), grid, block, g.lds_bytes, st, n, r, batch, A, B, info, region);  \
        break;
            GLASS_BUCKETS(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(posv_wg, grid, block, g.lds_bytes, st, n, r, batch, g.pack, A, B, info);
    }
    return finish();
}

int launch_potrs(const Shape& sh, const Geometry& g, int batch, const float* L, float* B, void* stream) {
    if (g.scope == GLASS_SCOPE_SUBWAVE) return launch_chol_subwave(sh, g, batch, const_cast<float*>(L), B, nullptr, stream);
    if (g.scope == GLASS_SCOPE_WAVE && sh.n >= kBlkMinN) return launch_chol_blk(sh, g, batch, const_cast<float*>(L), B, nullptr, stream);
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n, r = sh.nrhs;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD) {
        switch (n) {
#define X(N) \
    case N: hipLaunchKernelGGL(potrs_thread<N>, grid, block, g.lds_bytes, st, r, batch, L, B); break;
            GLASS_CASES_1_16(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_WAVE) {
        const int region = (int)wave_region_floats(sh);
        switch (bucket8(n)) {
#define X(NB) \
    case NB:                                                                                                  \
        if (r == 1)                                                                                           \
            hipLaunchKernelGGL((potrs_wave<NB, false>), grid, block, g.lds_bytes, st, n, r, batch, L, B, region); \
        else                                                                                                  \
            hipLaunchKernelGGL((potrs_wave<NB, true>), grid, block, g.lds_bytes, st, n, r, batch, L, B, region);  \
        break;
            GLASS_BUCKETS(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(potrs_wg, grid, block, g.lds_bytes, st, n, r, batch, g.pack, L, B);
    }
    return finish();
}

int launch_trsv(const Shape& sh, const Geometry& g, int batch, const float* L, float* x, void* stream) {
    if (g.scope == GLASS_SCOPE_SUBWAVE) return launch_chol_subwave(sh, g, batch, const_cast<float*>(L), x, nullptr, stream);
    if (g.scope == GLASS_SCOPE_WAVE && sh.n >= kBlkMinN) return launch_chol_blk(sh, g, batch, const_cast<float*>(L), x, nullptr, stream);
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n, tr = sh.trans;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD) {
        switch (n) {
#define X(N) \
    case N: hipLaunchKernelGGL(trsv_thread<N>, grid, block, g.lds_bytes, st, tr, batch, L, x); break;
            GLASS_CASES_1_16(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_WAVE) {
        const int region = (int)wave_region_floats(sh);
        switch (bucket8(n)) {
#define X(NB) \
    case NB: hipLaunchKernelGGL(trsv_wave<NB>, grid, block, g.lds_bytes, st, n, tr, batch, L, x, region); break;
            GLASS_BUCKETS(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(trsv_wg, grid, block, g.lds_bytes, st, n, tr, batch, g.pack, L, x);
    }
    return finish();
}

}  // namespace glass
