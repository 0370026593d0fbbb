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

namespace glass {
namespace {

#define TI(i, j) ((i) * ((i) + 1) / 2 + (j))

// ------------------------------------------------------------ thread scope --
__device__ __forceinline__ int stage_q(int threads, int elems) {
    int s = elems | 1;
    int q = kStagePassFloats / s;
    if (q < 1) q = 1;
    return q < threads ? q : threads;
}

template <int N>
GLASS_DEV void tri_load(float (&a)[N * (N + 1) / 2], const float* src) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) a[TI(i, j)] = src[i * N + j];
}

template <int N>
GLASS_DEV void tri_store_full(const float (&a)[N * (N + 1) / 2], float* dst) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) dst[i * N + j] = j <= i ? a[TI(i, j)] : 0.f;
}

// Left-looking Cholesky of the lane's triangle; returns info.
template <int N>
GLASS_DEV int tri_potrf(float (&a)[N * (N + 1) / 2], float (&dinv)[N]) {
    int info = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        float s = a[TI(j, j)];
#pragma unroll
        for (int p = 0; p < j; ++p) s = fmaf(-a[TI(j, p)], a[TI(j, p)], s);
        if (!(s > 0.f) && info == 0) info = j + 1;
        const float inv = rsq(s);
        const float l = s * inv;
        a[TI(j, j)] = l;
        dinv[j] = inv;
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            float t = a[TI(i, j)];
#pragma unroll
            for (int p = 0; p < j; ++p) t = fmaf(-a[TI(i, p)], a[TI(j, p)], t);
            a[TI(i, j)] = t * inv;
        }
    }
    return info;
}

// x <- L^{-1} x (fwd) and/or L^{-T} x (bwd) for one column held in VGPRs.
template <int N>
GLASS_DEV void tri_fwd(const float (&a)[N * (N + 1) / 2], const float (&dinv)[N], float (&y)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float t = y[i];
#pragma unroll
        for (int p = 0; p < i; ++p) t = fmaf(-a[TI(i, p)], y[p], t);
        y[i] = t * dinv[i];
    }
}

template <int N>
GLASS_DEV void tri_bwd(const float (&a)[N * (N + 1) / 2], const float (&dinv)[N], float (&y)[N]) {
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        float t = y[i];
#pragma unroll
        for (int p = i + 1; p < N; ++p) t = fmaf(-a[TI(p, i)], y[p], t);
        y[i] = t * dinv[i];
    }
}

// Stage the lanes' triangles in: passes of Q problems through LDS.
template <int N>
GLASS_DEV void thread_load_tri(float (&a)[N * (N + 1) / 2], const float* __restrict__ base, float* lds,
                               int cnt, int tid, int nt) {
    constexpr int SZ = N * N, S = SZ | 1;
    const int Q = stage_q(nt, SZ);
    const FastDiv fd = make_fastdiv(SZ);
    for (int s = 0; s < cnt; s += Q) {
        const int qn = min(Q, cnt - s);
        stage_in<(N <= 8 ? 8 : 4)>(lds, base + (size_t)s * SZ, qn * SZ, fd, S, tid, nt);
        __syncthreads();
        if (tid >= s && tid < s + qn) tri_load<N>(a, lds + (tid - s) * S);
        __syncthreads();
    }
}

template <int N>
GLASS_DEV void thread_store_tri(const float (&a)[N * (N + 1) / 2], float* __restrict__ base, float* lds,
                                int cnt, int tid, int nt) {
    constexpr int SZ = N * N, S = SZ | 1;
    const int Q = stage_q(nt, SZ);
    const FastDiv fd = make_fastdiv(SZ);
    for (int s = 0; s < cnt; s += Q) {
        const int qn = min(Q, cnt - s);
        if (tid >= s && tid < s + qn) tri_store_full<N>(a, lds + (tid - s) * S);
        __syncthreads();
        stage_out(base + (size_t)s * SZ, lds, qn * SZ, fd, S, tid, nt);
        __syncthreads();
    }
}

// Solve the staged right-hand sides of every lane (all columns) in place.
template <int N>
GLASS_DEV void thread_solve_rhs(const float (&a)[N * (N + 1) / 2], const float (&dinv)[N], float* __restrict__ Bg,
                                float* lds, int nrhs, int cnt, int tid, int nt, bool fwd, bool bwd,
                                bool active) {
    const int SZ = N * nrhs, S = SZ | 1;
    const FastDiv fd = make_fastdiv(SZ);
    stage_in<2>(lds, Bg, cnt * SZ, fd, S, tid, nt);
    __syncthreads();
    if (active) {
        float* b = lds + tid * S;
        for (int c = 0; c < nrhs; ++c) {
            float y[N];
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = b[i * nrhs + c];
            if (fwd) tri_fwd<N>(a, dinv, y);
            if (bwd) tri_bwd<N>(a, dinv, y);
#pragma unroll
            for (int i = 0; i < N; ++i) b[i * nrhs + c] = y[i];
        }
    }
    __syncthreads();
    stage_out(Bg, lds, cnt * SZ, fd, S, tid, nt);
}

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
    for (int i = 0; i < N; ++i) dinv[i] = 1.0f / a[TI(i, i)];
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
    for (int i = 0; i < N; ++i) dinv[i] = 1.0f / a[TI(i, i)];
    thread_solve_rhs<N>(a, dinv, x + p0 * N, lds, 1, cnt, tid, nt, trans == 0, trans != 0, tid < cnt);
}

// -------------------------------------------------------------- wave scope --
// Lane i owns row i.  Rows come straight from global memory with 16-byte
// buffer loads of only the column blocks at or left of the diagonal; rows and
// columns beyond n are padded with an identity block, so every column loop
// runs the full bucket width NB without a data-dependent exit and the leading
// n x n factor is unchanged (padded pivots are 1, padded couplings 0).
template <int NB>
GLASS_DEV void rows_load_lower(float (&a)[NB], const float* Ag, int n, int lane) {
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(Ag, (uint32_t)(n * n) * 4u);
    const bool row = lane < n;
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
        f4_t v = {0.f, 0.f, 0.f, 0.f};
        if (row && 4 * t <= lane) {
            if (lane * n + 4 * t + 4 <= n * n) {
                v = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, lane * n * 4, t * 16, 0));
            } else {  // last row, block past the end of the problem: element-wise
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * t + e < n)
                        v[e] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(rs, (lane * n + 4 * t + e) * 4, 0, 0));
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * t + e;
            a[j] = (row && j <= lane) ? v[e] : (j == lane ? 1.f : 0.f);
        }
    }
}

// One column step of the right-looking factorization: the pivot of column J
// comes from v_readlane, the scaled column is broadcast with DPP and each lane
// updates the rest of its row in VGPRs (a[K] -= l_iJ * l_KJ, one v_fmac each).
template <int NB, int J, int K>
struct WaveUpd {
    static GLASS_DEV void run(float (&a)[NB], const float (&R)[4], float nv) {
        fmac_bcast<K % 16>(a[K], R[K / 16], nv);
        WaveUpd<NB, J, K + 1>::run(a, R, nv);
    }
};
template <int NB, int J>
struct WaveUpd<NB, J, NB> {
    static GLASS_DEV void run(float (&)[NB], const float (&)[4], float) {}
};

template <int NB, int J>
struct WaveStep {
    static GLASS_DEV void run(float (&a)[NB], int lane, int& info, float& myinv) {
        const float d = readlane(a[J], J);
        if (!(d > 0.f) && info == 0) info = J + 1;
        const float inv = rsq(d);
        const float v = lane == J ? d * inv : a[J] * inv;
        myinv = lane == J ? inv : myinv;
        a[J] = v;
        float R[4];
        replicate_rows<(NB + 15) / 16>(v, R);
        WaveUpd<NB, J, J + 1>::run(a, R, -v);
        WaveStep<NB, J + 1>::run(a, lane, info, myinv);
    }
};
template <int NB>
struct WaveStep<NB, NB> {
    static GLASS_DEV void run(float (&)[NB], int, int&, float&) {}
};

// Factor the identity-padded rows in place; returns info, sets myinv = 1/L_ii
// and clears the strict upper part of every row.
template <int NB>
GLASS_DEV int wave_potrf(float (&a)[NB], int lane, float& myinv) {
    int info = 0;
    myinv = 1.f;
    WaveStep<NB, 0>::run(a, lane, info, myinv);
#pragma unroll
    for (int k = 0; k < NB; ++k) a[k] = k <= lane ? a[k] : 0.f;
    return info;
}

// Forward substitution L y = b for one right-hand side, b_i in lane i: the
// solved unknown is broadcast with v_readlane (rows hold L_ik with a zero
// strict upper part; padded lanes have b = 0 and L_ii = 1).
template <int NB>
GLASS_DEV float wave_fwd(const float (&a)[NB], float acc, float myinv, int lane) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const float yk = readlane(acc * myinv, k);
        acc = lane == k ? yk : fmaf(-a[k], yk, acc);
    }
    return acc;
}

// Rows r0 .. r0+7 (< n) of L (strict upper +0) from the owning lanes into
// the LDS chunk buffer, row-major with row stride n.
template <int NB>
GLASS_DEV void rows_to_lds(const float (&a)[NB], float* buf, int n, int r0, int lane) {
    if (lane >= r0 && lane < r0 + 8 && lane < n) {
        float* dst = buf + (lane - r0) * n;
        if ((n & 3) == 0) {
#pragma unroll
            for (int t = 0; t < NB / 4; ++t) {
                if (4 * t < n) {
                    f4_t v;
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = a[4 * t + e];
                    *reinterpret_cast<f4_t*>(dst + 4 * t) = v;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < n) dst[j] = a[j];
        }
    }
}

// Coalesced copy of len floats from the LDS chunk to global memory.
GLASS_DEV void chunk_to_global(float* __restrict__ dst, const float* buf, int len, bool vec, int lane) {
    if (vec) {
        for (int q = lane; q < (len >> 2); q += 64)
            reinterpret_cast<f4_t*>(dst)[q] = reinterpret_cast<const f4_t*>(buf)[q];
    } else {
        for (int g = lane; g < len; g += 64) dst[g] = buf[g];
    }
}

// Backward substitution L^T x = y for the rows of the chunk in LDS (rows
// r0 .. r1-1, descending); lane i < k reads L_ki from row k of the chunk.
GLASS_DEV float wave_bwd_chunk(const float* buf, int n, int r0, int r1, float acc, float myinv, int lane) {
    for (int k = r1 - 1; k >= r0; --k) {
        const float lki = lane < k ? buf[(k - r0) * n + lane] : 0.f;
        const float xk = readlane(acc * myinv, k);
        acc = lane == k ? xk : fmaf(-lki, xk, acc);
    }
    return acc;
}

// Walk the 8-row chunks of L from the bottom up: optionally store each chunk
// of L to global memory (coalesced) and optionally run the backward
// substitution steps of its rows.
template <int NB>
GLASS_DEV float wave_chunks_desc(const float (&a)[NB], float* buf, float* Lg, bool vec, int n, int lane, bool bwd,
                                 float acc, float myinv) {
    for (int r0 = (n - 1) & ~7; r0 >= 0; r0 -= 8) {
        const int r1 = min(r0 + 8, n);
        rows_to_lds<NB>(a, buf, n, r0, lane);
        wave_sync();
        if (Lg) chunk_to_global(Lg + r0 * n, buf, (r1 - r0) * n, vec, lane);
        if (bwd) acc = wave_bwd_chunk(buf, n, r0, r1, acc, myinv, lane);
        wave_sync();
    }
    return acc;
}

// 1 / L_ii of lane i's row (1 beyond n), read from global memory.
GLASS_DEV float diag_inv(const float* Lg, int n, int lane) {
    return lane < n ? 1.0f / Lg[lane * n + lane] : 1.f;
}

template <int NB>
__global__ void __launch_bounds__(512) potrf_wave(int n, int batch, float* __restrict__ A, int* __restrict__ info,
                                                  int region) {
    extern __shared__ float lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    float* Ag = A + p * n * n;
    float a[NB];
    rows_load_lower<NB>(a, Ag, n, lane);
    float myinv;
    const int inf = wave_potrf<NB>(a, lane, myinv);
    const bool vec = (n & 3) == 0 && aligned16(A);
    wave_chunks_desc<NB>(a, buf, Ag, vec, n, lane, false, 0.f, myinv);
    if (info && lane == 0) info[p] = inf;
}

template <int NB>
__global__ void __launch_bounds__(512) posv_wave(int n, int nrhs, int batch, float* __restrict__ A,
                                                 float* __restrict__ B, int* __restrict__ info, int region) {
    extern __shared__ float lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    float* Ag = A + p * n * n;
    float* Bg = B + p * n * nrhs;
    float a[NB];
    rows_load_lower<NB>(a, Ag, n, lane);
    float myinv;
    const int inf = wave_potrf<NB>(a, lane, myinv);
    const bool vec = (n & 3) == 0 && aligned16(A);
    if (inf != 0) {
        wave_chunks_desc<NB>(a, buf, Ag, vec, n, lane, false, 0.f, myinv);
    } else {
        for (int c = 0; c < nrhs; ++c) {
            float acc = lane < n ? Bg[lane * nrhs + c] : 0.f;
            acc = wave_fwd<NB>(a, acc, myinv, lane);
            acc = wave_chunks_desc<NB>(a, buf, c == 0 ? Ag : nullptr, vec, n, lane, true, acc, myinv);
            if (lane < n) Bg[lane * nrhs + c] = acc;
        }
    }
    if (info && lane == 0) info[p] = inf;
}

template <int NB>
__global__ void __launch_bounds__(512) potrs_wave(int n, int nrhs, int batch, const float* __restrict__ L,
                                                  float* __restrict__ B, int region) {
    extern __shared__ float lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    const float* Lg = L + p * n * n;
    float* Bg = B + p * n * nrhs;
    float a[NB];
    rows_load_lower<NB>(a, Lg, n, lane);
    const float myinv = diag_inv(Lg, n, lane);
    for (int c = 0; c < nrhs; ++c) {
        float acc = lane < n ? Bg[lane * nrhs + c] : 0.f;
        acc = wave_fwd<NB>(a, acc, myinv, lane);
        acc = wave_chunks_desc<NB>(a, buf, nullptr, false, n, lane, true, acc, myinv);
        if (lane < n) Bg[lane * nrhs + c] = acc;
    }
}

template <int NB>
__global__ void __launch_bounds__(512) trsv_wave(int n, int trans, int batch, const float* __restrict__ L,
                                                 float* __restrict__ x, int region) {
    extern __shared__ float lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    const float* Lg = L + p * n * n;
    float a[NB];
    rows_load_lower<NB>(a, Lg, n, lane);
    const float myinv = diag_inv(Lg, n, lane);
    float acc = lane < n ? x[p * n + lane] : 0.f;
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
    case NB: hipLaunchKernelGGL(posv_wave<NB>, grid, block, g.lds_bytes, st, n, r, batch, A, B, info, region); break;
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
    case NB: hipLaunchKernelGGL(potrs_wave<NB>, grid, block, g.lds_bytes, st, n, r, batch, L, B, region); break;
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
