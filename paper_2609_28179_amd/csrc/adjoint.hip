// adjoint.hip -- reverse mode of the batched Cholesky solve X = A^{-1} B.
//
// Given the factor L (A = L L^T), the solution X and the upstream gradient
// G = dl/dX of a scalar loss, one kernel returns
//   dB = A^{-1} G                       (forward + backward substitution)
//   dA = -(dB X^T + X dB^T) / 2         (the gradient over symmetric A)
// The paper validates derivatives by finite differences (Sec. III-C); the
// adjoint itself is the standard one of a linear solve, symmetrized because
// the factorization reads A as symmetric (only its lower triangle).
//
//   thread  (n <= 16) one problem per lane: L in VGPRs (compile-time n),
//           G and X staged through LDS, dA written through LDS passes as
//           coalesced stores.
//   wave    one problem per wavefront, the wave-scope substitutions of
//           chol.hip; lane i accumulates row i of dA from v_readlane
//           broadcasts of x_j and dB_j, rows leave through the 8-row LDS chunk.
//   sub-wave  (n <= 32) 64 / SEG problems per wavefront on SEG-lane segments
//           (SEG = 16 up to order 16, 32 above), the segment substitutions of
//           the sub-wave Cholesky kernels; x_j and dB_j reach lane i by
//           segment broadcasts, and dA leaves through the segments' LDS
//           blocks as one contiguous copy of the wavefront's problems.
// dB may be G itself (in place): at every scope an element of G is read
// before the same lane (or, at thread scope, the same workgroup after a
// barrier) writes that element of dB, so neither pointer is __restrict__.
#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"

namespace glass {
namespace {

// acc + (p * q + r * s) with both products rounded and no contraction: the
// (j, i) entry of dA forms the same two products in the other order, and
// addition commutes, so dA comes out bit-symmetric.
GLASS_DEV float sym_pair(float acc, float p, float q, float r, float s) {
#pragma clang fp contract(off)
    const float t = p * q + r * s;
    return acc + t;
}

// One right-hand side, every operand 16-byte aligned: the same arithmetic as
// adjoint_thread with no LDS.  Each lane loads its own problem's rows at or
// left of the diagonal, x and g, all issued before any is used, and stores
// dB and the rows of dA straight to memory, in pieces of AL floats: 4, 2 or 1
// as N allows (every row of every problem starts at a multiple of AL floats
// from the aligned base).  (dB may be G: a lane reads its g before it writes
// its dB.)  Entry (i, j) of dA is formed here as b_i x_j + x_i b_j for every
// j, which is the staged kernel's value of the (j, i) pair with the sum's
// terms swapped, so the result is the same bit for bit.
template <int AL>
GLASS_DEV void piece_get(float* v, const float* p) {
    if constexpr (AL == 4) {
        const f4_t x = *reinterpret_cast<const f4_t*>(p);
        v[0] = x[0], v[1] = x[1], v[2] = x[2], v[3] = x[3];
    } else if constexpr (AL == 2) {
        const float2 x = *reinterpret_cast<const float2*>(p);
        v[0] = x.x, v[1] = x.y;
    } else {
        v[0] = *p;
    }
}

template <int AL>
GLASS_DEV void piece_put(float* p, const float* v) {
    if constexpr (AL == 4)
        *reinterpret_cast<f4_t*>(p) = f4_t{v[0], v[1], v[2], v[3]};
    else if constexpr (AL == 2)
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    else
        *p = v[0];
}

template <int N>
__global__ void __launch_bounds__(512) adjoint_thread1(int batch, const float* __restrict__ L,
                                                       const float* __restrict__ X, const float* G, float* dB,
                                                       float* __restrict__ dA) {
    constexpr int AL = N % 4 == 0 ? 4 : N % 2 == 0 ? 2 : 1;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= batch) return;
    const float* Lp = L + p * (N * N);
    float a[N * (N + 1) / 2];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int t = 0; t <= i / AL; ++t) {
            float v[AL];
            piece_get<AL>(v, Lp + i * N + AL * t);
#pragma unroll
            for (int e = 0; e < AL; ++e)
                if (AL * t + e <= i) a[TI(i, AL * t + e)] = v[e];
        }
    float x[N], y[N];
#pragma unroll
    for (int t = 0; t < N / AL; ++t) {
        piece_get<AL>(x + AL * t, X + p * N + AL * t);
        piece_get<AL>(y + AL * t, G + p * N + AL * t);
    }
    float dinv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) dinv[i] = recip(a[TI(i, i)]);
    tri_fwd<N>(a, dinv, y);
    tri_bwd<N>(a, dinv, y);
#pragma unroll
    for (int t = 0; t < N / AL; ++t) piece_put<AL>(dB + p * N + AL * t, y + AL * t);
    float* Ap = dA + p * (N * N);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int t = 0; t < N / AL; ++t) {
            float o[AL];
#pragma unroll
            for (int e = 0; e < AL; ++e) o[e] = -0.5f * sym_pair(0.f, y[i], x[AL * t + e], x[i], y[AL * t + e]);
            piece_put<AL>(Ap + i * N + AL * t, o);
        }
}

template <int N>
__global__ void __launch_bounds__(512) adjoint_thread(int nrhs, int batch, const float* __restrict__ L,
                                                      const float* __restrict__ X, const float* G,
                                                      float* dB, float* __restrict__ dA) {
    extern __shared__ float lds[];
    constexpr int SZ = N * N, S = thread_stride(SZ);
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    const int Q = thread_stage_q_dev(nt, SZ);
    const int SBn = N * nrhs, SB = SBn | 1;
    float* gs = lds + Q * S;
    float* xs = gs + nt * SB;
    float a[N * (N + 1) / 2];
    float dinv[N];
    thread_load_tri<N>(a, L + p0 * SZ, lds, cnt, tid, nt);
#pragma unroll
    for (int i = 0; i < N; ++i) dinv[i] = recip(a[TI(i, i)]);
    const FastDiv fb = make_fastdiv(SBn);
    stage_in<2>(gs, G + p0 * SBn, cnt * SBn, fb, SB, tid, nt);
    stage_in<2>(xs, X + p0 * SBn, cnt * SBn, fb, SB, tid, nt);
    __syncthreads();
    const bool active = tid < cnt;
    if (active) {
        float* b = gs + tid * SB;
        for (int c = 0; c < nrhs; ++c) {
            float y[N];
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = b[i * nrhs + c];
            tri_fwd<N>(a, dinv, y);
            tri_bwd<N>(a, dinv, y);
#pragma unroll
            for (int i = 0; i < N; ++i) b[i * nrhs + c] = y[i];
        }
    }
    __syncthreads();
    stage_out(dB + p0 * SBn, gs, cnt * SBn, fb, SB, tid, nt);
    const FastDiv fa = make_fastdiv(SZ);
    for (int s = 0; s < cnt; s += Q) {
        const int qn = min(Q, cnt - s);
        if (tid >= s && tid < s + qn) {
            const float* b = gs + tid * SB;
            const float* x = xs + tid * SB;
            float* o = lds + (tid - s) * S;
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j) {
                    float v = 0.f;
                    for (int c = 0; c < nrhs; ++c)
                        v = sym_pair(v, b[i * nrhs + c], x[j * nrhs + c], x[i * nrhs + c], b[j * nrhs + c]);
                    o[i * N + j] = -0.5f * v;
                    o[j * N + i] = -0.5f * v;
                }
        }
        __syncthreads();
        stage_out(dA + (p0 + s) * SZ, lds, qn * SZ, fa, S, tid, nt);
        __syncthreads();
    }
}

template <int NB>
__global__ void __launch_bounds__(512) adjoint_wave(int n, int nrhs, int batch, const float* __restrict__ L,
                                                    const float* __restrict__ X, const float* G,
                                                    float* dB, float* __restrict__ dA, int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* buf = lds + (size_t)w * region;
    const float* Lg = L + p * n * n;
    const long long ob = p * n * nrhs;
    // the diagonal and the first column of g and x are issued with the rows;
    // each later column is loaded before the previous one's substitutions
    const int ro = (lane < n ? lane : 0) * nrhs;
    const float dg = diag_load(Lg, n, lane);
    float gn = G[ob + ro], xn = X[ob + ro];
    float a[NB];
    rows_load_lower<NB, true>(a, Lg, n, lane);
    const float myinv = diag_inv(dg, n, lane);
    float d[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) d[j] = 0.f;
    for (int c = 0; c < nrhs; ++c) {
        float acc = lane < n ? gn : 0.f;
        const float xc = lane < n ? xn : 0.f;
        if (c + 1 < nrhs) {
            gn = G[ob + ro + c + 1];
            xn = X[ob + ro + c + 1];
        }
        acc = wave_fwd<NB>(a, acc, myinv, lane);
        acc = wave_chunks_desc<NB>(a, buf, nullptr, false, n, lane, true, acc, myinv);
        if (lane < n) dB[ob + lane * nrhs + c] = acc;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const float xj = readlane(xc, j), bj = readlane(acc, j);
            d[j] = sym_pair(d[j], acc, xj, xc, bj);
        }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) d[j] *= -0.5f;
    const bool vec = (n & 3) == 0 && aligned16(dA);
    wave_chunks_desc<NB>(d, buf, dA + p * n * n, vec, n, lane, false, 0.f, 1.f);
}

template <int SEG, int NB, int J>
struct SegDa {
    // d[j] += dB_i x_j + x_i dB_j, x_j and dB_j broadcast from lane j of the segment
    static GLASS_DEV void run(float (&d)[NB], float b, float x) {
        const float xj = seg_bcast<SEG, J>(x), bj = seg_bcast<SEG, J>(b);
        d[J] = sym_pair(d[J], b, xj, x, bj);
        SegDa<SEG, NB, J + 1>::run(d, b, x);
    }
};
template <int SEG, int NB>
struct SegDa<SEG, NB, NB> {
    static GLASS_DEV void run(float (&)[NB], float, float) {}
};

template <int SEG, int NB>
__global__ void __launch_bounds__(512) adjoint_seg(int n, int nrhs, int batch, const float* __restrict__ L,
                                                   const float* __restrict__ X, const float* G,
                                                   float* dB, float* __restrict__ dA, int region) {
    extern __shared__ float lds[];
    constexpr int PPW = 64 / SEG;
    const int w = wave_index(), lane = threadIdx.x & 63;
    const int s = lane / SEG, i = lane % SEG;
    const long long p0 = ((long long)blockIdx.x * (blockDim.x >> 6) + w) * PPW;
    if (p0 >= batch) return;
    const int np = (int)min((long long)PPW, (long long)batch - p0);
    const bool row = s < np && i < n;
    float* buf = lds + (size_t)w * region;
    float* sb = buf + s * NB * (NB + 4);
    const float* Lb = L + p0 * n * n;
    // the diagonal and the first column of g and x are issued with the rows
    // (a lane without a row reads its wave's first problem's entries); each
    // later column is loaded before the previous one's substitutions
    const long long ob = (p0 + s) * n * nrhs, ob_safe = row ? ob + i * nrhs : p0 * n * nrhs;
    const float dg = Lb[row ? s * n * n + i * n + i : 0];
    float gn = G[ob_safe], xn = X[ob_safe];
    float a[NB];
    seg_load_rows<NB, true>(a, Lb, np, n, s, i);
    const float myinv = row ? recip(dg) : 1.f;
    seg_rows_to_lds<NB>(a, sb, i);
    wave_sync();
    seg_scale_row<NB>(a, myinv);
    float d[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) d[j] = 0.f;
    for (int c = 0; c < nrhs; ++c) {
        float y[1] = {(row ? gn : 0.f) * myinv};
        const float xc = row ? xn : 0.f;
        if (c + 1 < nrhs) {
            gn = G[ob_safe + (row ? c + 1 : 0)];
            xn = X[ob_safe + (row ? c + 1 : 0)];
        }
        SegFwdL<SEG, NB, 0, 1>::run(a, y);
        seg_bwd<SEG, NB, 1, true>(sb, i, y, myinv);
        if (row) dB[ob + i * nrhs + c] = y[0];
        SegDa<SEG, NB, 0>::run(d, y[0], xc);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) d[j] *= -0.5f;
    wave_sync();  // the segment blocks held L for the backward sweeps
    seg_rows_to_lds<NB>(d, sb, i);
    wave_sync();
    seg_store_L<NB>(dA + p0 * n * n, buf, np, n, (n & 3) == 0 && aligned16(dA), lane);
}

inline int bucket8(int n) { return ((n + 7) / 8) * 8; }

}  // namespace

int launch_posv_adjoint(const Shape& sh, const Geometry& g, int batch, const float* L, const float* X,
                        const float* G, float* dB, float* dA, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n, r = sh.nrhs;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD) {
        auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
        if (r == 1 && al16(L) && al16(X) && al16(G) && al16(dB) && al16(dA)) {
            switch (n) {
#define CASE1(N) \
    case N: hipLaunchKernelGGL(adjoint_thread1<N>, grid, block, 0, st, batch, L, X, G, dB, dA); return (int)hipGetLastError();
                CASE1(1) CASE1(2) CASE1(3) CASE1(4) CASE1(5) CASE1(6) CASE1(7) CASE1(8) CASE1(9) CASE1(10) CASE1(11)
                CASE1(12) CASE1(13) CASE1(14) CASE1(15) CASE1(16)
#undef CASE1
            }
        }
        switch (n) {
#define CASE(N) \
    case N: hipLaunchKernelGGL(adjoint_thread<N>, grid, block, g.lds_bytes, st, r, batch, L, X, G, dB, dA); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12)
            CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_WAVE) {
        const int region = (int)wave_region_floats(sh);
        switch (bucket8(n)) {
#define CASE(NB)                                                                                                 \
    case NB:                                                                                                     \
        hipLaunchKernelGGL(adjoint_wave<NB>, grid, block, g.lds_bytes, st, n, r, batch, L, X, G, dB, dA, region); \
        break;
            CASE(8) CASE(16) CASE(24) CASE(32) CASE(40) CASE(48) CASE(56) CASE(64)
#undef CASE
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_SUBWAVE) {
        const int region = (int)subwave_region_floats(n);
        switch (subwave_nb(n)) {
#define CASE(SEG, NB)                                                                                               \
    case NB:                                                                                                        \
        hipLaunchKernelGGL((adjoint_seg<SEG, NB>), grid, block, g.lds_bytes, st, n, r, batch, L, X, G, dB, dA, region); \
        break;
            CASE(16, 4) CASE(16, 8) CASE(16, 12) CASE(16, 16) CASE(32, 24) CASE(32, 32)
#undef CASE
        default: return (int)hipErrorInvalidValue;
        }
    } else {
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace glass
