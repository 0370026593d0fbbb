// gemv.hip -- batched y = alpha A x + beta y (Sec. III-B, BLAS L2) at the
// three scopes of Sec. III-A.  The thread and workgroup variants, and the
// wave variant of rectangular and small problems, stage A through LDS with
// coalesced loads of the contiguous batch span; the dot products then read
// A rows at an odd LDS stride (conflict-free) and x as broadcasts.
//   thread     (m = n <= 16) one problem per lane, A staged in passes.
//   wave       one problem per wavefront; lane i computes y_i, or (square,
//              orders 17 .. 64) A stays in registers and the rows are
//              reduced across lanes with DPP, no LDS.
//   workgroup  one problem per workgroup; T/64 lanes share a row and their
//              partial sums are combined through LDS.
#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {
namespace {

__device__ __forceinline__ int stage_q(int threads, int elems) {
    int s = thread_stride(elems);
    int q = kStagePassFloats / s;
    if (q < 1) q = 1;
    return q < threads ? q : threads;
}

template <int N>
__global__ void __launch_bounds__(512) gemv_thread(int batch, float alpha, const float* __restrict__ A,
                                                   const float* __restrict__ x, float beta, float* __restrict__ y) {
    extern __shared__ float lds[];
    // A at the stride thread_stride(SZ), rows read with the widest LDS
    // accesses their alignment allows (RA floats)
    constexpr int SZ = N * N, S = thread_stride(SZ), SV = N | 1, RA = N % 4 == 0 ? 4 : N % 2 == 0 ? 2 : 1;
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    const int Q = stage_q(nt, SZ);
    float* xs = lds + Q * S;
    float* ys = xs + nt * SV;
    const FastDiv fv = make_fastdiv(N);
    stage_in<2>(xs, x + p0 * N, cnt * N, fv, SV, tid, nt);
    __syncthreads();
    float xr[N];
    if (tid < cnt) {
#pragma unroll
        for (int j = 0; j < N; ++j) xr[j] = xs[tid * SV + j];
    }
    const FastDiv fa = make_fastdiv(SZ);
    for (int s = 0; s < cnt; s += Q) {
        const int qn = min(Q, cnt - s);
        stage_in<ThreadU<N>::v>(lds, A + (p0 + s) * SZ, qn * SZ, fa, S, tid, nt);
        __syncthreads();
        if (tid >= s && tid < s + qn) {
            const float* a = lds + (tid - s) * S;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float ar[N];
                lds_row_get<N, RA>(ar, a + i * N);
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < N; ++j) acc = fmaf(ar[j], xr[j], acc);
                ys[tid * SV + i] = alpha * acc;
            }
        }
        __syncthreads();
    }
    stage_out_beta(y + p0 * N, ys, cnt * N, fv, SV, beta, tid, nt);
}

template <int U>
__global__ void __launch_bounds__(512) gemv_wave(int m, int n, int batch, float alpha, const float* __restrict__ A,
                                                 const float* __restrict__ x, float beta, float* __restrict__ y,
                                                 int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* As = lds + (size_t)w * region;
    const int s = n | 1;
    float* xs = As + ((m * s + 3) & ~3);
    stage_in<U>(As, A + p * m * n, m * n, make_fastdiv(n), s, lane, 64);
    for (int j = lane; j < n; j += 64) xs[j] = x[p * n + j];
    wave_sync();
    if (lane < m) {
        float acc = 0.f;
        for (int j = 0; j < n; ++j) acc = fmaf(As[lane * s + j], xs[j], acc);
        float out = alpha * acc;
        if (beta != 0.f) out = fmaf(beta, y[p * m + lane], out);
        y[p * m + lane] = out;
    }
}

__global__ void __launch_bounds__(256) gemv_wg(int m, int n, int batch, int pack, float alpha,
                                               const float* __restrict__ A, const float* __restrict__ x, float beta,
                                               float* __restrict__ y) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const int s = n | 1;
    float* xs = lds + ((m * s + 3) & ~3);
    float* part = xs + ((n + 3) & ~3);
    const int parts = nt >> 6, row = tid & 63, pi = tid >> 6;
    const FastDiv fd = make_fastdiv(n);
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        stage_in<4>(lds, A + p * m * n, m * n, fd, s, tid, nt);
        for (int j = tid; j < n; j += nt) xs[j] = x[p * n + j];
        __syncthreads();
        if (row < m) {
            float acc = 0.f;
            for (int j = pi; j < n; j += parts) acc = fmaf(lds[row * s + j], xs[j], acc);
            part[pi * 64 + row] = acc;
        }
        __syncthreads();
        if (pi == 0 && row < m) {
            float acc = part[row];
            for (int t = 1; t < parts; ++t) acc += part[t * 64 + row];
            float out = alpha * acc;
            if (beta != 0.f) out = fmaf(beta, y[p * m + row], out);
            y[p * m + row] = out;
        }
        __syncthreads();
    }
}

// Square orders 12, 16 and 17 .. 64 at wave scope, with no LDS: one problem
// per wavefront, padded to N = 16, 32 or 64.  Every byte of A is loaded once into
// registers by instructions that cover whole consecutive rows: lane
// (g, c) = (lane / LPR, lane % LPR) takes row RPI k + g, columns
// 4 c .. 4 c + 3 in instruction k (LPR = N / 4 lanes per row, RPI = 64 / LPR
// rows per instruction, K = N / RPI instructions; rows and columns past n
// are zero), and its products with its fixed piece x[4 c .. 4 c + 3] give one
// partial sum of that row per instruction.  The LPR lanes of a row group
// then reduce their K partials with a transposing butterfly: each exchange
// step pairs a lane with one whose index differs in the step's bit (DPP
// row_mirror, row_half_mirror and quad permutations), the lane with the bit
// clear keeps the lower half of its values and the other the upper half,
// each adding its partner's copy.  Afterwards lane c of a group holds the
// whole dot product of row RPI k + g for k = c (N = 64) or k = c / 2 (N = 32;
// lanes c and c ^ 1 agree).  At N = 16 a row is one instruction's four lanes
// (K = 1) and two quad exchanges sum them.  VEC: n % 4 == 0 with A and x
// 16-byte aligned; FULL: besides, n == N (no padding, no masks).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}

// One butterfly step over M values: pairs (v[j], v[j + M / 2]); `hi` is the
// lane's bit of the step.
template <int M, int CTRL>
__device__ __forceinline__ void bfly_step(float (&v)[16], bool hi) {
    float send[M / 2];
#pragma unroll
    for (int j = 0; j < M / 2; ++j) send[j] = hi ? v[j] : v[j + M / 2];
#pragma unroll
    for (int j = 0; j < M / 2; ++j) v[j] = (hi ? v[j + M / 2] : v[j]) + dpp_mov<CTRL>(send[j]);
}

constexpr int kDppRowMirror = 0x140, kDppHalfMirror = 0x141, kDppXor3 = 0x1B, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

template <int N, bool VEC, bool FULL>
__global__ void __launch_bounds__(512) gemv_wave_dpp(int n, int batch, float alpha, const float* __restrict__ A,
                                                     const float* __restrict__ x, float beta,
                                                     float* __restrict__ y) {
    static_assert(N == 16 || N == 32 || N == 64, "padded orders 16, 32 and 64");
    static_assert(VEC || !FULL, "the unpadded form loads 16-byte pieces");
    if (FULL) n = N;
    constexpr int LPR = N / 4, RPI = 64 / LPR, K = N / RPI;
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    const int g = lane / LPR, c = lane % LPR;
    const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(A + p * n * n, (uint32_t)(n * n * 4));
    const __amdgpu_buffer_rsrc_t rx = buffer_rsrc(x + p * n, (uint32_t)(n * 4));
    f4_t a[K], xv = {0.f, 0.f, 0.f, 0.f};
    if (VEC) {
        const bool col = FULL || 4 * c < n;
        if (col) xv = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rx, 16 * c, 0, 0));
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int row = RPI * k + g;
            a[k] = f4_t{0.f, 0.f, 0.f, 0.f};
            if (FULL || (col && row < n))
                a[k] = __builtin_bit_cast(f4_t,
                                          __builtin_amdgcn_raw_buffer_load_b128(ra, (row * n + 4 * c) * 4, 0, 0));
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * c + e < n)
                xv[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, (4 * c + e) * 4, 0, 0));
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int row = RPI * k + g;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a[k][e] = 0.f;
                if (row < n && 4 * c + e < n)
                    a[k][e] = __builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(ra, (row * n + 4 * c + e) * 4, 0, 0));
            }
        }
    }
    float v[16];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float t = a[k][0] * xv[0];
        t = fmaf(a[k][1], xv[1], t);
        t = fmaf(a[k][2], xv[2], t);
        v[k] = fmaf(a[k][3], xv[3], t);
    }
    int row;
    bool owner = true;
    if (N == 64) {
        bfly_step<16, kDppRowMirror>(v, (c & 8) != 0);
        bfly_step<8, kDppHalfMirror>(v, (c & 4) != 0);
        bfly_step<4, kDppXor3>(v, (c & 2) != 0);
        bfly_step<2, kDppXor1>(v, (c & 1) != 0);
        row = RPI * c + g;
    } else if (N == 32) {
        bfly_step<4, kDppHalfMirror>(v, (c & 4) != 0);
        bfly_step<2, kDppXor3>(v, (c & 2) != 0);
        v[0] += dpp_mov<kDppXor1>(v[0]);
        row = RPI * (c >> 1) + g;
        owner = (c & 1) == 0;
    } else {
        v[0] += dpp_mov<kDppXor1>(v[0]);
        v[0] += dpp_mov<kDppXor2>(v[0]);
        row = g;
        owner = c == 0;
    }
    if (owner && (FULL || row < n)) {
        float out = alpha * v[0];
        if (beta != 0.f) out = fmaf(beta, y[p * n + row], out);
        y[p * n + row] = out;
    }
}

}  // namespace

int launch_gemv(const Shape& sh, const Geometry& g, int batch, float alpha, const float* A, const float* x,
                float beta, float* y, void* stream) {
    if (g.scope == GLASS_SCOPE_SUBWAVE) return launch_blas_subwave(sh, g, batch, alpha, A, x, beta, y, stream);
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD) {
        switch (sh.n) {
#define X(N) \
    case N: hipLaunchKernelGGL(gemv_thread<N>, grid, block, g.lds_bytes, st, batch, alpha, A, x, beta, y); break;
            X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
    } else if (g.scope == GLASS_SCOPE_WAVE && gemv_uses_dpp(sh)) {
        const bool vec = sh.n % 4 == 0 && (uintptr_t)A % 16 == 0 && (uintptr_t)x % 16 == 0;
        const int pad = sh.n <= 16 ? 16 : sh.n <= 32 ? 32 : 64;
        const bool full = vec && sh.n == pad;
#define X(N, V, F)                                                                                            \
    if (pad == N && vec == V && full == F)                                                                    \
        hipLaunchKernelGGL((gemv_wave_dpp<N, V, F>), grid, block, 0, st, sh.n, batch, alpha, A, x, beta, y);
        X(16, true, true) X(16, true, false) X(16, false, false) X(32, true, true) X(32, true, false)
        X(32, false, false) X(64, true, true) X(64, true, false) X(64, false, false)
#undef X
    } else if (g.scope == GLASS_SCOPE_WAVE) {
        const int mn = sh.m * sh.n;
        const int u = mn <= 512 ? 2 : mn <= 1024 ? 4 : mn <= 2048 ? 8 : 16;
        switch (u) {
#define X(U)                                                                                                  \
    case U:                                                                                                   \
        hipLaunchKernelGGL(gemv_wave<U>, grid, block, g.lds_bytes, st, sh.m, sh.n, batch, alpha, A, x, beta, y, \
                           (int)region_floats(sh));                                                           \
        break;
            X(2) X(4) X(8) X(16)
#undef X
        }
    } else {
        hipLaunchKernelGGL(gemv_wg, grid, block, g.lds_bytes, st, sh.m, sh.n, batch, g.pack, alpha, A, x, beta, y);
    }
    return (int)hipGetLastError();
}

}  // namespace glass
