// gemv.hip -- batched y = alpha A x + beta y (Sec. III-B, BLAS L2) at the
// three scopes of Sec. III-A.  Every variant stages A through LDS with
// coalesced loads of the contiguous batch span; the dot products then read
// A rows at an odd LDS stride (conflict-free) and x as broadcasts.
//   thread     (m = n <= 16) one problem per lane, A staged in passes.
//   wave       one problem per wavefront, lane i computes y_i.
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
