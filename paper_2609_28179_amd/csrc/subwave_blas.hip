// subwave_blas.hip -- sub-wave scope of GEMM and GEMV for orders up to 16:
// four problems per wavefront, one per 16-lane DPP row (the packing of
// Sec. IV-C below the warp granule).
//
// Lane (s, i) = (lane / 16, lane % 16) holds row i of problem s's A (and, for
// GEMM, row i of its B).  C_ij = sum_t A_it B_tj takes B_tj from lane t of
// the row with DPP row_newbcast folded into the v_fmac, so each lane issues
// one v_fmac per (t, j): 256 per wavefront at order 16, i.e. 64 per problem,
// against 4096 FMAs of work per problem.  GEMV broadcasts x_t the same way.
// The wavefront's four problems are adjacent in the batch, so one buffer
// descriptor covers their rows; rows are read with 16-byte buffer loads when
// the row length is a multiple of 4 (buffer loads need only 4-byte
// alignment) and element-wise otherwise.
#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {
namespace {

// Elements [0, len) of the row at float offset `off` of the descriptor into
// v (zero past len, and everywhere when !row).  vec: len % 4 == 0.
template <int NB>
GLASS_DEV void seg_row_load(float (&v)[NB], __amdgpu_buffer_rsrc_t rs, int off, int len, bool row, bool vec) {
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
        f4_t x = {0.f, 0.f, 0.f, 0.f};
        if (row && 4 * t < len) {
            if (vec) {
                x = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off * 4, t * 16, 0));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * t + e < len)
                        x[e] = __builtin_bit_cast(float,
                                                  __builtin_amdgcn_raw_buffer_load_b32(rs, (off + 4 * t + e) * 4, 0, 0));
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) v[4 * t + e] = x[e];
    }
}

// v read through DPP afterwards: a VALU write (the zero padding) needs two
// wait states before a DPP read, which the compiler does not insert for
// inline asm, so each register passes an s_nop 1 tied to it.
template <int NB>
GLASS_DEV void dpp_ready(float (&v)[NB]) {
#pragma unroll
    for (int j = 0; j < NB; ++j) asm volatile("s_nop 1" : "+v"(v[j]));
}

template <int NB, int T>
struct GemmStep {
    static GLASS_DEV void run(float (&acc)[NB], const float (&a)[NB], const float (&b)[NB]) {
#pragma unroll
        for (int j = 0; j < NB; ++j) fmac_bcast<T>(acc[j], b[j], a[T]);
        GemmStep<NB, T + 1>::run(acc, a, b);
    }
};
template <int NB>
struct GemmStep<NB, NB> {
    static GLASS_DEV void run(float (&)[NB], const float (&)[NB], const float (&)[NB]) {}
};

template <int NB, int T>
struct GemvStep {
    static GLASS_DEV void run(float& acc, const float (&a)[NB], float xv) {
        fmac_bcast<T>(acc, xv, a[T]);
        GemvStep<NB, T + 1>::run(acc, a, xv);
    }
};
template <int NB>
struct GemvStep<NB, NB> {
    static GLASS_DEV void run(float&, const float (&)[NB], float) {}
};

// NB: max(n, k) rounded up to 4.  vec: n % 4 == 0 and C 16-byte aligned.
template <int NB>
__global__ void __launch_bounds__(512) gemm_seg(int m, int n, int k, int batch, float alpha,
                                                const float* __restrict__ A, const float* __restrict__ B, float beta,
                                                float* __restrict__ C, int vec) {
    const int w = wave_index(), lane = threadIdx.x & 63, s = lane >> 4, i = lane & 15;
    const long long p0 = ((long long)blockIdx.x * (blockDim.x >> 6) + w) * 4;
    if (p0 >= batch) return;
    const int np = (int)min(4LL, (long long)batch - p0);
    const bool act = s < np;
    const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(A + p0 * m * k, (uint32_t)(np * m * k) * 4u);
    const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(B + p0 * k * n, (uint32_t)(np * k * n) * 4u);
    float a[NB], b[NB], acc[NB];
    seg_row_load<NB>(a, ra, s * m * k + i * k, k, act && i < m, (k & 3) == 0);
    seg_row_load<NB>(b, rb, s * k * n + i * n, n, act && i < k, (n & 3) == 0);
    dpp_ready<NB>(b);
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = 0.f;
    GemmStep<NB, 0>::run(acc, a, b);
    if (!(act && i < m)) return;
    float* Cr = C + (p0 + s) * m * n + i * n;
    if (vec) {
#pragma unroll
        for (int t = 0; t < NB / 4; ++t) {
            if (4 * t < n) {
                f4_t o;
                if (beta != 0.f) {
                    const f4_t c0 = *reinterpret_cast<const f4_t*>(Cr + 4 * t);
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = fmaf(beta, c0[e], alpha * acc[4 * t + e]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = alpha * acc[4 * t + e];
                }
                *reinterpret_cast<f4_t*>(Cr + 4 * t) = o;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < n) Cr[j] = beta != 0.f ? fmaf(beta, Cr[j], alpha * acc[j]) : alpha * acc[j];
    }
}

// NB: n rounded up to 4.
template <int NB>
__global__ void __launch_bounds__(512) gemv_seg(int m, int n, int batch, float alpha, const float* __restrict__ A,
                                                const float* __restrict__ x, float beta, float* __restrict__ y) {
    const int w = wave_index(), lane = threadIdx.x & 63, s = lane >> 4, i = lane & 15;
    const long long p0 = ((long long)blockIdx.x * (blockDim.x >> 6) + w) * 4;
    if (p0 >= batch) return;
    const int np = (int)min(4LL, (long long)batch - p0);
    const bool act = s < np;
    const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(A + p0 * m * n, (uint32_t)(np * m * n) * 4u);
    float a[NB];
    seg_row_load<NB>(a, ra, s * m * n + i * n, n, act && i < m, (n & 3) == 0);
    float xv = (act && i < n) ? x[(p0 + s) * n + i] : 0.f;
    asm volatile("s_nop 1" : "+v"(xv));
    float acc = 0.f;
    GemvStep<NB, 0>::run(acc, a, xv);
    if (act && i < m) {
        float* yr = y + (p0 + s) * m + i;
        *yr = beta != 0.f ? fmaf(beta, *yr, alpha * acc) : alpha * acc;
    }
}

}  // namespace

int launch_blas_subwave(const Shape& sh, const Geometry& g, int batch, float alpha, const float* A, const float* Bx,
                        float beta, float* Cy, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (sh.op == GLASS_OP_GEMM) {
        const int mx = sh.n > sh.k ? sh.n : sh.k;
        if (sh.trans != 0 || sh.m > 16 || mx > 16) return (int)hipErrorInvalidValue;
        const int vec = (sh.n & 3) == 0 && (reinterpret_cast<uintptr_t>(Cy) & 15) == 0;
        switch ((mx + 3) / 4) {
#define X(Q) \
    case Q: hipLaunchKernelGGL(gemm_seg<4 * Q>, grid, block, 0, st, sh.m, sh.n, sh.k, batch, alpha, A, Bx, beta, Cy, vec); break;
            X(1) X(2) X(3) X(4)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
        return (int)hipGetLastError();
    }
    if (sh.m > 16 || sh.n > 16) return (int)hipErrorInvalidValue;
    switch ((sh.n + 3) / 4) {
#define X(Q) \
    case Q: hipLaunchKernelGGL(gemv_seg<4 * Q>, grid, block, 0, st, sh.m, sh.n, batch, alpha, A, Bx, beta, Cy); break;
        X(1) X(2) X(3) X(4)
#undef X
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace glass
