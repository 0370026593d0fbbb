// gemm.hip -- batched C = alpha A B + beta C (Sec. III-B, BLAS L3) at the
// three scopes of Sec. III-A.
//
//   thread     (m = n = k = N <= 12) one problem per lane: B is staged
//              through LDS into VGPRs, A is staged whole and each lane turns
//              its A rows into C rows in place; the epilogue is fused into the
//              coalesced store.
//   wave / wg  max(m, n, k) >= 16: FP32 MFMA (v_mfma_f32_16x16x4_f32), the
//              operand fragments loaded straight from global memory (no LDS):
//              lane l = 16q + r holds A[row r][k0 + 4q .. k0 + 4q + 3] as one
//              16-byte load and feeds component c to MFMA step c, so step c
//              contracts k in {k0 + c, k0 + 4 + c, k0 + 8 + c, k0 + 12 + c};
//              the matching B fragment is B[k0 + 4q + c][col r].  The wave
//              scope runs one problem per wavefront; the workgroup scope
//              splits the 16-wide column tiles of one problem over its waves.
//   small n    max(m, n, k) < 16 at wave / wg scope: operands staged in LDS,
//              lanes over output elements.
#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int stage_q(int threads, int elems) {
    int s = thread_stride(elems);
    int q = kStagePassFloats / s;
    if (q < 1) q = 1;
    return q < threads ? q : threads;
}

// ------------------------------------------------------------ thread scope --
template <int N>
__global__ void __launch_bounds__(512) gemm_thread(int batch, float alpha, const float* __restrict__ A,
                                                   const float* __restrict__ B, float beta, float* __restrict__ C) {
    extern __shared__ float lds[];
    // problems at the stride thread_stride(SZ); each lane moves its own rows
    // with the widest LDS accesses their alignment allows (RA floats)
    constexpr int SZ = N * N, S = thread_stride(SZ), RA = N % 4 == 0 ? 4 : N % 2 == 0 ? 2 : 1;
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    const FastDiv fd = make_fastdiv(SZ);
    float b[SZ];
    const int Q = stage_q(nt, SZ);
    for (int s = 0; s < cnt; s += Q) {
        const int qn = min(Q, cnt - s);
        stage_in<ThreadU<N>::v>(lds, B + (p0 + s) * SZ, qn * SZ, fd, S, tid, nt);
        __syncthreads();
        if (tid >= s && tid < s + qn) lds_row_get<SZ, (S % 4 == 0 ? 4 : 1)>(b, lds + (tid - s) * S);
        __syncthreads();
    }
    stage_in<ThreadU<N>::v>(lds, A + p0 * SZ, cnt * SZ, fd, S, tid, nt);
    __syncthreads();
    if (tid < cnt) {
        float* a = lds + tid * S;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float ar[N], cr[N];
            lds_row_get<N, RA>(ar, a + i * N);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                float c = 0.f;
#pragma unroll
                for (int k = 0; k < N; ++k) c = fmaf(ar[k], b[k * N + j], c);
                cr[j] = alpha * c;
            }
            lds_row_put<N, RA>(a + i * N, cr);
        }
    }
    __syncthreads();
    stage_out_beta(C + p0 * SZ, lds, cnt * SZ, fd, S, beta, tid, nt);
}

// ------------------------------------------------- small n, wave / wg scope --
// TA / TBT: op(A) = A^T (A stored k x m) / op(B) = B^T (B stored n x k).
// Operands are staged as stored (rows padded to an odd stride).
template <bool TA, bool TBT>
GLASS_DEV void gemm_small_problem(int m, int n, int k, float alpha, const float* __restrict__ Ag,
                                  const float* __restrict__ Bg, float beta, float* __restrict__ Cg, float* As,
                                  int tid, int nt, bool wave) {
    const int arows = TA ? k : m, acols = TA ? m : k;
    const int brows = TBT ? n : k, bcols = TBT ? k : n;
    const int sa = acols | 1, sb = bcols | 1;
    float* Bs = As + ((arows * sa + 3) & ~3);
    stage_in<2>(As, Ag, arows * acols, make_fastdiv(acols), sa, tid, nt);
    stage_in<2>(Bs, Bg, brows * bcols, make_fastdiv(bcols), sb, tid, nt);
    if (wave) wave_sync(); else __syncthreads();
    const FastDiv fn = make_fastdiv(n);
    for (int e = tid; e < m * n; e += nt) {
        const int i = (int)fdiv((uint32_t)e, fn), j = e - i * n;
        float c = 0.f;
        for (int p = 0; p < k; ++p) {
            const float av = TA ? As[p * sa + i] : As[i * sa + p];
            const float bv = TBT ? Bs[j * sb + p] : Bs[p * sb + j];
            c = fmaf(av, bv, c);
        }
        float out = alpha * c;
        if (beta != 0.f) out = fmaf(beta, Cg[e], out);
        Cg[e] = out;
    }
}

template <bool TA, bool TBT>
__global__ void __launch_bounds__(512) gemm_small_wave(int m, int n, int k, int batch, float alpha,
                                                       const float* __restrict__ A, const float* __restrict__ B,
                                                       float beta, float* __restrict__ C, int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    gemm_small_problem<TA, TBT>(m, n, k, alpha, A + p * m * k, B + p * k * n, beta, C + p * m * n, lds + (size_t)w * region,
                       lane, 64, true);
}

template <bool TA, bool TBT>
__global__ void __launch_bounds__(256) gemm_small_wg(int m, int n, int k, int batch, int pack, float alpha,
                                                     const float* __restrict__ A, const float* __restrict__ B,
                                                     float beta, float* __restrict__ C) {
    extern __shared__ float lds[];
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        gemm_small_problem<TA, TBT>(m, n, k, alpha, A + p * m * k, B + p * k * n, beta, C + p * m * n, lds, threadIdx.x,
                           blockDim.x, false);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- MFMA path --
// One wave computes the 16x16 column tiles jt = jt0, jt0 + jstep, ... of one
// problem.  TB = ceil(max(m, n, k) / 16) <= 4 bounds the fragment arrays.
// Every A and B fragment the wave needs is loaded before the first MFMA, so
// all of a problem's loads are in flight together.  JJ bounds the number of
// column tiles one wave owns (TB at wave scope, 1 at workgroup scope where
// the T(n)/64 waves split the ceil(n/16) <= T(n)/64 column tiles).
// TA / TBT select transposed operands (A stored k x m, B stored n x k); the
// transposed A fragment is read element-wise (consecutive lanes take
// consecutive rows i, so the loads stay coalesced).
// Wave scope with a staged output (STG: n % 4 == 0, C 16-byte aligned): all
// column tiles of one 16-row block are accumulated, written to LDS in the
// MFMA output layout and stored back as whole rows with 16-byte stores (the
// output layout alone writes 64-byte half lines).
template <int TB, bool TA, bool TBT>
GLASS_DEV void mfma_store_block(int m, int n, float alpha, float beta, float* __restrict__ Cg, const float* stg,
                                int it, int lane) {
    const int n4 = n >> 2;
    const int rows = min(16, m - it * 16);
    for (int g = lane; g < 16 * n4; g += 64) {
        const int rr = g / n4, c4 = g - rr * n4;
        if (rr < rows) {
            const f4_t v = *reinterpret_cast<const f4_t*>(stg + rr * kGemmStageStride + 4 * c4);
            f4_t* dst = reinterpret_cast<f4_t*>(Cg + (size_t)(it * 16 + rr) * n) + c4;
            f4_t out;
            if (beta != 0.f) {
                const f4_t c0 = *dst;
#pragma unroll
                for (int e = 0; e < 4; ++e) out[e] = fmaf(beta, c0[e], alpha * v[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) out[e] = alpha * v[e];
            }
            *dst = out;
        }
    }
}

template <int TB, bool VEC, int JJ, bool TA = false, bool TBT = false, bool STG = false>
GLASS_DEV void mfma_problem(int m, int n, int k, float alpha, const float* __restrict__ Ag,
                            const float* __restrict__ Bg, float beta, float* __restrict__ Cg, int lane, int jt0,
                            int jstep, float* stg = nullptr) {
    const int q = lane >> 4, r = lane & 15;
    const int MT = (m + 15) >> 4, NT = (n + 15) >> 4, KT = (k + 15) >> 4;
    float af[TB][TB][4];
#pragma unroll
    for (int it = 0; it < TB; ++it) {
        const int i = it * 16 + r;
#pragma unroll
        for (int kb = 0; kb < TB; ++kb) {
            const int k0 = kb * 16 + 4 * q;
            const bool in = it < MT && kb < KT && i < m;
            if (TA) {
#pragma unroll
                for (int c = 0; c < 4; ++c) af[it][kb][c] = (in && k0 + c < k) ? Ag[(k0 + c) * m + i] : 0.f;
            } else if (VEC) {
                floatx4 v = {0.f, 0.f, 0.f, 0.f};
                if (in && k0 < k) v = *reinterpret_cast<const floatx4*>(Ag + i * k + k0);
#pragma unroll
                for (int c = 0; c < 4; ++c) af[it][kb][c] = v[c];
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) af[it][kb][c] = (in && k0 + c < k) ? Ag[i * k + k0 + c] : 0.f;
            }
        }
    }
    float bf[JJ][TB][4];
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
        const int j = (jt0 + jj * jstep) * 16 + r;
#pragma unroll
        for (int kb = 0; kb < TB; ++kb)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int kk = kb * 16 + 4 * q + c;
                bf[jj][kb][c] = (kb < KT && kk < k && j < n) ? (TBT ? Bg[j * k + kk] : Bg[kk * n + j]) : 0.f;
            }
    }
    if (STG) {
#pragma unroll
        for (int it = 0; it < TB; ++it) {
            if (it < MT) {
                floatx4 acc[JJ];
#pragma unroll
                for (int jj = 0; jj < JJ; ++jj) {
                    acc[jj] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < TB; ++kb) {
                        if (kb < KT) {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                acc[jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[it][kb][c], bf[jj][kb][c], acc[jj],
                                                                               0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int jj = 0; jj < JJ; ++jj)
                    if (jj < NT) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) stg[(4 * q + e) * kGemmStageStride + jj * 16 + r] = acc[jj][e];
                    }
                wave_sync();
                mfma_store_block<TB, TA, TBT>(m, n, alpha, beta, Cg, stg, it, lane);
                wave_sync();
            }
        }
        return;
    }
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
        const int jt = jt0 + jj * jstep;
        const int j = jt * 16 + r;
        if (jt < NT) {
#pragma unroll
            for (int it = 0; it < TB; ++it) {
                if (it < MT) {
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < TB; ++kb) {
                        if (kb < KT) {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[it][kb][c], bf[jj][kb][c], acc, 0, 0, 0);
                        }
                    }
                    if (j < n) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int row = it * 16 + 4 * q + e;
                            if (row < m) {
                                float out = alpha * acc[e];
                                if (beta != 0.f) out = fmaf(beta, Cg[row * n + j], out);
                                Cg[row * n + j] = out;
                            }
                        }
                    }
                }
            }
        }
    }
}

// The A fragments of row block `it` (all TB k-blocks), zero outside m x k.
template <int TB, bool VEC, bool TA>
GLASS_DEV void mfma_a_rows(float (&af)[TB][4], int m, int k, const float* __restrict__ Ag, int it, int q, int r) {
    const int MT = (m + 15) >> 4, KT = (k + 15) >> 4;
    const int i = it * 16 + r;
#pragma unroll
    for (int kb = 0; kb < TB; ++kb) {
        const int k0 = kb * 16 + 4 * q;
        const bool in = it < MT && kb < KT && i < m;
        if (TA) {
#pragma unroll
            for (int c = 0; c < 4; ++c) af[kb][c] = (in && k0 + c < k) ? Ag[(k0 + c) * m + i] : 0.f;
        } else if (VEC) {
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (in && k0 < k) v = *reinterpret_cast<const floatx4*>(Ag + i * k + k0);
#pragma unroll
            for (int c = 0; c < 4; ++c) af[kb][c] = v[c];
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) af[kb][c] = (in && k0 + c < k) ? Ag[i * k + k0 + c] : 0.f;
        }
    }
}

// Wave scope with a staged output at TB = 4 (orders 49..64): the B fragments
// of every column tile stay in VGPRs while A streams in by 16-row block,
// each block's fragments loaded before the previous block's products.  A
// block's products then run while the next block's loads are in flight and
// its stores overlap them; holding one A block at a time (two with the
// prefetch) instead of all four keeps the wave within 128 VGPRs, i.e. four
// waves per SIMD, so 4096 problems run in one round of waves.
template <int TB, bool VEC, bool TA, bool TBT>
GLASS_DEV void mfma_problem_rows(int m, int n, int k, float alpha, const float* __restrict__ Ag,
                                 const float* __restrict__ Bg, float beta, float* __restrict__ Cg, int lane,
                                 float* stg) {
    const int q = lane >> 4, r = lane & 15;
    const int MT = (m + 15) >> 4, NT = (n + 15) >> 4, KT = (k + 15) >> 4;
    float af[2][TB][4];
    mfma_a_rows<TB, VEC, TA>(af[0], m, k, Ag, 0, q, r);
    float bf[TB][TB][4];
#pragma unroll
    for (int jj = 0; jj < TB; ++jj) {
        const int j = jj * 16 + r;
#pragma unroll
        for (int kb = 0; kb < TB; ++kb)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int kk = kb * 16 + 4 * q + c;
                bf[jj][kb][c] = (kb < KT && kk < k && j < n) ? (TBT ? Bg[j * k + kk] : Bg[kk * n + j]) : 0.f;
            }
    }
#pragma unroll
    for (int it = 0; it < TB; ++it) {
        if (it + 1 < TB) mfma_a_rows<TB, VEC, TA>(af[(it + 1) & 1], m, k, Ag, it + 1, q, r);
        if (it < MT) {
            floatx4 acc[TB];
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) {
                acc[jj] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < TB; ++kb) {
                    if (kb < KT) {
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            acc[jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[it & 1][kb][c], bf[jj][kb][c], acc[jj],
                                                                           0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < TB; ++jj)
                if (jj < NT) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) stg[(4 * q + e) * kGemmStageStride + jj * 16 + r] = acc[jj][e];
                }
            wave_sync();
            mfma_store_block<TB, TA, TBT>(m, n, alpha, beta, Cg, stg, it, lane);
            wave_sync();
        }
    }
}

// Whole tiles (m = n = k = N = 16 TB, TB = 1..4, no transposes, every operand
// 16-byte aligned), the schedule of mfma_problem_rows with every bound known at
// compile time: fragments come from buffer loads at a per-lane offset plus a
// scalar block offset plus an immediate, with no guards and no 64-bit
// address arithmetic, and the staged rows leave as 16-byte buffer stores.
//   A block it, k-block kb: lane (q, r) reads row 16 it + r, columns
//     16 kb + 4 q .. + 3: byte r*4N + 16 q + it*64N + 64 kb;
//   B k-block kb, tile jj, step c: row 16 kb + 4 q + c, column 16 jj + r:
//     byte 16N q + 4 r + kb*64N + c*4N + 64 jj.
template <int TB>
GLASS_DEV void full_a_rows(float (&af)[TB][4], __amdgpu_buffer_rsrc_t ra, int lane_off, int it) {
    constexpr int N = 16 * TB;
#pragma unroll
    for (int kb = 0; kb < TB; ++kb) {
        const f4_t v = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(ra, lane_off + 64 * kb,
                                                                                        it * 64 * N, 0));
#pragma unroll
        for (int c = 0; c < 4; ++c) af[kb][c] = v[c];
    }
}

template <int TB>
__global__ void __launch_bounds__(512) gemm_mfma_wave_full(int batch, float alpha, const float* __restrict__ A,
                                                           const float* __restrict__ B, float beta,
                                                           float* __restrict__ C) {
    constexpr int N = 16 * TB;
    constexpr uint32_t PB = 4u * N * N;  // bytes per problem and operand
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* stg = lds + (size_t)w * 16 * kGemmStageStride;
    const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(A + p * N * N, PB);
    const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(B + p * N * N, PB);
    const __amdgpu_buffer_rsrc_t rc = buffer_rsrc(C + p * N * N, PB);
    const int a_off = r * 4 * N + 16 * q, b_off = 16 * N * q + 4 * r;
    float af[2][TB][4];
    full_a_rows<TB>(af[0], ra, a_off, 0);
    float bf[TB][TB][4];
#pragma unroll
    for (int jj = 0; jj < TB; ++jj)
#pragma unroll
        for (int kb = 0; kb < TB; ++kb)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                bf[jj][kb][c] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rb, b_off + c * 4 * N + 64 * jj, kb * 64 * N, 0));
#pragma unroll
    for (int it = 0; it < TB; ++it) {
        if (it + 1 < TB) full_a_rows<TB>(af[(it + 1) & 1], ra, a_off, it + 1);
        floatx4 acc[TB];
#pragma unroll
        for (int jj = 0; jj < TB; ++jj) {
            acc[jj] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < TB; ++kb)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[it & 1][kb][c], bf[jj][kb][c], acc[jj], 0, 0, 0);
        }
#pragma unroll
        for (int jj = 0; jj < TB; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) stg[(4 * q + e) * kGemmStageStride + jj * 16 + r] = acc[jj][e];
        wave_sync();
        // 16 rows of N floats = 4N 16-byte pieces, N / 16 per lane; piece g is
        // row g / (N/4), column piece g % (N/4)
#pragma unroll
        for (int u = 0; u < N / 16; ++u) {
            const int g = lane + 64 * u, rr = g / (N / 4), c4 = g % (N / 4);
            const f4_t v = *reinterpret_cast<const f4_t*>(stg + rr * kGemmStageStride + 4 * c4);
            const int off = (rr * N + 4 * c4) * 4;
            f4_t out;
            if (beta != 0.f) {
                const f4_t c0 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rc, off, it * 64 * N, 0));
#pragma unroll
                for (int e = 0; e < 4; ++e) out[e] = fmaf(beta, c0[e], alpha * v[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) out[e] = alpha * v[e];
            }
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, out),
                                                   rc, off, it * 64 * N, 0);
        }
        wave_sync();
    }
}

template <int TB, bool VEC, bool TA = false, bool TBT = false, bool STG = false>
__global__ void __launch_bounds__(512) gemm_mfma_wave(int m, int n, int k, int batch, float alpha,
                                                      const float* __restrict__ A, const float* __restrict__ B,
                                                      float beta, float* __restrict__ C) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    if constexpr (STG && TB == 4)
        mfma_problem_rows<TB, VEC, TA, TBT>(m, n, k, alpha, A + p * m * k, B + p * k * n, beta, C + p * m * n, lane,
                                            lds + (size_t)w * 16 * kGemmStageStride);
    else
        mfma_problem<TB, VEC, TB, TA, TBT, STG>(m, n, k, alpha, A + p * m * k, B + p * k * n, beta, C + p * m * n,
                                                lane, 0, 1, lds + (size_t)w * 16 * kGemmStageStride);
}

template <int TB, bool VEC, bool TA = false, bool TBT = false>
__global__ void __launch_bounds__(256) gemm_mfma_wg(int m, int n, int k, int batch, int pack, float alpha,
                                                    const float* __restrict__ A, const float* __restrict__ B,
                                                    float beta, float* __restrict__ C) {
    const int w = wave_index(), lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        mfma_problem<TB, VEC, 1, TA, TBT>(m, n, k, alpha, A + p * m * k, B + p * k * n, beta, C + p * m * n, lane,
                                          w, nw);
    }
}

#define GLASS_CASES_1_12(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

// Launch one GEMM kernel: TA / TBT are the transpose flags of the shape.
template <bool TA, bool TBT>
int launch_gemm_t(const Shape& sh, const Geometry& g, int batch, float alpha, const float* A, const float* B,
                  float beta, float* C, hipStream_t st) {
    const int m = sh.m, n = sh.n, k = sh.k;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (!gemm_uses_mfma(sh)) {
        if (g.scope == GLASS_SCOPE_WAVE)
            hipLaunchKernelGGL((gemm_small_wave<TA, TBT>), grid, block, g.lds_bytes, st, m, n, k, batch, alpha, A, B,
                               beta, C, (int)region_floats(sh));
        else
            hipLaunchKernelGGL((gemm_small_wg<TA, TBT>), grid, block, g.lds_bytes, st, m, n, k, batch, g.pack,
                               alpha, A, B, beta, C);
        return (int)hipGetLastError();
    }
    int mx = m > n ? m : n;
    mx = mx > k ? mx : k;
    const int tb = (mx + 15) / 16;
    const bool vec = !TA && (k % 4 == 0) && ((uintptr_t)A % 16 == 0);
    if (g.scope == GLASS_SCOPE_WAVE) {
        if (!TA && !TBT && m == n && n == k && (n == 16 || n == 32 || n == 48 || n == 64) && (uintptr_t)A % 16 == 0 &&
            (uintptr_t)B % 16 == 0 && (uintptr_t)C % 16 == 0) {
            switch (n) {
            case 16:
                hipLaunchKernelGGL(gemm_mfma_wave_full<1>, grid, block, g.lds_bytes, st, batch, alpha, A, B, beta, C);
                break;
            case 32:
                hipLaunchKernelGGL(gemm_mfma_wave_full<2>, grid, block, g.lds_bytes, st, batch, alpha, A, B, beta, C);
                break;
            case 48:
                hipLaunchKernelGGL(gemm_mfma_wave_full<3>, grid, block, g.lds_bytes, st, batch, alpha, A, B, beta, C);
                break;
            default:
                hipLaunchKernelGGL(gemm_mfma_wave_full<4>, grid, block, g.lds_bytes, st, batch, alpha, A, B, beta, C);
                break;
            }
            return (int)hipGetLastError();
        }
        // staged full-row stores when C rows are whole 16-byte units
        const bool stg = (n % 4 == 0) && ((uintptr_t)C % 16 == 0);
#define X(TB)                                                                                                   \
    case TB:                                                                                                    \
        if (vec && stg)                                                                                         \
            hipLaunchKernelGGL((gemm_mfma_wave<TB, true, TA, TBT, true>), grid, block, g.lds_bytes, st, m, n, k, \
                               batch, alpha, A, B, beta, C);                                                    \
        else if (stg)                                                                                           \
            hipLaunchKernelGGL((gemm_mfma_wave<TB, false, TA, TBT, true>), grid, block, g.lds_bytes, st, m, n,  \
                               k, batch, alpha, A, B, beta, C);                                                 \
        else if (vec)                                                                                           \
            hipLaunchKernelGGL((gemm_mfma_wave<TB, true, TA, TBT>), grid, block, g.lds_bytes, st, m, n, k,      \
                               batch, alpha, A, B, beta, C);                                                    \
        else                                                                                                    \
            hipLaunchKernelGGL((gemm_mfma_wave<TB, false, TA, TBT>), grid, block, g.lds_bytes, st, m, n, k,     \
                               batch, alpha, A, B, beta, C);                                                    \
        break;
        switch (tb) {
            X(1) X(2) X(3) X(4)
        default: return (int)hipErrorInvalidValue;
        }
#undef X
    } else {
#define X(TB)                                                                                                  \
    case TB:                                                                                                   \
        if (vec)                                                                                               \
            hipLaunchKernelGGL((gemm_mfma_wg<TB, true, TA, TBT>), grid, block, 0, st, m, n, k, batch, g.pack,  \
                               alpha, A, B, beta, C);                                                          \
        else                                                                                                   \
            hipLaunchKernelGGL((gemm_mfma_wg<TB, false, TA, TBT>), grid, block, 0, st, m, n, k, batch, g.pack, \
                               alpha, A, B, beta, C);                                                          \
        break;
        switch (tb) {
            X(1) X(2) X(3) X(4)
        default: return (int)hipErrorInvalidValue;
        }
#undef X
    }
    return (int)hipGetLastError();
}

}  // namespace

int launch_gemm(const Shape& sh, const Geometry& g, int batch, float alpha, const float* A, const float* B,
                float beta, float* C, void* stream) {
    if (g.scope == GLASS_SCOPE_SUBWAVE) return launch_blas_subwave(sh, g, batch, alpha, A, B, beta, C, stream);
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    if (g.scope == GLASS_SCOPE_THREAD) {  // square, no transposes (make_geometry)
        dim3 grid((unsigned)g.grid), block(g.threads);
        switch (sh.n) {
#define X(N) \
    case N: hipLaunchKernelGGL(gemm_thread<N>, grid, block, g.lds_bytes, st, batch, alpha, A, B, beta, C); break;
            GLASS_CASES_1_12(X)
#undef X
        default: return (int)hipErrorInvalidValue;
        }
        return (int)hipGetLastError();
    }
    switch (sh.trans & 3) {
    case 0: return launch_gemm_t<false, false>(sh, g, batch, alpha, A, B, beta, C, st);
    case 1: return launch_gemm_t<true, false>(sh, g, batch, alpha, A, B, beta, C, st);
    case 2: return launch_gemm_t<false, true>(sh, g, batch, alpha, A, B, beta, C, st);
    default: return launch_gemm_t<true, true>(sh, g, batch, alpha, A, B, beta, C, st);
    }
}

}  // namespace glass
