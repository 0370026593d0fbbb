// riccati.hip -- fused LQR feedback gain K = (R + B^T P B)^{-1} B^T P A
// (Sec. III-B names it as a fused composition of GEMM and solve primitives;
// Sec. IV-E measures fused against a chain of separate launches).
//
// One wavefront per problem (wave scope, P problems per workgroup), every
// intermediate on chip:
//   1. P (nx x nx) and B (nx x nu) are staged into LDS with coalesced loads,
//      rows padded with zeros to the 8-wide buckets NX8 / NU8;
//   2. lane c (c < nu + nx) loads column c of X = [B | A] into VGPRs and
//      accumulates z = B^T (P x): for each row i of P, y_i = P[i,:] x (P row
//      read as LDS broadcasts), then z_j += B[i][j] y_i.  Lane c < nu ends
//      with column c of B^T P B, lane nu + c with column c of T = B^T P A;
//   3. lanes c < nu add R[:, c] and hold S = R + B^T P B by columns (S is
//      symmetric, so a column serves as the row the wave Cholesky expects);
//      the existing DPP wave factorization gives L and 1/L_ii;
//   4. L goes to LDS; lane nu + c solves L L^T k = t for its own column t of
//      T (forward and backward substitution with L read as broadcasts) and
//      stores column c of K (K row-major nu x nx, so a row's stores are
//      consecutive lanes).
#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"

namespace glass {
namespace {

template <int NX8, int NU8>
__global__ void __launch_bounds__(512) riccati_wave(int nx, int nu, int batch, const float* __restrict__ A,
                                                    const float* __restrict__ B, const float* __restrict__ P,
                                                    const float* __restrict__ R, float* __restrict__ K,
                                                    int32_t* __restrict__ info, int region) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* Ps = lds + (size_t)w * region;  // [NX8][NX8]
    float* Bs = Ps + NX8 * NX8;            // [NX8][NU8]
    float* Ls = Bs + NX8 * NU8;            // [NU8][NU8] rows of L, then [NU8] of 1 / L_ii
    // (every offset is a multiple of 8 floats, so the f4_t accesses are aligned)
    const float* Pg = P + p * nx * nx;
    const float* Bg = B + p * nx * nu;
    const float* Ag = A + p * nx * nx;
    const float* Rg = R + p * nu * nu;

    for (int e = lane; e < NX8 * NX8; e += 64) {
        const int i = e / NX8, k = e - i * NX8;
        Ps[e] = (i < nx && k < nx) ? Pg[i * nx + k] : 0.f;
    }
    for (int e = lane; e < NX8 * NU8; e += 64) {
        const int i = e / NU8, j = e - i * NU8;
        Bs[e] = (i < nx && j < nu) ? Bg[i * nu + j] : 0.f;
    }
    const int c = lane;
    const bool colB = c < nu, colA = c >= nu && c < nu + nx;
    float x[NX8];
#pragma unroll
    for (int k = 0; k < NX8; ++k)
        x[k] = k < nx ? (colB ? Bg[k * nu + c] : (colA ? Ag[k * nx + (c - nu)] : 0.f)) : 0.f;
    wave_sync();

    float z[NU8];
#pragma unroll
    for (int j = 0; j < NU8; ++j) z[j] = 0.f;
    for (int i = 0; i < nx; ++i) {
        const float* pr = Ps + i * NX8;
        float y = 0.f;
#pragma unroll
        for (int k4 = 0; k4 < NX8 / 4; ++k4) {
            const f4_t pv = *reinterpret_cast<const f4_t*>(pr + 4 * k4);
#pragma unroll
            for (int e = 0; e < 4; ++e) y = fmaf(pv[e], x[4 * k4 + e], y);
        }
        const float* br = Bs + i * NU8;
#pragma unroll
        for (int j4 = 0; j4 < NU8 / 4; ++j4) {
            const f4_t bv = *reinterpret_cast<const f4_t*>(br + 4 * j4);
#pragma unroll
            for (int e = 0; e < 4; ++e) z[4 * j4 + e] = fmaf(bv[e], y, z[4 * j4 + e]);
        }
    }

    // S by columns in lanes < nu, identity rows up to the bucket, zero beyond
    float a[NU8];
#pragma unroll
    for (int j = 0; j < NU8; ++j) {
        if (colB)
            a[j] = j < nu ? z[j] + Rg[j * nu + c] : 0.f;
        else
            a[j] = (j == c) ? 1.f : 0.f;
    }
    float myinv;
    const int inf = wave_potrf<NU8>(a, lane, myinv);
    if (inf != 0) {
        if (info && lane == 0) info[p] = inf;
        return;
    }
    if (lane < NU8) {
#pragma unroll
        for (int j4 = 0; j4 < NU8 / 4; ++j4) {
            f4_t v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = a[4 * j4 + e];
            *reinterpret_cast<f4_t*>(Ls + lane * NU8 + 4 * j4) = v;
        }
        Ls[NU8 * NU8 + lane] = myinv;
    }
    wave_sync();
    if (colA) {
        float t[NU8];
#pragma unroll
        for (int i = 0; i < NU8; ++i) {  // L y = t (padded rows are identity, padded t is 0)
            float s = z[i];
#pragma unroll
            for (int j = 0; j < i; ++j) s = fmaf(-Ls[i * NU8 + j], t[j], s);
            t[i] = s * Ls[NU8 * NU8 + i];
        }
#pragma unroll
        for (int i = NU8 - 1; i >= 0; --i) {  // L^T k = y
            float s = t[i];
#pragma unroll
            for (int j = i + 1; j < NU8; ++j) s = fmaf(-Ls[j * NU8 + i], t[j], s);
            t[i] = s * Ls[NU8 * NU8 + i];
        }
        float* Kg = K + p * nu * nx + (c - nu);
#pragma unroll
        for (int i = 0; i < NU8; ++i)
            if (i < nu) Kg[i * nx] = t[i];
    }
    if (info && lane == 0) info[p] = 0;
}

}  // namespace

size_t riccati_region_floats(int nx, int nu) {
    const int x8 = bucket8_host(nx), u8 = bucket8_host(nu);
    return (size_t)x8 * x8 + (size_t)x8 * u8 + (size_t)u8 * u8 + u8;
}

int launch_riccati(int nx, int nu, int batch, int pack, const float* A, const float* B, const float* P,
                   const float* R, float* K, int32_t* info, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int region = (int)riccati_region_floats(nx, nu);
    dim3 grid((unsigned)((batch + pack - 1) / pack)), block(64 * pack);
    const size_t lds = sizeof(float) * (size_t)region * pack;
    const int x8 = bucket8_host(nx), u8 = bucket8_host(nu);
#define RK(X8, U8)                                                                                          \
    if (x8 == X8 && u8 == U8) {                                                                             \
        hipLaunchKernelGGL((riccati_wave<X8, U8>), grid, block, lds, st, nx, nu, batch, A, B, P, R, K, info, \
                           region);                                                                         \
        return (int)hipGetLastError();                                                                      \
    }
    RK(8, 8) RK(16, 8) RK(24, 8) RK(32, 8) RK(40, 8) RK(48, 8) RK(56, 8)
    RK(8, 16) RK(16, 16) RK(24, 16) RK(32, 16) RK(40, 16) RK(48, 16)
#undef RK
    return (int)hipErrorInvalidValue;
}

}  // namespace glass
