// riccati.hip -- fused LQR feedback gain K = (R + B^T P B)^{-1} B^T P A
// (Sec. III-B names it as a fused composition of GEMM and solve primitives;
// Sec. IV-E measures fused against a chain of separate launches).
//
// Every intermediate stays on chip.  At wave scope (one wavefront per
// problem, P problems per workgroup) in one of two forms, riccati_wave and
// riccati_mfma; at sub-wave scope riccati_seg; at thread scope riccati_thread.
//
// riccati_wave (LDS-staged, nx < kRiccatiMfmaMinNx):
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
//
// riccati_thread (thread scope, nx <= 8, nu <= 4): one problem per lane.  A
// lane loads its own P, B, R and A (every load issued before any is used),
// forms PB = P B, the lower triangle of S = R + B^T PB and the columns of
// T = PB^T A in VGPRs, factors S with the thread-scope Cholesky and solves
// S k = t for each column of T; its problem's K goes out in one run of stores.
//
// riccati_seg (sub-wave scope, nx <= 16, nu <= 8): four problems per
// wavefront, one per 16-lane row; lane i of a row holds row i of P, B and R
// and column i of A.  PB's row i takes B's rows as DPP row broadcasts;
// S = R + B^T PB sums each lane's outer product B_i PB_i^T over the row with
// four DPP exchanges; S is factored with the segment Cholesky (lane a holds
// row a of L); column i of T = PB^T A takes PB's rows as broadcasts, and
// lane i solves L L^T k = t for its own column of K with L's entries as
// broadcasts.  Every cross-lane move stays inside a 16-lane row.
//
// riccati_mfma (nx >= kRiccatiMfmaMinNx): every product on the matrix cores,
// in the blocked layouts of chol_blk.hpp (nx padded to 16-row blocks; nu <= 16
// is one block).  With B_k in accumulator layout (lane (q, r) holds B[16k+4q+c][r])
// the products chain without data movement:
//   PB_i = sum_k P_ik B_k                 P_ik loaded row-wise (T layout)
//   S    = R + sum_i B_i^T PB_i           B_i's registers are the T layout of B_i^T
//   T_j  = sum_i PB_i^T A_ij              PB_i's registers are the T layout of PB_i^T
//                                         (B^T P = (P B)^T: P is symmetric)
//   K_j  = L^{-T} L^{-1} T_j              S = L L^T factored as a diagonal block
// S's padded diagonal (orders nu..15) is the identity, so the solve runs on a
// full 16 x 16 block while the factorization and the inverse stop after nu
// rounded up to 4, 8 or 16 pivots (the rest would find unit pivots and zero
// coefficients).
#include <type_traits>

#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"
#include "chol_blk.hpp"
#include "riccati.hpp"

namespace glass {
namespace {

// One 16 x 16 block of a row-major [rows][ld] matrix in T layout (lane
// (q, r): row r0 + r, columns c0 + 4q .. c0 + 4q + 3; zero outside rows x cols).
GLASS_DEV f4_t load_t_block(__amdgpu_buffer_rsrc_t rs, int ld, int rows, int cols, int r0, int c0, bool vec, int q,
                            int r) {
    f4_t v = {0.f, 0.f, 0.f, 0.f};
    const int R = r0 + r, C = c0 + 4 * q;
    if (R < rows) {
        if (vec && C + 4 <= cols) {
            v = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, (R * ld + C) * 4, 0, 0));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (C + e < cols)
                    v[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (R * ld + C + e) * 4, 0, 0));
        }
    }
    return v;
}

// The same block in accumulator layout (lane (q, r): rows r0 + 4q .. r0 + 4q + 3,
// column c0 + r).
GLASS_DEV f4_t load_acc_block(const float* M, int ld, int rows, int cols, int r0, int c0, int q, int r) {
    f4_t v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int R = r0 + 4 * q + e, C = c0 + r;
        v[e] = (R < rows && C < cols) ? M[R * ld + C] : 0.f;
    }
    return v;
}

// L^{-1} of a 16 x 16 lower diagonal block whose rows and columns from NK on
// are the identity, in T layout: the substitution steps K >= NK add nothing
// (their coefficients are zero), so only the first NK run.
template <int K, int NK>
struct InvStepN {
    static GLASS_DEV void run(float (&u)[4], const float (&m)[16]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) fmac_self_bcast<K>(u[c], m[K]);
        InvStepN<K + 1, NK>::run(u, m);
    }
};
template <int NK>
struct InvStepN<NK, NK> {
    static GLASS_DEV void run(float (&)[4], const float (&)[16]) {}
};

template <int NK>
GLASS_DEV f4_t tri_inverse_l_first(const float (&m)[16], float myinv, int q, int r) {
    float u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (4 * q + c == r) ? myinv : 0.f;
    asm volatile("s_nop 1" : "+v"(u[0]), "+v"(u[1]), "+v"(u[2]), "+v"(u[3]));
    InvStepN<0, NK>::run(u, m);
    return f4_t{u[0], u[1], u[2], u[3]};
}

// NUB: nu rounded up to 4, 8 or 16.  S is the identity past nu, so its
// factorization and inverse run NUB pivot steps instead of 16.
template <int NXB, int NUB>
__global__ void __launch_bounds__(512) riccati_mfma(int nx, int nu, int batch, const float* __restrict__ A,
                                                    const float* __restrict__ B, const float* __restrict__ P,
                                                    const float* __restrict__ R, float* __restrict__ K,
                                                    int32_t* __restrict__ info) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float* xs = lds + (size_t)w * kRiccatiMfmaRegionFloats;
    const float* Ap = A + p * nx * nx;
    const float* Bp = B + p * nx * nu;
    const float* Pp = P + p * nx * nx;
    const float* Rp = R + p * nu * nu;
    f4_t Bb[NXB];
#pragma unroll
    for (int k = 0; k < NXB; ++k) Bb[k] = load_acc_block(Bp, nu, nx, nu, 16 * k, 0, q, r);
    const __amdgpu_buffer_rsrc_t rp = buffer_rsrc(Pp, (uint32_t)(nx * nx) * 4u);
    const bool vec = (nx & 3) == 0;
    f4_t PB[NXB];
#pragma unroll
    for (int i = 0; i < NXB; ++i) {
        f4_t acc = zero4();
#pragma unroll
        for (int k = 0; k < NXB; ++k) acc = mma(load_t_block(rp, nx, nx, nx, 16 * i, 16 * k, vec, q, r), Bb[k], acc);
        PB[i] = acc;
    }
    // S = R + B^T P B in accumulator layout, identity on the padded diagonal
    f4_t S = load_acc_block(Rp, nu, nu, nu, 0, 0, q, r);
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (4 * q + e == r && r >= nu) S[e] = 1.f;
#pragma unroll
    for (int i = 0; i < NXB; ++i) S = mma(Bb[i], PB[i], S);
    // rows of S to the lanes: lane (q, r) holds row r of S after the exchange
#pragma unroll
    for (int e = 0; e < 4; ++e) xs[(4 * q + e) * kXS + r] = S[e];
    wave_sync();
    float a[16];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const f4_t v = *reinterpret_cast<const f4_t*>(xs + r * kXS + 4 * u);
#pragma unroll
        for (int e = 0; e < 4; ++e) a[4 * u + e] = v[e];
    }
    wave_sync();
    int f = 0;
    float myinv = 1.f;
    {
        float as[NUB];  // the first NUB columns; rows from NUB on are identity rows
#pragma unroll
        for (int c = 0; c < NUB; ++c) as[c] = a[c];
        SegStep<16, NUB, 0>::run(as, f, myinv);
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = c < NUB ? (c <= r ? as[c] : 0.f) : (c == r ? 1.f : 0.f);
    }
    if (info && lane == 0) info[p] = f;
    if (f != 0) return;  // K is not written for an indefinite S
    float m[16];  // the rows again, diagonal entry cleared, scaled by -1 / L_rr
    rows_zero_diag<kXS, false>(a, m, xs, q, r);
#pragma unroll
    for (int j = 0; j < 16; ++j) m[j] *= -myinv;
    const f4_t linv = tri_inverse_l_first<NUB>(m, myinv, q, r);  // L^{-1} in T layout
    f4_t lt[4];
    lt[0] = linv;
    transpose_blocks<1>(lt, xs, q, r);  // lt[0]: L^{-T} in T layout
    float* Kp = K + p * nu * nx;
#pragma unroll
    for (int j = 0; j < NXB; ++j) {
        f4_t t = zero4();
#pragma unroll
        for (int i = 0; i < NXB; ++i) t = mma(PB[i], load_acc_block(Ap, nx, nx, nx, 16 * i, 16 * j, q, r), t);
        const f4_t kj = mma(lt[0], mma(linv, t, zero4()), zero4());  // L^{-T} (L^{-1} T_j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 4 * q + e, col = 16 * j + r;
            if (row < nu && col < nx) Kp[row * nx + col] = kj[e];
        }
    }
}

// L consecutive floats of one lane's problem at p, in accesses as wide as the
// problem's size allows when `wide` (the batch's base pointer is 16-byte
// aligned, so problem p starts at a multiple of L floats from it).
template <int L>
GLASS_DEV void lane_load(float (&v)[L], const float* __restrict__ p, bool wide) {
    constexpr int AL = L % 4 == 0 ? 4 : L % 2 == 0 ? 2 : 1;
    if (AL == 4 && wide) {
#pragma unroll
        for (int t = 0; t < L / 4; ++t) {
            const f4_t x = *reinterpret_cast<const f4_t*>(p + 4 * t);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[4 * t + e] = x[e];
        }
    } else if (AL == 2 && wide) {
#pragma unroll
        for (int t = 0; t < L / 2; ++t) {
            const float2 x = *reinterpret_cast<const float2*>(p + 2 * t);
            v[2 * t] = x.x;
            v[2 * t + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) v[t] = p[t];
    }
}

template <int L>
GLASS_DEV void lane_store(float* __restrict__ p, const float (&v)[L], bool wide) {
    constexpr int AL = L % 4 == 0 ? 4 : L % 2 == 0 ? 2 : 1;
    if (AL == 4 && wide) {
#pragma unroll
        for (int t = 0; t < L / 4; ++t) *reinterpret_cast<f4_t*>(p + 4 * t) = f4_t{v[4 * t], v[4 * t + 1], v[4 * t + 2], v[4 * t + 3]};
    } else if (AL == 2 && wide) {
#pragma unroll
        for (int t = 0; t < L / 2; ++t) *reinterpret_cast<float2*>(p + 2 * t) = make_float2(v[2 * t], v[2 * t + 1]);
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) p[t] = v[t];
    }
}

template <int NX, int NU>
__global__ void __launch_bounds__(512) riccati_thread(int batch, const float* __restrict__ A,
                                                      const float* __restrict__ B, const float* __restrict__ P,
                                                      const float* __restrict__ R, float* __restrict__ K,
                                                      int32_t* __restrict__ info, bool wide) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= batch) return;
    float pm[NX * NX], b[NX * NU], r[NU * NU], a[NX * NX];
    lane_load<NX * NX>(pm, P + p * (NX * NX), wide);
    lane_load<NX * NU>(b, B + p * (NX * NU), wide);
    lane_load<NU * NU>(r, R + p * (NU * NU), wide);
    lane_load<NX * NX>(a, A + p * (NX * NX), wide);
    float pb[NX * NU];  // P B
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NX; ++k) s = fmaf(pm[i * NX + k], b[k * NU + j], s);
            pb[i * NU + j] = s;
        }
    float sl[NU * (NU + 1) / 2];  // lower triangle of S = R + B^T (P B)
#pragma unroll
    for (int i = 0; i < NU; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            float s = r[i * NU + j];
#pragma unroll
            for (int k = 0; k < NX; ++k) s = fmaf(b[k * NU + i], pb[k * NU + j], s);
            sl[TI(i, j)] = s;
        }
    float dinv[NU];
    const int inf = tri_potrf<NU>(sl, dinv);
    if (info) info[p] = inf;
    if (inf != 0) return;
    float kk[NU * NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
        float y[NU];  // column c of T = (P B)^T A = B^T P A (P symmetric)
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NX; ++k) s = fmaf(pb[k * NU + i], a[k * NX + c], s);
            y[i] = s;
        }
        tri_fwd<NU>(sl, dinv, y);
        tri_bwd<NU>(sl, dinv, y);
#pragma unroll
        for (int i = 0; i < NU; ++i) kk[i * NX + c] = y[i];
    }
    lane_store<NU * NX>(K + p * (NU * NX), kk, wide);
}

template <int CTRL>
GLASS_DEV float row_dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
// lane K of the 16-lane row (row_newbcast)
template <int K>
GLASS_DEV float row_bcast(float v) {
    return row_dpp<0x150 + K>(v);
}
// the sum over the 16 lanes of a row, the same value in each: pairs, quads
// (quad_perm [1,0,3,2] and [2,3,0,1]), then half rows and rows (row_half_mirror,
// row_mirror); each step adds two equal-order operands, so every lane agrees
GLASS_DEV float row_sum16(float v) {
    v += row_dpp<0xB1>(v);
    v += row_dpp<0x4E>(v);
    v += row_dpp<0x141>(v);
    v += row_dpp<0x140>(v);
    return v;
}

template <int I, int N, class F>
GLASS_DEV void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <int NUB>
__global__ void __launch_bounds__(512) riccati_seg(int nx, int nu, int batch, const float* __restrict__ A,
                                                   const float* __restrict__ B, const float* __restrict__ P,
                                                   const float* __restrict__ R, float* __restrict__ K,
                                                   int32_t* __restrict__ info) {
    const int lane = threadIdx.x & 63, s = lane >> 4, i = lane & 15;
    const long long p0 = ((long long)blockIdx.x * (blockDim.x >> 6) + wave_index()) * 4;
    if (p0 >= batch) return;
    const long long ps = p0 + s;
    const bool act = ps < batch;
    const long long pp = act ? ps : p0;  // a row past the batch reads its wave's first problem
    const float* Pp = P + pp * nx * nx;
    const float* Ap = A + pp * nx * nx;
    const float* Bp = B + pp * nx * nu;
    const float* Rp = R + pp * nu * nu;
    const bool row = i < nx;
    float prow[16], acol[16], brow[NUB], rrow[NUB];
#pragma unroll
    for (int k = 0; k < 16; ++k) {  // unconditional loads (entry 0 for the rest), so that all issue at once
        const bool ok = act && row && k < nx;
        const float pv = Pp[ok ? k * nx + i : 0];  // P symmetric: row i read as column i (coalesced)
        const float av = Ap[ok ? k * nx + i : 0];
        prow[k] = ok ? pv : 0.f;
        acol[k] = ok ? av : 0.f;
    }
#pragma unroll
    for (int j = 0; j < NUB; ++j) {
        const bool okb = act && row && j < nu, okr = act && i < nu && j < nu;
        const float bv = Bp[okb ? i * nu + j : 0];
        const float rv = Rp[okr ? i * nu + j : 0];
        brow[j] = okb ? bv : 0.f;
        rrow[j] = okr ? rv : 0.f;
    }
    // row i of P B; the broadcasts are folded into the FMAs (one DPP op each,
    // so no broadcast value is held), after the wait states their sources need
    float pb[NUB];
#pragma unroll
    for (int j = 0; j < NUB; ++j) {
        pb[j] = 0.f;
        asm volatile("s_nop 1" : "+v"(brow[j]));
    }
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
#pragma unroll
        for (int j = 0; j < NUB; ++j) fmac_bcast<k>(pb[j], brow[j], prow[k]);
    });
    // S = R + B^T P B: lane i contributes B_i PB_i^T; row i of S to lane i
    // (identity rows from nu to NUB, zero rows past NUB)
    float srow[NUB];
#pragma unroll
    for (int c = 0; c < NUB; ++c) srow[c] = 0.f;
#pragma unroll
    for (int a = 0; a < NUB; ++a)
#pragma unroll
        for (int c = 0; c <= a; ++c) {
            const float v = row_sum16(brow[a] * pb[c]);
            if (i == a) srow[c] = a < nu ? rrow[c] + v : (c == a ? 1.f : 0.f);
            if (i == c && c != a) srow[a] = c < nu ? rrow[a] + v : 0.f;
        }
    int f = 0;
    float myinv = 1.f;
    SegStep<16, NUB, 0>::run(srow, f, myinv);
    if (act && i == 0 && info) info[ps] = f;
    if (f != 0) return;  // the row's problem is indefinite (or past the batch): K is not written
    // column i of T = (P B)^T A
    float t[NUB];
#pragma unroll
    for (int a = 0; a < NUB; ++a) {
        t[a] = 0.f;
        asm volatile("s_nop 1" : "+v"(pb[a]));
    }
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
#pragma unroll
        for (int a = 0; a < NUB; ++a) fmac_bcast<k>(t[a], pb[a], acol[k]);
    });
    // L's strictly lower entries and 1 / L_aa as broadcasts, then L L^T k = t
    float lo[NUB][NUB], inv[NUB];
    static_for<0, NUB>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        inv[a] = row_bcast<a>(myinv);
#pragma unroll
        for (int b = 0; b < a; ++b) lo[a][b] = row_bcast<a>(srow[b]);
    });
#pragma unroll
    for (int a = 0; a < NUB; ++a) {
        float v = t[a];
#pragma unroll
        for (int b = 0; b < a; ++b) v = fmaf(-lo[a][b], t[b], v);
        t[a] = v * inv[a];
    }
#pragma unroll
    for (int a = NUB - 1; a >= 0; --a) {
        float v = t[a];
#pragma unroll
        for (int b = a + 1; b < NUB; ++b) v = fmaf(-lo[b][a], t[b], v);
        t[a] = v * inv[a];
    }
    if (act && row) {
        float* Kp = K + ps * nu * nx + i;
#pragma unroll
        for (int a = 0; a < NUB; ++a)
            if (a < nu) Kp[a * nx] = t[a];
    }
}

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

static_assert(kRiccatiMfmaRegionFloats == 16 * kXS, "one exchange block");

size_t riccati_region_floats(int nx, int nu) {
    if (riccati_uses_mfma(nx)) return kRiccatiMfmaRegionFloats;
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
    if (riccati_uses_mfma(nx)) {
        const int nub = nu <= 4 ? 4 : nu <= 8 ? 8 : 16;
        switch ((nx + 15) / 16 * 100 + nub) {
#define RM(NXB, NUB)                                                                                            \
    case NXB * 100 + NUB:                                                                                       \
        hipLaunchKernelGGL((riccati_mfma<NXB, NUB>), grid, block, lds, st, nx, nu, batch, A, B, P, R, K, info); \
        break;
#define RM_NX(NXB) RM(NXB, 4) RM(NXB, 8) RM(NXB, 16)
            RM_NX(1) RM_NX(2) RM_NX(3) RM_NX(4)
#undef RM_NX
#undef RM
        default: return (int)hipErrorInvalidValue;
        }
        return (int)hipGetLastError();
    }
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

int launch_riccati_seg(int nx, int nu, int batch, int pack, const float* A, const float* B, const float* P,
                       const float* R, float* K, int32_t* info, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int per_wg = 4 * pack;
    dim3 grid((unsigned)((batch + per_wg - 1) / per_wg)), block(64 * pack);
    if (nu <= 4)
        hipLaunchKernelGGL((riccati_seg<4>), grid, block, 0, st, nx, nu, batch, A, B, P, R, K, info);
    else
        hipLaunchKernelGGL((riccati_seg<8>), grid, block, 0, st, nx, nu, batch, A, B, P, R, K, info);
    return (int)hipGetLastError();
}

int launch_riccati_thread(int nx, int nu, int batch, int pack, const float* A, const float* B, const float* P,
                          const float* R, float* K, int32_t* info, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int threads = 64 * pack;
    dim3 grid((unsigned)((batch + threads - 1) / threads)), block(threads);
    auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    const bool wide = al16(A) && al16(B) && al16(P) && al16(R) && al16(K);
#define RT(NX, NU)                                                                                          \
    if (nx == NX && nu == NU) {                                                                             \
        hipLaunchKernelGGL((riccati_thread<NX, NU>), grid, block, 0, st, batch, A, B, P, R, K, info, wide); \
        return (int)hipGetLastError();                                                                      \
    }
#define RT_NX(NX) RT(NX, 1) RT(NX, 2) RT(NX, 3) RT(NX, 4)
    RT_NX(1) RT_NX(2) RT_NX(3) RT_NX(4) RT_NX(5) RT_NX(6) RT_NX(7) RT_NX(8)
#undef RT_NX
#undef RT
    return (int)hipErrorInvalidValue;
}

}  // namespace glass
