// chol_blk.hpp -- device routines of the blocked MFMA Cholesky family
// (orders 25..64, one problem per wavefront); used by the batched kernels
// (chol_blk.hip) and the ragged solver (ragged.hip).
//
// POTRF / POSV / POTRS / TRSV of one problem of order 25..64 per wavefront,
// blocked in 16 x 16 tiles, with every block product on the matrix cores
// (v_mfma_f32_16x16x4_f32).
//
// Right-looking block Cholesky (the factorization of Sec. III-B, in blocks):
// for each block column k, factor the diagonal block A_kk = L_kk L_kk^T, form
// the panel L_ik = A_ik L_kk^{-T} for i > k, and update the trailing blocks
// A_ij -= L_ik L_jk^T for k < j <= i.  The unblocked row-per-lane kernel
// issues one v_fmac per lane for every (step, trailing column), two thirds of
// which fall on the upper part; here the trailing update is a dense
// 16 x 16 x 16 contraction per lower block.
//
// Register layout ("T layout"): block (i, j) of the lower triangle sits in
// four VGPRs per lane; lane (q, r) = (lane / 16, lane % 16) holds
// A[16 i + r][16 j + 4 q + c], c = 0..3 -- one 16-byte piece of a row, so
// loads and stores are row-major vectors.  Read as an MFMA accumulator
// (lane (q, r) holds D[4 q + c][r]) the same registers hold the block's
// transpose.  With M in T layout as the A operand and X in accumulator
// layout as the B operand, four v_mfma_f32_16x16x4_f32 (k = 4 q + c in step c)
// give D = M X + C in accumulator layout, and each product of the algorithm
// has that form with no data movement:
//   panel     L_ik^T  = L_kk^{-1} A_ik^T            M = L_kk^{-1}
//   update    A_ij^T -= L_jk L_ik^T                 M = -L_jk
//   forward   Y_k = L_kk^{-1} (B_k - sum_j L_kj Y_j)  M = L_kk^{-1}, -L_kj
// The backward substitution needs L_ik^T and L_kk^{-T} as M; those come from
// a transpose through LDS.  A diagonal block goes through LDS into
// row-per-lane form (each 16-lane row of the wavefront receives all 16 rows),
// is factored with the 16-lane DPP column steps, and is inverted by forward
// substitution against the identity, which yields L_kk^{-1} in T layout.
//
// Rows past n are identity rows (unit pivots that leave the real rows alone;
// L = I there for the solves) and columns past n are zero.
#pragma once

#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"

namespace glass {

constexpr int kXS = kBlkXS;
static_assert(16 * blk_row_stride(4) <= kBlkRegionFloats && 4 * 16 * kXS <= kBlkRegionFloats, "LDS region");
static_assert(16 * kXS <= kBlkSolve1Floats, "LDS region of the one-column solves");
static_assert(16 * kXS <= 16 * blk_row_stride(2), "exchange block inside the staging area");

constexpr int BI(int i, int j) { return i * (i + 1) / 2 + j; }

GLASS_DEV f4_t zero4() { return f4_t{0.f, 0.f, 0.f, 0.f}; }
GLASS_DEV f4_t neg4(const f4_t& v) { return f4_t{-v[0], -v[1], -v[2], -v[3]}; }

// D = M X + C for 16 x 16 blocks: M in T layout, X and C in accumulator layout.
GLASS_DEV f4_t mma(const f4_t& m, const f4_t& x, f4_t c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(m[s], x[s], c, 0, 0, 0);
    return c;
}

// The lower blocks of the problem at Ag in T layout.  FULL: n == 16 NBLK.
// The strict upper part of a diagonal block is not read (zero).  Otherwise
// every lane still issues one 16-byte load per piece into registers of its
// own, all before any is read (loads under a per-lane branch, or a separate
// element-wise load of a row's last piece, made the compiler wait for each
// piece in turn): a piece past the problem reads the first one (in range)
// and is cleared, the piece of the last row that would run past the problem
// is loaded as its last 16 bytes and moved down, and the entries past
// column n of the other rows are cleared; loads are 4-byte aligned.
template <int NBLK, bool FULL>
GLASS_DEV void blk_load(f4_t (&T)[NBLK * (NBLK + 1) / 2], const float* Ag, int n, int q, int r) {
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(Ag, (uint32_t)(n * n) * 4u);
#pragma unroll
    for (int i = 0; i < NBLK; ++i) {
        const int R = 16 * i + r;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const int C = 16 * j + 4 * q;
            f4_t v = zero4();
            if (FULL) {
                v = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, (R * n + C) * 4, 0, 0));
            } else {  // a piece past the problem loads the first one (in range) and is cleared below
                const int off = !(R < n && C < n) ? 0 : (R == n - 1 && C + 4 > n) ? n * n - 4 : R * n + C;
                v = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off * 4, 0, 0));
            }
            T[BI(i, j)] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < NBLK; ++i) {
        const int R = 16 * i + r;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const int C = 16 * j + 4 * q;
            f4_t v = T[BI(i, j)];
            if (!FULL) {
                if (!(R < n && C < n)) v = zero4();
                if (16 * j < n && 16 * j + 16 > n) {  // the block column that holds column n - 1
                    const int over = C + 4 - n;          // entries of the piece past column n
                    const f4_t d = over == 1   ? f4_t{v[1], v[2], v[3], 0.f}
                                   : over == 2 ? f4_t{v[2], v[3], 0.f, 0.f}
                                               : f4_t{v[3], 0.f, 0.f, 0.f};
                    const f4_t k = f4_t{C < n ? v[0] : 0.f, C + 1 < n ? v[1] : 0.f, C + 2 < n ? v[2] : 0.f,
                                        C + 3 < n ? v[3] : 0.f};
                    v = (R == n - 1 && over > 0 && over < 4) ? d : k;
                }
                if (i == j && R >= n) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (4 * q + e == r) ? 1.f : 0.f;
                }
            }
            if (i == j) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (4 * q + e <= r) ? v[e] : 0.f;
            }
            T[BI(i, j)] = v;
        }
    }
}

// Diagonal block (T layout) to row-per-lane form: lane (q, r) receives row r
// (every 16-lane row of the wavefront a full copy).  Returns the lane's
// diagonal entry; ZD: the rows come with that entry cleared.
template <bool ZD = false>
GLASS_DEV float diag_rows(const f4_t& t, float (&a)[16], float* xs, int q, int r) {
    *reinterpret_cast<f4_t*>(xs + r * kXS + 4 * q) = t;
    wave_sync();
    float d = 0.f;
    if (ZD) {
        d = xs[r * kXS + r];
        xs[r * kXS + r] = 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const f4_t v = *reinterpret_cast<const f4_t*>(xs + r * kXS + 4 * u);
#pragma unroll
        for (int e = 0; e < 4; ++e) a[4 * u + e] = v[e];
    }
    if (!ZD) d = xs[r * kXS + r];
    wave_sync();
    return d;
}

// acc += bcast_K(acc) * m, the broadcast of lane K of the 16-lane row folded
// into the v_fmac.  Consecutive calls on one register are three instructions
// apart (four accumulators in turn), above the two wait states a DPP read of a
// just-written VGPR needs.
template <int K>
GLASS_DEV void fmac_self_bcast(float& acc, float m) {
    asm volatile("v_fmac_f32_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(m), "n"(K));
}

template <int K>
struct InvStep {
    static GLASS_DEV void run(float (&u)[4], const float (&m)[16]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) fmac_self_bcast<K>(u[c], m[K]);
        InvStep<K + 1>::run(u, m);
    }
};
template <>
struct InvStep<16> {
    static GLASS_DEV void run(float (&)[4], const float (&)[16]) {}
};

// X = L^{-1} of a 16 x 16 lower diagonal block, in T layout: lane (q, r)
// returns row r, columns 4 q .. 4 q + 3.  Forward substitution against the
// identity with the lane's own coefficients m_K = -L_rK / L_rr (zero in lane
// K and above the diagonal) and myinv = 1 / L_rr reads
// X_r = e_r / L_rr + sum_{K<r} m_K X_K, so the rows are finished in order
// K = 0..15 and each step is one v_fmac per column with lane K's row
// broadcast.
GLASS_DEV f4_t tri_inverse_l(const float (&m)[16], float myinv, int q, int r) {
    float u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (4 * q + c == r) ? myinv : 0.f;
    asm volatile("s_nop 1" : "+v"(u[0]), "+v"(u[1]), "+v"(u[2]), "+v"(u[3]));
    InvStep<0>::run(u, m);
    return f4_t{u[0], u[1], u[2], u[3]};
}

// Row r of a factored diagonal block with its diagonal entry cleared, read
// back through LDS at xs (row stride S).  STAGED: the rows are already there
// (the staged block row); otherwise the lanes of row 0 write them first.
// Leaves the cleared rows in LDS.
template <int S, bool STAGED>
GLASS_DEV void rows_zero_diag(const float (&a)[16], float (&az)[16], float* xs, int q, int r) {
    if (!STAGED) {
        if (q == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                *reinterpret_cast<f4_t*>(xs + r * S + 4 * u) = f4_t{a[4 * u], a[4 * u + 1], a[4 * u + 2], a[4 * u + 3]};
        }
        wave_sync();
    }
    xs[r * S + r] = 0.f;
    wave_sync();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const f4_t v = *reinterpret_cast<const f4_t*>(xs + r * S + 4 * u);
#pragma unroll
        for (int e = 0; e < 4; ++e) az[4 * u + e] = v[e];
    }
    wave_sync();
}

// Block row k of L (rows 16 k .. 16 k + 15): the finished blocks left of the
// diagonal, the diagonal block from its rows and +0 to the right, staged in
// LDS and stored as whole rows.
template <int NBLK, bool FULL>
GLASS_DEV void store_block_row(const f4_t (&T)[NBLK * (NBLK + 1) / 2], int k, const float (&a)[16], float* Ag,
                               int n, float* xs, int q, int r, int lane, bool vec) {
    constexpr int kRS = blk_row_stride(NBLK);
#pragma unroll
    for (int j = 0; j < NBLK; ++j) {
        if (j < k) *reinterpret_cast<f4_t*>(xs + r * kRS + 16 * j + 4 * q) = T[BI(k, j)];
        if (j > k) *reinterpret_cast<f4_t*>(xs + r * kRS + 16 * j + 4 * q) = zero4();
    }
    if (q == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            *reinterpret_cast<f4_t*>(xs + r * kRS + 16 * k + 4 * u) =
                f4_t{a[4 * u], a[4 * u + 1], a[4 * u + 2], a[4 * u + 3]};
    }
    wave_sync();
    float* dst = Ag + (size_t)16 * k * n;
    if (FULL) {
        constexpr int N4 = 4 * NBLK;  // 16-byte pieces per row
#pragma unroll
        for (int g = lane; g < 16 * N4; g += 64) {
            const int rr = g / N4, c4 = g % N4;
            reinterpret_cast<f4_t*>(dst)[g] = *reinterpret_cast<const f4_t*>(xs + rr * kRS + 4 * c4);
        }
    } else {
        const int rows = min(16, n - 16 * k);
        if (vec) {
            const int n4 = n >> 2;
            const FastDiv f4 = make_fastdiv((uint32_t)n4);
            for (int g = lane; g < rows * n4; g += 64) {
                const int rr = (int)fdiv((uint32_t)g, f4), c4 = g - rr * n4;
                reinterpret_cast<f4_t*>(dst)[g] = *reinterpret_cast<const f4_t*>(xs + rr * kRS + 4 * c4);
            }
        } else {
            const FastDiv fn = make_fastdiv((uint32_t)n);
            for (int g = lane; g < rows * n; g += 64) {
                const int rr = (int)fdiv((uint32_t)g, fn), cc = g - rr * n;
                dst[g] = xs[rr * kRS + cc];
            }
        }
    }
    wave_sync();
}

// Transposes of up to four blocks through LDS (exchange areas of 16 x kXS):
// a block in T layout comes back in T layout of its transpose.
template <int NB>
GLASS_DEV void transpose_blocks(f4_t (&v)[4], float* xs, int q, int r) {
#pragma unroll
    for (int b = 0; b < NB; ++b) *reinterpret_cast<f4_t*>(xs + b * 16 * kXS + r * kXS + 4 * q) = v[b];
    wave_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) v[b][c] = xs[b * 16 * kXS + (4 * q + c) * kXS + r];
    wave_sync();
}

// Columns cb .. cb + 15 of the row-major [n][nr] right-hand sides, in
// accumulator layout per block row (lane (q, r), element e: row 16 k + 4 q + e,
// column cb + r).
template <int NBLK, bool FULL>
GLASS_DEV void rhs_load(f4_t (&Y)[NBLK], const float* Bg, int n, int nr, int cb, int q, int r) {
    const int col = cb + r;
#pragma unroll
    for (int k = 0; k < NBLK; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int R = 16 * k + 4 * q + e;
            Y[k][e] = ((FULL || R < n) && col < nr) ? Bg[R * nr + col] : 0.f;
        }
}

template <int NBLK, bool FULL>
GLASS_DEV void rhs_store(const f4_t (&Y)[NBLK], float* Bg, int n, int nr, int cb, int q, int r) {
    const int col = cb + r;
#pragma unroll
    for (int k = 0; k < NBLK; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int R = 16 * k + 4 * q + e;
            if ((FULL || R < n) && col < nr) Bg[R * nr + col] = Y[k][e];
        }
}

template <int NBLK, int K>
struct BwdBlk {
    // X_K = L_KK^{-T} (Y_K - sum_{i>K} L_iK^T X_i); nT holds -L blocks.
    static GLASS_DEV void run(const f4_t (&nT)[NBLK * (NBLK + 1) / 2], const f4_t (&linv)[NBLK], f4_t (&Y)[NBLK],
                              float* xs, int q, int r) {
        constexpr int NI = NBLK - 1 - K;
        f4_t v[4];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = nT[BI(K + 1 + i, K)];
        v[NI] = linv[K];
        transpose_blocks<NI + 1>(v, xs, q, r);
        f4_t s = Y[K];
#pragma unroll
        for (int i = 0; i < NI; ++i) s = mma(v[i], Y[K + 1 + i], s);
        Y[K] = mma(v[NI], s, zero4());
        BwdBlk<NBLK, K - 1>::run(nT, linv, Y, xs, q, r);
    }
};
template <int NBLK>
struct BwdBlk<NBLK, -1> {
    static GLASS_DEV void run(const f4_t (&)[NBLK * (NBLK + 1) / 2], const f4_t (&)[NBLK], f4_t (&)[NBLK], float*,
                              int, int) {}
};

// --------------------------------------------- one right-hand side, no inverses
// A single right-hand side (TRSV; POTRS with nrhs = 1) gains nothing from the
// matrix cores: an MFMA product spends 15 of its 16 columns on padding, and
// the 16 x 16 diagonal-block inverses cost more VALU than the substitution
// itself.  This path keeps L in T layout and runs everything on VALU:
//   R form: a 16-vector of block row k with lane (q, r) holding v[r] in
//           every one of the four 16-lane rows q;
//   diagonal block: plain substitution on its rows (forward) or columns
//           (backward) in row-per-lane form, one DPP step per unknown on
//           s = b_r / L_rr: s += bcast_K(s) * m_K with m_K = -L_rK / L_rr
//           (forward) or -L_Kr / L_rr (backward), the lane's own entries
//           times its own -1 / L_rr (the diagonal entry is cleared on the
//           way through LDS, so m_K is zero in lane K with no select);
//   off-diagonal blocks: a lane's four T-layout entries times the matching
//           four unknowns, summed across the four rows q (two permlane
//           swaps) for L_kj x_j, or across the 16 lanes of a row (four DPP
//           steps) for L_ik^T x_i.
// Pending products are accumulated as soon as a block of x is known
// (right-looking), so only one partial sum per later block stays live.

// acc += bcast_K(acc) * m with the two wait states the DPP read of a
// just-written acc needs.
template <int K>
GLASS_DEV void fmac_self_bcast_w(float& acc, float m) {
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(m), "n"(K));
}

template <int K, int DIR>
struct DiagSub {
    static GLASS_DEV void run(float& s, const float (&m)[16]) {
        fmac_self_bcast_w<K>(s, m[K]);
        DiagSub<K + DIR, DIR>::run(s, m);
    }
};
template <>
struct DiagSub<16, 1> {
    static GLASS_DEV void run(float&, const float (&)[16]) {}
};
template <>
struct DiagSub<-1, -1> {
    static GLASS_DEV void run(float&, const float (&)[16]) {}
};

// v summed over the four 16-lane rows (lanes r, r + 16, r + 32, r + 48), in
// every lane: each v_permlane*_swap exchanges half of v with half of a copy,
// and the VALU write of the copy gets its two wait states before the swap.
GLASS_DEV float sum_rows4(float v) {
    float t;
    asm volatile(
        "v_mov_b32 %1, %0\n"
        "s_nop 1\n"
        "v_permlane32_swap_b32 %0, %1\n"
        "v_add_f32 %0, %0, %1\n"
        "v_mov_b32 %1, %0\n"
        "s_nop 1\n"
        "v_permlane16_swap_b32 %0, %1\n"
        "v_add_f32 %0, %0, %1\n"
        : "+v"(v), "=&v"(t));
    return v;
}

// Each of z[0..3] summed over the 16 lanes of its row, in every lane of the
// row (quad swaps, then the half-row and row mirrors).  The four registers
// take turns, so every DPP read is three instructions after the write of its
// source; the leading s_nop covers the caller's last writes.
GLASS_DEV void sum_row16(float (&z)[4]) {
    asm volatile(
        "s_nop 1\n"
        "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 row_half_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_mirror row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 row_mirror row_mask:0xf bank_mask:0xf\n"
        : "+v"(z[0]), "+v"(z[1]), "+v"(z[2]), "+v"(z[3]));
}

// xc[c] = v[4 q + c] of an R-form v (lane (q, 4 q + c) holds it).
GLASS_DEV void r_to_c(float v, float (&xc)[4], int q) {
    const int vi = __float_as_int(v);
#pragma unroll
    for (int c = 0; c < 4; ++c) xc[c] = __int_as_float(__builtin_amdgcn_ds_bpermute((20 * q + c) * 4, vi));
}

// R form of w with w[4 q + c] = z[c] in every lane of row q: lane (q', r')
// takes z[r' % 4] from lane r' % 4 of row r' / 4.
GLASS_DEV float c_to_r(const float (&z)[4], int r) {
    const int c = r & 3;
    const float w = c == 0 ? z[0] : c == 1 ? z[1] : c == 2 ? z[2] : z[3];
    return __int_as_float(__builtin_amdgcn_ds_bpermute((16 * (r >> 2) + c) * 4, __float_as_int(w)));
}

// Diagonal block k of L (T layout) transposed through LDS: lane (q, r)
// receives column r (col[j] = L_kk[j][r]) with its diagonal entry cleared;
// returns L_kk[r][r].
GLASS_DEV float diag_cols(const f4_t& t, float (&col)[16], float* xs, int q, int r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) xs[(4 * q + c) * kXS + r] = t[c];
    wave_sync();
    const float d = xs[r * kXS + r];
    xs[r * kXS + r] = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const f4_t v = *reinterpret_cast<const f4_t*>(xs + r * kXS + 4 * u);
#pragma unroll
        for (int e = 0; e < 4; ++e) col[4 * u + e] = v[e];
    }
    wave_sync();
    return d;
}

// The pieces of the single-column solve; x[k] is block k of the vector in R
// form (lane (q, r) holds element 16 k + r in every row q).
template <int NBLK, bool FULL>
GLASS_DEV void blk_x_load(float (&x)[NBLK], const float* bg, int n, int r) {
#pragma unroll
    for (int k = 0; k < NBLK; ++k) {
        const int R = 16 * k + r;
        x[k] = (FULL || R < n) ? bg[R] : 0.f;
    }
}

template <int NBLK, bool FULL>
GLASS_DEV void blk_x_store(const float (&x)[NBLK], float* bg, int n, int q, int r) {
    if (q == 0) {
#pragma unroll
        for (int k = 0; k < NBLK; ++k) {
            const int R = 16 * k + r;
            if (FULL || R < n) bg[R] = x[k];
        }
    }
}

// Forward step k: block k of y from its pending sum p[k], the diagonal
// block's lane-local coefficients m_K = -L_rK / L_rr and 1 / L_rr (the
// right-hand side is scaled by it first), then its contributions L_ik y_k to
// the pending sums of the later blocks (right-looking, p[i] split over the
// rows q).
template <int NBLK>
GLASS_DEV void blk_fwd_step(const f4_t (&T)[NBLK * (NBLK + 1) / 2], int k, const float (&m)[16], float myinv,
                            float (&x)[NBLK], float (&p)[NBLK], int q) {
    float s = k > 0 ? x[k] - sum_rows4(p[k]) : x[k];
    s *= myinv;
    DiagSub<0, 1>::run(s, m);
    x[k] = s;
    if (k + 1 < NBLK) {
        float xc[4];
        r_to_c(x[k], xc, q);
#pragma unroll
        for (int i = k + 1; i < NBLK; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) p[i] = fmaf(T[BI(i, k)][c], xc[c], p[i]);
    }
}

// L^T x = y, bottom block first (left-looking over the columns: z[j] collects
// sum_i L_ij^T x_i split over the lanes of a row).
template <int NBLK>
GLASS_DEV void blk_bwd1(const f4_t (&T)[NBLK * (NBLK + 1) / 2], float (&x)[NBLK], float* xs, int q, int r) {
    float z[NBLK][4];
#pragma unroll
    for (int k = 0; k < NBLK; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) z[k][c] = 0.f;
#pragma unroll
    for (int k = NBLK - 1; k >= 0; --k) {
        float s = x[k];
        if (k + 1 < NBLK) {
            sum_row16(z[k]);
            s -= c_to_r(z[k], r);
        }
        float col[16];
        const float myinv = recip(diag_cols(T[BI(k, k)], col, xs, q, r)), nmy = -myinv;
#pragma unroll
        for (int j = 0; j < 16; ++j) col[j] *= nmy;  // -L_jr / L_rr
        s *= myinv;
        DiagSub<15, -1>::run(s, col);
        x[k] = s;
#pragma unroll
        for (int j = 0; j < k; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) z[j][c] = fmaf(T[BI(k, j)][c], x[k], z[j][c]);
    }
}

// The backward pass of op 4 (POSV, one right-hand side), L^T x = y with y in
// R form in x, on what the factorization leaves behind:
//   last block K: the rows of L_KK are still staged in LDS (xs, row stride
//       blk_row_stride(NBLK)) with the diagonal entry cleared, so lane r
//       reads column r and scales it by its own -1 / L_rr, the coefficients
//       of blk_bwd1: x_r = s_r / L_rr + sum_{j>r} (-L_jr / L_rr) x_j, one
//       DPP step per unknown;
//   blocks k < K: L_kk^{-1} is in LDS at lt (T layout, 16 x kXS floats per
//       block), so lane (q, r) reads its column r, rows 4 q .. 4 q + 3, and
//       x_k = L_kk^{-T} s is four FMAs on s in C form (the form the sum of
//       the pending products L_ik^T x_i already has) and one sum over the
//       four rows q -- no substitution chain.
template <int NBLK>
GLASS_DEV void blk_bwd1_posv(const f4_t (&T)[NBLK * (NBLK + 1) / 2], float (&x)[NBLK], float myinv_last,
                             const float* lt, float* xs, int q, int r) {
    constexpr int K = NBLK - 1;
    constexpr int RS = blk_row_stride(NBLK);
    float z[NBLK][4];
#pragma unroll
    for (int k = 0; k < NBLK; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) z[k][c] = 0.f;
    {
        const float* colr = xs + 16 * K + r;  // column r of the staged L_KK
        const float nmy = -myinv_last;
        float mt[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) mt[j] = colr[j * RS] * nmy;
        float s = x[K] * myinv_last;
        DiagSub<15, -1>::run(s, mt);
        x[K] = s;
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) z[j][c] = fmaf(T[BI(K, j)][c], x[K], z[j][c]);
    }
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
        float yc[4];
        r_to_c(x[k], yc, q);
        sum_row16(z[k]);
        float part = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) part = fmaf(lt[k * 16 * kXS + (4 * q + c) * kXS + r], yc[c] - z[k][c], part);
        x[k] = sum_rows4(part);
#pragma unroll
        for (int j = 0; j < k; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) z[j][c] = fmaf(T[BI(k, j)][c], x[k], z[j][c]);
    }
}

// L x = b (FWD) and / or L^T x = b (BWD) for one right-hand side bg[0..n)
// (unit stride), in place; T: L in T layout (diagonal blocks with a zero
// strict upper part, identity rows past n).
template <int NBLK, bool FULL, bool FWD, bool BWD>
GLASS_DEV void blk_solve1(const f4_t (&T)[NBLK * (NBLK + 1) / 2], float* bg, int n, float* xs, int q, int r) {
    float x[NBLK];
    blk_x_load<NBLK, FULL>(x, bg, n, r);
    if (FWD) {
        float p[NBLK];  // pending sum_j L_kj x_j of block row k, split over the rows q
#pragma unroll
        for (int k = 0; k < NBLK; ++k) p[k] = 0.f;
#pragma unroll
        for (int k = 0; k < NBLK; ++k) {
            float a[16];
            const float myinv = recip(diag_rows<true>(T[BI(k, k)], a, xs, q, r)), nmy = -myinv;
#pragma unroll
            for (int j = 0; j < 16; ++j) a[j] *= nmy;  // -L_rj / L_rr
            blk_fwd_step<NBLK>(T, k, a, myinv, x, p, q);
        }
    }
    if (BWD) blk_bwd1<NBLK>(T, x, xs, q, r);
    blk_x_store<NBLK, FULL>(x, bg, n, q, r);
}

// One problem: factor (POTRF, POSV) or take L as given (POTRS, TRSV), then
// solve.  op: 0 POTRF, 1 POSV, 2 POTRS, 3 TRSV (trans: 0 forward, 1 backward),
// 4 POSV with one right-hand side (the factorization of op 1 with VALU
// substitutions on the factor in registers: each forward step runs inside its
// factorization step with the block inverse's coefficients, the backward pass
// of blk_bwd1_posv after it on the inverses the panels used; no inverse of
// the last diagonal block and no block transposes).  Every op forms the
// diagonal blocks' inverses with tri_inverse_l on lane-local coefficients:
// after a factorization from the factored rows read back through LDS with
// their diagonal cleared (the staged block row itself when it is already
// out: two tiles per side, and the last block), for the solves from rows
// read without it.  Ag is A (L for the
// solves), Bg the problem's [n][nr] right-hand sides (nr = 1 for TRSV and op
// 4); vec: Ag 16-byte aligned with n % 4 == 0.  xs: the wavefront's LDS,
// kBlkRegionFloats (op 4: blk_posv1_floats(NBLK)).  Returns info (0 for the
// solves); a failed factorization leaves B untouched.
template <int NBLK, int OP, bool FULL>
GLASS_DEV int blk_one(float* Ag, float* Bg, int n, int nrhs, int trans, bool vec, float* xs, int lane) {
    constexpr int NT = NBLK * (NBLK + 1) / 2;
    constexpr bool FACTOR = OP == 0 || OP == 1 || OP == 4;
    constexpr bool MFMA_SOLVE = OP >= 1 && OP <= 3;
    const int q = lane >> 4, r = lane & 15;
    f4_t T[NT];
    blk_load<NBLK, FULL>(T, Ag, n, q, r);
    // op 4: the right-hand side, loaded with A, and the forward substitution's
    // pending sums; step k of the substitution runs inside factorization step k
    float x1[NBLK], p1[NBLK], myinv_last = 1.f;
    float* lt = xs + 16 * blk_row_stride(NBLK);  // op 4: L_kk^{-1} of the blocks k < NBLK - 1
    if (OP == 4) {
        blk_x_load<NBLK, FULL>(x1, Bg, n, r);
#pragma unroll
        for (int k = 0; k < NBLK; ++k) p1[k] = 0.f;
    }
    f4_t linv[NBLK];
    int inf = 0;
#pragma unroll
    for (int k = 0; k < NBLK; ++k) {
        // Block row k is final once its diagonal block is factored.  On three
        // or four tiles per side it is staged and stored while the matrix
        // cores run the panel products (3 % on POTRF / POSV n = 64 x 4096,
        // whose waves are bound by this chain); on two tiles, memory-bound
        // at large batches, and for the last block it goes out first.
        const bool early = NBLK < 3 || k + 1 == NBLK;
        float a[16];
        const float d = diag_rows<!FACTOR>(T[BI(k, k)], a, xs, q, r);
        float myinv = 1.f;
        if (FACTOR) {
            int f = 0;
            SegStep<16, 16, 0>::run(a, f, myinv);
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = c <= r ? a[c] : 0.f;
            if (inf == 0 && f != 0) inf = 16 * k + f;
            if (early) store_block_row<NBLK, FULL>(T, k, a, Ag, n, xs, q, r, lane, vec);
        } else {
            myinv = recip(d);
        }
        // The coefficients -L_rj / L_rr of the block's substitutions (its
        // inverse; op 4's forward step): the rows with their diagonal entry
        // cleared, read back through LDS after a factorization (from the
        // staged block row when it is already out), as they come for the
        // solves.
        const bool need_inv = MFMA_SOLVE || k + 1 < NBLK;
        float m[16];
        if (need_inv || OP == 4) {
            if (FACTOR) {
                if (early)
                    rows_zero_diag<blk_row_stride(NBLK), true>(a, m, xs + 16 * k, q, r);
                else
                    rows_zero_diag<kXS, false>(a, m, xs, q, r);
            } else {
#pragma unroll
                for (int j = 0; j < 16; ++j) m[j] = a[j];
            }
            const float nmy = -myinv;
#pragma unroll
            for (int j = 0; j < 16; ++j) m[j] *= nmy;
        }
        if (need_inv) {
            linv[k] = tri_inverse_l(m, myinv, q, r);
            if (OP == 4) *reinterpret_cast<f4_t*>(lt + k * 16 * kXS + r * kXS + 4 * q) = linv[k];
        }
        if (OP == 4 && k + 1 == NBLK) myinv_last = myinv;
        if (FACTOR) {
#pragma unroll
            for (int i = k + 1; i < NBLK; ++i) T[BI(i, k)] = mma(linv[k], T[BI(i, k)], zero4());
            if (!early) store_block_row<NBLK, FULL>(T, k, a, Ag, n, xs, q, r, lane, vec);
#pragma unroll
            for (int j = k + 1; j < NBLK; ++j) {
                const f4_t nq = neg4(T[BI(j, k)]);
#pragma unroll
                for (int i = j; i < NBLK; ++i) T[BI(i, j)] = mma(nq, T[BI(i, k)], T[BI(i, j)]);
            }
            // op 4: forward step k (needs this step's panel L_ik), on VALU
            // while the matrix cores run the trailing products
            if (OP == 4) blk_fwd_step<NBLK>(T, k, m, myinv, x1, p1, q);
        }
    }
    if (OP == 4) {  // a failed factorization leaves B untouched
        if (inf == 0) {
            blk_bwd1_posv<NBLK>(T, x1, myinv_last, lt, xs, q, r);
            blk_x_store<NBLK, FULL>(x1, Bg, n, q, r);
        }
        return inf;
    }
    if (OP == 0 || inf != 0) return inf;  // a failed factorization leaves B untouched
    // off-diagonal blocks of L, negated: the forward pass subtracts L_kj Y_j
#pragma unroll
    for (int k = 1; k < NBLK; ++k)
#pragma unroll
        for (int j = 0; j < k; ++j) T[BI(k, j)] = neg4(T[BI(k, j)]);
    const int nr = OP == 3 ? 1 : nrhs;
    const bool fwd = OP != 3 || trans == 0, bwd = OP != 3 || trans != 0;
    for (int cb = 0; cb < nr; cb += 16) {
        f4_t Y[NBLK];
        rhs_load<NBLK, FULL>(Y, Bg, n, nr, cb, q, r);
        if (fwd) {
#pragma unroll
            for (int k = 0; k < NBLK; ++k) {
                f4_t s = Y[k];
#pragma unroll
                for (int j = 0; j < k; ++j) s = mma(T[BI(k, j)], Y[j], s);
                Y[k] = mma(linv[k], s, zero4());
            }
        }
        if (bwd) BwdBlk<NBLK, NBLK - 1>::run(T, linv, Y, xs, q, r);
        rhs_store<NBLK, FULL>(Y, Bg, n, nr, cb, q, r);
    }
    return 0;
}

}  // namespace glass
