// chol_device.hpp -- device routines of the Cholesky family shared by the
// factor / solve kernels (chol.hip) and the adjoint kernels (adjoint.hip).
//
// Thread scope: one problem per lane, its lower triangle in VGPRs at
// compile-time order N, staged in and out through LDS passes.
// Wave scope: one problem per wavefront, lane i owning row i in VGPRs.
#pragma once

#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {

// ------------------------------------------------------------ thread scope --
#define TI(i, j) ((i) * ((i) + 1) / 2 + (j))

GLASS_DEV int thread_stage_q_dev(int threads, int elems) {
    int s = thread_stride(elems);
    int q = kStagePassFloats / s;
    if (q < 1) q = 1;
    return q < threads ? q : threads;
}

// The lane's problem in LDS at src / dst, at the stride thread_stride(N * N)
// (16-byte aligned for even N): even orders move whole 16-byte pieces (the
// pieces wholly above the diagonal are not read), odd orders single floats.
template <int N>
GLASS_DEV void tri_load(float (&a)[N * (N + 1) / 2], const float* src) {
    if constexpr (N % 2 == 0) {
#pragma unroll
        for (int t = 0; t < N * N / 4; ++t) {
            if (4 * t / N == (4 * t + 3) / N && 4 * t % N > 4 * t / N) continue;  // one row, wholly above
            const f4_t v = *reinterpret_cast<const f4_t*>(src + 4 * t);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int g = 4 * t + e, gi = g / N, gj = g % N;
                if (gj <= gi) a[TI(gi, gj)] = v[e];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) a[TI(i, j)] = src[i * N + j];
    }
}

template <int N>
GLASS_DEV void tri_store_full(const float (&a)[N * (N + 1) / 2], float* dst) {
    if constexpr (N % 2 == 0) {
#pragma unroll
        for (int t = 0; t < N * N / 4; ++t) {
            f4_t v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int g = 4 * t + e, gi = g / N, gj = g % N;
                v[e] = gj <= gi ? a[TI(gi, gj)] : 0.f;
            }
            *reinterpret_cast<f4_t*>(dst + 4 * t) = v;
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) dst[i * N + j] = j <= i ? a[TI(i, j)] : 0.f;
    }
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
    constexpr int SZ = N * N, S = thread_stride(SZ);
    const int Q = thread_stage_q_dev(nt, SZ);
    const FastDiv fd = make_fastdiv(SZ);
    for (int s = 0; s < cnt; s += Q) {
        const int qn = min(Q, cnt - s);
        stage_in<ThreadU<N>::v>(lds, base + (size_t)s * SZ, qn * SZ, fd, S, tid, nt);
        __syncthreads();
        if (tid >= s && tid < s + qn) tri_load<N>(a, lds + (tid - s) * S);
        __syncthreads();
    }
}

template <int N>
GLASS_DEV void thread_store_tri(const float (&a)[N * (N + 1) / 2], float* __restrict__ base, float* lds,
                                int cnt, int tid, int nt) {
    constexpr int SZ = N * N, S = thread_stride(SZ);
    const int Q = thread_stage_q_dev(nt, SZ);
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


// The 16-byte pieces t = 0 .. NB / 4 - 1 of row r of the n x n row-major
// problem at float offset pb of the descriptor: the pieces at or left of the
// diagonal (4 t <= r) of a row that exists (ld), zero elsewhere.  Every lane
// issues one 16-byte load per piece into registers of its own (a lane with
// nothing to load reads the descriptor's first piece, which is in range),
// and all loads go out before any is read; the selects come after.  A piece
// of the problem's last row that would run past the problem is loaded as
// the problem's last 16 bytes and moved down by 4 t + 4 - n elements (zero
// above).  (Loads under a per-lane branch, or an element-wise load of that
// piece into the registers of the vector load, made the compiler wait for
// each piece before issuing the next.)  Elements past n of the other rows
// hold the next row's entries; loads are 4-byte aligned.
template <int NB>
GLASS_DEV void row_pieces(f4_t (&w)[NB / 4], __amdgpu_buffer_rsrc_t rs, int pb, int n, int r, bool ld) {
    if (n == 1) {  // the whole problem is one element
        const float x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ld ? pb * 4 : 0, 0, 0));
        w[0] = f4_t{ld && r == 0 ? x : 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 1; t < NB / 4; ++t) w[t] = f4_t{0.f, 0.f, 0.f, 0.f};
        return;
    }
    const bool last = r == n - 1;
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
        const bool want = ld && 4 * t <= r;
        const int off = !want ? 0 : (last && 4 * t + 4 > n) ? pb + n * n - 4 : pb + r * n + 4 * t;
        w[t] = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off * 4, 0, 0));
    }
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
        const bool want = ld && 4 * t <= r;
        const int sh = 4 * t + 4 - n;  // wave-uniform; 1..3 for the piece that holds column n - 1
        f4_t v = w[t];
        if (sh > 0 && sh < 4) {
            const f4_t d = sh == 1   ? f4_t{v[1], v[2], v[3], 0.f}
                           : sh == 2 ? f4_t{v[2], v[3], 0.f, 0.f}
                                     : f4_t{v[3], 0.f, 0.f, 0.f};
            v = last ? d : v;
        }
        w[t] = want ? v : f4_t{0.f, 0.f, 0.f, 0.f};
    }
}

// -------------------------------------------------------------- wave scope --
// Lane i owns row i.  Rows come straight from global memory with 16-byte
// buffer loads of only the column blocks at or left of the diagonal; blocks
// right of the diagonal block are zero.
//   MASK (L used as stored: POTRS, TRSV, the adjoint): the diagonal block is
//     cut at the diagonal and rows past n are zero.
//   !MASK (a factorization): the diagonal block keeps whatever the row holds
//     past the diagonal -- it stays in the upper part (an update of row i
//     writes only columns past the current step, and those of row i's lower
//     part use only lower entries) and wave_potrf clears it at the end -- and
//     rows past n are identity rows, so their steps take a unit pivot and
//     leave every other row unchanged.  The identity is built from the lane's
//     own 4-wide block and element (no compare per column, which would stay
//     live across the unrolled factorization).
template <int NB, bool MASK>
GLASS_DEV void rows_load_lower(float (&a)[NB], const float* Ag, int n, int lane) {
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(Ag, (uint32_t)(n * n) * 4u);
    const bool row = lane < n;
    f4_t w[NB / 4];
    row_pieces<NB>(w, rs, 0, n, lane, row);
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
        const f4_t v = w[t];
        if (MASK) {
#pragma unroll
            for (int e = 0; e < 4; ++e) a[4 * t + e] = (4 * t + e <= lane) ? v[e] : 0.f;
        } else {
            const bool dblk = !row && t == (lane >> 2);
#pragma unroll
            for (int e = 0; e < 4; ++e) a[4 * t + e] = (dblk && e == (lane & 3)) ? 1.f : v[e];
        }
    }
}

// v in the lane whose bit is set in the constant mask 1 << J, `other` in the
// rest: one v_cndmask on a scalar literal mask (a lane compare per step would
// keep 64 compare results alive across the unrolled factorization).  The
// compiler does not insert wait states for operands read inside inline asm:
// v comes straight from v_rsq (a transcendental result needs one wait state
// before a VALU reads it), so the block starts with s_nop 1.
template <int J>
GLASS_DEV float lane_select(float other, float v) {
    float r;
    asm("s_nop 1\n\tv_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(other), "v"(v), "s"(1ull << J));
    return r;
}

// The scalar v written into lane K of `old` (immediate lane select).  v is
// the SGPR a v_readlane has just written; a VALU read of an SGPR written by a
// VALU needs wait states the compiler does not insert for inline asm, so the
// block starts with s_nop 4 (five wait states, above every such requirement).
template <int K>
GLASS_DEV float writelane(float v, float old) {
    asm("s_nop 4\n\tv_writelane_b32 %0, %1, %2" : "+v"(old) : "s"(v), "i"(K));
    return old;
}

// One column step of the right-looking factorization: the pivot of column J
// comes from v_readlane, the scaled column is broadcast with DPP and each lane
// updates the rest of its row in VGPRs (a[K] -= l_iJ * l_KJ, one v_fmac each).
template <int NB, int J, int K>
struct WaveUpd {
    static GLASS_DEV void run(float (&a)[NB], const float (&R)[4], float m) {
        fnmac_bcast<K % 16>(a[K], R[K / 16], m);
        WaveUpd<NB, J, K + 1>::run(a, R, m);
    }
};
template <int NB, int J>
struct WaveUpd<NB, J, NB> {
    static GLASS_DEV void run(float (&)[NB], const float (&)[4], float) {}
};

// A step does not test its pivot: 1/L_JJ = rsq(d) is kept per lane, and rsq
// is not finite exactly when !(d > 0) (+inf at +0, -inf at -0, NaN below 0
// and at NaN, finite and positive for every positive finite d, +0 at +inf),
// so the first non-finite lane after the last step is info - 1.
template <int NB, int J>
struct WaveStep {
    static GLASS_DEV void run(float (&a)[NB], int lane, int& info, float& myinv) {
        const float d = readlane(a[J], J);
        const float inv = rsq(d);
        float v = a[J] * inv;  // in lane J, a[J] is the pivot itself: v = sqrt(d)
        myinv = lane_select<J>(myinv, inv);
        float R[4];
        if ((NB + 15) / 16 == 1) {
            asm volatile("s_nop 1" : "+v"(v));  // wait states before the DPP reads of v
            R[0] = R[1] = R[2] = R[3] = v;
        } else {
            replicate_rows<(NB + 15) / 16>(v, R);
        }
        a[J] = v;
        WaveUpd<NB, J, J + 1>::run(a, R, v);
        WaveStep<NB, J + 1>::run(a, lane, info, myinv);
    }
};
template <int NB>
struct WaveStep<NB, NB> {
    static GLASS_DEV void run(float (&)[NB], int, int& info, float& myinv) { info = first_nonfinite<64>(myinv); }
};

// Factor the rows in place (identity rows past the order); returns info, sets
// myinv = 1 / L_ii and clears the strict upper part of every row.
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
// Each solved unknown is written into its lane with v_writelane; the update
// runs in every lane (lane k's own accumulator is not used again).
template <int NB, int K, int RG>
struct FwdStep {
    static GLASS_DEV void run(const float (&a)[NB], float (&acc)[RG], float (&y)[RG], float myinv) {
        float yk[RG];
#pragma unroll
        for (int c = 0; c < RG; ++c) yk[c] = readlane(acc[c] * myinv, K);
#pragma unroll
        for (int c = 0; c < RG; ++c) {
            acc[c] = fmaf(-a[K], yk[c], acc[c]);
            y[c] = writelane<K>(yk[c], y[c]);
        }
        FwdStep<NB, K + 1, RG>::run(a, acc, y, myinv);
    }
};
template <int NB, int RG>
struct FwdStep<NB, NB, RG> {
    static GLASS_DEV void run(const float (&)[NB], float (&)[RG], float (&)[RG], float) {}
};

template <int NB>
GLASS_DEV float wave_fwd(const float (&a)[NB], float acc, float myinv, int lane) {
    float accv[1] = {acc}, y[1] = {0.f};
    FwdStep<NB, 0, 1>::run(a, accv, y, myinv);
    return y[0];
}

// Rows r0 .. r0+7 of L (strict upper +0, identity padding past n) from the
// owning lanes into the LDS chunk buffer, row stride NB: every lane of the
// chunk writes its whole padded row with 16-byte stores and no per-element
// predicate (a predicate per column of a runtime n spilled scalar registers).
template <int NB>
GLASS_DEV void rows_to_lds(const float (&a)[NB], float* buf, int r0, int lane) {
    if (lane >= r0 && lane < r0 + 8) {
        float* dst = buf + (lane - r0) * NB;
#pragma unroll
        for (int t = 0; t < NB / 4; ++t) {
            f4_t v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = a[4 * t + e];
            *reinterpret_cast<f4_t*>(dst + 4 * t) = v;
        }
    }
}

// Coalesced copy of `rows` rows of n floats from the LDS chunk (row stride
// NB) to contiguous global memory (row stride n).  vec: n % 4 == 0 and dst
// 16-byte aligned.
template <int NB>
GLASS_DEV void chunk_to_global(float* __restrict__ dst, const float* buf, int rows, int n, bool vec, int lane) {
    if (vec) {
        const int n4 = n >> 2;
        const FastDiv f4 = make_fastdiv((uint32_t)n4);
        for (int q = lane; q < rows * n4; q += 64) {
            const int rr = (int)fdiv((uint32_t)q, f4), c4 = q - rr * n4;
            reinterpret_cast<f4_t*>(dst)[q] = *reinterpret_cast<const f4_t*>(buf + rr * NB + 4 * c4);
        }
    } else {
        const FastDiv fn = make_fastdiv((uint32_t)n);
        for (int g = lane; g < rows * n; g += 64) {
            const int rr = (int)fdiv((uint32_t)g, fn), cc = g - rr * n;
            dst[g] = buf[rr * NB + cc];
        }
    }
}

// Backward substitution L^T x = y for the rows of the chunk in LDS (rows
// r0 .. r1-1, descending, row stride NB); lane i < k reads L_ki from row k.
template <int NB>
GLASS_DEV float wave_bwd_chunk(const float* buf, int r0, int r1, float acc, float myinv, int lane) {
    // the chunk's eight entries of column `lane` are read before the steps
    // (a read at each step put an LDS round trip on the dependent chain)
    float lk[8];
    const int col = lane < NB ? lane : 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) lk[j] = buf[j * NB + col];
#pragma unroll
    for (int j = 7; j >= 0; --j) {
        if (j < r1 - r0) {  // wave-uniform
            const int k = r0 + j;
            const float lki = lane < k ? lk[j] : 0.f;
            const float xk = readlane(acc * myinv, k);
            acc = lane == k ? xk : fmaf(-lki, xk, acc);
        }
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
        rows_to_lds<NB>(a, buf, r0, lane);
        wave_sync();
        if (Lg) chunk_to_global<NB>(Lg + r0 * n, buf, r1 - r0, n, vec, lane);
        if (bwd) acc = wave_bwd_chunk<NB>(buf, r0, r1, acc, myinv, lane);
        wave_sync();
    }
    return acc;
}

// ------------------------------------------- several right-hand sides at once
// The substitutions for RG columns run in one sweep: each step broadcasts RG
// unknowns (independent v_readlane) and updates RG accumulators, so the
// dependent chain is n steps for the whole group instead of n per column.
template <int NB, int RG>
GLASS_DEV void wave_fwd_rg(const float (&a)[NB], float (&acc)[RG], float (&y)[RG], float myinv, int lane) {
#pragma unroll
    for (int c = 0; c < RG; ++c) y[c] = 0.f;
    FwdStep<NB, 0, RG>::run(a, acc, y, myinv);
}

template <int NB, int RG>
GLASS_DEV void wave_bwd_chunk_rg(const float* buf, int r0, int r1, float (&acc)[RG], float myinv, int lane) {
    float lk[8];  // read before the steps, as in wave_bwd_chunk
    const int col = lane < NB ? lane : 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) lk[j] = buf[j * NB + col];
#pragma unroll
    for (int j = 7; j >= 0; --j) {
        if (j < r1 - r0) {  // wave-uniform
            const int k = r0 + j;
            const float lki = lane < k ? lk[j] : 0.f;
            float xk[RG];
#pragma unroll
            for (int c = 0; c < RG; ++c) xk[c] = readlane(acc[c] * myinv, k);
#pragma unroll
            for (int c = 0; c < RG; ++c) acc[c] = lane == k ? xk[c] : fmaf(-lki, xk[c], acc[c]);
        }
    }
}

// Columns c0 .. c0+RG-1 of the row-major [n][nrhs] block Bg (columns past
// nrhs are zero padding and are not stored); the backward sweep walks the
// 8-row chunks of L bottom-up and, when Lg is given, also stores L.
template <int NB, int RG>
GLASS_DEV void wave_solve_cols(const float (&a)[NB], float* buf, float* Lg, bool vec, float* Bg, int n, int nrhs,
                               int c0, float myinv, int lane) {
    float acc[RG], y[RG];
#pragma unroll
    for (int c = 0; c < RG; ++c) {  // unconditional loads (Bg[0] for the rest), so that all issue at once
        const bool ok = lane < n && c0 + c < nrhs;
        const float v = Bg[ok ? lane * nrhs + c0 + c : 0];
        acc[c] = ok ? v : 0.f;
    }
    wave_fwd_rg<NB, RG>(a, acc, y, myinv, lane);
    for (int r0 = (n - 1) & ~7; r0 >= 0; r0 -= 8) {
        const int r1 = min(r0 + 8, n);
        rows_to_lds<NB>(a, buf, r0, lane);
        wave_sync();
        if (Lg) chunk_to_global<NB>(Lg + r0 * n, buf, r1 - r0, n, vec, lane);
        wave_bwd_chunk_rg<NB, RG>(buf, r0, r1, y, myinv, lane);
        wave_sync();
    }
#pragma unroll
    for (int c = 0; c < RG; ++c)
        if (lane < n && c0 + c < nrhs) Bg[lane * nrhs + c0 + c] = y[c];
}

// All nrhs columns in groups of 8, 4 or 1 (L stored during the first group).
template <int NB>
GLASS_DEV void wave_solve_all(const float (&a)[NB], float* buf, float* Lg, bool vec, float* Bg, int n, int nrhs,
                              float myinv, int lane) {
    for (int c0 = 0; c0 < nrhs;) {
        float* L = c0 == 0 ? Lg : nullptr;
        const int left = nrhs - c0;
        if (left >= 5) {
            wave_solve_cols<NB, 8>(a, buf, L, vec, Bg, n, nrhs, c0, myinv, lane);
            c0 += 8;
        } else if (left >= 2) {
            wave_solve_cols<NB, 4>(a, buf, L, vec, Bg, n, nrhs, c0, myinv, lane);
            c0 += 4;
        } else {
            wave_solve_cols<NB, 1>(a, buf, L, vec, Bg, n, nrhs, c0, myinv, lane);
            c0 += 1;
        }
    }
}

// --------------------------------------------------- segments of a wavefront
// A wavefront split into 64 / SEG segments of SEG lanes (SEG = 16: the four
// 16-lane DPP rows; SEG = 32: the two halves), each running its own problem
// with lane i of the segment owning row i.  Broadcasts stay inside a segment.

template <int SEG>
constexpr unsigned long long seg_mask() {
    return SEG == 16 ? 0x0001000100010001ull : 0x0000000100000001ull;
}

// Lane K of every segment, broadcast to its segment.  Inline asm gets no
// compiler wait states: the DPP read is preceded by s_nop 1.
template <int SEG, int K>
GLASS_DEV float seg_bcast(float v) {
    float src = v;
    if (SEG == 32) {
        float R[4];
        replicate_rows<2>(v, R);  // ends with the wait states a DPP read needs
        src = R[K / 16];
    }
    float r;
    asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                 : "=v"(r)
                 : "v"(src), "n"(K % 16));
    return r;
}

// v in lane K of every segment, `other` elsewhere (literal mask; s_nop 1 covers
// a transcendental or DPP result read as an operand).
template <int SEG, int K>
GLASS_DEV float seg_select(float other, float v) {
    float r;
    asm("s_nop 1\n\tv_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(other), "v"(v), "s"(seg_mask<SEG>() << K));
    return r;
}

// One column step.  SEG = 16: the pivot is one DPP broadcast and the scaled
// column l_iJ = a_iJ / sqrt(d) is broadcast for the update.  SEG = 32: a
// cross-row broadcast needs a permlane16 swap first, so the raw column a_iJ is
// replicated once and serves both the pivot and the update, which then scales
// by a_iJ / d in the lane (a_iK -= a_KJ * (a_iJ / d), the same product as
// l_iJ * l_KJ).
template <int SEG, int NB, int J>
struct SegStep {
    static GLASS_DEV void run(float (&a)[NB], int& info, float& myinv) {
        float R[4];
        float d, m;
        if (SEG == 16) {
            d = seg_bcast<SEG, J>(a[J]);
        } else {
            replicate_rows<2>(a[J], R);
            asm volatile("v_mov_b32_dpp %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                         : "=v"(d)
                         : "v"(R[J / 16]), "n"(J % 16));
        }
        const float inv = rsq(d);
        myinv = seg_select<SEG, J>(myinv, inv);
        if (SEG == 16) {
            float v = a[J] * inv;  // in lane J of the segment, a[J] is the pivot itself
            asm volatile("s_nop 1" : "+v"(v));  // wait states before the DPP reads of v
            a[J] = v;
            R[0] = R[1] = R[2] = R[3] = v;
            m = v;
        } else {
            m = a[J] * (inv * inv);
            a[J] *= inv;
        }
        WaveUpd<NB, J, J + 1>::run(a, R, m);
        SegStep<SEG, NB, J + 1>::run(a, info, myinv);
    }
};
// The pivots are tested once, after the last step, as in WaveStep: myinv of
// a segment's lane i is 1 / L_ii (1 past the order), not finite exactly for
// the failed pivots.
template <int SEG, int NB>
struct SegStep<SEG, NB, NB> {
    static GLASS_DEV void run(float (&)[NB], int& info, float& myinv) { info = first_nonfinite<SEG>(myinv); }
};

// acc -= bcast_K(acc) * m within the segment: lane K's own value, broadcast
// from the accumulating register itself (SEG = 32: replicated across the two
// 16-lane rows first); s_nop 1 gives the DPP read of acc its wait states.
template <int SEG, int K>
GLASS_DEV void seg_fnmac_self(float& acc, float m) {
    if (SEG == 16) {
        asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, -%1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(m), "n"(K));
    } else {
        float R[4];
        replicate_rows<2>(acc, R);  // ends with the wait states a DPP read needs
        fnmac_bcast<K % 16>(acc, R[K / 16], m);
    }
}

// Forward substitution L y = b on the lane's own coefficients: w holds
// b_i / L_ii on entry and y_i on exit; step K subtracts m_K y_K with
// m_K = L_iK / L_ii (row i scaled by its own 1 / L_ii, diagonal entry and
// upper part zero, so lane K and the lanes above it are left alone), y_K
// being lane K's w, final by then.  One DPP FMA per unknown on the
// dependent chain.
template <int SEG, int NB, int K, int RG>
struct SegFwdL {
    static GLASS_DEV void run(const float (&m)[NB], float (&w)[RG]) {
#pragma unroll
        for (int c = 0; c < RG; ++c) seg_fnmac_self<SEG, K>(w[c], m[K]);
        SegFwdL<SEG, NB, K + 1, RG>::run(m, w);
    }
};
template <int SEG, int NB, int RG>
struct SegFwdL<SEG, NB, NB, RG> {
    static GLASS_DEV void run(const float (&)[NB], float (&)[RG]) {}
};

// Row i of L scaled by 1 / L_ii, in place: the coefficients of SegFwdL.
template <int NB>
GLASS_DEV void seg_scale_row(float (&a)[NB], float myinv) {
#pragma unroll
    for (int k = 0; k < NB; ++k) a[k] *= myinv;
}

// Backward substitution L^T x = y; row K of the segment's L is read from its
// LDS block (row stride NB + 4; lane i takes L_Ki, zero for K <= i), AHEAD
// steps before row K is used (the first AHEAD rows by the prologue).  In the
// one-column solves (EARLY, AHEAD = kSegBwdAhead) a read at its own step,
// behind the inline-asm DPP steps, put one LDS round trip on every step of
// the dependent chain.  The column groups of seg_solve_all read at the step
// (AHEAD = 0): they share each read among their columns, and there the rows
// of L stay live for the next group, so reads moved up would add NB
// registers to the kernel.
constexpr int kSegBwdAhead = 8;

// COND: a read under the lane's condition, which the compiler leaves at its
// step; otherwise an unconditional read of an in-range entry and a select.
template <int NB, int K, bool COND>
GLASS_DEV void seg_col_read(const float* sb, int i, float (&lc)[NB]) {
    if (K >= 0) {
        if (COND) {
            lc[K] = i < K ? sb[K * (NB + 4) + i] : 0.f;
        } else {
            const float v = sb[K * (NB + 4) + (i < K ? i : 0)];
            lc[K] = i < K ? v : 0.f;
        }
    }
}

template <int NB, int K, int STOP>
struct SegBwdPrologue {
    static GLASS_DEV void run(const float* sb, int i, float (&lc)[NB]) {
        seg_col_read<NB, K, false>(sb, i, lc);
        SegBwdPrologue<NB, K - 1, STOP>::run(sb, i, lc);
    }
};
template <int NB, int STOP>
struct SegBwdPrologue<NB, STOP, STOP> {
    static GLASS_DEV void run(const float*, int, float (&)[NB]) {}
};

// Step K on the lane's own coefficients: w_i -= (L_Ki / L_ii) x_K with x_K
// lane K's w (L_Ki is read as zero for K <= i, so lane K and the lanes below
// it are left alone).
template <int SEG, int NB, int K, int RG, int AHEAD>
struct SegBwd {
    static GLASS_DEV void run(const float* sb, int i, float (&lc)[NB], float (&w)[RG], float myinv) {
        seg_col_read<NB, (K - AHEAD >= 0 ? K - AHEAD : -1), AHEAD == 0>(sb, i, lc);
        const float m = lc[K] * myinv;
#pragma unroll
        for (int c = 0; c < RG; ++c) seg_fnmac_self<SEG, K>(w[c], m);
        SegBwd<SEG, NB, K - 1, RG, AHEAD>::run(sb, i, lc, w, myinv);
    }
};
template <int SEG, int NB, int RG, int AHEAD>
struct SegBwd<SEG, NB, -1, RG, AHEAD> {
    static GLASS_DEV void run(const float*, int, float (&)[NB], float (&)[RG], float) {}
};

// L^T x = y for the segment (sb: its L in LDS).
template <int SEG, int NB, int RG, bool EARLY>
GLASS_DEV void seg_bwd(const float* sb, int i, float (&y)[RG], float myinv) {
    constexpr int AHEAD = EARLY ? (kSegBwdAhead < NB ? kSegBwdAhead : NB) : 0;
    float lc[NB];
    // the early reads start here, not above the forward pass (where the
    // rows of L are still live)
    if (AHEAD > 0) asm volatile("" ::: "memory");
    SegBwdPrologue<NB, NB - 1, NB - 1 - AHEAD>::run(sb, i, lc);
#pragma unroll
    for (int c = 0; c < RG; ++c) y[c] *= myinv;  // x_i = y_i / L_ii - sum_{K>i} (L_Ki / L_ii) x_K
    SegBwd<SEG, NB, NB - 1, RG, AHEAD>::run(sb, i, lc, y, myinv);
}

// Columns c0 .. c0+RG-1 of segment-local right-hand sides Bs (row-major
// [n][r]; columns past r and rows past n are zero padding and are not
// stored); act: this lane's segment has a problem to solve.  sb: the
// segment's L in LDS, row stride NB + 4.  a: row i of L for the forward
// pass with its diagonal entry zero, scaled by 1 / L_ii (the coefficients of
// SegFwdL).
template <int SEG, int NB, int RG>
GLASS_DEV void seg_solve_cols(const float (&a)[NB], const float* sb, float* Bs, int n, int r, int c0, int i,
                              float myinv, bool act, bool fwd, bool bwd, const float* Bsafe) {
    float y[RG];
#pragma unroll
    for (int c = 0; c < RG; ++c) {  // unconditional loads (Bsafe for the rest), so that all issue at once
        const bool ok = act && i < n && c0 + c < r;
        const float v = *(ok ? Bs + i * r + c0 + c : Bsafe);
        y[c] = ok ? v : 0.f;
    }
    if (fwd) {
#pragma unroll
        for (int c = 0; c < RG; ++c) y[c] *= myinv;
        SegFwdL<SEG, NB, 0, RG>::run(a, y);
    }
    if (bwd) seg_bwd<SEG, NB, RG, false>(sb, i, y, myinv);
#pragma unroll
    for (int c = 0; c < RG; ++c)
        if (act && i < n && c0 + c < r) Bs[i * r + c0 + c] = y[c];
}

// One right-hand side, already in b (lane i of the segment: b_i, zero past
// n), so that its load could issue with the rows: solved and stored to Bs.
// a as for seg_solve_cols.
template <int SEG, int NB>
GLASS_DEV void seg_solve_one(const float (&a)[NB], const float* sb, float* Bs, int n, int i, float myinv, bool act,
                             bool fwd, bool bwd, float b) {
    float y[1] = {b};
    if (fwd) {
        y[0] *= myinv;
        SegFwdL<SEG, NB, 0, 1>::run(a, y);
    }
    if (bwd) seg_bwd<SEG, NB, 1, true>(sb, i, y, myinv);
    if (act && i < n) Bs[i] = y[0];
}

// All columns of every segment in groups of 8 / 4 / 1.  r is this lane's
// segment's column count (the row stride of its Bs); the groups run to
// rloop, which must be wave-uniform and at least every segment's r (every
// DPP step runs in all lanes): the batch's nrhs for a uniform batch (the
// default), the wavefront's largest count for a ragged one.  Bsafe: an
// address every lane may read, which lanes with nothing to load read instead
// so that the loads need no branch (default Bs, when every lane's Bs is
// valid).  a as for seg_solve_cols.
template <int SEG, int NB>
GLASS_DEV void seg_solve_all(const float (&a)[NB], const float* sb, float* Bs, int n, int r, int i, float myinv,
                             bool act, bool fwd, bool bwd, int rloop = -1, const float* Bsafe = nullptr) {
    if (rloop < 0) rloop = r;
    if (!Bsafe) Bsafe = Bs;
    for (int c0 = 0; c0 < rloop;) {
        const int left = rloop - c0;
        if (left >= 5) {
            seg_solve_cols<SEG, NB, 8>(a, sb, Bs, n, r, c0, i, myinv, act, fwd, bwd, Bsafe);
            c0 += 8;
        } else if (left >= 2) {
            seg_solve_cols<SEG, NB, 4>(a, sb, Bs, n, r, c0, i, myinv, act, fwd, bwd, Bsafe);
            c0 += 4;
        } else {
            seg_solve_cols<SEG, NB, 1>(a, sb, Bs, n, r, c0, i, myinv, act, fwd, bwd, Bsafe);
            c0 += 1;
        }
    }
}

// Row i of segment s's problem (lane 16s + i or 32s + i) from the wavefront's
// np adjacent problems starting at base.  The padding follows
// rows_load_lower (identity rows for a factorization, zero rows otherwise;
// a segment past np holds only padding rows).  MASK (L as stored: the
// solves, the adjoint): the strict lower part only -- the callers load the
// diagonal apart, and the lane-local substitutions want it zero in the row.
// !MASK (a factorization): as rows_load_lower.
template <int NB, bool MASK>
GLASS_DEV void seg_load_rows(float (&a)[NB], const float* base, int np, int n, int s, int i) {
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(base, (uint32_t)(np * n * n) * 4u);
    const bool row = s < np && i < n;
    f4_t w[NB / 4];
    row_pieces<NB>(w, rs, s * n * n, n, i, row);
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
        const f4_t v = w[t];
        if (MASK) {
#pragma unroll
            for (int e = 0; e < 4; ++e) a[4 * t + e] = (4 * t + e < i) ? v[e] : 0.f;
        } else {
            const bool dblk = !row && t == (i >> 2);
#pragma unroll
            for (int e = 0; e < 4; ++e) a[4 * t + e] = (dblk && e == (i & 3)) ? 1.f : v[e];
        }
    }
}

// Rows of L (strict upper +0) into the segment's LDS block.
template <int NB>
GLASS_DEV void seg_rows_to_lds(const float (&a)[NB], float* sb, int i) {
    if (i < NB) {
#pragma unroll
        for (int t = 0; t < NB / 4; ++t) {
            f4_t v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = a[4 * t + e];
            *reinterpret_cast<f4_t*>(sb + i * (NB + 4) + 4 * t) = v;
        }
    }
}

// The wavefront's np n x n problems (contiguous in global memory: L, or the
// adjoint's dA) from the segment blocks: one flat, coalesced copy (16-byte stores when n % 4 == 0
// and dst is 16-byte aligned, so four consecutive elements share a row).
template <int NB>
GLASS_DEV void seg_store_L(float* __restrict__ dst, const float* buf, int np, int n, bool vec, int lane) {
    const int nn = n * n;
    const FastDiv fnn = make_fastdiv((uint32_t)nn), fn = make_fastdiv((uint32_t)n);
    if (vec) {
        for (int q = lane; q < np * nn / 4; q += 64) {
            const int g = 4 * q;
            const int s = (int)fdiv((uint32_t)g, fnn), rem = g - s * nn;
            const int i = (int)fdiv((uint32_t)rem, fn), j = rem - i * n;
            reinterpret_cast<f4_t*>(dst)[q] =
                *reinterpret_cast<const f4_t*>(buf + s * NB * (NB + 4) + i * (NB + 4) + j);
        }
        return;
    }
    for (int g = lane; g < np * nn; g += 64) {
        const int s = (int)fdiv((uint32_t)g, fnn), rem = g - s * nn;
        const int i = (int)fdiv((uint32_t)rem, fn), j = rem - i * n;
        dst[g] = buf[s * NB * (NB + 4) + i * (NB + 4) + j];
    }
}

// 1 / L_ii of lane i's row (1 beyond n), read from global memory.
// L_ii of the lane's row, loaded unconditionally (a lane past n reads L_00)
// so that the load can issue with the row loads; diag_inv of it.
GLASS_DEV float diag_load(const float* Lg, int n, int lane) { return Lg[(lane < n ? lane : 0) * (n + 1)]; }
GLASS_DEV float diag_inv(float d, int n, int lane) { return lane < n ? recip(d) : 1.f; }

// x[lane] for lane < n, else 0, loaded unconditionally (x[0] is read instead).
GLASS_DEV float lane_elem(const float* x, int n, int lane) {
    const float v = x[lane < n ? lane : 0];
    return lane < n ? v : 0.f;
}


}  // namespace glass
