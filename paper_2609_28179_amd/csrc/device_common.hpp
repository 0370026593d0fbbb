// device_common.hpp -- device helpers shared by the gfx950 kernels:
// exact division by a small runtime divisor, coalesced staging of a
// batch-contiguous span into padded LDS rows (and back), wavefront-local
// synchronisation and lane broadcast.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GLASS_DEV __device__ __forceinline__

namespace glass {

// q = g / d for 0 <= g < 2^20 and 1 <= d <= 4096: m = ceil(2^32 / d) gives
// m*d = 2^32 + e with 0 <= e < d, so g*m / 2^32 = g/d + g*e/(d 2^32) and the
// error term stays below 1/d whenever g*e < 2^32.
struct FastDiv {
    uint32_t d;
    uint32_t m;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    f.m = d <= 1 ? 0u : (uint32_t)((0x100000000ull + d - 1) / d);
    return f;
}

GLASS_DEV uint32_t fdiv(uint32_t g, FastDiv f) { return f.d <= 1 ? g : __umulhi(g, f.m); }

// Wavefront-local barrier: orders this wave's LDS writes before its later LDS
// reads by other lanes (LDS instructions of one wave complete in order; the
// fences keep the compiler from moving accesses across this point).
GLASS_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of this thread's wavefront within its workgroup as a wave-uniform
// (scalar) value.  Addresses and buffer descriptors derived from it then live
// in SGPRs; derived from threadIdx.x directly they are per-lane values to the
// compiler, which wraps every buffer load in a readfirstlane loop.
GLASS_DEV int wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// A value the caller knows to be equal in every active lane, as a scalar.
GLASS_DEV int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
GLASS_DEV long long uniform_i64(long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

GLASS_DEV float readlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));

GLASS_DEV bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// 1 / x by v_rcp_f32 (1 ulp; +-inf at +-0, NaN at NaN), the reciprocal of a
// given diagonal entry in the solves, as the factorizations take their pivots'
// reciprocal square roots from v_rsq_f32.  A correctly rounded division is a
// sequence of about ten instructions.
GLASS_DEV float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Write 4 consecutive span elements starting at element g into the padded
// LDS layout (rows of cols.d floats at stride ldst).
GLASS_DEV void lds_put4(float* dst, int g, const f4_t& v, FastDiv cols, int ldst) {
    int r = (int)fdiv((uint32_t)g, cols), c = g - r * (int)cols.d;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        dst[r * ldst + c] = v[e];
        if (++c == (int)cols.d) {
            c = 0;
            ++r;
        }
    }
}

GLASS_DEV f4_t lds_get4(const float* src, int g, FastDiv cols, int ldst) {
    int r = (int)fdiv((uint32_t)g, cols), c = g - r * (int)cols.d;
    f4_t v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] = src[r * ldst + c];
        if (++c == (int)cols.d) {
            c = 0;
            ++r;
        }
    }
    return v;
}

// Raw buffer descriptor over `bytes` bytes at p (dword 3 = 0x00020000: 32-bit
// data format, the raw-buffer setting of gfx9-family parts).  Loads outside
// [0, bytes) return 0 and do not touch memory.
GLASS_DEV __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Copy src[0 .. len) (contiguous, global) into LDS re-laid as rows of
// `cols.d` floats at row stride `ldst`: element g lands at
// dst[(g / cols) * ldst + g % cols].  `nt` cooperating lanes, this one is
// `tid`.  All loads are 16-byte buffer loads from the 16-byte-aligned
// address at or below src (that block lies in the same page as src, and the
// up to 12 extra bytes on either side are loaded but never stored), and every
// lane issues its U loads of a chunk before the first LDS write, so a
// wavefront keeps U KiB in flight: the staging of a batch span is bandwidth-,
// not latency-bound.  The per-load offsets are scalar, so the loads in flight
// cost only their data VGPRs.
//
// When src and dst are 16-byte aligned and every 16-byte piece lands whole
// at a 16-byte-aligned LDS address (rows unpadded, or rows and stride both
// multiples of 4 floats), each piece is one 16-byte LDS write: consecutive
// lanes then fill consecutive bank groups.  Otherwise the piece is split
// into four 4-byte writes, which conflict (lanes 16 bytes apart).
template <int U>
GLASS_DEV void stage_in(float* dst, const float* __restrict__ src, int len, FastDiv cols, int ldst, int tid,
                        int nt) {
    const uintptr_t addr = reinterpret_cast<uintptr_t>(src);
    const int shift = (int)((addr & 15) >> 2);
    const float* base_p = reinterpret_cast<const float*>(addr & ~(uintptr_t)15);
    const int n4 = (shift + len + 3) >> 2;
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(base_p, (uint32_t)n4 * 16u);
    const int d = (int)cols.d, pad = ldst - d;
    const bool wide = shift == 0 && aligned16(dst) && (pad == 0 || ((d & 3) == 0 && (ldst & 3) == 0));
    for (int base = 0; base < n4; base += U * nt) {
        f4_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, tid * 16, (base + u * nt) * 16, 0));
        if (wide) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int g = 4 * (base + u * nt + tid);
                if (g < len) {
                    const int off = pad == 0 ? g : g + (int)fdiv((uint32_t)g, cols) * pad;
                    if (g + 4 <= len) {
                        *reinterpret_cast<f4_t*>(dst + off) = v[u];
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (g + e < len) dst[off + e] = v[u][e];
                    }
                }
            }
            continue;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = base + u * nt + tid;
            if (q < n4) {
                int g = 4 * q - shift;
                const int g0 = g < 0 ? 0 : g;
                int r = (int)fdiv((uint32_t)g0, cols), c = g0 - r * d;
#pragma unroll
                for (int e = 0; e < 4; ++e, ++g) {
                    if (g >= 0 && g < len) {
                        dst[r * ldst + c] = v[u][e];
                        if (++c == d) {
                            c = 0;
                            ++r;
                        }
                    }
                }
            }
        }
    }
}

// Loads per lane (U of stage_in) that cover an n x n problem staged by one
// wavefront in a single chunk, for the largest n of a size bucket.
template <int NB>
struct WaveU {
    static constexpr int v = NB * NB <= 512 ? 2 : NB * NB <= 1024 ? 4 : NB * NB <= 2048 ? 8 : 16;
};

// Loads per lane of stage_in for the thread scope at order N: the whole
// pass in one round of loads up to order 8 (N * N / 4 pieces per lane).
template <int N>
struct ThreadU {
    static constexpr int v = N * N <= 64 ? (N * N + 3) / 4 : 8;
};

// A lane's own row of L floats in LDS at p, whose float offset from a
// 16-byte boundary is a multiple of AL (4, 2 or 1): 16-, 8- or 4-byte
// accesses, the widest the alignment and length allow.  Used on the thread
// scope's staged problems, whose stride (thread_stride) makes the wide
// accesses of a wavefront's lanes fall on distinct bank groups.
template <int L, int AL>
GLASS_DEV void lds_row_get(float* v, const float* p) {
    if constexpr (AL % 4 == 0 && L % 4 == 0) {
#pragma unroll
        for (int t = 0; t < L / 4; ++t) {
            const f4_t x = *reinterpret_cast<const f4_t*>(p + 4 * t);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[4 * t + e] = x[e];
        }
    } else if constexpr (AL % 2 == 0 && L % 2 == 0) {
#pragma unroll
        for (int t = 0; t < L / 2; ++t) {
            const f2_t x = *reinterpret_cast<const f2_t*>(p + 2 * t);
            v[2 * t] = x[0];
            v[2 * t + 1] = x[1];
        }
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) v[t] = p[t];
    }
}

template <int L, int AL>
GLASS_DEV void lds_row_put(float* p, const float* v) {
    if constexpr (AL % 4 == 0 && L % 4 == 0) {
#pragma unroll
        for (int t = 0; t < L / 4; ++t)
            *reinterpret_cast<f4_t*>(p + 4 * t) = f4_t{v[4 * t], v[4 * t + 1], v[4 * t + 2], v[4 * t + 3]};
    } else if constexpr (AL % 2 == 0 && L % 2 == 0) {
#pragma unroll
        for (int t = 0; t < L / 2; ++t) *reinterpret_cast<f2_t*>(p + 2 * t) = f2_t{v[2 * t], v[2 * t + 1]};
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) p[t] = v[t];
    }
}

// Inverse of stage_in: dst[g] = src_lds[(g / cols) * ldst + g % cols], with
// 16-byte stores when dst is 16-byte aligned (and 16-byte LDS reads under
// the same condition as stage_in's 16-byte writes).
GLASS_DEV void stage_out(float* __restrict__ dst, const float* src, int len, FastDiv cols, int ldst, int tid,
                         int nt) {
    const int d = (int)cols.d, pad = ldst - d;
    if (aligned16(dst) && aligned16(src) && (pad == 0 || ((d & 3) == 0 && (ldst & 3) == 0))) {
        const int len4 = len >> 2;
        f4_t* d4 = reinterpret_cast<f4_t*>(dst);
        for (int q = tid; q < len4; q += nt) {
            const int g = 4 * q;
            d4[q] = *reinterpret_cast<const f4_t*>(src + (pad == 0 ? g : g + (int)fdiv((uint32_t)g, cols) * pad));
        }
        const int g = (len4 << 2) + tid;
        if (g < len) dst[g] = src[g + (int)fdiv((uint32_t)g, cols) * pad];
        return;
    }
    if (aligned16(dst)) {
        const int len4 = len >> 2;
        f4_t* d4 = reinterpret_cast<f4_t*>(dst);
        for (int q = tid; q < len4; q += nt) d4[q] = lds_get4(src, q * 4, cols, ldst);
        const int g = (len4 << 2) + tid;
        if (g < len) dst[g] = src[g + (int)fdiv((uint32_t)g, cols) * (ldst - (int)cols.d)];
    } else {
        const int pad = ldst - (int)cols.d;
        for (int g = tid; g < len; g += nt) dst[g] = src[g + (int)fdiv((uint32_t)g, cols) * pad];
    }
}

// stage_out with a BLAS epilogue: dst[g] = v + beta * dst_old[g] (dst_old not
// read when beta == 0).  `v` already carries alpha.
GLASS_DEV void stage_out_beta(float* __restrict__ dst, const float* src, int len, FastDiv cols, int ldst,
                              float beta, int tid, int nt) {
    if (beta == 0.f) {
        stage_out(dst, src, len, cols, ldst, tid, nt);
        return;
    }
    const int d = (int)cols.d, pad = ldst - d;
    if (aligned16(dst) && aligned16(src) && (pad == 0 || ((d & 3) == 0 && (ldst & 3) == 0))) {
        const int len4 = len >> 2;
        f4_t* d4 = reinterpret_cast<f4_t*>(dst);
        for (int q = tid; q < len4; q += nt) {
            const int g = 4 * q;
            const f4_t s = *reinterpret_cast<const f4_t*>(src + (pad == 0 ? g : g + (int)fdiv((uint32_t)g, cols) * pad));
            f4_t o = d4[q];
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = fmaf(beta, o[e], s[e]);
            d4[q] = o;
        }
        const int g = (len4 << 2) + tid;
        if (g < len) dst[g] = fmaf(beta, dst[g], src[g + (int)fdiv((uint32_t)g, cols) * pad]);
        return;
    }
    for (int g = tid; g < len; g += nt) dst[g] = fmaf(beta, dst[g], src[g + (int)fdiv((uint32_t)g, cols) * pad]);
}

// Reciprocal square root of a positive pivot (v_rsq_f32, about 1 ulp).
GLASS_DEV float rsq(float x) { return __builtin_amdgcn_rsqf(x); }


// ---------------------------------------------------------------------------
// Wavefront broadcast without LDS.  DPP row_newbcast:c hands every lane the
// value of lane c of its own 16-lane row, and it can be folded into the
// v_fmac_f32 that consumes it.  To broadcast lane k = 16 r + c to the whole
// wave, row r is first replicated into all four rows (R[r]); two
// v_permlane32_swap / v_permlane16_swap steps build R[0..3] from one VGPR.

// R[r][lane] = v[16 r + lane % 16] for r < NR (NR 16-lane rows in use).  The
// trailing s_nop provides the two wait states between the VALU writes of R
// and their DPP reads; it is tied to R so the compiler cannot reorder them.
template <int NR>
GLASS_DEV void replicate_rows(float v, float (&R)[4]) {
    if (NR == 1) {
        float r0 = v;
        asm volatile("s_nop 1" : "+v"(r0));
        R[0] = r0;
        R[1] = R[2] = R[3] = r0;
    } else if (NR == 2) {
        float r0, r1;
        asm volatile(
            "v_mov_b32 %0, %2\n"
            "v_mov_b32 %1, %2\n"
            "s_nop 1\n"
            "v_permlane16_swap_b32 %0, %1\n"
            "s_nop 1\n"
            : "=&v"(r0), "=&v"(r1)
            : "v"(v));
        R[0] = r0;
        R[1] = r1;
        R[2] = R[3] = r0;
    } else {
        float r0, r1, r2, r3;
        asm volatile(
            "v_mov_b32 %0, %4\n"
            "v_mov_b32 %1, %4\n"
            "s_nop 1\n"
            "v_permlane32_swap_b32 %0, %1\n"
            "v_mov_b32 %2, %0\n"
            "v_mov_b32 %3, %1\n"
            "s_nop 1\n"
            "v_permlane16_swap_b32 %0, %2\n"
            "v_permlane16_swap_b32 %1, %3\n"
            "s_nop 1\n"
            : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
            : "v"(v));
        // r0 = row 0, r2 = row 1 (from the first swap's low half), r1 = row 2, r3 = row 3
        R[0] = r0;
        R[1] = r2;
        R[2] = r1;
        R[3] = r3;
    }
}

// acc += bcast_c(src) * m, where bcast_c is DPP row_newbcast:C (one VALU op).
template <int C>
GLASS_DEV void fmac_bcast(float& acc, float src, float m) {
    asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(src), "v"(m), "n"(C));
}

// acc -= bcast_c(src) * m: the same op with the negate modifier on m.
template <int C>
GLASS_DEV void fnmac_bcast(float& acc, float src, float m) {
    asm volatile("v_fmac_f32_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(src), "v"(m), "n"(C));
}

// 1 + the position within its group of `width` lanes (16, 32 or 64) of the
// first lane whose v is not finite, 0 if there is none; every lane of a
// group gets its group's value.  Lanes the wave does not execute count as
// finite.
template <int W>
GLASS_DEV int first_nonfinite(float v) {
    const unsigned long long m = __ballot(!__builtin_isfinite(v));
    if constexpr (W == 64) {
        return m ? __ffsll((long long)m) : 0;
    } else {
        const int shift = (int)(__lane_id() & ~(W - 1));
        const unsigned int bits = (unsigned int)(m >> shift) & (unsigned int)((1ull << W) - 1);
        return bits ? __ffs(bits) : 0;
    }
}

}  // namespace glass
