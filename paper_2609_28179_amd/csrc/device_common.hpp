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

GLASS_DEV float readlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Copy src[0 .. len) (contiguous, global) into LDS re-laid as rows of
// `cols.d` floats at row stride `ldst`: element g lands at
// dst[(g / cols) * ldst + g % cols].  `nt` cooperating lanes, this one is
// `tid`.  Four loads are issued before their LDS writes.
GLASS_DEV void stage_in(float* dst, const float* __restrict__ src, int len, FastDiv cols, int ldst,
                        int tid, int nt) {
    const int pad = ldst - (int)cols.d;
    for (int base = 0; base < len; base += 4 * nt) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int g = base + u * nt + tid;
            v[u] = g < len ? src[g] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int g = base + u * nt + tid;
            if (g < len) dst[g + (int)fdiv((uint32_t)g, cols) * pad] = v[u];
        }
    }
}

// Inverse of stage_in: dst[g] = src_lds[(g / cols) * ldst + g % cols].
GLASS_DEV void stage_out(float* __restrict__ dst, const float* src, int len, FastDiv cols, int ldst,
                         int tid, int nt) {
    const int pad = ldst - (int)cols.d;
    for (int g = tid; g < len; g += nt) dst[g] = src[g + (int)fdiv((uint32_t)g, cols) * pad];
}

// stage_out with a BLAS epilogue: dst[g] = v + beta * dst_old[g] (dst_old not
// read when beta == 0).  `v` already carries alpha.
GLASS_DEV void stage_out_beta(float* __restrict__ dst, const float* src, int len, FastDiv cols,
                              int ldst, float beta, int tid, int nt) {
    const int pad = ldst - (int)cols.d;
    if (beta == 0.f) {
        for (int g = tid; g < len; g += nt) dst[g] = src[g + (int)fdiv((uint32_t)g, cols) * pad];
    } else {
        for (int g = tid; g < len; g += nt)
            dst[g] = fmaf(beta, dst[g], src[g + (int)fdiv((uint32_t)g, cols) * pad]);
    }
}

}  // namespace glass
