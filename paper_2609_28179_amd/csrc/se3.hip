// se3.hip -- batched SE(3) homogeneous-transform compose and closed-form
// inverse (Sec. III-B) at the three scopes of Sec. III-A.  A transform is a
// row-major 4x4 [R t; 0 0 0 1]; row 3 of the inputs is never read and row 3
// of the output is written as exactly (0, 0, 0, 1).
//   thread     one transform (pair) per lane, staged through LDS with
//              coalesced loads, composed in VGPRs, written back in place.
//   wave       one problem per wavefront, lane e < 16 produces entry e.
//   workgroup  one problem at a time per 64-lane workgroup, P back to back.
#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {
namespace {

// LDS stride of one staged transform: 16-byte aligned, and 4 x an odd number
// so the lanes' 16-byte row accesses fall on distinct bank groups.
constexpr int kS = kSe3Stride;
static_assert(kS == thread_stride(16), "transform stride");

GLASS_DEV void compose_regs(const float (&a)[12], const float (&b)[12], float (&o)[12]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float s = a[i * 4 + 0] * b[0 * 4 + j];
            s = fmaf(a[i * 4 + 1], b[1 * 4 + j], s);
            s = fmaf(a[i * 4 + 2], b[2 * 4 + j], s);
            if (j == 3) s += a[i * 4 + 3];
            o[i * 4 + j] = s;
        }
    }
}

GLASS_DEV void inverse_regs(const float (&a)[12], float (&o)[12]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) o[i * 4 + j] = a[j * 4 + i];
        float s = a[0 * 4 + i] * a[0 * 4 + 3];
        s = fmaf(a[1 * 4 + i], a[1 * 4 + 3], s);
        s = fmaf(a[2 * 4 + i], a[2 * 4 + 3], s);
        o[i * 4 + 3] = -s;
    }
}

__global__ void __launch_bounds__(512) se3_thread(int inverse, int batch, const float* Ta,
                                                  const float* Tb, float* Tout) {
    extern __shared__ float lds[];
    const int nt = blockDim.x, tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * nt;
    const int cnt = (int)min((long long)nt, (long long)batch - p0);
    const FastDiv f16 = make_fastdiv(16);
    float* sa = lds;
    float* sb = lds + nt * kS;
    stage_in<4>(sa, Ta + p0 * 16, cnt * 16, f16, kS, tid, nt);
    if (!inverse) stage_in<4>(sb, Tb + p0 * 16, cnt * 16, f16, kS, tid, nt);
    __syncthreads();
    if (tid < cnt) {
        float a[12], o[12];
        lds_row_get<12, 4>(a, sa + tid * kS);
        if (inverse) {
            inverse_regs(a, o);
        } else {
            float b[12];
            lds_row_get<12, 4>(b, sb + tid * kS);
            compose_regs(a, b, o);
        }
        float w[16];
#pragma unroll
        for (int e = 0; e < 12; ++e) w[e] = o[e];
        w[12] = 0.f;
        w[13] = 0.f;
        w[14] = 0.f;
        w[15] = 1.f;
        lds_row_put<16, 4>(sa + tid * kS, w);
    }
    __syncthreads();
    stage_out(Tout + p0 * 16, sa, cnt * 16, f16, kS, tid, nt);
}

// Entry e (< 16) of one problem's output, computed from global memory.
GLASS_DEV float se3_entry(int inverse, const float* a, const float* b, int e) {
    const int i = e >> 2, j = e & 3;
    if (i == 3) return j == 3 ? 1.f : 0.f;
    if (inverse) {
        if (j < 3) return a[j * 4 + i];
        float s = a[0 * 4 + i] * a[0 * 4 + 3];
        s = fmaf(a[1 * 4 + i], a[1 * 4 + 3], s);
        s = fmaf(a[2 * 4 + i], a[2 * 4 + 3], s);
        return -s;
    }
    float s = a[i * 4 + 0] * b[0 * 4 + j];
    s = fmaf(a[i * 4 + 1], b[1 * 4 + j], s);
    s = fmaf(a[i * 4 + 2], b[2 * 4 + j], s);
    if (j == 3) s += a[i * 4 + 3];
    return s;
}

__global__ void __launch_bounds__(512) se3_wave(int inverse, int batch, const float* Ta,
                                                const float* Tb, float* Tout) {
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    float v = 0.f;
    if (lane < 16) v = se3_entry(inverse, Ta + p * 16, inverse ? nullptr : Tb + p * 16, lane);
    wave_sync();
    if (lane < 16) Tout[p * 16 + lane] = v;
}

__global__ void __launch_bounds__(64) se3_wg(int inverse, int batch, int pack, const float* Ta,
                                             const float* Tb, float* Tout) {
    const int tid = threadIdx.x;
    for (int q = 0; q < pack; ++q) {
        const long long p = (long long)blockIdx.x * pack + q;
        if (p >= batch) break;
        float v = 0.f;
        if (tid < 16) v = se3_entry(inverse, Ta + p * 16, inverse ? nullptr : Tb + p * 16, tid);
        __syncthreads();
        if (tid < 16) Tout[p * 16 + tid] = v;
        __syncthreads();
    }
}

}  // namespace

int launch_se3(const Shape& sh, const Geometry& g, int batch, const float* Ta, const float* Tb, float* Tout,
               void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int inv = sh.op == GLASS_OP_SE3_INVERSE;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (g.scope == GLASS_SCOPE_THREAD)
        hipLaunchKernelGGL(se3_thread, grid, block, g.lds_bytes, st, inv, batch, Ta, Tb, Tout);
    else if (g.scope == GLASS_SCOPE_WAVE)
        hipLaunchKernelGGL(se3_wave, grid, block, 0, st, inv, batch, Ta, Tb, Tout);
    else
        hipLaunchKernelGGL(se3_wg, grid, block, 0, st, inv, batch, g.pack, Ta, Tb, Tout);
    return (int)hipGetLastError();
}

}  // namespace glass
