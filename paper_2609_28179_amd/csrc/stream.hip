// stream.hip -- plain streaming kernels that measure the attainable HBM
// bandwidth of the access mixes the batched ops run at (read only, write
// only, copy, two reads per write).  The roofline fractions of the batched
// kernels are quoted against the 8 TB/s spec peak; these measured ceilings
// say how much of that a kernel with the same read/write mix can reach.
//
// Every kernel is grid-stride over 16-byte elements, one access per lane per
// iteration, in workgroups of 1024 lanes; with a grid of one element per
// lane it is a single sweep.  (Measured on gfx950 over 1 GiB: 1024-lane
// workgroups with one element per lane read at 6.8 TB/s and copy at
// 5.9 TB/s, above 256-lane workgroups and above four or eight unrolled
// accesses per lane.)  The read-only kernel keeps its loads alive by writing
// its sum only when it equals a value the data never produce.
#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {
namespace {

constexpr int kStreamThreads = 1024;

__global__ void __launch_bounds__(kStreamThreads) stream_read(const f4_t* __restrict__ a, float* __restrict__ sink,
                                                              long long n4) {
    const long long stride = (long long)gridDim.x * kStreamThreads;
    f4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n4; i += stride) acc += a[i];
    const float s = acc[0] + acc[1] + acc[2] + acc[3];
    if (s == -1234.5f) sink[threadIdx.x & 255] = s;
}

__global__ void __launch_bounds__(kStreamThreads) stream_write(f4_t* __restrict__ c, long long n4) {
    const long long stride = (long long)gridDim.x * kStreamThreads;
    const f4_t v = {1.f, 1.f, 1.f, 1.f};
    for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n4; i += stride) c[i] = v;
}

__global__ void __launch_bounds__(kStreamThreads) stream_copy(const f4_t* __restrict__ a, f4_t* __restrict__ c,
                                                              long long n4) {
    const long long stride = (long long)gridDim.x * kStreamThreads;
    for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n4; i += stride) c[i] = a[i];
}

__global__ void __launch_bounds__(kStreamThreads) stream_add(const f4_t* __restrict__ a, const f4_t* __restrict__ b,
                                                             f4_t* __restrict__ c, long long n4) {
    const long long stride = (long long)gridDim.x * kStreamThreads;
    for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n4; i += stride) c[i] = a[i] + b[i];
}

}  // namespace

int launch_stream_probe(int kind, const float* a, const float* b, float* c, long long n4, int blocks, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)blocks), block(kStreamThreads);
    const f4_t* a4 = reinterpret_cast<const f4_t*>(a);
    const f4_t* b4 = reinterpret_cast<const f4_t*>(b);
    f4_t* c4 = reinterpret_cast<f4_t*>(c);
    switch (kind) {
    case 0: hipLaunchKernelGGL(stream_read, grid, block, 0, st, a4, c, n4); break;
    case 1: hipLaunchKernelGGL(stream_write, grid, block, 0, st, c4, n4); break;
    case 2: hipLaunchKernelGGL(stream_copy, grid, block, 0, st, a4, c4, n4); break;
    default: hipLaunchKernelGGL(stream_add, grid, block, 0, st, a4, b4, c4, n4); break;
    }
    return (int)hipGetLastError();
}

}  // namespace glass
