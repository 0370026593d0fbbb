// ragged.hip -- factor-and-solve of a ragged batch (problems of mixed order n
// and right-hand-side count) in one launch sequence.
//
// Problems are grouped into eight size classes k = ceil(n/8) - 1 (orders
// 8k+1 .. 8k+8).  Every class has one placement (Sec. III-A, Sec. IV-C):
// thread scope (class 0 only: a wavefront takes 64 problems, one per lane),
// sub-wave scope (classes 0 and 1: four problems per wavefront, one per
// 16-lane row; class 2: two, one per 32-lane half) or wave scope (a
// wavefront takes one problem; orders above 24 run the blocked MFMA routines
// of chol_blk.hpp).  Within a class a problem is padded with an identity
// block up to the class order, so one code path serves all its n.  (Thread
// scope stops at order 8 here because every path of a solve kernel shares
// one register allocation.)
//
// Launch sequence (all on one stream, no host synchronisation, capturable):
//   1. ragged_count    per-chunk class histograms (each block a fixed chunk);
//   2. ragged_scan     one block: class totals, class bases in descending
//                      class order (largest problems first), per-chunk bases,
//                      work-item bases;
//   3. ragged_scatter  stable counting-sort scatter of problem indices into
//                      perm[] (ranks from wavefront ballots, so the permutation
//                      is deterministic: equal classes keep index order);
//   4. ragged_solve    one wavefront per work item of the class-sorted list
//                      (64 problems of a thread-scope class, four at sub-wave
//                      scope, or one problem), every class in one launch, so
//                      the small classes fill the slots that the blocked
//                      classes' last round leaves idle.
#include <atomic>
#include <mutex>

#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"
#include "chol_blk.hpp"

namespace glass {

namespace {

constexpr int kClasses = 8;
constexpr int kChunk = 1024;        // problems per histogram / scatter block
constexpr int kScanThreads = 256;
constexpr int kBigClass = 3;        // classes from here on (orders above 24) run the blocked routines
// LDS floats per wavefront of the small-class solve: the segments' L blocks
// (row stride NB + 4) of the sub-wave path, or the wave path's 8-row chunk
constexpr int kRaggedSegFloats = 2 * 24 * 28;
static_assert(4 * 16 * 20 <= kRaggedSegFloats && 8 * 24 <= kRaggedSegFloats, "ragged LDS");

// Work items of class k holding `cnt` problems: 64 problems per item at
// thread scope, 4 (classes 0, 1) or 2 (class 2) at sub-wave scope, 1 at wave
// scope.
GLASS_DEV int items_of(int scope, int k, int cnt) {
    if (scope == GLASS_SCOPE_THREAD) return (cnt + 63) / 64;
    if (scope == kScopeSubwave) return k <= 1 ? (cnt + 3) / 4 : (cnt + 1) / 2;
    return cnt;
}

// Size class of order n; orders outside 1..64 are clamped into a class here
// and flagged (info = -1, problem skipped) by the solve kernel.
GLASS_DEV int class_of(int n) {
    const int k = (n - 1) >> 3;
    return k < 0 ? 0 : (k > kClasses - 1 ? kClasses - 1 : k);
}

__global__ void __launch_bounds__(256) ragged_count(int count, const int32_t* __restrict__ nvec, int32_t* hist) {
    __shared__ int32_t h[kClasses];
    const int tid = threadIdx.x;
    if (tid < kClasses) h[tid] = 0;
    __syncthreads();
    const int base = blockIdx.x * kChunk;
    for (int e = base + tid; e < min(base + kChunk, count); e += blockDim.x) atomicAdd(&h[class_of(nvec[e])], 1);
    __syncthreads();
    if (tid < kClasses) hist[blockIdx.x * kClasses + tid] = h[tid];
}

// One block of 8 x 32 threads: thread (c, t) owns class c's counts in a
// contiguous range of chunks (ceil(nchunks / 32) of them), so every thread
// reads only its own range.  Classes are laid out largest first.  meta:
// [0..8) class count, [8..16) class base in perm, [16..24) work-item base per
// class, [24] total work items.  Every value is formed in LDS and registers of
// this block; the per-chunk bases are derived from those, not re-read.
__global__ void __launch_bounds__(kScanThreads) ragged_scan(int nchunks, int32_t* hist, int32_t* meta,
                                                           RaggedScopes scopes) {
    static_assert(kScanThreads == kClasses * 32, "one 32-thread group per class");
    __shared__ int32_t part[kClasses][32];
    __shared__ int32_t tot[kClasses];
    __shared__ int32_t cbase[kClasses];
    const int tid = threadIdx.x, c = tid >> 5, t = tid & 31;
    const int per = (nchunks + 31) / 32;
    const int b0 = min(t * per, nchunks), b1 = min(b0 + per, nchunks);
    int s = 0;
    for (int b = b0; b < b1; ++b) s += hist[b * kClasses + c];
    part[c][t] = s;
    __syncthreads();
    if (tid < kClasses) {
        int sum = 0;
        for (int u = 0; u < 32; ++u) sum += part[tid][u];
        tot[tid] = sum;
    }
    __syncthreads();
    if (tid == 0) {
        int base = 0, items = 0;
        for (int k = kClasses - 1; k >= 0; --k) {
            cbase[k] = base;
            meta[k] = tot[k];
            meta[kClasses + k] = base;
            meta[2 * kClasses + k] = items;
            base += tot[k];
            items += items_of(scopes.s[k], k, tot[k]);
        }
        meta[3 * kClasses] = items;  // total work items
    }
    __syncthreads();
    // per-chunk bases: class base + counts of that class in earlier chunks
    int run = cbase[c];
    for (int u = 0; u < t; ++u) run += part[c][u];
    for (int b = b0; b < b1; ++b) {
        const int v = hist[b * kClasses + c];
        hist[b * kClasses + c] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(256) ragged_scatter(int count, const int32_t* __restrict__ nvec,
                                                      const int32_t* __restrict__ hist, int32_t* __restrict__ perm) {
    __shared__ int32_t off[kClasses];
    __shared__ int32_t wcnt[4][kClasses];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < kClasses) off[tid] = hist[blockIdx.x * kClasses + tid];
    __syncthreads();
    const int base = blockIdx.x * kChunk;
    const int end = min(base + kChunk, count);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int s = base; s < end; s += 256) {
        const int e = s + tid;
        const int k = e < end ? class_of(nvec[e]) : -1;
        int rank = 0;
#pragma unroll
        for (int c = 0; c < kClasses; ++c) {
            const uint64_t m = __ballot(k == c);
            if (k == c) rank = __popcll(m & lt);
            if (lane == 0) wcnt[w][c] = __popcll(m);
        }
        __syncthreads();
        if (k >= 0) {
            int before = 0;
            for (int ww = 0; ww < w; ++ww) before += wcnt[ww][k];
            perm[off[k] + before + rank] = e;
        }
        __syncthreads();
        if (tid < kClasses) off[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- solve --
// Thread scope: lane q solves one problem of order n <= N, padded with an
// identity block to N; its own rows are read and written with direct loads.
template <int N>
GLASS_DEV void ragged_thread_one(float* __restrict__ Ag, float* __restrict__ Bg, int n, int nrhs, int32_t* info) {
    float a[N * (N + 1) / 2];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {  // unconditional loads (Ag[0] past n), so that all issue at once
            const float v = Ag[i < n ? i * n + j : 0];
            a[TI(i, j)] = (i < n) ? v : (i == j ? 1.f : 0.f);
        }
    float dinv[N];
    const int inf = tri_potrf<N>(a, dinv);
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < n) {
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (j < n) Ag[i * n + j] = j <= i ? a[TI(i, j)] : 0.f;
        }
    *info = inf;
    if (inf != 0) return;
    for (int c = 0; c < nrhs; ++c) {
        float y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float v = Bg[i < n ? i * nrhs + c : 0];
            y[i] = i < n ? v : 0.f;
        }
        tri_fwd<N>(a, dinv, y);
        tri_bwd<N>(a, dinv, y);
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (i < n) Bg[i * nrhs + c] = y[i];
    }
}

template <int NB>
GLASS_DEV void ragged_wave_one(float* __restrict__ Ag, float* __restrict__ Bg, int n, int nrhs, int32_t* info,
                               float* buf, int lane) {
    float a[NB];
    rows_load_lower<NB, false>(a, Ag, n, lane);
    float myinv;
    const int inf = wave_potrf<NB>(a, lane, myinv);
    const bool vec = false;  // problem offsets are arbitrary: 4-byte stores
    if (inf != 0) {
        wave_chunks_desc<NB>(a, buf, Ag, vec, n, lane, false, 0.f, myinv);
    } else {
        wave_solve_all<NB>(a, buf, Ag, vec, Bg, n, nrhs, myinv, lane);
    }
    if (lane == 0) *info = inf;
}

// Sub-wave scope (classes 0 to 2): 64 / SEG problems per wavefront, SEG = 16
// for classes 0 and 1 (orders <= 16), 32 for class 2 (orders 17..24); lane
// SEG s + i owns row i of problem s.  Pivots and solved unknowns move with the
// segment broadcasts of chol_device.hpp, so the problems never mix; rows past
// a problem's n are identity rows.  Problems of one wavefront differ in n and
// nrhs: loads and stores are per lane, and the column groups run to the
// wavefront's largest nrhs so every DPP step is uniform.
template <int SEG, int NB>
GLASS_DEV void ragged_seg(float* A, float* B, const int64_t* offA, const int64_t* offB, int e, int n, int r,
                          int32_t* info, float* sbuf, int lane) {
    const int s = lane / SEG, i = lane % SEG;
    const bool act = e >= 0;
    const int nn = act ? n : 0;
    float* Ag = act ? A + offA[e] : A;
    float* Bg = act ? B + offB[e] : B;
    float a[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {  // unconditional loads (Ag[0] for the rest), so that all issue at once
        const bool ok = i < nn && j <= i;
        const float v = Ag[ok ? i * nn + j : 0];
        a[j] = ok ? v : (j == i ? 1.f : 0.f);
    }
    int inf = 0;
    float myinv = 1.f;
    SegStep<SEG, NB, 0>::run(a, inf, myinv);
#pragma unroll
    for (int j = 0; j < NB; ++j) a[j] = j <= i ? a[j] : 0.f;
    float* sb = sbuf + s * NB * (NB + 4);
    if (i < NB) {
#pragma unroll
        for (int t = 0; t < NB / 4; ++t) {
            f4_t v;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = a[4 * t + q];
            *reinterpret_cast<f4_t*>(sb + i * (NB + 4) + 4 * t) = v;
        }
    }
    wave_sync();
    if (i < nn) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < nn) Ag[i * nn + j] = a[j];
    }
    if (act && i == 0) info[e] = inf;
    // the rows again from the segment's block, diagonal entry cleared and
    // scaled by 1 / L_ii: the coefficients of the lane-local forward pass
    if (i < NB) sb[i * (NB + 4) + i] = 0.f;
    wave_sync();
    if (i < NB) {
#pragma unroll
        for (int t = 0; t < NB / 4; ++t) {
            const f4_t v = *reinterpret_cast<const f4_t*>(sb + i * (NB + 4) + 4 * t);
#pragma unroll
            for (int q = 0; q < 4; ++q) a[4 * t + q] = v[q];
        }
    }
    wave_sync();
    seg_scale_row<NB>(a, myinv);
    // a failed or empty segment solves zero columns and stores nothing
    const int reff = (act && inf == 0) ? r : 0;
    int rmax = 0;
#pragma unroll
    for (int t = 0; t < 64 / SEG; ++t) rmax = max(rmax, __builtin_amdgcn_readlane(reff, t * SEG));
    seg_solve_all<SEG, NB>(a, sb, Bg, nn, reff, i, myinv, reff > 0, true, true, rmax);
}

// One work item per wavefront: wavefront g of the launch takes item g of the
// class-sorted work list (largest class first) and exits; waves past the
// list's end exit at once.  There is no work-queue loop: a loop drawing items
// from an atomic counter in lane 0 compiled to a per-lane exit in which lanes
// 1..63 never saw a new item and could not leave, so the launch covers the
// list instead and hardware dispatch order provides the largest-first order.
__global__ void __launch_bounds__(256, 3) ragged_solve(const int32_t* __restrict__ nvec,
                                                    const int32_t* __restrict__ rvec,
                                                    const int64_t* __restrict__ offA,
                                                    const int64_t* __restrict__ offB, float* A, float* B,
                                                    int32_t* info, const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ meta, RaggedScopes scopes) {
    // per wavefront, the largest of: 8 rows of up to 24 (the row-per-lane wave
    // path), the segments' L blocks (sub-wave) and the blocked routines'
    // staging (orders above 24)
    constexpr int kFloats = kBlkRegionFloats > kRaggedSegFloats ? kBlkRegionFloats : kRaggedSegFloats;
    __shared__ float chunk[4][kFloats];
    const int lane = threadIdx.x & 63, w = wave_index();
    const int item = blockIdx.x * 4 + w;
    if (item >= meta[3 * kClasses]) return;
    int k = kClasses - 1;
#pragma unroll
    for (int c = 0; c < kClasses; ++c) {
        const int cnt = meta[c], ib = meta[2 * kClasses + c];
        const int nit = items_of(scopes.s[c], c, cnt);
        if (cnt > 0 && item >= ib && item < ib + nit) k = c;
    }
    const bool big = k >= kBigClass;
    const int rel = item - meta[2 * kClasses + k];
    const int cbase = meta[kClasses + k];
    if (!big && scopes.s[k] == kScopeSubwave) {  // classes 0 to 2 only (checked by the caller)
        const int seg = k <= 1 ? 16 : 32;
        const int q = rel * (64 / seg) + lane / seg;
        int e = -1, n = 0, r = 0;
        if (q < meta[k]) {
            e = perm[cbase + q];
            n = nvec[e];
            r = rvec[e];
            if (n < 1 || n > kMaxN || r < 1 || r > kMaxN) {
                if (lane % seg == 0) info[e] = -1;
                e = -1;
            }
        }
        if (k <= 1)
            ragged_seg<16, 16>(A, B, offA, offB, e, n, r, info, chunk[w], lane);
        else
            ragged_seg<32, 24>(A, B, offA, offB, e, n, r, info, chunk[w], lane);
        return;
    }
    if (!big && scopes.s[k] == GLASS_SCOPE_THREAD) {
        const int q = rel * 64 + lane;
        if (q < meta[k]) {
            const int e = perm[cbase + q];
            const int n = nvec[e], r = rvec[e];
            if (n < 1 || n > kMaxN || r < 1 || r > kMaxN) {
                info[e] = -1;
            } else {
                ragged_thread_one<8>(A + offA[e], B + offB[e], n, r, info + e);  // class 0 only
            }
        }
        return;
    }
    // one problem per wavefront: its index, sizes and offsets are wave-uniform
    const int e = uniform_i32(perm[cbase + rel]);
    const int n = uniform_i32(nvec[e]), r = uniform_i32(rvec[e]);
    if (n < 1 || n > kMaxN || r < 1 || r > kMaxN) {
        if (lane == 0) info[e] = -1;
        return;
    }
    float* Ag = A + uniform_i64(offA[e]);
    float* Bg = B + uniform_i64(offB[e]);
    float* buf = chunk[w];
    if (big) {  // problem offsets are arbitrary: 4-byte stores
        const int inf = k == 3   ? blk_one<2, 1, false>(Ag, Bg, n, r, 0, false, buf, lane)
                        : k <= 5 ? blk_one<3, 1, false>(Ag, Bg, n, r, 0, false, buf, lane)
                                 : blk_one<4, 1, false>(Ag, Bg, n, r, 0, false, buf, lane);
        if (lane == 0) info[e] = inf;
        return;
    }
    switch (k) {
    case 0: ragged_wave_one<8>(Ag, Bg, n, r, info + e, buf, lane); break;
    case 1: ragged_wave_one<16>(Ag, Bg, n, r, info + e, buf, lane); break;
    default: ragged_wave_one<24>(Ag, Bg, n, r, info + e, buf, lane); break;  // class 2
    }
}

}  // namespace

size_t ragged_workspace_bytes(int count) {
    const int nchunks = (count + kChunk - 1) / kChunk;
    return sizeof(int32_t) * ((size_t)nchunks * kClasses + 32 + (size_t)count);
}

// ------------------------------------------------------- no-allocation form --
// Workspace of the ragged solve for callers that cannot allocate: a static
// device array sized for kRaggedNoAllocMaxCount problems (about 4 MiB), one
// copy per device that the library runs on, kept until the process ends.
// Host code never passes `scratch` itself (on the host it is only a stand-in
// for the symbol); it passes the device address hipGetSymbolAddress returns,
// looked up once per device with that device current.  Every call on a
// device shares its copy; the planning kernels rewrite every word they read
// (histograms, class metadata, permutation), so nothing needs clearing.
namespace {
constexpr size_t kNoAllocWords =
    (size_t)((kRaggedNoAllocMaxCount + kChunk - 1) / kChunk) * kClasses + 32 + (size_t)kRaggedNoAllocMaxCount;
static __device__ __align__(256) int32_t scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;
}  // namespace

int ragged_noalloc_workspace(void** ptr, size_t* bytes) {
    static_assert(sizeof(scratch) == kNoAllocWords * sizeof(int32_t), "scratch size");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return (int)e;
            if (!p) return (int)hipErrorInvalidSymbol;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *ptr = p;
    *bytes = sizeof(scratch);
    return 0;
}

int launch_posv_ragged(int count, const int32_t* n, const int32_t* nrhs, const int64_t* offA, const int64_t* offB,
                       float* A, float* B, int32_t* info, void* workspace, const RaggedScopes& scopes,
                       void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int nchunks = (count + kChunk - 1) / kChunk;
    int32_t* hist = reinterpret_cast<int32_t*>(workspace);
    int32_t* meta = hist + (size_t)nchunks * kClasses;
    int32_t* perm = meta + 32;
    hipLaunchKernelGGL(ragged_count, dim3(nchunks), dim3(256), 0, st, count, n, hist);
    hipLaunchKernelGGL(ragged_scan, dim3(1), dim3(kScanThreads), 0, st, nchunks, hist, meta, scopes);
    hipLaunchKernelGGL(ragged_scatter, dim3(nchunks), dim3(256), 0, st, count, n, hist, perm);
    // work items never outnumber problems: ceil(count / 4) four-wave blocks cover the list
    hipLaunchKernelGGL(ragged_solve, dim3((count + 3) / 4), dim3(256), 0, st, n, nrhs, offA, offB, A, B, info, perm,
                       meta, scopes);
    return (int)hipGetLastError();
}

}  // namespace glass
