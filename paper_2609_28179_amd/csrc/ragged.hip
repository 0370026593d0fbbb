// ragged.hip -- factor-and-solve of a ragged batch (problems of mixed order n
// and right-hand-side count) in one launch sequence.
//
// Problems are grouped into eight size classes k = ceil(n/8) - 1 (orders
// 8k+1 .. 8k+8).  Every class has one placement (Sec. III-A, Sec. IV-C):
// thread scope (class 0 only: a wavefront takes 64 problems, one per lane),
// sub-wave scope (classes 0 and 1: four problems per wavefront, one per
// 16-lane row) or wave scope (a wavefront takes one problem; orders above 32
// run the blocked MFMA routines of chol_blk.hpp).  Within a class a problem is
// padded with an identity block up to the class order, so one code path
// serves all its n.  (Thread scope stops at order 8 here because every path
// of a solve kernel shares one register allocation.)
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
//                      scope, or one problem), in two launches: the classes
//                      above order 32 (the blocked routines need more
//                      registers), then the rest at the smaller allocation.
#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"
#include "chol_blk.hpp"

namespace glass {

namespace {

constexpr int kClasses = 8;
constexpr int kChunk = 1024;        // problems per histogram / scatter block
constexpr int kScanThreads = 256;
constexpr int kBigClass = 4;        // classes from here on (orders above 32) run the blocked routines

// Work items of a class of `cnt` problems: 64 problems per item at thread
// scope, 4 at sub-wave scope, 1 at wave scope.
GLASS_DEV int items_of(int scope, int cnt) {
    return scope == GLASS_SCOPE_THREAD ? (cnt + 63) / 64 : (scope == kScopeSubwave ? (cnt + 3) / 4 : cnt);
}

// Size class of order n; orders outside 1..64 are clamped into a class here
// and flagged (info = -1, problem skipped) by the solve kernel.
GLASS_DEV int class_of(int n) {
    const int k = (n - 1) >> 3;
    return k < 0 ? 0 : (k > kClasses - 1 ? kClasses - 1 : k);
}

__global__ void __launch_bounds__(256) ragged_count(int count, const int32_t* __restrict__ nvec, int32_t* hist,
                                                    int32_t* meta) {
    __shared__ int32_t h[kClasses];
    const int tid = threadIdx.x;
    if (tid < kClasses) h[tid] = 0;
    __syncthreads();
    const int base = blockIdx.x * kChunk;
    for (int e = base + tid; e < min(base + kChunk, count); e += blockDim.x) atomicAdd(&h[class_of(nvec[e])], 1);
    __syncthreads();
    if (tid < kClasses) hist[blockIdx.x * kClasses + tid] = h[tid];
}

// One block.  Classes are laid out largest first.  meta: [0..8) class count,
// [8..16) class base in perm, [16..24) work-item base per class, [24] total
// work items.  Every value is formed in LDS and registers of this block; the
// per-chunk bases are derived from those, not re-read from global memory.
__global__ void __launch_bounds__(kScanThreads) ragged_scan(int nchunks, int32_t* hist, int32_t* meta,
                                                           RaggedScopes scopes) {
    __shared__ int32_t tot[kClasses];
    __shared__ int32_t cbase[kClasses];
    const int tid = threadIdx.x;
    if (tid < kClasses) {
        int s = 0;
        for (int b = 0; b < nchunks; ++b) s += hist[b * kClasses + tid];
        tot[tid] = s;
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
            items += items_of(scopes.s[k], tot[k]);
        }
        meta[3 * kClasses] = items;  // total work items
    }
    __syncthreads();
    // per-chunk bases: class base + counts of that class in earlier chunks
    if (tid < kClasses) {
        int run = cbase[tid];
        for (int b = 0; b < nchunks; ++b) {
            const int c = hist[b * kClasses + tid];
            hist[b * kClasses + tid] = run;
            run += c;
        }
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
        for (int j = 0; j <= i; ++j) a[TI(i, j)] = (i < n) ? Ag[i * n + j] : (i == j ? 1.f : 0.f);
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
        for (int i = 0; i < N; ++i) y[i] = i < n ? Bg[i * nrhs + c] : 0.f;
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

// Sub-wave scope (classes 0 and 1, orders <= 16): four problems per
// wavefront, one per 16-lane row; lane 16s + i owns row i of problem s.
// Pivots and solved unknowns reach the other lanes of their row with DPP
// row_newbcast, so the four problems never mix; rows past n are identity.
// Inline asm operands get no compiler wait states, so each block starts with
// the ones its inputs need (a VALU result read through DPP: two).
template <int C>
GLASS_DEV float row_bcast(float v) {
    float r;
    asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                 : "=v"(r)
                 : "v"(v), "n"(C));
    return r;
}

// v in lane J of every 16-lane row, `other` elsewhere (literal lane mask).
template <int J>
GLASS_DEV float rows_select(float other, float v) {
    float r;
    asm("s_nop 1\n\tv_cndmask_b32_e64 %0, %1, %2, %3"
        : "=v"(r)
        : "v"(other), "v"(v), "s"(0x0001000100010001ull << J));
    return r;
}

template <int J, int K>
struct SubUpd {
    static GLASS_DEV void run(float (&a)[16], float R, float nv) {
        fmac_bcast<K>(a[K], R, nv);
        SubUpd<J, K + 1>::run(a, R, nv);
    }
};
template <int J>
struct SubUpd<J, 16> {
    static GLASS_DEV void run(float (&)[16], float, float) {}
};

template <int J>
struct SubStep {
    static GLASS_DEV void run(float (&a)[16], int& info, float& myinv) {
        const float d = row_bcast<J>(a[J]);
        if (!(d > 0.f) && info == 0) info = J + 1;
        const float inv = rsq(d);
        const float v = a[J] * inv;  // in lane J of the row, a[J] is the pivot itself
        myinv = rows_select<J>(myinv, inv);
        a[J] = v;
        float R[4];
        replicate_rows<1>(v, R);  // wait states before the DPP reads of v
        SubUpd<J, J + 1>::run(a, R[0], -v);
        SubStep<J + 1>::run(a, info, myinv);
    }
};
template <>
struct SubStep<16> {
    static GLASS_DEV void run(float (&)[16], int&, float&) {}
};

template <int K, int RG>
struct SubFwd {
    static GLASS_DEV void run(const float (&a)[16], float (&acc)[RG], float (&y)[RG], float myinv) {
#pragma unroll
        for (int c = 0; c < RG; ++c) {
            const float yk = row_bcast<K>(acc[c] * myinv);
            acc[c] = fmaf(-a[K], yk, acc[c]);
            y[c] = rows_select<K>(y[c], yk);
        }
        SubFwd<K + 1, RG>::run(a, acc, y, myinv);
    }
};
template <int RG>
struct SubFwd<16, RG> {
    static GLASS_DEV void run(const float (&)[16], float (&)[RG], float (&)[RG], float) {}
};

// Backward substitution L^T x = y; row K of the problem's L is read from its
// 16 x 16 LDS block (lane i takes L_Ki).
template <int K, int RG>
struct SubBwd {
    static GLASS_DEV void run(const float* sb, int i, float (&acc)[RG], float myinv) {
        const float lki = i < K ? sb[K * 16 + i] : 0.f;
#pragma unroll
        for (int c = 0; c < RG; ++c) {
            const float xk = row_bcast<K>(acc[c] * myinv);
            acc[c] = rows_select<K>(fmaf(-lki, xk, acc[c]), xk);
        }
        SubBwd<K - 1, RG>::run(sb, i, acc, myinv);
    }
};
template <int RG>
struct SubBwd<-1, RG> {
    static GLASS_DEV void run(const float*, int, float (&)[RG], float) {}
};

template <int RG>
GLASS_DEV void sub_solve_cols(const float (&a)[16], const float* sb, float* Bg, int n, int r, int c0, int i,
                              float myinv) {
    float acc[RG], y[RG];
#pragma unroll
    for (int c = 0; c < RG; ++c) {
        acc[c] = (i < n && c0 + c < r) ? Bg[i * r + c0 + c] : 0.f;
        y[c] = 0.f;
    }
    SubFwd<0, RG>::run(a, acc, y, myinv);
    SubBwd<15, RG>::run(sb, i, y, myinv);
#pragma unroll
    for (int c = 0; c < RG; ++c)
        if (i < n && c0 + c < r) Bg[i * r + c0 + c] = y[c];
}

// Row s of the wavefront solves problem e (e < 0: an empty row, all identity).
GLASS_DEV void ragged_subwave(float* A, float* B, const int64_t* offA, const int64_t* offB, int e, int n, int r,
                              int32_t* info, float* sbuf, int lane) {
    const int seg = lane >> 4, i = lane & 15;
    const bool act = e >= 0;
    const int nn = act ? n : 0;
    float* Ag = act ? A + offA[e] : A;
    float* Bg = act ? B + offB[e] : B;
    float a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = (i < nn && j <= i) ? Ag[i * nn + j] : (j == i ? 1.f : 0.f);
    int inf = 0;
    float myinv = 1.f;
    SubStep<0>::run(a, inf, myinv);
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = j <= i ? a[j] : 0.f;
    float* sb = sbuf + seg * 256;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f4_t v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = a[4 * t + q];
        *reinterpret_cast<f4_t*>(sb + i * 16 + 4 * t) = v;
    }
    wave_sync();
    if (i < nn) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < nn) Ag[i * nn + j] = a[j];
    }
    if (act && i == 0) info[e] = inf;
    // column groups up to the largest right-hand-side count of the four rows
    // (uniform, so every DPP step runs in all lanes); a failed or empty row
    // solves zero columns and stores nothing
    const int reff = (act && inf == 0) ? r : 0;
    int rmax = max(max(__builtin_amdgcn_readlane(reff, 0), __builtin_amdgcn_readlane(reff, 16)),
                   max(__builtin_amdgcn_readlane(reff, 32), __builtin_amdgcn_readlane(reff, 48)));
    for (int c0 = 0; c0 < rmax;) {
        const int left = rmax - c0;
        if (left >= 5) {
            sub_solve_cols<8>(a, sb, Bg, nn, reff, c0, i, myinv);
            c0 += 8;
        } else if (left >= 2) {
            sub_solve_cols<4>(a, sb, Bg, nn, reff, c0, i, myinv);
            c0 += 4;
        } else {
            sub_solve_cols<1>(a, sb, Bg, nn, reff, c0, i, myinv);
            c0 += 1;
        }
    }
}

// One work item per wavefront: wavefront g of the launch takes item g of the
// class-sorted work list (largest class first) and exits; waves past the
// list's end exit at once.  There is no work-queue loop: a loop drawing items
// from an atomic counter in lane 0 compiled to a per-lane exit in which lanes
// 1..63 never saw a new item and could not leave, so the launch covers the
// list instead and hardware dispatch order provides the largest-first order.
// BIG selects the classes of orders above 32 (blocked MFMA routines, which
// need more registers) or the rest; the two instances are launched over the
// same item range, the BIG one first, and each leaves the other's items.
template <bool BIG>
__global__ void __launch_bounds__(256) ragged_solve(const int32_t* __restrict__ nvec,
                                                    const int32_t* __restrict__ rvec,
                                                    const int64_t* __restrict__ offA,
                                                    const int64_t* __restrict__ offB, float* A, float* B,
                                                    int32_t* info, const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ meta, RaggedScopes scopes) {
    // per wavefront: 8 rows of 64 (wave, orders <= 32), four 16 x 16 blocks
    // (sub-wave) or the blocked routines' staging (orders above 32)
    __shared__ float chunk[4][BIG ? kBlkRegionFloats : 1024];
    const int lane = threadIdx.x & 63, w = wave_index();
    const int item = blockIdx.x * 4 + w;
    if (item >= meta[3 * kClasses]) return;
    int k = kClasses - 1;
#pragma unroll
    for (int c = 0; c < kClasses; ++c) {
        const int cnt = meta[c], ib = meta[2 * kClasses + c];
        const int nit = items_of(scopes.s[c], cnt);
        if (cnt > 0 && item >= ib && item < ib + nit) k = c;
    }
    if (BIG != (k >= kBigClass)) return;
    const int rel = item - meta[2 * kClasses + k];
    const int cbase = meta[kClasses + k];
    if (scopes.s[k] == kScopeSubwave) {  // classes 0 and 1 only (checked by the caller)
        const int q = rel * 4 + (lane >> 4);
        int e = -1, n = 0, r = 0;
        if (q < meta[k]) {
            e = perm[cbase + q];
            n = nvec[e];
            r = rvec[e];
            if (n < 1 || n > 16 || r < 1 || r > kMaxN) {
                if ((lane & 15) == 0) info[e] = -1;
                e = -1;
            }
        }
        ragged_subwave(A, B, offA, offB, e, n, r, info, chunk[w], lane);
        return;
    }
    if (scopes.s[k] == GLASS_SCOPE_THREAD) {
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
    if (BIG) {  // problem offsets are arbitrary: 4-byte stores
        const int inf = k <= 5 ? blk_one<3, 1, false>(Ag, Bg, n, r, 0, false, buf, lane)
                               : blk_one<4, 1, false>(Ag, Bg, n, r, 0, false, buf, lane);
        if (lane == 0) info[e] = inf;
        return;
    }
    switch (k) {
    case 0: ragged_wave_one<8>(Ag, Bg, n, r, info + e, buf, lane); break;
    case 1: ragged_wave_one<16>(Ag, Bg, n, r, info + e, buf, lane); break;
    case 2: ragged_wave_one<24>(Ag, Bg, n, r, info + e, buf, lane); break;
    default: ragged_wave_one<32>(Ag, Bg, n, r, info + e, buf, lane); break;
    }
}

}  // namespace

size_t ragged_workspace_bytes(int count) {
    const int nchunks = (count + kChunk - 1) / kChunk;
    return sizeof(int32_t) * ((size_t)nchunks * kClasses + 32 + (size_t)count);
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
    hipLaunchKernelGGL(ragged_count, dim3(nchunks), dim3(256), 0, st, count, n, hist, meta);
    hipLaunchKernelGGL(ragged_scan, dim3(1), dim3(kScanThreads), 0, st, nchunks, hist, meta, scopes);
    hipLaunchKernelGGL(ragged_scatter, dim3(nchunks), dim3(256), 0, st, count, n, hist, perm);
    // work items never outnumber problems: ceil(count / 4) four-wave blocks cover the list
    hipLaunchKernelGGL(ragged_solve<true>, dim3((count + 3) / 4), dim3(256), 0, st, n, nrhs, offA, offB, A, B, info,
                       perm, meta, scopes);
    hipLaunchKernelGGL(ragged_solve<false>, dim3((count + 3) / 4), dim3(256), 0, st, n, nrhs, offA, offB, A, B, info,
                       perm, meta, scopes);
    return (int)hipGetLastError();
}

}  // namespace glass
