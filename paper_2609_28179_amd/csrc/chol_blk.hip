// chol_blk.hip -- batched wave-scope kernels of POTRF / POSV / POTRS / TRSV
// for orders 25..64 on the blocked routines of chol_blk.hpp (one problem per
// wavefront; 2, 3 or 4 tiles of 16 per side): the MFMA kernel for the
// factorizations and multi-column solves, the VALU substitution for one
// right-hand side.
#include "chol_blk.hpp"

namespace glass {
namespace {

// op: 0 POTRF, 1 POSV, 2 POTRS, 3 TRSV (trans: 0 forward, 1 backward), 4 POSV
// with one right-hand side.
template <int NBLK, int OP, bool FULL>
__global__ void __launch_bounds__(512) chol_blk(int n, int nrhs, int trans, int batch, float* __restrict__ A,
                                                float* __restrict__ B, int32_t* __restrict__ info) {
    extern __shared__ float lds[];
    // POTRF on whole 16 x 16 tiles above order 32 (n = 48, 64) is write-bound
    // and runs 1.5-3 % faster at 4 waves per SIMD than at the 5-7 its
    // registers allow (at n = 40 the extra waves pay instead): reserving VGPRs
    // up to v103 makes the allocation 104 registers, which caps the occupancy.
    if (OP == 0 && FULL && NBLK >= 3) asm volatile("" ::: "v103");
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    const int nr = OP >= 3 ? 1 : nrhs;
    const bool vec = FULL || ((n & 3) == 0 && aligned16(A));
    constexpr int region = OP == 4 ? blk_posv1_floats(NBLK) : kBlkRegionFloats;
    const int inf = blk_one<NBLK, OP, FULL>(A + p * n * n, OP == 0 ? nullptr : B + p * n * nr, n, nrhs, trans, vec,
                                            lds + (size_t)w * region, lane);
    if ((OP <= 1 || OP == 4) && info && lane == 0) info[p] = inf;
}

// One right-hand side (TRSV; POTRS with nrhs = 1) on VALU, no inverses:
// FWD solves L y = b, BWD L^T x = y.  L is read, B[batch][n] overwritten.
template <int NBLK, bool FULL, bool FWD, bool BWD>
__global__ void __launch_bounds__(512) chol_blk_solve1(int n, int batch, const float* __restrict__ L,
                                                       float* __restrict__ B) {
    extern __shared__ float lds[];
    const int w = wave_index(), lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + w;
    if (p >= batch) return;
    const int q = lane >> 4, r = lane & 15;
    f4_t T[NBLK * (NBLK + 1) / 2];
    blk_load<NBLK, FULL>(T, L + p * n * n, n, q, r);
    blk_solve1<NBLK, FULL, FWD, BWD>(T, B + p * n, n, lds + (size_t)w * kBlkSolve1Floats, q, r);
}

}  // namespace

int launch_chol_blk(const Shape& sh, const Geometry& g, int batch, float* A, float* B, int32_t* info,
                    void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n;
    if (n < kBlkMinN || n > kMaxN) return (int)hipErrorInvalidValue;
    const int nblk = n <= 32 ? 2 : n <= 48 ? 3 : 4;
    const bool full = n == 16 * nblk && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
    const int op = sh.op == GLASS_OP_POTRF ? 0
                   : sh.op == GLASS_OP_POSV ? (sh.nrhs == 1 ? 4 : 1)
                   : sh.op == GLASS_OP_POTRS ? 2
                                             : 3;
    dim3 grid((unsigned)g.grid), block(g.threads);
    if (op == 3 || (op == 2 && sh.nrhs == 1)) {
        const int mode = op == 2 ? 3 : sh.trans == 0 ? 1 : 2;  // 1: L y = b, 2: L^T x = b, 3: both
#define ONE(NBLK, FULL, MODE)                                                                                   \
    if (nblk == NBLK && full == FULL && mode == MODE) {                                                         \
        hipLaunchKernelGGL((chol_blk_solve1<NBLK, FULL, (MODE & 1) != 0, (MODE & 2) != 0>), grid, block,          \
                           g.lds_bytes, st, n, batch, A, B);                                                    \
        return (int)hipGetLastError();                                                                          \
    }
#define ONE_MODES(NBLK, FULL) ONE(NBLK, FULL, 1) ONE(NBLK, FULL, 2) ONE(NBLK, FULL, 3)
        ONE_MODES(2, false) ONE_MODES(2, true) ONE_MODES(3, false) ONE_MODES(3, true) ONE_MODES(4, false)
        ONE_MODES(4, true)
#undef ONE_MODES
#undef ONE
        return (int)hipErrorInvalidValue;
    }
#define BLK(NBLK, OP, FULL)                                                                                    \
    if (nblk == NBLK && op == OP && full == FULL) {                                                            \
        hipLaunchKernelGGL((chol_blk<NBLK, OP, FULL>), grid, block, g.lds_bytes, st, n, sh.nrhs, sh.trans, batch, \
                           A, B, info);                                                                        \
        return (int)hipGetLastError();                                                                         \
    }
#define BLK_OPS(NBLK, FULL) \
    BLK(NBLK, 0, FULL) BLK(NBLK, 1, FULL) BLK(NBLK, 2, FULL) BLK(NBLK, 3, FULL) BLK(NBLK, 4, FULL)
    BLK_OPS(2, false) BLK_OPS(2, true) BLK_OPS(3, false) BLK_OPS(3, true) BLK_OPS(4, false) BLK_OPS(4, true)
#undef BLK_OPS
#undef BLK
    return (int)hipErrorInvalidValue;
}

}  // namespace glass
