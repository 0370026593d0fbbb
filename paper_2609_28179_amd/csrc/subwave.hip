// subwave.hip -- sub-wave scope of the batched Cholesky family: 64 / SEG
// problems per wavefront, one per SEG-lane segment (SEG = 16 for orders up to
// 16, 32 for orders up to 32; Sec. IV-C packing below the warp granule).
//
// A problem of order n <= SEG uses only n rows of a wavefront at wave scope;
// here every segment runs its own problem with lane i of the segment owning
// row i.  Broadcasts stay inside a segment: DPP row_newbcast reaches the 16
// lanes of a row, and for SEG = 32 v_permlane16_swap first replicates each
// 16-lane row across its 32-lane half (replicate_rows<2>), so the two halves
// of the wavefront never mix.  The per-segment pivot and 1 / L_ii use the
// same broadcast and a literal lane mask that repeats every SEG lanes; the
// substitutions scale each row by its own 1 / L_ii, so that a solved unknown
// is its lane's running value, broadcast in the FMA that consumes it (rows
// with the diagonal entry cleared: read so for the solves, read back from
// LDS after the factorization).  The backward substitution reads L from a
// per-segment LDS block;
// L leaves through that block as one contiguous copy of the wavefront's
// problems (they are adjacent in the batch).
#include "device_common.hpp"
#include "glass_internal.hpp"
#include "chol_device.hpp"

namespace glass {
namespace {

// op: 0 POTRF, 1 POSV, 2 POTRS, 3 TRSV (trans selects forward 0 / backward 1).
template <int SEG, int NB, int OP>
__global__ void __launch_bounds__(512) chol_seg(int n, int nrhs, int trans, int batch, float* __restrict__ A,
                                                float* __restrict__ B, int32_t* __restrict__ info, int region) {
    extern __shared__ float lds[];
    constexpr int PPW = 64 / SEG;
    const int w = wave_index(), lane = threadIdx.x & 63;
    const int s = lane / SEG, i = lane % SEG;
    const long long p0 = ((long long)blockIdx.x * (blockDim.x >> 6) + w) * PPW;
    if (p0 >= batch) return;
    const int np = (int)min((long long)PPW, (long long)batch - p0);
    const bool act = s < np;
    float* buf = lds + (size_t)w * region;
    float* sb = buf + s * NB * (NB + 4);
    float* Ab = A + p0 * n * n;
    const int r = OP == 3 ? 1 : nrhs;
    float* Bs = B + (p0 + s) * n * r;
    // With one right-hand side its entry, and for the solves the diagonal,
    // are loaded with the rows (a lane without a row reads its wave's first
    // problem's entries).
    const bool row = act && i < n, one = OP >= 1 && r == 1;
    const float b1 = one ? B[row ? (p0 + s) * n + i : p0 * n] : 0.f;
    const float dg = OP >= 2 ? Ab[row ? s * n * n + i * n + i : 0] : 1.f;
    float a[NB];
    float myinv = 1.f;
    int inf = 0;
    if (OP <= 1) {
        seg_load_rows<NB, false>(a, Ab, np, n, s, i);
        SegStep<SEG, NB, 0>::run(a, inf, myinv);
#pragma unroll
        for (int k = 0; k < NB; ++k) a[k] = k <= i ? a[k] : 0.f;
    } else {
        seg_load_rows<NB, true>(a, Ab, np, n, s, i);
        myinv = row ? recip(dg) : 1.f;
    }
    const bool fwd = OP != 3 || trans == 0, bwd = OP != 3 || trans == 1;
    if (OP <= 1 || bwd) {
        seg_rows_to_lds<NB>(a, sb, i);
        wave_sync();
    }
    if (OP <= 1) {
        seg_store_L<NB>(Ab, buf, np, n, (n & 3) == 0 && aligned16(A), lane);
        if (info && act && i == 0) info[p0 + s] = inf;
    }
    if (OP == 0) return;
    if (OP == 1) {  // the factored rows again, diagonal entry cleared, for the lane-local forward pass
        if (i < NB) sb[i * (NB + 4) + i] = 0.f;
        wave_sync();
        if (i < NB) {
#pragma unroll
            for (int t = 0; t < NB / 4; ++t) {
                const f4_t v = *reinterpret_cast<const f4_t*>(sb + i * (NB + 4) + 4 * t);
#pragma unroll
                for (int e = 0; e < 4; ++e) a[4 * t + e] = v[e];
            }
        }
        wave_sync();
    }
    seg_scale_row<NB>(a, myinv);
    const bool solve = act && inf == 0;  // a failed factorization leaves B untouched
    if (one)
        seg_solve_one<SEG, NB>(a, sb, Bs, n, i, myinv, solve, fwd, bwd, row ? b1 : 0.f);
    else
        seg_solve_all<SEG, NB>(a, sb, Bs, n, r, i, myinv, solve, fwd, bwd, -1, B + p0 * n * r);
}

}  // namespace

int launch_chol_subwave(const Shape& sh, const Geometry& g, int batch, float* A, float* B, int32_t* info,
                        void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipStream_t st = (hipStream_t)stream;
    const int n = sh.n, nb = subwave_nb(n);
    if (n > kSubwaveMaxN) return (int)hipErrorInvalidValue;
    const int region = (int)subwave_region_floats(n);
    dim3 grid((unsigned)g.grid), block(g.threads);
    const int op = sh.op == GLASS_OP_POTRF ? 0 : sh.op == GLASS_OP_POSV ? 1 : sh.op == GLASS_OP_POTRS ? 2 : 3;
#define SW(SEG, NB, OP)                                                                                         \
    if (nb == NB && op == OP) {                                                                                 \
        hipLaunchKernelGGL((chol_seg<SEG, NB, OP>), grid, block, g.lds_bytes, st, n, sh.nrhs, sh.trans, batch, A, \
                           B, info, region);                                                                    \
        return (int)hipGetLastError();                                                                          \
    }
#define SW_OPS(SEG, NB) SW(SEG, NB, 0) SW(SEG, NB, 1) SW(SEG, NB, 2) SW(SEG, NB, 3)
    SW_OPS(16, 4) SW_OPS(16, 8) SW_OPS(16, 12) SW_OPS(16, 16) SW_OPS(32, 24) SW_OPS(32, 32)
#undef SW_OPS
#undef SW
    return (int)hipErrorInvalidValue;
}

}  // namespace glass
