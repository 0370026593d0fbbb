// riccati.hpp -- launch interface of the thread-scope form of the fused LQR
// gain (riccati.hip); the wave-scope forms are declared with the other
// launchers in glass_internal.hpp.
#pragma once
#include "glass_internal.hpp"

namespace glass {

// Thread scope: one problem per lane with every operand and intermediate in
// VGPRs, at compile-time orders up to these.
constexpr int kRiccatiThreadMaxNx = 8;
constexpr int kRiccatiThreadMaxNu = 4;

inline bool riccati_thread_ok(int nx, int nu) {
    return nx >= 1 && nu >= 1 && nx <= kRiccatiThreadMaxNx && nu <= kRiccatiThreadMaxNu;
}

// Sub-wave scope: four problems per wavefront, one per 16-lane row.
constexpr int kRiccatiSegMaxNx = 16;
constexpr int kRiccatiSegMaxNu = 8;

inline bool riccati_seg_ok(int nx, int nu) {
    return nx >= 1 && nu >= 1 && nx <= kRiccatiSegMaxNx && nu <= kRiccatiSegMaxNu;
}

// pack wavefronts (4 * pack problems) per workgroup; the caller has checked
// riccati_seg_ok.
int launch_riccati_seg(int nx, int nu, int batch, int pack, const float* A, const float* B, const float* P,
                       const float* R, float* K, int32_t* info, void* stream);

// 64 * pack lanes per workgroup; the caller has checked riccati_thread_ok.
int launch_riccati_thread(int nx, int nu, int batch, int pack, const float* A, const float* B, const float* P,
                          const float* R, float* K, int32_t* info, void* stream);

}  // namespace glass
