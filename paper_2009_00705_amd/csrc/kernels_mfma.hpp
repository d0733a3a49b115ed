// MFMA element operator of the fine levels (see kernels_mfma.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace pmg {

// MF_F32G16: FP32 MFMA arithmetic reading the BF16 lane-native copy of G;
// MF_BF16X3: split-BF16 products (three BF16 MFMAs each) on the BF16 copy of G
// and the hi / lo BF16 tables; MF_BF16X2: split vectors on the BF16 tables (two)
enum MfmaFlavour { MF_F64 = 0, MF_F32 = 1, MF_BF16 = 2, MF_F32G16 = 3, MF_BF16X3 = 4, MF_BF16X2 = 5 };

// vertical interpolation/derivative matrices at the Gauss points (Bz[k][c],
// Dz[k][c]), the same with row k scaled by the Gauss weight zw_k (Bzw, Dzw),
// and the weights zw and positions zh = (1 + zq) / 2 in [0, 1], passed by value
template <typename T> struct VertMats {
  T Bz[81];
  T Dz[81];
  T Bzw[81];
  T Dzw[81];
  T zw[9];
  T zh[9];
};

template <typename TO> __device__ __forceinline__ TO cvt_out(double v);
template <> __device__ __forceinline__ double cvt_out<double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt_out<float>(double v) { return float(v); }
template <> __device__ __forceinline__ bf16_t cvt_out<bf16_t>(double v) {
  uint32_t u = __float_as_uint(float(v));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16_t(u >> 16);
}
__device__ __forceinline__ double gld_any(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float gld_any(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float gld_any(const bf16_t* p, int64_t i) { return __uint_as_float(uint32_t(p[i]) << 16); }

// (triangle, vertical) orders with an MFMA kernel for a flavour
inline bool mfma_available(int PT, int PZ, int flavour) {
  const bool order = (PT == 3 && PZ == 3) || (PT == 6 && PZ == 6) || (PT == 3 && PZ == 6) ||
                     (PT == 4 && PZ == 8) || (PT == 2 && PZ == 8) || (PT == 8 && PZ == 8);
  // split-BF16 kernels at in-plane order 6 only: at lower orders the K = 16 steps
  // pad the few triangle nodes and FP32 MFMA is faster; at 8 the tables do not fit
  if (flavour == MF_BF16X3 || flavour == MF_BF16X2) return order && PT == 6;
  return order;
}
// lane-native copy of G for a flavour, from the standard FP64 G, or (geo given)
// formed from the FP64 column factors of an L-layer column with vertical Gauss
// points zq and weights zw (device arrays)
void launch_g_native(int PT, int PZ, int64_t n_elem, const double* G, void* out, int flavour, hipStream_t st,
                     const double* geo = nullptr, int L = 1, const double* zq = nullptr,
                     const double* zw = nullptr);
// tab2lo / tab4lo: the lo tables of MF_BF16X3 (unused by the other flavours).
// geo (optional): column factors of the level (FP64 for MF_F64, FP32 for MF_F32
// and the split-BF16 flavours; ignored by MF_BF16 and MF_F32G16, which read
// their stored BF16 G), from which the kernel computes G in place of reading
// Gnat.
// colsum: write column sums (the layout of launch_col_sum) instead of the
// element layout; returns false, launching nothing, when the level has no
// such kernel (the level's colsum flag, orders with more (node, prism) pairs
// per batch than threads, stored-G FP64/FP32, MF_BF16X2); otherwise true.
bool launch_ax_mfma(const LevelView& lv, const void* Gnat, int flavour, const void* tab2, const void* tab4,
                    const void* vmats, const void* u, void* Y, hipStream_t st, const void* tab2lo = nullptr,
                    const void* tab4lo = nullptr, const void* geo = nullptr, bool colsum = false);

}  // namespace pmg
