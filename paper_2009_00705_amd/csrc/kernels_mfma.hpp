// MFMA element operator of the fine levels (see kernels_mfma.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace pmg {

// MF_F32G16: FP32 MFMA arithmetic reading the BF16 lane-native copy of G;
// MF_BF16X3: split-BF16 products (three BF16 MFMAs each) on the BF16 copy of G
// and the hi / lo BF16 tables
enum MfmaFlavour { MF_F64 = 0, MF_F32 = 1, MF_BF16 = 2, MF_F32G16 = 3, MF_BF16X3 = 4 };

// vertical interpolation/derivative matrices at the Gauss points, passed by value
template <typename T> struct VertMats {
  T Bz[81];
  T Dz[81];
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
  if ((PT == 3 && PZ == 3) || (PT == 6 && PZ == 6) || (PT == 3 && PZ == 6)) return true;
  if (PT == 8 && PZ == 8) return flavour != MF_BF16X3;  // LDS
  return false;
}
void launch_g_native(int PT, int PZ, int64_t n_elem, const double* G, void* out, int flavour, hipStream_t st);
// tab2lo / tab4lo: the lo tables of MF_BF16X3 (unused by the other flavours)
void launch_ax_mfma(const LevelView& lv, const void* Gnat, int flavour, const void* tab2, const void* tab4,
                    const void* vmats, const void* u, void* Y, hipStream_t st, const void* tab2lo = nullptr,
                    const void* tab4lo = nullptr);

}  // namespace pmg
