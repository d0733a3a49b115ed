// Warm-start network kernels (FP32).  See mlp.hip.
//
// Features of a coarsest-level (P = 1) node g = (vertex v, level z), with the
// finest-level node gf at the same point, top = the finest surface node of
// column v, p1/p2 the two previous solutions and surf the new surface data:
//   x0..x3 constants: sigma = z / L, x and y scaled to [-1, 1], distance to
//          the nearest curved boundary circle (0 without one)
//   x4 = p1[gf] - p2[gf]                       (local rate)
//   x5 = surf[v] - base[top]                   (new surface data minus its extrapolation)
//   x6 = p1[top] - p2[top]                     (surface rate)
// target T = pnow[gf] - base[gf]               (the correction of the extrapolation)
// with base = 2 p1 - p2, or 3 p1 - 3 p2 + p3 when a third previous solution p3 is given
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmg {

constexpr int NET_DIN = 7;
constexpr int MLP_RED = 256;

// Allocation-free forward: rows go through the network in chunks of at most
// NET_NOALLOC_ROWS, their hidden activations ping-ponging between two
// [NET_NOALLOC_ROWS][NET_NOALLOC_WIDTH] FP32 halves of a file-scope device
// array (8 MiB per GPU, held until the process ends).  Networks wider than
// NET_NOALLOC_WIDTH are rejected by that entry point.
constexpr int NET_NOALLOC_ROWS = 4096;
constexpr int NET_NOALLOC_WIDTH = 256;
// Device address of this GPU's activation array (the current device's copy),
// looked up once per device with hipGetSymbolAddress; null (with the HIP error
// in *err) if the lookup fails.
float* net_scratch_ptr(int device, hipError_t* err);

void launch_gemm(int M, int N, int K, const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk,
                 int64_t sbj, const float* bias, float* Z, float* C, int64_t ldc, bool silu, hipStream_t st);
void launch_silu_back(const float* dH, const float* Z, float* dZ, int64_t n, hipStream_t st);
void launch_mse(const float* y, const float* t, float* dy, int64_t n, double* partial, hipStream_t st);
void launch_red_final(const double* partial, int np, double* out, hipStream_t st);
void launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t st);
void launch_adam(float* th, const float* g, float* m, float* v, int64_t n, double lr, int t, hipStream_t st);
void launch_gather_batch(const float* X, const float* T, int64_t n, int d, int B, uint64_t seed, uint64_t step,
                         const float* mean, const float* inv_std, float tinv, float* Xb, float* Tb, hipStream_t st);
void launch_normalize(const float* X, int64_t n, int d, const float* mean, const float* inv_std, float* Xn,
                      hipStream_t st);
void launch_colstats(const float* X, int64_t n, int d, double* out, hipStream_t st);
void launch_features(int64_t n1, int nz1, int nzf, int Pf, const float* cst, const double* surf, const double* p1,
                     const double* p2, const double* p3, const double* pnow, float* X, float* T, hipStream_t st);
void launch_scale_out(const float* y, double s, int64_t n, double* out, hipStream_t st);
void launch_corr_surface(int64_t n1, int nz1, int nzf, const double* surf, const double* p1, const double* p2,
                         const double* p3, double* delta, hipStream_t st);
void launch_extrap(const double* p1, const double* p2, const double* p3, double* out, int64_t n, hipStream_t st);

}  // namespace pmg
