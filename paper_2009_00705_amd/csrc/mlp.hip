// Kernels of the warm-start network (FP32): MFMA GEMM with fused bias and
// SiLU epilogue, SiLU backward, MSE loss with deterministic reductions,
// column sums, Adam, counter-based mini-batch gather, feature assembly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "mlp.hpp"

namespace pmg {

// Hidden activations of the allocation-free forward: two halves of
// NET_NOALLOC_ROWS x NET_NOALLOC_WIDTH floats.  In host code this name is a
// stand-in, not a device address; kernels receive the address returned by
// net_scratch_ptr.  Every call on one GPU shares that GPU's copy, so calls that
// overlap on a GPU race.
static __device__ __align__(256) float scratch[2 * NET_NOALLOC_ROWS * NET_NOALLOC_WIDTH];

float* net_scratch_ptr(int device, hipError_t* err) {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static float* ptr[MAX_DEV] = {};
  *err = hipSuccess;
  if (device < 0 || device >= MAX_DEV) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    ptr[device] = static_cast<float*>(p);
  }
  return ptr[device];
}

typedef float f4m_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_d(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C = act(A B + bias); A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj].
// One wave per 16x16 tile of C, v_mfma_f32_16x16x4f32; lane l supplies
// A(i0 + l%16, k0 + l/16), B(k0 + l/16, j0 + l%16) and receives
// C(i0 + 4(l/16) + r, j0 + l%16), r = 0..3.  Z (nullable) keeps A B + bias.
template <int ACT>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int64_t sai,
                                              int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbj,
                                              const float* __restrict__ bias, float* __restrict__ Z,
                                              float* __restrict__ Cm, int64_t ldc) {
  const int tiles_n = (N + 15) / 16;
  const int64_t tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t ntile = int64_t((M + 15) / 16) * tiles_n;
  if (tile >= ntile) return;
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int i0 = int(tile / tiles_n) * 16, j0 = int(tile % tiles_n) * 16;
  f4m_t acc = {0.f, 0.f, 0.f, 0.f};
  const int ia = i0 + j, jb = j0 + j;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + g;
    const float a = (ia < M && k < K) ? A[ia * sai + k * sak] : 0.f;
    const float b = (k < K && jb < N) ? B[k * sbk + jb * sbj] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * g + r;
    if (i < M && jb < N) {
      float c = acc[r] + (bias ? bias[jb] : 0.f);
      if (Z) Z[int64_t(i) * ldc + jb] = c;
      if (ACT == 1) c = silu_f(c);
      Cm[int64_t(i) * ldc + jb] = c;
    }
  }
}

// Row-contiguous A (sak = 1), K a multiple of 16: one wave per 16 x 64 block
// of C (four MFMA chains sharing the A operand).  Every lane loads four
// consecutive k of its A row at once; step s of a group of four uses k =
// k0 + 4 g + s in lane group g for both operands (the sum over k does not
// depend on the order in which its terms are grouped).
template <int ACT>
__global__ __launch_bounds__(256) void k_gemm_rc(int M, int N, int K, const float* __restrict__ A, int64_t sai,
                                                 const float* __restrict__ B, int64_t sbk, int64_t sbj,
                                                 const float* __restrict__ bias, float* __restrict__ Z,
                                                 float* __restrict__ Cm, int64_t ldc) {
  const int tiles_n = (N + 63) / 64;
  const int64_t tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t ntile = int64_t((M + 15) / 16) * tiles_n;
  if (tile >= ntile) return;
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int i0 = int(tile / tiles_n) * 16, j0 = int(tile % tiles_n) * 64;
  f4m_t acc[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) acc[n] = f4m_t{0.f, 0.f, 0.f, 0.f};
  const int ia = i0 + j;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kb = k0 + 4 * g;
    float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ia < M) a4 = *reinterpret_cast<const float4*>(A + int64_t(ia) * sai + kb);
    const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int jb = j0 + 16 * n + j;
        const float b = jb < N ? B[int64_t(kb + s) * sbk + int64_t(jb) * sbj] : 0.f;
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], b, acc[n], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const int jb = j0 + 16 * n + j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * g + r;
      if (i < M && jb < N) {
        float c = acc[n][r] + (bias ? bias[jb] : 0.f);
        if (Z) Z[int64_t(i) * ldc + jb] = c;
        if (ACT == 1) c = silu_f(c);
        Cm[int64_t(i) * ldc + jb] = c;
      }
    }
  }
}

void launch_gemm(int M, int N, int K, const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk,
                 int64_t sbj, const float* bias, float* Z, float* C, int64_t ldc, bool silu, hipStream_t st) {
  if (sak == 1 && K % 16 == 0 && sai % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0) {
    const int64_t nt = int64_t((M + 15) / 16) * ((N + 63) / 64);
    const int grid = int((nt + 3) / 4);
    if (silu)
      hipLaunchKernelGGL(k_gemm_rc<1>, dim3(grid), dim3(256), 0, st, M, N, K, A, sai, B, sbk, sbj, bias, Z, C, ldc);
    else
      hipLaunchKernelGGL(k_gemm_rc<0>, dim3(grid), dim3(256), 0, st, M, N, K, A, sai, B, sbk, sbj, bias, Z, C, ldc);
    return;
  }
  const int64_t ntile = int64_t((M + 15) / 16) * ((N + 15) / 16);
  const int grid = int((ntile + 3) / 4);
  if (silu)
    hipLaunchKernelGGL(k_gemm<1>, dim3(grid), dim3(256), 0, st, M, N, K, A, sai, sak, B, sbk, sbj, bias, Z, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm<0>, dim3(grid), dim3(256), 0, st, M, N, K, A, sai, sak, B, sbk, sbj, bias, Z, C, ldc);
}

// dZ = dH .* silu'(Z)
__global__ void k_silu_back(const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ,
                            int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    dZ[i] = dH[i] * silu_d(Z[i]);
}
void launch_silu_back(const float* dH, const float* Z, float* dZ, int64_t n, hipStream_t st) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_silu_back, dim3(g < 1 ? 1 : g), dim3(256), 0, st, dH, Z, dZ, n);
}

// deterministic block sum of 256 doubles (thread 0)
__device__ double mlp_block_sum(double v) {
  __shared__ double sh[4];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return threadIdx.x == 0 ? (sh[0] + sh[1]) + (sh[2] + sh[3]) : 0.0;
}

// r = y - t; dY = 2 r / n; partial[b] = sum r^2 (fixed MLP_RED blocks)
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, int64_t n, double* __restrict__ partial) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float r = y[i] - t[i];
    if (dy) dy[i] = 2.0f * r / float(n);
    acc += double(r) * double(r);
  }
  const double s = mlp_block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
void launch_mse(const float* y, const float* t, float* dy, int64_t n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(MLP_RED), dim3(256), 0, st, y, t, dy, n, partial);
}
__global__ __launch_bounds__(256) void k_red_final(const double* __restrict__ partial, int np, double* __restrict__ out) {
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) a += partial[i];
  const double s = mlp_block_sum(a);
  if (threadIdx.x == 0) *out = s;
}
void launch_red_final(const double* partial, int np, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_red_final, dim3(1), dim3(256), 0, st, partial, np, out);
}

// db[j] = sum_i dZ[i][j] (thread per column, rows in ascending order)
__global__ void k_colsum(const float* __restrict__ dZ, int M, int N, float* __restrict__ db) {
  const int jcol = blockIdx.x * 256 + threadIdx.x;
  if (jcol >= N) return;
  double s = 0.0;
  for (int i = 0; i < M; ++i) s += dZ[int64_t(i) * N + jcol];
  db[jcol] = float(s);
}
void launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, st, dZ, M, N, db);
}

// Adam with bias correction (step t >= 1)
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}
void launch_adam(float* th, const float* g, float* m, float* v, int64_t n, double lr, int t, hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = float(1.0 - std::pow(b1, t)), c2 = float(1.0 - std::pow(b2, t));
  int64_t gsz = (n + 255) / 256;
  if (gsz > 4096) gsz = 4096;
  hipLaunchKernelGGL(k_adam, dim3(gsz < 1 ? 1 : gsz), dim3(256), 0, st, th, g, m, v, n, float(lr), float(b1),
                     float(b2), 1e-8f, c1, c2);
}

// mini-batch gather with a counter-based index: idx = floor(u(seed + step*B + i) * n),
// normalised inputs (x - mean) / std and scaled targets t / tscale
__device__ __forceinline__ double sm64_unit(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return double(z >> 11) * (1.0 / 9007199254740992.0);
}
__global__ void k_gather_batch(const float* __restrict__ X, const float* __restrict__ T, int64_t n, int d, int B,
                               uint64_t seed, uint64_t step, const float* __restrict__ mean,
                               const float* __restrict__ inv_std, float tinv, float* __restrict__ Xb,
                               float* __restrict__ Tb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= B) return;
  int64_t r = int64_t(sm64_unit(seed, step * uint64_t(B) + uint64_t(i)) * double(n));
  if (r >= n) r = n - 1;
  for (int c = 0; c < d; ++c) Xb[int64_t(i) * d + c] = (X[r * d + c] - mean[c]) * inv_std[c];
  Tb[i] = T[r] * tinv;
}
void launch_gather_batch(const float* X, const float* T, int64_t n, int d, int B, uint64_t seed, uint64_t step,
                         const float* mean, const float* inv_std, float tinv, float* Xb, float* Tb, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_batch, dim3((B + 255) / 256), dim3(256), 0, st, X, T, n, d, B, seed, step, mean,
                     inv_std, tinv, Xb, Tb);
}

// x_norm = (x - mean) * inv_std for all rows
__global__ void k_normalize(const float* __restrict__ X, int64_t n, int d, const float* __restrict__ mean,
                            const float* __restrict__ inv_std, float* __restrict__ Xn) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n * d; i += int64_t(gridDim.x) * 256) {
    const int c = int(i % d);
    Xn[i] = (X[i] - mean[c]) * inv_std[c];
  }
}
void launch_normalize(const float* X, int64_t n, int d, const float* mean, const float* inv_std, float* Xn,
                      hipStream_t st) {
  int64_t g = (n * d + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_normalize, dim3(g < 1 ? 1 : g), dim3(256), 0, st, X, n, d, mean, inv_std, Xn);
}

// column statistics: out[2c] = mean, out[2c+1] = mean of squares (block per column)
__global__ __launch_bounds__(256) void k_colstats(const float* __restrict__ X, int64_t n, int d, double* __restrict__ out) {
  const int c = blockIdx.x;
  double s = 0.0, s2 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = X[i * d + c];
    s += v;
    s2 += v * v;
  }
  const double a = mlp_block_sum(s);
  const double b = mlp_block_sum(s2);
  if (threadIdx.x == 0) {
    out[2 * c] = a / double(n);
    out[2 * c + 1] = b / double(n);
  }
}
void launch_colstats(const float* X, int64_t n, int d, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colstats, dim3(d), dim3(256), 0, st, X, n, d, out);
}

// features of the coarsest (P = 1) nodes, see mlp.hpp
// base extrapolation of the guess: 2 p1 - p2, or 3 p1 - 3 p2 + p3 when p3 is given
__device__ __forceinline__ double base_ex(const double* __restrict__ p1, const double* __restrict__ p2,
                                          const double* __restrict__ p3, int64_t i) {
  return p3 ? 3.0 * p1[i] - 3.0 * p2[i] + p3[i] : 2.0 * p1[i] - p2[i];
}

__global__ void k_features(int64_t n1, int nz1, int nzf, int Pf, const float* __restrict__ cst,
                           const double* __restrict__ surf, const double* __restrict__ p1,
                           const double* __restrict__ p2, const double* __restrict__ p3,
                           const double* __restrict__ pnow, float* __restrict__ X, float* __restrict__ T) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n1; g += int64_t(gridDim.x) * 256) {
    const int64_t v = g / nz1;
    const int zl = int(g - v * nz1);
    const int64_t gf = v * nzf + int64_t(zl) * Pf;   // the same point on the finest level
    const int64_t top = v * nzf + (nzf - 1);
    float* x = X + g * NET_DIN;
    x[0] = cst[g * 4 + 0];
    x[1] = cst[g * 4 + 1];
    x[2] = cst[g * 4 + 2];
    x[3] = cst[g * 4 + 3];
    x[4] = float(p1[gf] - p2[gf]);
    x[5] = float(surf[v] - base_ex(p1, p2, p3, top));
    x[6] = float(p1[top] - p2[top]);
    if (T) T[g] = float(pnow[gf] - base_ex(p1, p2, p3, gf));
  }
}
void launch_features(int64_t n1, int nz1, int nzf, int Pf, const float* cst, const double* surf, const double* p1,
                     const double* p2, const double* p3, const double* pnow, float* X, float* T, hipStream_t st) {
  int64_t g = (n1 + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_features, dim3(g < 1 ? 1 : g), dim3(256), 0, st, n1, nz1, nzf, Pf, cst, surf, p1, p2, p3,
                     pnow, X, T);
}

// u_coarse (double) = out_scale * y (float) on free nodes of the coarsest level
__global__ void k_scale_out(const float* __restrict__ y, double s, int64_t n, double* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    out[i] = s * double(y[i]);
}
void launch_scale_out(const float* y, double s, int64_t n, double* out, hipStream_t st) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_scale_out, dim3(g < 1 ? 1 : g), dim3(256), 0, st, y, s, n, out);
}

// correction of the base extrapolation at the coarsest surface nodes is known exactly:
// delta = surf[v] - base(top)
__global__ void k_corr_surface(int64_t n1, int nz1, int nzf, const double* __restrict__ surf,
                               const double* __restrict__ p1, const double* __restrict__ p2,
                               const double* __restrict__ p3, double* __restrict__ delta) {
  for (int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x; v * nz1 < n1; v += int64_t(gridDim.x) * 256) {
    const int64_t top = v * nzf + (nzf - 1);
    delta[v * nz1 + (nz1 - 1)] = surf[v] - base_ex(p1, p2, p3, top);
  }
}
void launch_corr_surface(int64_t n1, int nz1, int nzf, const double* surf, const double* p1, const double* p2,
                         const double* p3, double* delta, hipStream_t st) {
  int64_t g = (n1 / nz1 + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_corr_surface, dim3(g < 1 ? 1 : g), dim3(256), 0, st, n1, nz1, nzf, surf, p1, p2, p3, delta);
}

// out = 2 p1 - p2, or 3 p1 - 3 p2 + p3 (p3 given)
__global__ void k_extrap(const double* __restrict__ p1, const double* __restrict__ p2,
                         const double* __restrict__ p3, double* __restrict__ out, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    out[i] = base_ex(p1, p2, p3, i);
}
void launch_extrap(const double* p1, const double* p2, const double* p3, double* out, int64_t n, hipStream_t st) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_extrap, dim3(g < 1 ? 1 : g), dim3(256), 0, st, p1, p2, p3, out, n);
}

}  // namespace pmg
