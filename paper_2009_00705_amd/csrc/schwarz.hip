// Overlapping Schwarz smoother kernels (see schwarz.hpp): set-up (element
// matrices, local matrices, blocked Gauss-Jordan inverses) and application
// (batched dense matrix-vector product, node-centric weighted sum).
#include "schwarz.hpp"

namespace pmg {

namespace {

__device__ __forceinline__ bf16_t sz_f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16_t(u >> 16);
}

int grid_of(int64_t n) { return int(n < 65536 ? (n < 1 ? 1 : n) : 65536); }

}  // namespace

// ---------------------------------------------------------------------------
// element matrices: K[i][j] = sum_q sum_ab D_a(q, i) G_ab(q) D_b(q, j), the
// reference gradients of the prism basis being products of the triangle
// tables (Dr, Ds, B at the triangle points) and the vertical ones (Bz, Dz).
// Upper triangle computed, mirrored.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_elem_mats(int64_t n_elem, int npt, int nqt, int n1, int tab_lds,
                                                   const double* __restrict__ mats, const double* __restrict__ G,
                                                   double* __restrict__ K) {
  extern __shared__ double sm[];
  const int nq = nqt * n1, np = npt * n1;
  const int ntab = tab_lds ? 3 * nqt * npt + 2 * n1 * n1 : 0;
  double* sT = sm;
  double* sG = sm + ntab;
  for (int i = threadIdx.x; i < ntab; i += 256) sT[i] = mats[i];
  const double* Dr = tab_lds ? sT : mats;
  const double* Ds = Dr + nqt * npt;
  const double* Bt = Ds + nqt * npt;
  const double* Bz = Bt + nqt * npt;
  const double* Dz = Bz + n1 * n1;
  const int npair = np * (np + 1) / 2;
  for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
    __syncthreads();
    for (int i = threadIdx.x; i < 6 * nq; i += 256) sG[i] = G[size_t(e) * 6 * nq + i];
    __syncthreads();
    double* Ke = K + size_t(e) * np * np;
    for (int idx = threadIdx.x; idx < npair; idx += 256) {
      // idx = j (j + 1) / 2 + i, i <= j
      int j = int((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (j * (j + 1) / 2 > idx) --j;
      while ((j + 1) * (j + 2) / 2 <= idx) ++j;
      const int i = idx - j * (j + 1) / 2;
      const int ci = i / npt, ai = i - ci * npt, cj = j / npt, aj = j - cj * npt;
      double s = 0.0;
      for (int k = 0; k < n1; ++k) {
        const double bzi = Bz[k * n1 + ci], dzi = Dz[k * n1 + ci];
        const double bzj = Bz[k * n1 + cj], dzj = Dz[k * n1 + cj];
        const double* g = sG + k * nqt;
        for (int q = 0; q < nqt; ++q) {
          const double xi = Dr[q * npt + ai] * bzi, yi = Ds[q * npt + ai] * bzi, zi = Bt[q * npt + ai] * dzi;
          const double xj = Dr[q * npt + aj] * bzj, yj = Ds[q * npt + aj] * bzj, zj = Bt[q * npt + aj] * dzj;
          s += g[q] * xi * xj + g[nq + q] * (xi * yj + yi * xj) + g[2 * nq + q] * (xi * zj + zi * xj) +
               g[3 * nq + q] * yi * yj + g[4 * nq + q] * (yi * zj + zi * yj) + g[5 * nq + q] * zi * zj;
        }
      }
      Ke[size_t(i) * np + j] = s;
      Ke[size_t(j) * np + i] = s;
    }
  }
}

void launch_elem_mats(const LevelView& lv, const double* mats, const double* G64, double* K, hipStream_t st) {
  const int npt = lv.np_tri, n1 = lv.PZ + 1, nqt = (lv.P + 1) * (lv.P + 1);
  // tables in LDS beside G when both fit in 64 KB, else read through the caches
  const size_t ltab = sizeof(double) * (3 * size_t(nqt) * npt + 2 * size_t(n1) * n1);
  const size_t lg = sizeof(double) * 6 * size_t(nqt) * n1;
  const int tab_lds = ltab + lg <= 65536 ? 1 : 0;
  hipLaunchKernelGGL(k_elem_mats, dim3(grid_of(lv.n_elem)), dim3(256), tab_lds ? ltab + lg : lg, st, lv.n_elem, npt,
                     nqt, n1, tab_lds, mats, G64, K);
}

// ---------------------------------------------------------------------------
// local matrices: every prism block adds its entries; blocks in ascending
// prism order (fixed summation order), no two entries of a block collide.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sd_assemble(int64_t k0, int64_t k1, int64_t base,
                                                     const int32_t* __restrict__ sd_ptr,
                                                     const int32_t* __restrict__ msz,
                                                     const int64_t* __restrict__ inv_off,
                                                     const int32_t* __restrict__ blk_ptr,
                                                     const int32_t* __restrict__ blk_elem,
                                                     const int32_t* __restrict__ blk_ent,
                                                     const int32_t* __restrict__ ent, int np,
                                                     const double* __restrict__ K, double* __restrict__ A) {
  for (int64_t k = k0 + blockIdx.x; k < k1; k += gridDim.x) {
    const int m = msz[k], n = sd_ptr[k + 1] - sd_ptr[k];
    double* Ak = A + (inv_off[k] - base);
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * m; idx += 256) {
      const int i = idx / m, j = idx - i * m;
      Ak[idx] = (i == j && i >= n) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int b = blk_ptr[k]; b < blk_ptr[k + 1]; ++b) {
      const int e0 = blk_ent[b], ne = blk_ent[b + 1] - e0;
      const double* Ke = K + size_t(blk_elem[b]) * np * np;
      for (int idx = threadIdx.x; idx < ne * ne; idx += 256) {
        const int u = idx / ne, v = idx - u * ne;
        const int eu = ent[e0 + u], ev = ent[e0 + v];
        Ak[size_t(eu & 0xFFFF) * m + (ev & 0xFFFF)] += Ke[size_t(eu >> 16) * np + (ev >> 16)];
      }
      __syncthreads();
    }
  }
}

void launch_sd_assemble(const SchwarzView& sv, int64_t k0, int64_t k1, int64_t base, int np, const double* K,
                        double* A, hipStream_t st) {
  hipLaunchKernelGGL(k_sd_assemble, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.sd_ptr, sv.msz,
                     sv.inv_off, sv.blk_ptr, sv.blk_elem, sv.blk_ent, sv.ent, np, K, A);
}

// ---------------------------------------------------------------------------
// blocked Gauss-Jordan inversion in place (pivot blocks of GJ_B, no pivoting).
// Per pivot block K: A_KK <- A_KK^-1 (in LDS); A_KJ <- A_KK^-1 A_KJ;
// A_IJ <- A_IJ - A_IK A_KJ; A_IK <- -A_IK A_KK^-1, rows in chunks of GJ_RC
// whose A_IK is staged in LDS.  One workgroup per matrix.
// ---------------------------------------------------------------------------
constexpr int GJ_B = 16, GJ_RC = 256;

__global__ __launch_bounds__(256) void k_sd_invert(int64_t k0, int64_t k1, int64_t base,
                                                   const int32_t* __restrict__ sd_ptr,
                                                   const int32_t* __restrict__ msz,
                                                   const int64_t* __restrict__ inv_off, double* __restrict__ A,
                                                   int* __restrict__ bad) {
  __shared__ double sKK[GJ_B][GJ_B + 1];
  __shared__ double sCol[GJ_RC][GJ_B + 1];
  const int tid = threadIdx.x;
  for (int64_t k = k0 + blockIdx.x; k < k1; k += gridDim.x) {
    const int m = msz[k], n = sd_ptr[k + 1] - sd_ptr[k];
    double* Ak = A + (inv_off[k] - base);
    for (int p0 = 0; p0 < n; p0 += GJ_B) {
      const int bb = n - p0 < GJ_B ? n - p0 : GJ_B;
      const int r = tid / GJ_B, c = tid - r * GJ_B;
      __syncthreads();
      if (r < bb && c < bb) sKK[r][c] = Ak[size_t(p0 + r) * m + p0 + c];
      __syncthreads();
      // 1. A_KK^-1 by unblocked Gauss-Jordan
      for (int p = 0; p < bb; ++p) {
        const double piv = sKK[p][p];
        if (tid == 0 && !(piv > 0.0)) atomicOr(bad, 1);
        const double d = 1.0 / piv;
        double v = 0.0;
        if (r < bb && c < bb) {
          if (r == p && c == p) v = d;
          else if (r == p) v = sKK[p][c] * d;
          else if (c == p) v = -sKK[r][p] * d;
          else v = sKK[r][c] - sKK[r][p] * (sKK[p][c] * d);
        }
        __syncthreads();
        if (r < bb && c < bb) sKK[r][c] = v;
        __syncthreads();
      }
      // 2. row panel A_KJ <- A_KK^-1 A_KJ
      for (int j = tid; j < n; j += 256) {
        if (j >= p0 && j < p0 + bb) continue;
        double x[GJ_B], y[GJ_B];
#pragma unroll
        for (int s = 0; s < GJ_B; ++s) x[s] = s < bb ? Ak[size_t(p0 + s) * m + j] : 0.0;
#pragma unroll
        for (int s = 0; s < GJ_B; ++s) {
          double a = 0.0;
#pragma unroll
          for (int u = 0; u < GJ_B; ++u)
            if (u < bb) a += sKK[s][u] * x[u];
          y[s] = a;
        }
#pragma unroll
        for (int s = 0; s < GJ_B; ++s)
          if (s < bb) Ak[size_t(p0 + s) * m + j] = y[s];
      }
      __syncthreads();
      // 3. rank-bb update and column panel, by row chunks
      for (int i0 = 0; i0 < n; i0 += GJ_RC) {
        const int nr = n - i0 < GJ_RC ? n - i0 : GJ_RC;
        for (int idx = tid; idx < nr * GJ_B; idx += 256) {
          const int ii = idx / GJ_B, s = idx - ii * GJ_B;
          const int i = i0 + ii;
          sCol[ii][s] = (s < bb && !(i >= p0 && i < p0 + bb)) ? Ak[size_t(i) * m + p0 + s] : 0.0;
        }
        __syncthreads();
        for (int j = tid; j < n; j += 256) {
          if (j >= p0 && j < p0 + bb) continue;
          double rp[GJ_B];
#pragma unroll
          for (int s = 0; s < GJ_B; ++s) rp[s] = s < bb ? Ak[size_t(p0 + s) * m + j] : 0.0;
          int ii = 0;
          for (; ii + 4 <= nr; ii += 4) {
            double a[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) a[h] = Ak[size_t(i0 + ii + h) * m + j];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
#pragma unroll
              for (int s = 0; s < GJ_B; ++s) a[h] -= sCol[ii + h][s] * rp[s];
            }
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              const int i = i0 + ii + h;
              if (!(i >= p0 && i < p0 + bb)) Ak[size_t(i) * m + j] = a[h];
            }
          }
          for (; ii < nr; ++ii) {
            const int i = i0 + ii;
            if (i >= p0 && i < p0 + bb) continue;
            double a = Ak[size_t(i) * m + j];
#pragma unroll
            for (int s = 0; s < GJ_B; ++s) a -= sCol[ii][s] * rp[s];
            Ak[size_t(i) * m + j] = a;
          }
        }
        for (int idx = tid; idx < nr * GJ_B; idx += 256) {
          const int ii = idx / GJ_B, s = idx - ii * GJ_B;
          const int i = i0 + ii;
          if (s >= bb || (i >= p0 && i < p0 + bb)) continue;
          double a = 0.0;
#pragma unroll
          for (int u = 0; u < GJ_B; ++u) a -= sCol[ii][u] * sKK[u][s];
          Ak[size_t(i) * m + p0 + s] = a;
        }
        __syncthreads();
      }
      if (r < bb && c < bb) Ak[size_t(p0 + r) * m + p0 + c] = sKK[r][c];
    }
  }
}

// (A + A^T)/2 on the n x n block, written to the kept copies of the whole
// padded block (FP64 may be the work block itself)
__global__ __launch_bounds__(256) void k_sd_symm(int64_t k0, int64_t k1, int64_t base,
                                                 const int32_t* __restrict__ sd_ptr,
                                                 const int32_t* __restrict__ msz,
                                                 const int64_t* __restrict__ inv_off, double* A, double* A64,
                                                 float* __restrict__ A32, bf16_t* __restrict__ A16) {
  for (int64_t k = k0 + blockIdx.x; k < k1; k += gridDim.x) {
    const int m = msz[k], n = sd_ptr[k + 1] - sd_ptr[k];
    const int64_t off = inv_off[k];
    double* Ak = A + (off - base);
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * m; idx += 256) {
      const int i = idx / m, j = idx - i * m;
      if (j < i) continue;
      double v = Ak[size_t(i) * m + j];
      if (j < n) v = 0.5 * (v + Ak[size_t(j) * m + i]);
      if (A64) {
        A64[off + size_t(i) * m + j] = v;
        A64[off + size_t(j) * m + i] = v;
      }
      if (A32) {
        A32[off + size_t(i) * m + j] = float(v);
        A32[off + size_t(j) * m + i] = float(v);
      }
      if (A16) {
        A16[off + size_t(i) * m + j] = sz_f32_to_bf16(float(v));
        A16[off + size_t(j) * m + i] = sz_f32_to_bf16(float(v));
      }
    }
  }
}

void launch_sd_invert(const SchwarzView& sv, int64_t k0, int64_t k1, int64_t base, double* A, double* A64,
                      float* A32, bf16_t* A16, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_sd_invert, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.sd_ptr, sv.msz,
                     sv.inv_off, A, bad);
  hipLaunchKernelGGL(k_sd_symm, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.sd_ptr, sv.msz,
                     sv.inv_off, A, A64, A32, A16);
}

// ---------------------------------------------------------------------------
// application: one workgroup per subdomain.  The local vector x is gathered
// into LDS; lane l owns rows VR*l .. VR*l+VR-1 and streams the (symmetric)
// inverse column by column, one 8-byte load per column (VR = 8/sizeof(TI)),
// so a wave reads 512 contiguous bytes per column.  When the row vectors fill
// at most half the workgroup (BF16 inverses: up to 128 vectors = 512 rows), the
// columns are split in two halves, one per half of the workgroup, and the two
// partial sums are added in a fixed order through LDS: every thread streams,
// twice the loads are in flight.
// ---------------------------------------------------------------------------
template <typename TI> struct Vec8;
template <> struct Vec8<double> { typedef double type; static constexpr int VR = 1; };
template <> struct Vec8<float> { typedef float2 type; static constexpr int VR = 2; };
template <> struct Vec8<bf16_t> { typedef uint2 type; static constexpr int VR = 4; };

template <typename T>
__device__ __forceinline__ void unpack(const double& v, T* o) { o[0] = T(v); }
template <typename T>
__device__ __forceinline__ void unpack(const float2& v, T* o) { o[0] = v.x; o[1] = v.y; }
template <typename T>
__device__ __forceinline__ void unpack(const uint2& v, T* o) {
  o[0] = __uint_as_float(v.x << 16);
  o[1] = __uint_as_float(v.x & 0xFFFF0000u);
  o[2] = __uint_as_float(v.y << 16);
  o[3] = __uint_as_float(v.y & 0xFFFF0000u);
}

// acc[0..VR) += sum over columns j in [j0, j1) of A[j][rows of vector l] x[j]
template <typename T, typename V, int VR>
__device__ __forceinline__ void sd_columns(const V* __restrict__ Ak, int mv, int l, int j0, int j1,
                                           const T* __restrict__ sx, T (&acc)[VR]) {
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    V a[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) a[h] = Ak[size_t(j + h) * mv + l];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      T e[VR];
      unpack<T>(a[h], e);
      const T x = sx[j + h];
#pragma unroll
      for (int v = 0; v < VR; ++v) acc[v] += e[v] * x;
    }
  }
  for (; j < j1; ++j) {
    T e[VR];
    unpack<T>(Ak[size_t(j) * mv + l], e);
    const T x = sx[j];
#pragma unroll
    for (int v = 0; v < VR; ++v) acc[v] += e[v] * x;
  }
}

template <typename T, typename TI>
__global__ __launch_bounds__(256) void k_sd_apply(int64_t n_sub, const int32_t* __restrict__ sd_ptr,
                                                  const int32_t* __restrict__ sd_node,
                                                  const int32_t* __restrict__ msz,
                                                  const int64_t* __restrict__ inv_off, const TI* __restrict__ inv,
                                                  const T* __restrict__ r, const T* __restrict__ w,
                                                  T* __restrict__ zS) {
  typedef typename Vec8<TI>::type V;
  constexpr int VR = Vec8<TI>::VR;
  extern __shared__ unsigned char smraw[];
  T* sx = reinterpret_cast<T*>(smraw);
  __shared__ T spart[128 * VR];  // second half's partial sums (split columns)
  const int tid = threadIdx.x;
  for (int64_t k = blockIdx.x; k < n_sub; k += gridDim.x) {
    const int32_t b = sd_ptr[k];
    const int n = sd_ptr[k + 1] - b, m = msz[k];
    __syncthreads();
    for (int j = tid; j < n; j += 256) {
      const int32_t g = sd_node[b + j];
      sx[j] = w ? r[g] * w[g] : r[g];
    }
    __syncthreads();
    const V* Ak = reinterpret_cast<const V*>(inv + inv_off[k]);
    const int mv = m / VR;        // vectors per column
    const int nv = (n + VR - 1) / VR;
    if (nv <= 128) {
      // split columns: threads 0..127 take [0, n/2), threads 128..255 take [n/2, n)
      const int half = tid >> 7, l = tid & 127, jm = n >> 1;
      T acc[VR];
#pragma unroll
      for (int v = 0; v < VR; ++v) acc[v] = T(0);
      if (l < nv) sd_columns<T, V, VR>(Ak, mv, l, half ? jm : 0, half ? n : jm, sx, acc);
      if (half && l < nv) {
#pragma unroll
        for (int v = 0; v < VR; ++v) spart[l * VR + v] = acc[v];
      }
      __syncthreads();
      if (!half && l < nv) {
#pragma unroll
        for (int v = 0; v < VR; ++v)
          if (VR * l + v < n) zS[b + VR * l + v] = acc[v] + spart[l * VR + v];
      }
    } else {
      for (int l = tid; l < nv; l += 256) {
        T acc[VR];
#pragma unroll
        for (int v = 0; v < VR; ++v) acc[v] = T(0);
        sd_columns<T, V, VR>(Ak, mv, l, 0, n, sx, acc);
#pragma unroll
        for (int v = 0; v < VR; ++v)
          if (VR * l + v < n) zS[b + VR * l + v] = acc[v];
      }
    }
  }
}

template <typename T, typename TI>
void launch_sd_apply(const SchwarzView& sv, const TI* inv, const T* r, const T* w, T* zS, hipStream_t st) {
  hipLaunchKernelGGL((k_sd_apply<T, TI>), dim3(grid_of(sv.n_sub)), dim3(256), sizeof(T) * size_t(sv.max_m), st,
                     sv.n_sub, sv.sd_ptr, sv.sd_node, sv.msz, sv.inv_off, inv, r, w, zS);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sd_sum(int64_t n_dof, const int32_t* __restrict__ node_ptr,
                                                const int32_t* __restrict__ node_pos, const T* __restrict__ zS,
                                                const T* __restrict__ w, T omega, int accumulate,
                                                T* __restrict__ u) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n_dof; g += int64_t(gridDim.x) * 256) {
    T s = T(0);
    for (int32_t p = node_ptr[g]; p < node_ptr[g + 1]; ++p) s += zS[node_pos[p]];
    if (w) s *= w[g];
    u[g] = accumulate ? u[g] + omega * s : omega * s;
  }
}

template <typename T>
void launch_sd_sum(const SchwarzView& sv, int64_t n_dof, const T* zS, const T* w, T omega, bool accumulate, T* u,
                   hipStream_t st) {
  const int64_t nb = (n_dof + 255) / 256;
  hipLaunchKernelGGL((k_sd_sum<T>), dim3(int(nb < 65536 ? (nb < 1 ? 1 : nb) : 65536)), dim3(256), 0, st, n_dof,
                     sv.node_ptr, sv.node_pos, zS, w, omega, int(accumulate), u);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sd_scale(T* __restrict__ x, T s, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) x[i] *= s;
}

template <typename T>
void launch_sd_scale(T* x, double s, int64_t n, hipStream_t st) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL((k_sd_scale<T>), dim3(int(nb < 65536 ? (nb < 1 ? 1 : nb) : 65536)), dim3(256), 0, st, x, T(s), n);
}

template void launch_sd_scale<double>(double*, double, int64_t, hipStream_t);
template void launch_sd_scale<float>(float*, double, int64_t, hipStream_t);
template void launch_sd_apply<double, double>(const SchwarzView&, const double*, const double*, const double*,
                                              double*, hipStream_t);
template void launch_sd_apply<float, float>(const SchwarzView&, const float*, const float*, const float*, float*,
                                            hipStream_t);
template void launch_sd_apply<float, bf16_t>(const SchwarzView&, const bf16_t*, const float*, const float*, float*,
                                             hipStream_t);
template void launch_sd_sum<double>(const SchwarzView&, int64_t, const double*, const double*, double, bool,
                                    double*, hipStream_t);
template void launch_sd_sum<float>(const SchwarzView&, int64_t, const float*, const float*, float, bool, float*,
                                   hipStream_t);

}  // namespace pmg
