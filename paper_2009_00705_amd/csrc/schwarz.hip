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

// (A + A^T)/2 on the n x n block, written as the packed upper block-triangle
// tiles of the kept copies (zero outside n x n)
__global__ __launch_bounds__(256) void k_sd_symm(int64_t k0, int64_t k1, int64_t base,
                                                 const int32_t* __restrict__ sd_ptr,
                                                 const int32_t* __restrict__ msz,
                                                 const int64_t* __restrict__ inv_off,
                                                 const int64_t* __restrict__ tile_off, const double* __restrict__ A,
                                                 double* __restrict__ A64, float* __restrict__ A32,
                                                 bf16_t* __restrict__ A16) {
  for (int64_t k = k0 + blockIdx.x; k < k1; k += gridDim.x) {
    const int m = msz[k], n = sd_ptr[k + 1] - sd_ptr[k];
    const int nt = (n + SZ_TS - 1) / SZ_TS;
    const double* Ak = A + (inv_off[k] - base);
    int64_t off = tile_off[k];
    for (int J = 0; J < nt; ++J)
      for (int I = 0; I <= J; ++I, off += SZ_TS * SZ_TS)
        for (int e = threadIdx.x; e < SZ_TS * SZ_TS; e += 256) {
          const int i = I * SZ_TS + (e / SZ_TS), j = J * SZ_TS + (e % SZ_TS);
          const int lo = i < j ? i : j, hi = i < j ? j : i;
          const double v = hi < n ? 0.5 * (Ak[size_t(lo) * m + hi] + Ak[size_t(hi) * m + lo]) : 0.0;
          if (A64) A64[off + e] = v;
          if (A32) A32[off + e] = float(v);
          if (A16) A16[off + e] = sz_f32_to_bf16(float(v));
        }
  }
}

void launch_sd_invert(const SchwarzView& sv, int64_t k0, int64_t k1, int64_t base, double* A, double* A64,
                      float* A32, bf16_t* A16, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_sd_invert, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.sd_ptr, sv.msz,
                     sv.inv_off, A, bad);
  hipLaunchKernelGGL(k_sd_symm, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.sd_ptr, sv.msz,
                     sv.inv_off, sv.tile_off, A, A64, A32, A16);
}

// ---------------------------------------------------------------------------
// application: one workgroup per subdomain, z = inv x with inv stored as the
// tiles (I, J), I <= J, of its upper block triangle.  A tile off the diagonal
// serves twice: z_I += A_IJ x_J (row pass) and z_J += A_IJ^T x_I (column
// pass); a diagonal tile (stored whole) only in the row pass.  Each wave takes
// a contiguous run of the tiles in their storage order (J-major), so x_J sits
// in registers and z_J accumulates in registers until the column ends.  A tile
// is read from HBM once, with 16-byte loads (the next tile's are issued before
// the current one is used), and staged in the wave's own LDS slice (rows
// padded by 16 bytes: both passes read it without bank conflicts).  Lane l
// takes row l mod 32 over the column half l / 32 in the row pass and column
// l mod 32 over the row half l / 32 in the column pass; one cross-half
// exchange completes both sums.  z_I goes to the wave's own LDS accumulator;
// the four accumulators are added in a fixed order at the end.
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Entries of a staged tile: get(p, i) one entry, row(p, o) the 16 entries at
// p (16-byte aligned) read as 16-byte words.
template <typename TI> struct TileT;
template <> struct TileT<double> {
  static __device__ __forceinline__ double get(const double* p, int i) { return p[i]; }
  static __device__ __forceinline__ void row(const double* p, double (&o)[16]) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const u32x4 v = q[h];
      o[2 * h] = __hiloint2double(int(v.y), int(v.x));
      o[2 * h + 1] = __hiloint2double(int(v.w), int(v.z));
    }
  }
};
template <> struct TileT<float> {
  static __device__ __forceinline__ float get(const float* p, int i) { return p[i]; }
  static __device__ __forceinline__ void row(const float* p, float (&o)[16]) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const u32x4 v = q[h];
      o[4 * h] = __uint_as_float(v.x);
      o[4 * h + 1] = __uint_as_float(v.y);
      o[4 * h + 2] = __uint_as_float(v.z);
      o[4 * h + 3] = __uint_as_float(v.w);
    }
  }
};
template <> struct TileT<bf16_t> {
  static __device__ __forceinline__ float get(const bf16_t* p, int i) { return __uint_as_float(uint32_t(p[i]) << 16); }
  static __device__ __forceinline__ void row(const bf16_t* p, float (&o)[16]) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const u32x4 v = q[h];
      const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        o[8 * h + 2 * c] = __uint_as_float(wd[c] << 16);
        o[8 * h + 2 * c + 1] = __uint_as_float(wd[c] & 0xFFFF0000u);
      }
    }
  }
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, typename TI>
__global__ __launch_bounds__(256) void k_sd_apply(int64_t n_sub, int ntm, const int32_t* __restrict__ sd_ptr,
                                                  const int32_t* __restrict__ sd_node,
                                                  const int64_t* __restrict__ tile_off, const TI* __restrict__ inv,
                                                  const T* __restrict__ r, const T* __restrict__ w,
                                                  T* __restrict__ zS) {
  constexpr int TS = SZ_TS;
  constexpr int EC = 16 / int(sizeof(TI));   // entries per 16-byte chunk
  constexpr int NCH = int(sizeof(TI));       // 16-byte chunks per lane and tile (TS*TS/64 entries)
  constexpr int RS = TS + EC;                // padded LDS row (entries)
  static_assert(TS * TS * int(sizeof(TI)) == 64 * 16 * NCH, "tile = 64 lanes x NCH chunks");
  extern __shared__ __align__(16) unsigned char smraw[];
  T* sx = reinterpret_cast<T*>(smraw);                       // [ntm*TS]
  T* zacc = sx + size_t(ntm) * TS;                           // [4][ntm*TS]
  TI* stile = reinterpret_cast<TI*>(zacc + 4 * size_t(ntm) * TS);  // [4][TS*RS]
  const int tid = threadIdx.x, l = tid & 63, lr = l & 31, lh = l >> 5;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: the tile loop is scalar
  T* zw = zacc + size_t(wv) * ntm * TS;
  TI* st = stile + wv * TS * RS;
  for (int64_t k = blockIdx.x; k < n_sub; k += gridDim.x) {
    const int32_t b = sd_ptr[k];
    const int n = sd_ptr[k + 1] - b, nt = (n + TS - 1) / TS, np = nt * TS;
    __syncthreads();
    for (int j = tid; j < np; j += 256) {
      T x = T(0);
      if (j < n) {
        const int32_t g = sd_node[b + j];
        x = w ? r[g] * w[g] : r[g];
      }
      sx[j] = x;
    }
    for (int j = tid; j < 4 * np; j += 256) zacc[(j / np) * ntm * TS + j % np] = T(0);
    __syncthreads();
    const int ntl = nt * (nt + 1) / 2;
    const int t0 = ntl * wv / 4, t1 = ntl * (wv + 1) / 4;
    if (t0 < t1) {
      const u32x4* At = reinterpret_cast<const u32x4*>(inv + tile_off[k]);
      int J = 0;
      while ((J + 1) * (J + 2) / 2 <= t0) ++J;
      int I = t0 - J * (J + 1) / 2;
      u32x4 a[NCH];
#pragma unroll
      for (int h = 0; h < NCH; ++h) a[h] = At[size_t(t0) * 64 * NCH + h * 64 + l];
      T xj[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) xj[i] = sx[J * TS + lh * 16 + i];
      T zj = T(0);
      for (int t = t0; t < t1; ++t) {
        wave_sync();
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
          const int e = (h * 64 + l) * EC;  // first entry of the chunk
          *reinterpret_cast<u32x4*>(st + (e / TS) * RS + e % TS) = a[h];
        }
        if (t + 1 < t1) {
#pragma unroll
          for (int h = 0; h < NCH; ++h) a[h] = At[size_t(t + 1) * 64 * NCH + h * 64 + l];
        }
        wave_sync();
        // row pass: row lr, columns lh*16 .. lh*16+15
        T pr = T(0);
        {
          T e[16];
          TileT<TI>::row(st + lr * RS + lh * 16, e);
#pragma unroll
          for (int i = 0; i < 16; ++i) pr += e[i] * xj[i];
        }
        const bool diag = I == J;
        T pc = T(0);
        if (!diag) {
          // column pass: column lr, rows lh*16 .. lh*16+15
          const TI* col = st + lh * 16 * RS + lr;
          const T* xi = sx + I * TS + lh * 16;
#pragma unroll
          for (int i = 0; i < 16; ++i) pc += T(TileT<TI>::get(col, i * RS)) * xi[i];
        }
        // lanes < 32 complete row sums, lanes >= 32 column sums
        const T o = __shfl_xor((lh == 0 && !diag) ? pc : pr, 32);
        // at the diagonal the upper lanes hand over the column's z_J (same rows)
        const T oz = diag ? __shfl_xor(zj, 32) : T(0);
        if (lh == 0) {
          zw[I * TS + lr] += (pr + o) + oz;
        } else if (!diag) {
          zj += pc + o;
        }
        if (diag) {
          // next column
          ++J;
          I = 0;
          zj = T(0);
          if (t + 1 < t1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) xj[i] = sx[J * TS + lh * 16 + i];
          }
        } else {
          ++I;
        }
      }
      // run ended inside a column: flush the upper lanes' z_J
      if (I != 0 && lh == 1) zw[J * TS + lr] += zj;
    }
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
      const size_t q = size_t(ntm) * TS;
      zS[b + i] = ((zacc[i] + zacc[q + i]) + zacc[2 * q + i]) + zacc[3 * q + i];
    }
  }
}

template <typename T, typename TI>
void launch_sd_apply(const SchwarzView& sv, const TI* inv, const T* r, const T* w, T* zS, hipStream_t st) {
  const int ntm = (sv.max_n + SZ_TS - 1) / SZ_TS;
  hipLaunchKernelGGL((k_sd_apply<T, TI>), dim3(grid_of(sv.n_sub)), dim3(256), sd_apply_lds(sv.max_n, sizeof(T), sizeof(TI)), st,
                     sv.n_sub, ntm, sv.sd_ptr, sv.sd_node, sv.tile_off, inv, r, w, zS);
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
