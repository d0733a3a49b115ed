// Overlapping Schwarz smoother kernels (see schwarz.hpp): set-up (element
// matrices, local matrices, blocked Gauss-Jordan inverses) and application
// (batched dense matrix-vector product, node-centric weighted sum).
#include "schwarz.hpp"

#include <stdexcept>

namespace pmg {

namespace {

__device__ __forceinline__ bf16_t sz_f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16_t(u >> 16);
}

int grid_of(int64_t n) { return int(n < 65536 ? (n < 1 ? 1 : n) : 65536); }

// orders this wave's LDS accesses (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

// ---------------------------------------------------------------------------
// element matrices: K[i][j] = sum_q sum_ab D_a(q, i) G_ab(q) D_b(q, j), the
// reference gradients of the prism basis being products of triangle tables
// (Dr, Ds, Bt at the triangle points) and vertical ones (Bz, Dz): x = Dr Bz,
// y = Ds Bz, z = Bt Dz.  Sum-factorised: one thread per triangle-node pair
// (ai <= aj) of one element forms, per vertical point k, the four in-plane
// sums S_BB, S_BD, S_DB, S_DD over the triangle points and spreads them to
// every vertical pair (ci, cj) through Bz / Dz.  Exactly symmetric output.
// ---------------------------------------------------------------------------
template <int N1>
__global__ __launch_bounds__(256) void k_elem_mats(int64_t n_elem, int npt, int nqt, int epb, int tab_lds,
                                                   const double* __restrict__ mats, const double* __restrict__ G,
                                                   double* __restrict__ K) {
  extern __shared__ double sm[];
  const int nq = nqt * N1, np = npt * N1, npair = npt * (npt + 1) / 2;
  const int ntab = tab_lds ? 3 * nqt * npt + 2 * N1 * N1 : 0;
  double* sT = sm;
  double* sG = sm + ntab;
  for (int i = threadIdx.x; i < ntab; i += 256) sT[i] = mats[i];
  const double* Dr = tab_lds ? sT : mats;
  const double* Ds = Dr + nqt * npt;
  const double* Bt = Ds + nqt * npt;
  const double* Bz = Bt + nqt * npt;
  const double* Dz = Bz + N1 * N1;
  for (int64_t e0 = int64_t(blockIdx.x) * epb; e0 < n_elem; e0 += int64_t(gridDim.x) * epb) {
    const int ne = int(n_elem - e0 < epb ? n_elem - e0 : epb);
    __syncthreads();
    for (int i = threadIdx.x; i < ne * 6 * nq; i += 256) sG[i] = G[size_t(e0) * 6 * nq + i];
    __syncthreads();
    for (int w = threadIdx.x; w < ne * npair; w += 256) {
      const int le = w / npair, pr = w - le * npair;
      int aj = int((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
      while (aj * (aj + 1) / 2 > pr) --aj;
      while ((aj + 1) * (aj + 2) / 2 <= pr) ++aj;
      const int ai = pr - aj * (aj + 1) / 2;
      const double* g = sG + le * 6 * nq;
      double acc[N1][N1];
      #pragma unroll
      for (int ci = 0; ci < N1; ++ci)
        #pragma unroll
        for (int cj = 0; cj < N1; ++cj) acc[ci][cj] = 0.0;
#pragma unroll 1
      for (int k = 0; k < N1; ++k) {
        double sbb = 0.0, sbd = 0.0, sdb = 0.0, sdd = 0.0;
        const double* gk = g + k * nqt;
        for (int q = 0; q < nqt; ++q) {
          const double ri = Dr[q * npt + ai], si = Ds[q * npt + ai], ti = Bt[q * npt + ai];
          const double rj = Dr[q * npt + aj], sj = Ds[q * npt + aj], tj = Bt[q * npt + aj];
          const double g0 = gk[q], g1 = gk[nq + q], g2 = gk[2 * nq + q];
          const double g3 = gk[3 * nq + q], g4 = gk[4 * nq + q], g5 = gk[5 * nq + q];
          sbb += g0 * ri * rj + g1 * (ri * sj + si * rj) + g3 * si * sj;
          sbd += tj * (g2 * ri + g4 * si);
          sdb += ti * (g2 * rj + g4 * sj);
          sdd += g5 * ti * tj;
        }
        #pragma unroll
        for (int cj = 0; cj < N1; ++cj) {
          const double vb = Bz[k * N1 + cj] * sbb + Dz[k * N1 + cj] * sbd;
          const double vd = Bz[k * N1 + cj] * sdb + Dz[k * N1 + cj] * sdd;
          #pragma unroll
          for (int ci = 0; ci < N1; ++ci) acc[ci][cj] += Bz[k * N1 + ci] * vb + Dz[k * N1 + ci] * vd;
        }
      }
      double* Ke = K + size_t(e0 + le) * np * np;
      #pragma unroll
      for (int ci = 0; ci < N1; ++ci)
        #pragma unroll
        for (int cj = 0; cj < N1; ++cj) {
          if (ai == aj && cj < ci) continue;  // diagonal triangle block: its upper half, mirrored
          const int i = ci * npt + ai, j = cj * npt + aj;
          Ke[size_t(i) * np + j] = acc[ci][cj];
          Ke[size_t(j) * np + i] = acc[ci][cj];
        }
    }
  }
}

void launch_elem_mats(const LevelView& lv, const double* mats, const double* G64, double* K, hipStream_t st) {
  const int npt = lv.np_tri, n1 = lv.PZ + 1, nqt = (lv.P + 1) * (lv.P + 1);
  const int npair = npt * (npt + 1) / 2;
  const size_t lg = sizeof(double) * 6 * size_t(nqt) * n1;  // one element's factors
  // elements per workgroup: fill the 256 threads with node pairs, within 64 KB of LDS
  int epb = npair >= 256 ? 1 : 256 / npair;
  while (epb > 1 && lg * epb > 32768) --epb;
  // tables in LDS beside G when both fit in 64 KB, else read through the caches
  const size_t ltab = sizeof(double) * (3 * size_t(nqt) * npt + 2 * size_t(n1) * n1);
  const int tab_lds = ltab + lg * epb <= 65536 ? 1 : 0;
  const size_t lds = (tab_lds ? ltab : 0) + lg * size_t(epb);
  const int64_t nb = (lv.n_elem + epb - 1) / epb;
  const dim3 grid(grid_of(nb));
  switch (n1) {
#define PMG_EM(N)                                                                                        \
  case N:                                                                                                \
    hipLaunchKernelGGL(k_elem_mats<N>, grid, dim3(256), lds, st, lv.n_elem, npt, nqt, epb, tab_lds, mats, \
                       G64, K);                                                                          \
    break;
    PMG_EM(2) PMG_EM(3) PMG_EM(4) PMG_EM(5) PMG_EM(6) PMG_EM(7) PMG_EM(8) PMG_EM(9)
#undef PMG_EM
    default: throw std::runtime_error("element matrices: vertical order outside 1..8");
  }
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
// blocked Gauss-Jordan inversion in place (pivot blocks of GJ_T = 32, no
// pivoting: the blocks are SPD; m a multiple of 32, identity on the padding).
// Per pivot block K:
//   (a) every wave inverts its own LDS copy of A_KK (unblocked Gauss-Jordan);
//   (b) row panel A_KJ <- A_KK^-1 A_KJ;
//   (c) A_IJ <- A_IJ - A_IK A_KJ for I, J != K, each wave a contiguous run of
//       the tiles in row order (A_IK stays in registers along a row);
//   (d) column panel A_IK <- -A_IK A_KK^-1, and A_KK <- A_KK^-1.
// The 32 x 32 tile products run on v_mfma_f64_16x16x4f64 (2 x 2 blocks of
// 16 x 16, eight K = 4 steps).  One workgroup per matrix.
// Register layouts (g = lane / 16, j = lane % 16): A operand A[j][g], B operand
// B[g][j], accumulator D[g + 4r][j], r = 0..3.
// ---------------------------------------------------------------------------
constexpr int GJ_T = 32;
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void k_sd_invert(int64_t k0, int64_t k1, int64_t base,
                                                   const int32_t* __restrict__ msz,
                                                   const int64_t* __restrict__ inv_off, double* __restrict__ A,
                                                   int* __restrict__ bad) {
  __shared__ double sK[4][GJ_T][GJ_T + 1];
  const int tid = threadIdx.x, l = tid & 63, lj = l & 15, lg = l >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  double(*Kw)[GJ_T + 1] = sK[wv];
  for (int64_t k = k0 + blockIdx.x; k < k1; k += gridDim.x) {
    const int m = msz[k], mt = m / GJ_T;
    double* Ak = A + (inv_off[k] - base);
    auto at = [&](int r, int c) -> double& { return Ak[size_t(r) * m + c]; };
    for (int kb = 0; kb < mt; ++kb) {
      const int p0 = kb * GJ_T;
      // (a) A_KK^-1 in this wave's LDS copy; lane l owns column l % 32 of rows 2t + l / 32
      for (int t = 0; t < 16; ++t) Kw[2 * t + (l >> 5)][l & 31] = at(p0 + 2 * t + (l >> 5), p0 + (l & 31));
      wave_sync();
      for (int p = 0; p < GJ_T; ++p) {
        const double piv = Kw[p][p];
        if (wv == 0 && l == 0 && !(piv > 0.0)) atomicOr(bad, 1);
        const double d = 1.0 / piv;
        const int c = l & 31;
        const double pc = Kw[p][c] * d;
        double v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int r = 2 * t + (l >> 5);
          const double rp = Kw[r][p];
          v[t] = r == p ? (c == p ? d : pc) : (c == p ? -rp * d : Kw[r][c] - rp * pc);
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < 16; ++t) Kw[2 * t + (l >> 5)][c] = v[t];
        wave_sync();
      }
      // (b) row panel
      for (int J = wv; J < mt; J += 4) {
        if (J == kb) continue;
        double bo[2][8];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int s = 0; s < 8; ++s) bo[bj][s] = at(p0 + 4 * s + lg, J * GJ_T + 16 * bj + lj);
        d4_t acc[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int bi = 0; bi < 2; ++bi) {
            const double a = Kw[16 * bi + lj][4 * s + lg];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma_f64(a, bo[bj][s], acc[bi][bj]);
          }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) at(p0 + 16 * bi + lg + 4 * r, J * GJ_T + 16 * bj + lj) = acc[bi][bj][r];
      }
      __syncthreads();
      // (c) trailing update
      const int mo = mt - 1, nu = mo * mo;
      const int u0 = nu * wv / 4, u1 = nu * (wv + 1) / 4;
      int Ic = -1;
      double ao[2][8];
      for (int u = u0; u < u1; ++u) {
        int I = u / mo, J = u - (u / mo) * mo;
        I += I >= kb ? 1 : 0;
        J += J >= kb ? 1 : 0;
        if (I != Ic) {
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int s = 0; s < 8; ++s) ao[bi][s] = -at(I * GJ_T + 16 * bi + lj, p0 + 4 * s + lg);
          Ic = I;
        }
        double bo[2][8];
        d4_t acc[2][2];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int s = 0; s < 8; ++s) bo[bj][s] = at(p0 + 4 * s + lg, J * GJ_T + 16 * bj + lj);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = at(I * GJ_T + 16 * bi + lg + 4 * r, J * GJ_T + 16 * bj + lj);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma_f64(ao[bi][s], bo[bj][s], acc[bi][bj]);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) at(I * GJ_T + 16 * bi + lg + 4 * r, J * GJ_T + 16 * bj + lj) = acc[bi][bj][r];
      }
      __syncthreads();
      // (d) column panel, and the inverted pivot block
      for (int I = wv; I < mt; I += 4) {
        if (I == kb) {
          for (int t = 0; t < 16; ++t) at(p0 + 2 * t + (l >> 5), p0 + (l & 31)) = Kw[2 * t + (l >> 5)][l & 31];
          continue;
        }
        double a2[2][8];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int s = 0; s < 8; ++s) a2[bi][s] = -at(I * GJ_T + 16 * bi + lj, p0 + 4 * s + lg);
        d4_t acc[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            const double b = Kw[4 * s + lg][16 * bj + lj];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) acc[bi][bj] = mfma_f64(a2[bi][s], b, acc[bi][bj]);
          }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) at(I * GJ_T + 16 * bi + lg + 4 * r, p0 + 16 * bj + lj) = acc[bi][bj][r];
      }
      __syncthreads();
    }
  }
}

// (A + A^T)/2 on the n x n block, written as the packed upper block-triangle
// tiles of the kept copies (zero outside n x n; entry order sz_tile_pos)
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
          const int r = e / SZ_TS, c = e % SZ_TS;
          if (A64) A64[off + sz_tile_pos(r, c, 8)] = v;
          if (A32) A32[off + sz_tile_pos(r, c, 4)] = float(v);
          if (A16) A16[off + sz_tile_pos(r, c, 2)] = sz_f32_to_bf16(float(v));
        }
  }
}

void launch_sd_invert(const SchwarzView& sv, int64_t k0, int64_t k1, int64_t base, double* A, double* A64,
                      float* A32, bf16_t* A16, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_sd_invert, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.msz, sv.inv_off, A,
                     bad);
  hipLaunchKernelGGL(k_sd_symm, dim3(grid_of(k1 - k0)), dim3(256), 0, st, k0, k1, base, sv.sd_ptr, sv.msz,
                     sv.inv_off, sv.tile_off, A, A64, A32, A16);
}

// ---------------------------------------------------------------------------
// application: one workgroup per subdomain, z = inv x with inv stored as the
// tiles (I, J), I <= J, of its upper block triangle.  A tile off the diagonal
// serves twice: z_I += A_IJ x_J (row pass) and z_J += A_IJ^T x_I (column
// pass); a diagonal tile (stored whole) only in the row pass.  Each wave takes
// a contiguous run of the tiles in their storage order (J-major) and keeps
// two tiles in flight.  Lane l holds the strip of row l % 32, columns
// 16 (l / 32) .. +15 of the tile (the tile is stored so that every load of a
// wave reads 1 KB contiguously, see sz_tile_pos), and uses it for both passes:
//   row pass: one dot product with x_J (in registers for the whole column),
//     the two half rows joined by one cross-half exchange, added to the
//     wave's LDS accumulator of z_I;
//   column pass: 16 running sums x_I[row] A[row][c] in registers, reduced
//     over the 32 rows once per column (at its diagonal tile or where the
//     wave's run ends) and added to z_J.
// The four wave accumulators are added in a fixed order at the end.
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The 16 entries of a strip from its NCH = sizeof(TI) 16-byte chunks.
template <typename TI> struct Strip;
template <> struct Strip<double> {
  static __device__ __forceinline__ void get(const u32x4 (&q)[8], double (&o)[16]) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      o[2 * h] = __hiloint2double(int(q[h].y), int(q[h].x));
      o[2 * h + 1] = __hiloint2double(int(q[h].w), int(q[h].z));
    }
  }
};
template <> struct Strip<float> {
  static __device__ __forceinline__ void get(const u32x4 (&q)[4], float (&o)[16]) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      o[4 * h] = __uint_as_float(q[h].x);
      o[4 * h + 1] = __uint_as_float(q[h].y);
      o[4 * h + 2] = __uint_as_float(q[h].z);
      o[4 * h + 3] = __uint_as_float(q[h].w);
    }
  }
};
template <> struct Strip<bf16_t> {
  static __device__ __forceinline__ void get(const u32x4 (&q)[2], float (&o)[16]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t wd[4] = {q[h].x, q[h].y, q[h].z, q[h].w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        o[8 * h + 2 * c] = __uint_as_float(wd[c] << 16);
        o[8 * h + 2 * c + 1] = __uint_as_float(wd[c] & 0xFFFF0000u);
      }
    }
  }
};

template <typename T, typename TI>
__global__ __launch_bounds__(256) void k_sd_apply(int64_t n_sub, int ntm, const int32_t* __restrict__ sd_ptr,
                                                  const int32_t* __restrict__ sd_node,
                                                  const int64_t* __restrict__ tile_off, const TI* __restrict__ inv,
                                                  const T* __restrict__ r, const T* __restrict__ w,
                                                  T* __restrict__ zS) {
  constexpr int TS = SZ_TS;
  constexpr int NCH = int(sizeof(TI));  // 16-byte chunks of a 16-entry strip
  extern __shared__ __align__(16) unsigned char smraw[];
  T* sx = reinterpret_cast<T*>(smraw);  // [ntm*TS]
  T* zacc = sx + size_t(ntm) * TS;      // [4][ntm*TS]
  T* red = zacc + 4 * size_t(ntm) * TS;  // [4][16][SD_RED]
  const int tid = threadIdx.x, l = tid & 63, lr = l & 31, lh = l >> 5;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: the tile loop is scalar
  T* zw = zacc + size_t(wv) * ntm * TS;
  T* rw = red + wv * 16 * SD_RED;
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
      T xj[16], zc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        xj[i] = sx[J * TS + lh * 16 + i];
        zc[i] = T(0);
      }
      auto load = [&](u32x4(&a)[NCH], int t) {
#pragma unroll
        for (int h = 0; h < NCH; ++h) a[h] = At[size_t(t) * 64 * NCH + h * 64 + l];
      };
      // column J's running sums of this run: reduce over the 32 rows, add to z_J
      auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < 16; ++i) rw[i * SD_RED + l] = zc[i];
        wave_sync();
        const int c = lr;  // lane l sums column c over rows 16 lh .. 16 lh + 15
        const T* q = rw + (c & 15) * SD_RED + (c >> 4) * 32 + 16 * lh;
        T s = T(0);
#pragma unroll
        for (int i = 0; i < 16; ++i) s += q[i];
        s += __shfl_xor(s, 32);
        if (lh == 0) zw[J * TS + c] += s;
        wave_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) zc[i] = T(0);
      };
      auto tile = [&](u32x4(&a)[NCH], int t) {
        T e[16];
        Strip<TI>::get(a, e);
        if (t + 2 < t1) load(a, t + 2);
        T pr = T(0);
#pragma unroll
        for (int i = 0; i < 16; ++i) pr += e[i] * xj[i];
        const bool diag = I == J;
        if (!diag) {
          const T xr = sx[I * TS + lr];
#pragma unroll
          for (int i = 0; i < 16; ++i) zc[i] += e[i] * xr;
        }
        const T o = __shfl_xor(pr, 32);
        if (lh == 0) zw[I * TS + lr] += pr + o;
        if (diag) {
          flush();
          ++J;
          I = 0;
          if (t + 1 < t1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) xj[i] = sx[J * TS + lh * 16 + i];
          }
        } else {
          ++I;
        }
      };
      u32x4 a0[NCH], a1[NCH];
      load(a0, t0);
      if (t0 + 1 < t1) load(a1, t0 + 1);
      for (int t = t0; t < t1; t += 2) {
        tile(a0, t);
        if (t + 1 < t1) tile(a1, t + 1);
      }
      if (I != 0) flush();  // run ended inside column J
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
  const size_t lds = sd_apply_lds(sv.max_n, sizeof(T));
  hipLaunchKernelGGL((k_sd_apply<T, TI>), dim3(grid_of(sv.n_sub)), dim3(256), lds, st, sv.n_sub, ntm, sv.sd_ptr,
                     sv.sd_node, sv.tile_off, inv, r, w, zS);
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
