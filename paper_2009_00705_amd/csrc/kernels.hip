// Device kernels of the p-multigrid SEM Laplace solve (gfx950, wave64).
//
// Layouts (all chosen by this library):
//  * L-vectors: global node g = id2d*(L*P+1) + z, columns contiguous.
//  * E-vectors ("Y"): [t][a][layer][c] so that the column of triangle node a
//    of triangle t is contiguous (L*(P+1) values) and the node-centric sum
//    reads it with unit stride.
//  * G: [e][6][Nq] with components (rr, rs, rt, ss, st, tt) and cubature index
//    k*Nq_tri + q (levels that keep it stored).
//  * Column factors: [t][q][8], seven factors per triangle cubature point from
//    which G of every layer and vertical point of the column follows (k_geom).
//  * Reference matrices ("mats"): [Dr | Ds | B] (Nq_tri x Np_tri each, row
//    major) followed by [Bz | Dz] ((P+1) x (P+1) each).
#include <hip/hip_runtime.h>

#include <cmath>

#include "epilogue.hpp"
#include "kernels.hpp"

namespace pmg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(bf16_t h) {
  return __uint_as_float(uint32_t(h) << 16);
}
__device__ __forceinline__ bf16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return bf16_t(u >> 16);
}
template <typename T> __device__ __forceinline__ T ldg(const double* p, size_t i) { return T(p[i]); }
template <typename T> __device__ __forceinline__ T ldg(const float* p, size_t i) { return T(p[i]); }
template <typename T> __device__ __forceinline__ T ldg(const bf16_t* p, size_t i) { return T(bf16_to_f32(p[i])); }

// deterministic block sum (256 threads); result valid in thread 0
__device__ double block_sum256(double v) {
  __shared__ double sh[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return threadIdx.x == 0 ? (sh[0] + sh[1]) + (sh[2] + sh[3]) : 0.0;
}

static inline int grid_for(int64_t n, int per = 256, int cap = 65535 * 4) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

// position of vertical level z inside a column of L*(P+1) element values (P the
// vertical order); p2 >= 0 when z is an interior layer interface (two copies)
__device__ __forceinline__ void column_pos(int z, int P, int L, int& p1, int& p2) {
  if (z == 0) { p1 = 0; p2 = -1; return; }
  const int layer = (z - 1) / P;
  const int c = z - layer * P;
  p1 = layer * (P + 1) + c;
  p2 = (c == P && layer + 1 < L) ? p1 + 1 : -1;
}

// ---------------------------------------------------------------------------
// generic element operator (all orders, LDS staged)
// ---------------------------------------------------------------------------
// PT: triangle order, PZ: vertical order (N1 = PZ + 1 vertical nodes / points)
template <int PT, int PZ> struct Dims {
  static constexpr int N1 = PZ + 1, NPT = (PT + 1) * (PT + 2) / 2, NP = NPT * N1;
  static constexpr int NQT = (PT + 1) * (PT + 1), NQ = NQT * N1;
  static constexpr int NMAT = 3 * NQT * NPT + 2 * N1 * N1;
  static constexpr int PER_EL = (NP > 3 * NQ ? NP : 3 * NQ) + 2 * N1 * NPT;
  static constexpr int NEB = (4096 / PER_EL) < 1 ? 1 : ((4096 / PER_EL) > 64 ? 64 : (4096 / PER_EL));
};

template <int PT, int PZ, typename T, typename TG>
__global__ __launch_bounds__(256) void k_ax(const int32_t* __restrict__ map2d, int L, int nz,
                                            int64_t n_elem, const T* __restrict__ mats,
                                            const TG* __restrict__ G, const T* __restrict__ u,
                                            T* __restrict__ Y) {
  using D = Dims<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NP = D::NP, NQT = D::NQT, NQ = D::NQ, NEB = D::NEB;
  constexpr int SA = (NP > 3 * NQ ? NP : 3 * NQ), SB = 2 * N1 * NPT;
  __shared__ T sm_mat[D::NMAT];
  __shared__ T sm_a[NEB * SA];
  __shared__ T sm_b[NEB * SB];
  for (int i = threadIdx.x; i < D::NMAT; i += 256) sm_mat[i] = mats[i];
  const T* Dr = sm_mat;
  const T* Ds = Dr + NQT * NPT;
  const T* Bt = Ds + NQT * NPT;
  const T* Bz = Bt + NQT * NPT;
  const T* Dz = Bz + N1 * N1;
  for (int64_t e0 = int64_t(blockIdx.x) * NEB; e0 < n_elem; e0 += int64_t(gridDim.x) * NEB) {
    const int ne = int(n_elem - e0 < NEB ? n_elem - e0 : NEB);
    __syncthreads();
    // gather: item (el, a, c), c fastest (contiguous in the L-vector)
    for (int i = threadIdx.x; i < ne * NP; i += 256) {
      const int el = i / NP, r = i - el * NP, a = r / N1, c = r - a * N1;
      const int64_t e = e0 + el;
      const int t = int(e / L), layer = int(e - int64_t(t) * L);
      const int64_t g = int64_t(map2d[size_t(t) * NPT + a]) * nz + layer * PZ + c;
      sm_a[el * SA + c * NPT + a] = u[g];
    }
    __syncthreads();
    // vertical: W[k][a] = sum_c Bz[k][c] U[c][a], Wz with Dz
    for (int i = threadIdx.x; i < ne * N1 * NPT; i += 256) {
      const int el = i / (N1 * NPT), r = i - el * N1 * NPT, k = r / NPT, a = r - k * NPT;
      const T* U = sm_a + el * SA;
      T w = 0, wz = 0;
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        const T uv = U[c * NPT + a];
        w += Bz[k * N1 + c] * uv;
        wz += Dz[k * N1 + c] * uv;
      }
      sm_b[el * SB + k * NPT + a] = w;
      sm_b[el * SB + N1 * NPT + k * NPT + a] = wz;
    }
    __syncthreads();
    // triangle contractions + geometric factors at every cubature point
    for (int i = threadIdx.x; i < ne * NQ; i += 256) {
      const int el = i / NQ, r = i - el * NQ, k = r / NQT, q = r - k * NQT;
      const T* W = sm_b + el * SB + k * NPT;
      const T* Wz = W + N1 * NPT;
      T ur = 0, us = 0, ut = 0;
#pragma unroll 4
      for (int a = 0; a < NPT; ++a) {
        ur += Dr[q * NPT + a] * W[a];
        us += Ds[q * NPT + a] * W[a];
        ut += Bt[q * NPT + a] * Wz[a];
      }
      const size_t gb = size_t(e0 + el) * 6 * NQ + r;
      const T g0 = ldg<T>(G, gb), g1 = ldg<T>(G, gb + NQ), g2 = ldg<T>(G, gb + 2 * NQ);
      const T g3 = ldg<T>(G, gb + 3 * NQ), g4 = ldg<T>(G, gb + 4 * NQ), g5 = ldg<T>(G, gb + 5 * NQ);
      T* V = sm_a + el * SA;
      V[r] = g0 * ur + g1 * us + g2 * ut;
      V[NQ + r] = g1 * ur + g3 * us + g4 * ut;
      V[2 * NQ + r] = g2 * ur + g4 * us + g5 * ut;
    }
    __syncthreads();
    // transposed triangle contractions
    for (int i = threadIdx.x; i < ne * N1 * NPT; i += 256) {
      const int el = i / (N1 * NPT), r = i - el * N1 * NPT, k = r / NPT, a = r - k * NPT;
      const T* vr = sm_a + el * SA + k * NQT;
      const T* vs = vr + NQ;
      const T* vt = vr + 2 * NQ;
      T yr = 0, yt = 0;
#pragma unroll 4
      for (int q = 0; q < NQT; ++q) {
        yr += Dr[q * NPT + a] * vr[q] + Ds[q * NPT + a] * vs[q];
        yt += Bt[q * NPT + a] * vt[q];
      }
      sm_b[el * SB + k * NPT + a] = yr;
      sm_b[el * SB + N1 * NPT + k * NPT + a] = yt;
    }
    __syncthreads();
    // vertical transpose, store E-layout
    for (int i = threadIdx.x; i < ne * NP; i += 256) {
      const int el = i / NP, r = i - el * NP, a = r / N1, c = r - a * N1;
      const T* Yr = sm_b + el * SB;
      const T* Yt = Yr + N1 * NPT;
      T y = 0;
#pragma unroll
      for (int k = 0; k < N1; ++k) y += Bz[k * N1 + c] * Yr[k * NPT + a] + Dz[k * N1 + c] * Yt[k * NPT + a];
      const int64_t e = e0 + el;
      const int t = int(e / L), layer = int(e - int64_t(t) * L);
      Y[((size_t(t) * NPT + a) * L + layer) * N1 + c] = y;
    }
  }
}

template <int PT, int PZ, typename T>
static void ax_dispatch_g(const LevelView& lv, const T* mats, const void* G, int gstore, const T* u,
                          T* Y, hipStream_t st) {
  constexpr int NEB = Dims<PT, PZ>::NEB;
  const int64_t nb = (lv.n_elem + NEB - 1) / NEB;
  const int grid = int(nb < 262144 ? nb : 262144);
  if (gstore == G_F64)
    hipLaunchKernelGGL((k_ax<PT, PZ, T, double>), dim3(grid), dim3(256), 0, st, lv.map2d, lv.L, int(lv.nz),
                       lv.n_elem, mats, (const double*)G, u, Y);
  else if (gstore == G_F32)
    hipLaunchKernelGGL((k_ax<PT, PZ, T, float>), dim3(grid), dim3(256), 0, st, lv.map2d, lv.L, int(lv.nz),
                       lv.n_elem, mats, (const float*)G, u, Y);
  else
    hipLaunchKernelGGL((k_ax<PT, PZ, T, bf16_t>), dim3(grid), dim3(256), 0, st, lv.map2d, lv.L, int(lv.nz),
                       lv.n_elem, mats, (const bf16_t*)G, u, Y);
}

template <typename T>
void launch_ax(const LevelView& lv, const T* mats, const void* G, int gstore, const T* u, T* Y,
               hipStream_t st) {
#define PMG_AX(PTV, PZV) \
  if (lv.P == PTV && lv.PZ == PZV) return ax_dispatch_g<PTV, PZV, T>(lv, mats, G, gstore, u, Y, st);
  PMG_ORDERS(PMG_AX)
#undef PMG_AX
}
bool order_supported(int PT, int PZ) {
#define PMG_OS(PTV, PZV) \
  if (PT == PTV && PZ == PZV) return true;
  PMG_ORDERS(PMG_OS)
#undef PMG_OS
  return false;
}
bool pair_supported(int PFT, int PFZ, int PCT, int PCZ) {
#define PMG_PS(A, B, C, D) \
  if (PFT == A && PFZ == B && PCT == C && PCZ == D) return true;
  PMG_PAIRS(PMG_PS)
#undef PMG_PS
  return false;
}
template void launch_ax<double>(const LevelView&, const double*, const void*, int, const double*, double*, hipStream_t);
template void launch_ax<float>(const LevelView&, const float*, const void*, int, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// node-centric direct-stiffness sum with fused epilogues
// ---------------------------------------------------------------------------
// Thread per global node g = n nz + z (32-bit: every level has fewer than 2^32
// nodes, pmg_create).  The node's epilogue inputs and the element values of its
// first two incidences are read first, with no read waiting on another beyond
// the incidence ids; nodes of more triangle columns (triangle vertices) read
// the next ASM_UNROLL together the same way, and any further ones in a loop.
// The sum runs in ascending incidence order.
constexpr int ASM_UNROLL = 6;
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_assemble(uint32_t n_dof, uint32_t nz, int L, int P,
                                                  const int32_t* __restrict__ inc_ptr,
                                                  const int32_t* __restrict__ inc,
                                                  const uint8_t* __restrict__ dir2d, int top_dir,
                                                  const T* __restrict__ Y, T* __restrict__ out,
                                                  const T* __restrict__ a1, const T* __restrict__ a2,
                                                  T* __restrict__ a3, T omega, T c1,
                                                  double* __restrict__ partial, T* __restrict__ a4) {
  const uint32_t colen = uint32_t(L * (P + 1));
  double acc = 0.0;
  for (uint64_t gl = uint64_t(blockIdx.x) * 256 + threadIdx.x; gl < n_dof; gl += uint64_t(gridDim.x) * 256) {
    const uint32_t g = uint32_t(gl), g2 = g / nz, z = g - g2 * nz;
    const int j0 = inc_ptr[g2], n = inc_ptr[g2 + 1] - j0;
    const bool dir = dir2d[g2] || (top_dir && z == nz - 1);
    const NodeIn<T> in = node_in<T, OP>(g, out, a1, a2, a3);
    int p1, p2;
    column_pos(int(z), P, L, p1, p2);
    // p2 read as p1 off an interface (same line, not added); every node has n >= 1
    const int q2 = p2 >= 0 ? p2 : p1;
    T s;
    {
      const T* ca = Y + size_t(uint32_t(inc[j0])) * colen;
      const T* cb = Y + size_t(uint32_t(inc[j0 + (n > 1 ? 1 : 0)])) * colen;
      const T xa = ca[p1], ya = ca[q2], xb = cb[p1], yb = cb[q2];
      s = xa;
      if (p2 >= 0) s += ya;
      if (n > 1) {
        s += xb;
        if (p2 >= 0) s += yb;
      }
    }
    if (n > 2) {  // vertex columns: the next ASM_UNROLL incidences at once, clamped in bounds
      T x[ASM_UNROLL], y[ASM_UNROLL];
#pragma unroll
      for (int u = 0; u < ASM_UNROLL; ++u) {
        const T* col = Y + size_t(uint32_t(inc[j0 + 2 + (u < n - 3 ? u : n - 3)])) * colen;
        x[u] = col[p1];
        y[u] = col[q2];
      }
#pragma unroll
      for (int u = 0; u < ASM_UNROLL; ++u) {
        if (u + 2 < n) {
          s += x[u];
          if (p2 >= 0) s += y[u];
        }
      }
      for (int j = j0 + 2 + ASM_UNROLL; j < j0 + n; ++j) {
        const T* col = Y + size_t(uint32_t(inc[j])) * colen;
        s += col[p1];
        if (p2 >= 0) s += col[p2];
      }
    }
    if constexpr (OP == OP_AVG_RAW) {
      out[g] = s / T(n * (p2 >= 0 ? 2 : 1));
    } else if constexpr (OP == OP_AVG_ADD || OP == OP_AVG_STORE) {
      const T m = T(n * (p2 >= 0 ? 2 : 1));
      const T v = dir ? T(0) : s / m;
      if (OP == OP_AVG_ADD) out[g] = in.o + v; else out[g] = v;
    } else {
      node_epilogue<T, OP>(g, dir, s, in, out, const_cast<T*>(a1), a3, a4, omega, c1, acc);
    }
  }
  if (OP == OP_STORE_DOT) {
    const double b = block_sum256(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
  }
}

template <typename T>
void launch_assemble(const LevelView& lv, int op, const T* Y, T* out, const T* a1, const T* a2, T* a3,
                     double omega, double c1, double* partial, hipStream_t st, T* a4) {
  const int grid = op == OP_STORE_DOT ? RED_BLOCKS : grid_for(lv.n_dof);
#define PMG_ASM(OPV)                                                                                   \
  hipLaunchKernelGGL((k_assemble<T, OPV>), dim3(grid), dim3(256), 0, st, uint32_t(lv.n_dof),           \
                     uint32_t(lv.nz), lv.L,                                                           \
                     lv.PZ, lv.inc_ptr, lv.inc, lv.dir2d, lv.top_dir, Y, out, a1, a2, a3, T(omega),   \
                     T(c1), partial, a4)
  switch (op) {
    case OP_STORE: PMG_ASM(OP_STORE); break;
    case OP_AVG_ADD: PMG_ASM(OP_AVG_ADD); break;
    case OP_RESID: PMG_ASM(OP_RESID); break;
    case OP_JACOBI: PMG_ASM(OP_JACOBI); break;
    case OP_STORE_DOT: PMG_ASM(OP_STORE_DOT); break;
    case OP_AVG_STORE: PMG_ASM(OP_AVG_STORE); break;
    case OP_CHEB: PMG_ASM(OP_CHEB); break;
    case OP_RAW: PMG_ASM(OP_RAW); break;
    case OP_AVG_RAW: PMG_ASM(OP_AVG_RAW); break;
    case OP_CHEB0: PMG_ASM(OP_CHEB0); break;
    default: break;
  }
#undef PMG_ASM
}
template void launch_assemble<double>(const LevelView&, int, const double*, double*, const double*, const double*, double*, double, double, double*, hipStream_t, double*);
template void launch_assemble<float>(const LevelView&, int, const float*, float*, const float*, const float*, float*, double, double, double*, hipStream_t, float*);

// ---------------------------------------------------------------------------
// Coloured direct-stiffness sum (see launch_dss in kernels.hpp)
// ---------------------------------------------------------------------------
// One colour: item (i, a, z), z fastest, of the colour's triangles tri[i]: the
// node's value in the triangle's column (its two layers' values at a layer
// interface) added to S at the node.  Reads and writes run along z.
template <typename T>
__global__ __launch_bounds__(256) void k_dss_colour(uint32_t n_items, uint32_t nz, int L, int P, int np_tri,
                                                    const int32_t* __restrict__ tri,
                                                    const int32_t* __restrict__ map2d, const T* __restrict__ Y,
                                                    T* __restrict__ S) {
  const uint32_t colen = uint32_t(L * (P + 1));
  for (uint64_t it = uint64_t(blockIdx.x) * 256 + threadIdx.x; it < n_items; it += uint64_t(gridDim.x) * 256) {
    const uint32_t q = uint32_t(it) / nz, z = uint32_t(it) - q * nz;
    const uint32_t i = q / uint32_t(np_tri), a = q - i * uint32_t(np_tri);
    const uint32_t inc = uint32_t(tri[i]) * uint32_t(np_tri) + a;
    int p1, p2;
    column_pos(int(z), P, L, p1, p2);
    const T* col = Y + size_t(inc) * colen;
    T v = col[p1];
    if (p2 >= 0) v += col[p2];
    T* sp = S + size_t(uint32_t(map2d[inc])) * nz + z;
    *sp += v;
  }
}

// Epilogue per node from the summed S (then S back to zero); the averaging ops
// divide by the node's number of element values, as k_assemble does.
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_dss_finish(uint32_t n_dof, uint32_t nz, int L, int P,
                                                    const int32_t* __restrict__ inc_ptr,
                                                    const uint8_t* __restrict__ dir2d, int top_dir,
                                                    T* __restrict__ S, T* __restrict__ out,
                                                    const T* __restrict__ a1, const T* __restrict__ a2,
                                                    T* __restrict__ a3, T omega, T c1,
                                                    double* __restrict__ partial, T* __restrict__ a4) {
  double acc = 0.0;
  for (uint64_t gl = uint64_t(blockIdx.x) * 256 + threadIdx.x; gl < n_dof; gl += uint64_t(gridDim.x) * 256) {
    const uint32_t g = uint32_t(gl), g2 = g / nz, z = g - g2 * nz;
    const bool dir = dir2d[g2] || (top_dir && z == nz - 1);
    const NodeIn<T> in = node_in<T, OP>(g, out, a1, a2, a3);
    const T s = S[g];
    S[g] = T(0);
    if constexpr (OP == OP_AVG_RAW || OP == OP_AVG_ADD || OP == OP_AVG_STORE) {
      int p1, p2;
      column_pos(int(z), P, L, p1, p2);
      const T m = T((inc_ptr[g2 + 1] - inc_ptr[g2]) * (p2 >= 0 ? 2 : 1));
      if constexpr (OP == OP_AVG_RAW) {
        out[g] = s / m;
      } else {
        const T v = dir ? T(0) : s / m;
        if (OP == OP_AVG_ADD) out[g] = in.o + v; else out[g] = v;
      }
    } else {
      node_epilogue<T, OP>(g, dir, s, in, out, const_cast<T*>(a1), a3, a4, omega, c1, acc);
    }
  }
  if constexpr (OP == OP_STORE_DOT) {
    const double b = block_sum256(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
  }
}

template <typename T>
void launch_dss(const LevelView& lv, const std::vector<int64_t>& tcol_ptr, int op, const T* Y, T* S, T* out,
                const T* a1, const T* a2, T* a3, double omega, double c1, double* partial, hipStream_t st, T* a4) {
  const int npt = lv.np_tri;
  for (size_t c = 0; c + 1 < tcol_ptr.size(); ++c) {
    const int64_t n_items = (tcol_ptr[c + 1] - tcol_ptr[c]) * npt * lv.nz;
    if (n_items <= 0) continue;
    hipLaunchKernelGGL((k_dss_colour<T>), dim3(grid_for(n_items)), dim3(256), 0, st, uint32_t(n_items),
                       uint32_t(lv.nz), lv.L, lv.PZ, npt, lv.tcol_list + tcol_ptr[c], lv.map2d, Y, S);
  }
  const int grid = op == OP_STORE_DOT ? RED_BLOCKS : grid_for(lv.n_dof);
#define PMG_DF(OPV)                                                                                          \
  hipLaunchKernelGGL((k_dss_finish<T, OPV>), dim3(grid), dim3(256), 0, st, uint32_t(lv.n_dof), uint32_t(lv.nz), \
                     lv.L, lv.PZ, lv.inc_ptr, lv.dir2d, lv.top_dir, S, out, a1, a2, a3, T(omega), T(c1), partial, \
                     a4)
  switch (op) {
    case OP_STORE: PMG_DF(OP_STORE); break;
    case OP_AVG_ADD: PMG_DF(OP_AVG_ADD); break;
    case OP_RESID: PMG_DF(OP_RESID); break;
    case OP_JACOBI: PMG_DF(OP_JACOBI); break;
    case OP_STORE_DOT: PMG_DF(OP_STORE_DOT); break;
    case OP_AVG_STORE: PMG_DF(OP_AVG_STORE); break;
    case OP_CHEB: PMG_DF(OP_CHEB); break;
    case OP_RAW: PMG_DF(OP_RAW); break;
    case OP_AVG_RAW: PMG_DF(OP_AVG_RAW); break;
    case OP_CHEB0: PMG_DF(OP_CHEB0); break;
    default: break;
  }
#undef PMG_DF
}
template void launch_dss<double>(const LevelView&, const std::vector<int64_t>&, int, const double*, double*, double*,
                                 const double*, const double*, double*, double, double, double*, hipStream_t,
                                 double*);
template void launch_dss<float>(const LevelView&, const std::vector<int64_t>&, int, const float*, float*, float*,
                                const float*, const float*, float*, double, double, double*, hipStream_t, float*);

// ---------------------------------------------------------------------------
// Node sum from column sums (see launch_col_sum in kernels.hpp).  Thread per
// global node g = n nz + z: a triangle-interior node (n >= n_bnd) reads its one
// value, cv[g - n_bnd nz], in global order; a vertex or edge node adds the
// column sums cv_b[(t 3P + s) nz + z] of the triangles holding it (ascending
// triangle order).  Then the node epilogue.  z is fastest across a wave, so
// every read is a contiguous run.
// ---------------------------------------------------------------------------
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_col_sum(int64_t n_dof, uint32_t nz, int64_t n_bnd,
                                                 const T* __restrict__ cv, const T* __restrict__ cv_b,
                                                 const int32_t* __restrict__ sh_ptr,
                                                 const int32_t* __restrict__ sh_idx,
                                                 const uint8_t* __restrict__ dir2d, int top_dir,
                                                 T* __restrict__ out, const T* __restrict__ a1,
                                                 const T* __restrict__ a2, T* __restrict__ a3, T omega, T c1,
                                                 double* __restrict__ partial, T* __restrict__ a4) {
  double acc = 0.0;
  const int64_t g_bnd = n_bnd * int64_t(nz);
  for (uint64_t gl = uint64_t(blockIdx.x) * 256 + threadIdx.x; gl < n_dof; gl += uint64_t(gridDim.x) * 256) {
    const uint32_t g = uint32_t(gl), n2 = g / nz, z = g - n2 * nz;  // n_dof < 2^32 (pmg_create)
    const NodeIn<T> in = node_in<T, OP>(g, out, a1, a2, a3);
    T s;
    if (int64_t(g) >= g_bnd) {
      s = cv[g - g_bnd];
    } else {
      s = 0;
      const int j1 = sh_ptr[n2 + 1];
      for (int j = sh_ptr[n2]; j < j1; ++j) s += cv_b[size_t(sh_idx[j]) * nz + z];
    }
    const bool dir = dir2d[n2] || (top_dir && z == nz - 1);
    node_epilogue<T, OP>(g, dir, s, in, out, const_cast<T*>(a1), a3, a4, omega, c1, acc);
  }
  if constexpr (OP == OP_STORE_DOT) {
    const double b = block_sum256(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
  }
}

template <typename T>
void launch_col_sum(const LevelView& lv, int op, const T* cv, T* out, const T* a1, const T* a2, T* a3,
                    double omega, double c1, double* partial, hipStream_t st, T* a4) {
  const int grid = op == OP_STORE_DOT ? RED_BLOCKS : grid_for(lv.n_dof);
  const T* cv_b = cv + int64_t(lv.nt) * lv.nint * lv.nz;
#define PMG_CS(OPV)                                                                                     \
  hipLaunchKernelGGL((k_col_sum<T, OPV>), dim3(grid), dim3(256), 0, st, lv.n_dof, uint32_t(lv.nz), lv.n_bnd, \
                     cv, cv_b, lv.sh_ptr, lv.sh_idx, lv.dir2d, lv.top_dir, out, a1, a2, a3, T(omega), T(c1), \
                     partial, a4)
  switch (op) {
    case OP_STORE: PMG_CS(OP_STORE); break;
    case OP_RESID: PMG_CS(OP_RESID); break;
    case OP_JACOBI: PMG_CS(OP_JACOBI); break;
    case OP_STORE_DOT: PMG_CS(OP_STORE_DOT); break;
    case OP_CHEB: PMG_CS(OP_CHEB); break;
    case OP_RAW: PMG_CS(OP_RAW); break;
    case OP_CHEB0: PMG_CS(OP_CHEB0); break;
    default: break;
  }
#undef PMG_CS
}
template void launch_col_sum<double>(const LevelView&, int, const double*, double*, const double*, const double*,
                                     double*, double, double, double*, hipStream_t, double*);
template void launch_col_sum<float>(const LevelView&, int, const float*, float*, const float*, const float*,
                                    float*, double, double, double*, hipStream_t, float*);

// ---------------------------------------------------------------------------
// geometric factors (thread per triangle x triangle cubature point)
// ---------------------------------------------------------------------------
template <int PF>
__global__ __launch_bounds__(256) void k_geom(int nt, int L, int nqtl, int n1l, double depth,
                                              const double* __restrict__ xyt,
                                              const double* __restrict__ eta,
                                              const int32_t* __restrict__ map2d_f,
                                              const double* __restrict__ gmats,
                                              const double* __restrict__ wq,
                                              const double* __restrict__ zq,
                                              const double* __restrict__ zw, double* __restrict__ G64,
                                              float* __restrict__ G32, bf16_t* __restrict__ G16,
                                              int* __restrict__ bad, double* __restrict__ geo64,
                                              float* __restrict__ geo32) {
  // fine map of order PF, evaluated at the level's nqtl triangle points and n1l vertical points
  constexpr int NPTF = (PF + 1) * (PF + 2) / 2;
  const int NQTL = nqtl, N1L = n1l, NQL = nqtl * n1l;
  const int64_t item = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (item >= int64_t(nt) * NQTL) return;
  const int t = int(item / NQTL), q = int(item - int64_t(t) * NQTL);
  const double* Bf = gmats;
  const double* Drf = Bf + NQTL * NPTF;
  const double* Dsf = Drf + NQTL * NPTF;
  double xr = 0, xs = 0, yr = 0, ys = 0, eq = 0, er = 0, es = 0;
  for (int a = 0; a < NPTF; ++a) {
    const double x = xyt[(size_t(t) * NPTF + a) * 2], y = xyt[(size_t(t) * NPTF + a) * 2 + 1];
    const double h = eta[map2d_f[size_t(t) * NPTF + a]];
    const double br = Drf[q * NPTF + a], bs = Dsf[q * NPTF + a], bb = Bf[q * NPTF + a];
    xr += br * x; xs += bs * x; yr += br * y; ys += bs * y;
    eq += bb * h; er += br * h; es += bs * h;
  }
  const double j2 = xr * ys - xs * yr;
  const double Krx = ys / j2, Kry = -xs / j2, Ksx = -yr / j2, Ksy = xr / j2;
  const double zt = (eq + depth) / (2.0 * L);
  int badv = (j2 <= 0.0 || zt <= 0.0 || !(j2 == j2) || !(zt == zt)) ? 1 : 0;
  if (geo64 || geo32) {
    // column factors: every (layer, k) of this column shares x_r .. y_s, eta and its
    // gradient; z_t = (eta + h) / 2L is the same in every layer and
    // grad t = -s grad(eta) / z_t + e_z / z_t
    const double c0 = wq[q] * j2;
    const double ex = er * Krx + es * Ksx, ey = er * Kry + es * Ksy;
    double bq[8];
    bq[0] = c0 * zt * (Krx * Krx + Kry * Kry);
    bq[1] = c0 * zt * (Krx * Ksx + Kry * Ksy);
    bq[2] = -c0 * (Krx * ex + Kry * ey);
    bq[3] = c0 * zt * (Ksx * Ksx + Ksy * Ksy);
    bq[4] = -c0 * (Ksx * ex + Ksy * ey);
    bq[5] = c0 * (ex * ex + ey * ey) / zt;
    bq[6] = c0 / zt;
    bq[7] = 0.0;
    const size_t o = (size_t(t) * NQTL + q) * 8;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (geo64) geo64[o + m] = bq[m];
      if (geo32) geo32[o + m] = float(bq[m]);
    }
  }
  for (int layer = 0; layer < ((G64 || G32 || G16) ? L : 0); ++layer) {
    const size_t e = size_t(t) * L + layer;
    for (int k = 0; k < N1L; ++k) {
      const double sig = (layer + 0.5 * (1.0 + zq[k])) / L;
      const double zr = sig * er, zs = sig * es;
      const double Ktx = -(zr * Krx + zs * Ksx) / zt, Kty = -(zr * Kry + zs * Ksy) / zt, Ktz = 1.0 / zt;
      const double w = wq[q] * zw[k] * zt * j2;
      double g[6];
      g[0] = w * (Krx * Krx + Kry * Kry);
      g[1] = w * (Krx * Ksx + Kry * Ksy);
      g[2] = w * (Krx * Ktx + Kry * Kty);
      g[3] = w * (Ksx * Ksx + Ksy * Ksy);
      g[4] = w * (Ksx * Ktx + Ksy * Kty);
      g[5] = w * (Ktx * Ktx + Kty * Kty + Ktz * Ktz);
      const size_t base = e * 6 * NQL + size_t(k) * NQTL + q;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        if (G64) G64[base + size_t(m) * NQL] = g[m];
        if (G32) G32[base + size_t(m) * NQL] = float(g[m]);
        if (G16) G16[base + size_t(m) * NQL] = f32_to_bf16(float(g[m]));
      }
    }
  }
  if (badv) atomicOr(bad, 1);
}

void launch_geom(const LevelView& fine, const LevelView& lvl, double depth, const double* xyt,
                 const double* eta, const double* gmats, const double* wq, const double* zq,
                 const double* zw, double* G64, float* G32, bf16_t* G16, int* bad, hipStream_t st,
                 double* geo64, float* geo32) {
  const int nqtl = (lvl.P + 1) * (lvl.P + 1), n1l = lvl.PZ + 1;
  const int64_t items = int64_t(fine.nt) * nqtl;
  const int grid = int((items + 255) / 256);
#define PMG_GEOM(PFV)                                                                               \
  case PFV:                                                                                         \
    hipLaunchKernelGGL((k_geom<PFV>), dim3(grid), dim3(256), 0, st, fine.nt, fine.L, nqtl, n1l, depth, xyt, \
                       eta, fine.map2d, gmats, wq, zq, zw, G64, G32, G16, bad, geo64, geo32);       \
    break;
  switch (fine.P) {
    PMG_GEOM(1) PMG_GEOM(2) PMG_GEOM(3) PMG_GEOM(4) PMG_GEOM(5) PMG_GEOM(6) PMG_GEOM(7) PMG_GEOM(8)
    default: break;
  }
#undef PMG_GEOM
}

// ---------------------------------------------------------------------------
// diagonal of the element matrices, E-layout.  With the tensor structure
// D_r = B_z (x) Dr, D_s = B_z (x) Ds, D_t = D_z (x) B:
//   diag[c][a] = sum_k Bz[k][c]^2 S1[k][a] + 2 Bz[k][c] Dz[k][c] S2[k][a] + Dz[k][c]^2 S3[k][a]
//   S1 = sum_q G_rr Dr^2 + 2 G_rs Dr Ds + G_ss Ds^2,  S2 = sum_q (G_rt Dr + G_st Ds) B,
//   S3 = sum_q G_tt B^2   (q over the triangle points of vertical point k).
// One element per block iteration with its G staged in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag(int64_t n_elem, int L, int npt, int nqt, int n1,
                                              const double* __restrict__ mats, const double* __restrict__ G,
                                              double* __restrict__ Y) {
  extern __shared__ double dsm[];
  const int nq = nqt * n1;
  double* sG = dsm;               // [6][nq]
  double* sS = sG + 6 * nq;       // [3][n1][npt]
  const double* Dr = mats;
  const double* Ds = Dr + nqt * npt;
  const double* Bt = Ds + nqt * npt;
  const double* Bz = Bt + nqt * npt;
  const double* Dz = Bz + n1 * n1;
  for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
    __syncthreads();
    for (int i = threadIdx.x; i < 6 * nq; i += 256) sG[i] = G[size_t(e) * 6 * nq + i];
    __syncthreads();
    for (int i = threadIdx.x; i < n1 * npt; i += 256) {
      const int k = i / npt, a = i - k * npt;
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int q = 0; q < nqt; ++q) {
        const int p = k * nqt + q;
        const double dr = Dr[q * npt + a], ds = Ds[q * npt + a], b = Bt[q * npt + a];
        s1 += dr * (sG[p] * dr + 2.0 * sG[nq + p] * ds) + ds * sG[3 * nq + p] * ds;
        s2 += (sG[2 * nq + p] * dr + sG[4 * nq + p] * ds) * b;
        s3 += sG[5 * nq + p] * b * b;
      }
      sS[i] = s1;
      sS[n1 * npt + i] = s2;
      sS[2 * n1 * npt + i] = s3;
    }
    __syncthreads();
    const int t = int(e / L), layer = int(e - int64_t(t) * L);
    for (int i = threadIdx.x; i < npt * n1; i += 256) {
      const int a = i / n1, c = i - a * n1;
      double d = 0.0;
      for (int k = 0; k < n1; ++k) {
        const double bz = Bz[k * n1 + c], dz = Dz[k * n1 + c];
        d += bz * bz * sS[k * npt + a] + 2.0 * bz * dz * sS[n1 * npt + k * npt + a] +
             dz * dz * sS[2 * n1 * npt + k * npt + a];
      }
      Y[((size_t(t) * npt + a) * L + layer) * n1 + c] = d;
    }
  }
}

// Diagonal from the column factors geo[t][q][8] (see launch_geom).  The four
// triangle sums T1 = sum_q B0 Dr^2 + 2 B1 Dr Ds + B3 Ds^2, T2 = sum_q (B2 Dr + B4 Ds) B,
// T5 = sum_q B5 B^2 and T6 = sum_q B6 B^2 are shared by every layer and vertical
// point of the column, so that, with s_k the sigma of Gauss point k in layer l,
//   diag[c][a] = sum_k zw_k (Bz^2 T1 + 2 Bz Dz s_k T2 + Dz^2 (s_k^2 T5 + T6)).
// DIAG_TB triangle columns per block iteration (one thread per (column, node a)
// for the triangle sums).
constexpr int DIAG_TB = 8;
__global__ __launch_bounds__(256) void k_diag_col(int nt, int L, int npt, int nqt, int n1,
                                                  const double* __restrict__ mats, const double* __restrict__ zq,
                                                  const double* __restrict__ zw, const double* __restrict__ geo,
                                                  double* __restrict__ Y) {
  extern __shared__ double dsm[];
  double* sB = dsm;                         // [DIAG_TB][nqt][8]
  double* sT = sB + DIAG_TB * nqt * 8;      // [DIAG_TB][4][npt]
  const double* Dr = mats;
  const double* Ds = Dr + nqt * npt;
  const double* Bt = Ds + nqt * npt;
  const double* Bz = Bt + nqt * npt;
  const double* Dz = Bz + n1 * n1;
  for (int t0 = blockIdx.x * DIAG_TB; t0 < nt; t0 += gridDim.x * DIAG_TB) {
    const int nb = nt - t0 < DIAG_TB ? nt - t0 : DIAG_TB;
    __syncthreads();
    for (int i = threadIdx.x; i < nb * nqt * 8; i += 256) sB[i] = geo[size_t(t0) * nqt * 8 + i];
    __syncthreads();
    for (int i = threadIdx.x; i < nb * npt; i += 256) {
      const int tl = i / npt, a = i - tl * npt;
      double t1 = 0.0, t2 = 0.0, t5 = 0.0, t6 = 0.0;
      for (int q = 0; q < nqt; ++q) {
        const double* g = sB + (tl * nqt + q) * 8;
        const double dr = Dr[q * npt + a], ds = Ds[q * npt + a], b = Bt[q * npt + a];
        t1 += dr * (g[0] * dr + 2.0 * g[1] * ds) + ds * g[3] * ds;
        t2 += (g[2] * dr + g[4] * ds) * b;
        t5 += g[5] * b * b;
        t6 += g[6] * b * b;
      }
      double* T = sT + tl * 4 * npt;
      T[a] = t1;
      T[npt + a] = t2;
      T[2 * npt + a] = t5;
      T[3 * npt + a] = t6;
    }
    __syncthreads();
    const int per = L * npt * n1;
    for (int i = threadIdx.x; i < nb * per; i += 256) {
      const int tl = i / per, rr = i - tl * per;
      const int layer = rr / (npt * n1), r = rr - layer * npt * n1, a = r / n1, c = r - a * n1;
      const double* T = sT + tl * 4 * npt;
      double d = 0.0;
      for (int k = 0; k < n1; ++k) {
        const double s = (layer + 0.5 * (1.0 + zq[k])) / L;
        const double bz = Bz[k * n1 + c], dz = Dz[k * n1 + c];
        d += zw[k] * (bz * bz * T[a] + 2.0 * bz * dz * s * T[npt + a] + dz * dz * (s * s * T[2 * npt + a] + T[3 * npt + a]));
      }
      Y[((size_t(t0 + tl) * npt + a) * L + layer) * n1 + c] = d;
    }
  }
}

void launch_diag_col(const LevelView& lv, const double* mats, const double* zq, const double* zw, const double* geo,
                     double* Y, hipStream_t st) {
  const int npt = lv.np_tri, n1 = lv.PZ + 1, nqt = (lv.P + 1) * (lv.P + 1);
  const size_t lds = sizeof(double) * DIAG_TB * (8 * size_t(nqt) + 4 * size_t(npt));
  const int nblk = (lv.nt + DIAG_TB - 1) / DIAG_TB;
  const int grid = nblk < 65536 ? nblk : 65536;
  hipLaunchKernelGGL(k_diag_col, dim3(grid < 1 ? 1 : grid), dim3(256), lds, st, lv.nt, lv.L, npt, nqt, n1, mats, zq,
                     zw, geo, Y);
}

void launch_diag(const LevelView& lv, const double* mats, const double* G64, double* Y, hipStream_t st) {
  const int npt = lv.np_tri, n1 = lv.PZ + 1, nqt = (lv.P + 1) * (lv.P + 1);
  const size_t lds = sizeof(double) * (6 * size_t(nqt) * n1 + 3 * size_t(n1) * npt);
  const int grid = int(lv.n_elem < 65536 ? lv.n_elem : 65536);
  hipLaunchKernelGGL(k_diag, dim3(grid < 1 ? 1 : grid), dim3(256), lds, st, lv.n_elem, lv.L, npt, nqt, n1, mats,
                     G64, Y);
}

// ---------------------------------------------------------------------------
// transfers: per-element interpolation Pi = Pi_z (x) Pi_tri
// ---------------------------------------------------------------------------
// Per-element transfers between consecutive orders, NEB prisms per round.
// Loads: one thread per (prism, triangle node) pair reads the map once and
// issues the whole vertical column of the prism at once.
constexpr int XFER_NEB = 16;

template <int PFT, int PFZ, int PCT, int PCZ, typename T>
__global__ __launch_bounds__(256) void k_prolong_elem(int64_t n_elem, int L, int nzc,
                                                      const int32_t* __restrict__ map2d_c,
                                                      const T* __restrict__ pit,
                                                      const T* __restrict__ piz,
                                                      const T* __restrict__ uc, T* __restrict__ Yf) {
  constexpr int N1F = PFZ + 1, NPTF = (PFT + 1) * (PFT + 2) / 2, NPF = NPTF * N1F;
  constexpr int N1C = PCZ + 1, NPTC = (PCT + 1) * (PCT + 2) / 2, NPC = NPTC * N1C;
  constexpr int NEB = XFER_NEB;
  __shared__ T sUc[NEB * NPC];
  __shared__ T sT1[NEB * N1C * NPTF];
  __shared__ T sPt[NPTF * NPTC];
  __shared__ T sPz[N1F * N1C];
  for (int i = threadIdx.x; i < NPTF * NPTC; i += 256) sPt[i] = pit[i];
  for (int i = threadIdx.x; i < N1F * N1C; i += 256) sPz[i] = piz[i];
  for (int64_t e0 = int64_t(blockIdx.x) * NEB; e0 < n_elem; e0 += int64_t(gridDim.x) * NEB) {
    const int ne = int(n_elem - e0 < NEB ? n_elem - e0 : NEB);
    __syncthreads();
    // coarse nodal values U[el][c][a]
    for (int pr = threadIdx.x; pr < ne * NPTC; pr += 256) {
      const int el = pr / NPTC, a = pr - el * NPTC;
      const int64_t e = e0 + el;
      const int t = int(e / L), layer = int(e - int64_t(t) * L);
      const T* col = uc + int64_t(map2d_c[size_t(t) * NPTC + a]) * nzc + layer * PCZ;
      T v[N1C];
#pragma unroll
      for (int c = 0; c < N1C; ++c) v[c] = col[c];
#pragma unroll
      for (int c = 0; c < N1C; ++c) sUc[el * NPC + c * NPTC + a] = v[c];
    }
    __syncthreads();
    // triangle factor: T1[el][c][a] = sum_b Pi_tri[a][b] U[el][c][b]
    for (int i = threadIdx.x; i < ne * N1C * NPTF; i += 256) {
      const int el = i / (N1C * NPTF), r = i - el * N1C * NPTF, c = r / NPTF, a = r - c * NPTF;
      T s = 0;
#pragma unroll 4
      for (int b = 0; b < NPTC; ++b) s += sPt[a * NPTC + b] * sUc[el * NPC + c * NPTC + b];
      sT1[el * N1C * NPTF + c * NPTF + a] = s;
    }
    __syncthreads();
    // vertical factor and E-layout output: one thread per (prism, fine triangle node)
    for (int pr = threadIdx.x; pr < ne * NPTF; pr += 256) {
      const int el = pr / NPTF, a = pr - el * NPTF;
      T t1[N1C];
#pragma unroll
      for (int cc = 0; cc < N1C; ++cc) t1[cc] = sT1[el * N1C * NPTF + cc * NPTF + a];
      const int64_t e = e0 + el;
      const int t = int(e / L), layer = int(e - int64_t(t) * L);
      T* out = Yf + ((size_t(t) * NPTF + a) * L + layer) * N1F;
#pragma unroll
      for (int c = 0; c < N1F; ++c) {
        T s = 0;
#pragma unroll
        for (int cc = 0; cc < N1C; ++cc) s += sPz[c * N1C + cc] * t1[cc];
        out[c] = s;
      }
    }
  }
}

template <int PFT, int PFZ, int PCT, int PCZ, typename T>
__global__ __launch_bounds__(256) void k_restrict_elem(int64_t n_elem, int L, int nzf,
                                                       const int32_t* __restrict__ map2d_f,
                                                       const int32_t* __restrict__ inc_ptr_f,
                                                       const uint8_t* __restrict__ dir2d_f, int top_dir,
                                                       const T* __restrict__ pit,
                                                       const T* __restrict__ piz,
                                                       const T* __restrict__ rf, T* __restrict__ Yc) {
  constexpr int N1F = PFZ + 1, NPTF = (PFT + 1) * (PFT + 2) / 2, NPF = NPTF * N1F;
  constexpr int N1C = PCZ + 1, NPTC = (PCT + 1) * (PCT + 2) / 2;
  constexpr int NEB = XFER_NEB;
  __shared__ T sRf[NEB * NPF];
  __shared__ T sT1[NEB * N1F * NPTC];
  __shared__ T sPt[NPTF * NPTC];
  __shared__ T sPz[N1F * N1C];
  for (int i = threadIdx.x; i < NPTF * NPTC; i += 256) sPt[i] = pit[i];
  for (int i = threadIdx.x; i < N1F * N1C; i += 256) sPz[i] = piz[i];
  for (int64_t e0 = int64_t(blockIdx.x) * NEB; e0 < n_elem; e0 += int64_t(gridDim.x) * NEB) {
    const int ne = int(n_elem - e0 < NEB ? n_elem - e0 : NEB);
    __syncthreads();
    // fine values weighted by the inverse multiplicity (the transpose of the averaged
    // prolongation), zero at Dirichlet nodes
    for (int pr = threadIdx.x; pr < ne * NPTF; pr += 256) {
      const int el = pr / NPTF, a = pr - el * NPTF;
      const int64_t e = e0 + el;
      const int t = int(e / L), layer = int(e - int64_t(t) * L);
      const int g2 = map2d_f[size_t(t) * NPTF + a];
      const T* col = rf + int64_t(g2) * nzf + layer * PFZ;
      T v[N1F];
#pragma unroll
      for (int c = 0; c < N1F; ++c) v[c] = col[c];
      const bool dcol = dir2d_f[g2] != 0;
      const int cnt = inc_ptr_f[g2 + 1] - inc_ptr_f[g2];
      const T inv1 = T(1) / T(cnt), inv2 = T(1) / T(2 * cnt);
#pragma unroll
      for (int c = 0; c < N1F; ++c) {
        const int z = layer * PFZ + c;
        const bool dir = dcol || (top_dir && z == nzf - 1);
        const bool iface = (c == 0 && z > 0) || (c == PFZ && z < nzf - 1);
        sRf[el * NPF + c * NPTF + a] = dir ? T(0) : v[c] * (iface ? inv2 : inv1);
      }
    }
    __syncthreads();
    // triangle factor: T1[el][c][b] = sum_a Pi_tri[a][b] R[el][c][a]
    for (int i = threadIdx.x; i < ne * N1F * NPTC; i += 256) {
      const int el = i / (N1F * NPTC), r = i - el * N1F * NPTC, c = r / NPTC, b = r - c * NPTC;
      T s = 0;
#pragma unroll 4
      for (int a = 0; a < NPTF; ++a) s += sPt[a * NPTC + b] * sRf[el * NPF + c * NPTF + a];
      sT1[el * N1F * NPTC + c * NPTC + b] = s;
    }
    __syncthreads();
    // vertical factor and E-layout output: one thread per (prism, coarse triangle node)
    for (int pr = threadIdx.x; pr < ne * NPTC; pr += 256) {
      const int el = pr / NPTC, b = pr - el * NPTC;
      T t1[N1F];
#pragma unroll
      for (int c = 0; c < N1F; ++c) t1[c] = sT1[el * N1F * NPTC + c * NPTC + b];
      const int64_t e = e0 + el;
      const int t = int(e / L), layer = int(e - int64_t(t) * L);
      T* out = Yc + ((size_t(t) * NPTC + b) * L + layer) * N1C;
#pragma unroll
      for (int cc = 0; cc < N1C; ++cc) {
        T s = 0;
#pragma unroll
        for (int c = 0; c < N1F; ++c) s += sPz[c * N1C + cc] * t1[c];
        out[cc] = s;
      }
    }
  }
}


template <typename T>
void launch_prolong_elem(const LevelView& f, const LevelView& c, const T* pit, const T* piz, const T* uc,
                         T* Yf, hipStream_t st) {
  const int grid = grid_for(f.n_elem, XFER_NEB, 262144);
#define PMG_PRO(PFT, PFZ, PCT, PCZ)                                                                  \
  if (f.P == PFT && f.PZ == PFZ && c.P == PCT && c.PZ == PCZ) {                                       \
    hipLaunchKernelGGL((k_prolong_elem<PFT, PFZ, PCT, PCZ, T>), dim3(grid), dim3(256), 0, st, f.n_elem, f.L, \
                       int(c.nz), c.map2d, pit, piz, uc, Yf);                                        \
    return;                                                                                          \
  }
  PMG_PAIRS(PMG_PRO)
#undef PMG_PRO
}

// Node-wise prolongation for level pairs where one factor of the transfer is
// the identity (the in-plane-first sequence: the vertical order kept while the
// triangle order halves, then the triangle order kept).  The coarse space is
// continuous and nested in the fine one, so every element holding a fine node
// interpolates the same value there: the element average of the element-wise
// path equals the value from any one element, here the first incidence of the
// node's column (the node's triangle t and local node a) in the layer holding
// it.  One thread per (fine 2D node, layer): the incidence and the coarse map
// are read once, then the PZ+1 (PZ for layers above the first, whose bottom
// node the layer below writes) nodes of the layer are formed from independent
// loads, and the result goes straight to the nodes (OP: OP_AVG_ADD out +=
// mask v, OP_AVG_STORE out = mask v, OP_AVG_RAW out = v).  Consecutive threads
// take the layers of one column, so a wave writes runs of whole columns.
template <int PFT, int PFZ, int PCT, int PCZ, typename T, int OP>
__global__ __launch_bounds__(256) void k_prolong_node(uint32_t n_col, uint32_t nz, int L,
                                                      const int32_t* __restrict__ inc_ptr,
                                                      const int32_t* __restrict__ inc,
                                                      const uint8_t* __restrict__ dir2d, int top_dir, int nzc,
                                                      const int32_t* __restrict__ map2d_c,
                                                      const T* __restrict__ pit, const T* __restrict__ piz,
                                                      const T* __restrict__ uc, T* __restrict__ out) {
  constexpr int N1F = PFZ + 1, NPTF = (PFT + 1) * (PFT + 2) / 2;
  constexpr int N1C = PCZ + 1, NPTC = (PCT + 1) * (PCT + 2) / 2;
  static_assert(PFT == PCT || PFZ == PCZ, "one factor of the transfer is the identity");
  __shared__ T sPt[NPTF * NPTC];
  __shared__ T sPz[N1F * N1C];
  for (int i = threadIdx.x; i < NPTF * NPTC; i += 256) sPt[i] = pit[i];
  for (int i = threadIdx.x; i < N1F * N1C; i += 256) sPz[i] = piz[i];
  __syncthreads();
  for (uint64_t il = uint64_t(blockIdx.x) * 256 + threadIdx.x; il < n_col; il += uint64_t(gridDim.x) * 256) {
    const uint32_t item = uint32_t(il), n2 = item / uint32_t(L);
    const int layer = int(item - n2 * uint32_t(L));
    const uint32_t id = uint32_t(inc[inc_ptr[n2]]), t = id / NPTF, a = id - t * NPTF;
    const bool dcol = OP != OP_AVG_RAW && dir2d[n2];
    const int c0 = layer > 0 ? 1 : 0;
    T v[N1F];
    if constexpr (PFZ == PCZ) {
      // vertical factor the identity: at each level c, sum over the coarse triangle nodes
      int64_t base[NPTC];
#pragma unroll
      for (int b = 0; b < NPTC; ++b) base[b] = int64_t(map2d_c[size_t(t) * NPTC + b]) * nzc + layer * PCZ;
      T w[NPTC];
#pragma unroll
      for (int b = 0; b < NPTC; ++b) w[b] = sPt[a * NPTC + b];
#pragma unroll
      for (int c = 0; c < N1F; ++c) {
        T x[NPTC];
#pragma unroll
        for (int b = 0; b < NPTC; ++b) x[b] = uc[base[b] + c];
        T s = 0;
#pragma unroll
        for (int b = 0; b < NPTC; ++b) s += w[b] * x[b];
        v[c] = s;
      }
    } else {
      // triangle factor the identity: the coarse column of node a, vertical factor
      const T* col = uc + int64_t(map2d_c[size_t(t) * NPTC + a]) * nzc + layer * PCZ;
      T x[N1C];
#pragma unroll
      for (int cc = 0; cc < N1C; ++cc) x[cc] = col[cc];
#pragma unroll
      for (int c = 0; c < N1F; ++c) {
        T s = 0;
#pragma unroll
        for (int cc = 0; cc < N1C; ++cc) s += sPz[c * N1C + cc] * x[cc];
        v[c] = s;
      }
    }
    T* o = out + size_t(n2) * nz + layer * PFZ;
#pragma unroll
    for (int c = 0; c < N1F; ++c) {
      if (c < c0) continue;
      if constexpr (OP == OP_AVG_RAW) {
        o[c] = v[c];
      } else {
        const bool dir = dcol || (top_dir && layer == L - 1 && c == PFZ);
        if constexpr (OP == OP_AVG_ADD) {
          if (!dir) o[c] += v[c];
        } else {
          o[c] = dir ? T(0) : v[c];
        }
      }
    }
  }
}

template <typename T>
bool launch_prolong_node(const LevelView& f, const LevelView& c, const T* pit, const T* piz, const T* uc, T* out,
                         int op, hipStream_t st) {
  if (!(f.P == c.P || f.PZ == c.PZ)) return false;
  const int64_t n_col = f.n2d * f.L;
  const int grid = grid_for(n_col);
#define PMG_PRN(PFT, PFZ, PCT, PCZ)                                                                           \
  if constexpr (PFT == PCT || PFZ == PCZ) {                                                                    \
    if (f.P == PFT && f.PZ == PFZ && c.P == PCT && c.PZ == PCZ) {                                              \
      if (op == OP_AVG_ADD)                                                                                    \
        hipLaunchKernelGGL((k_prolong_node<PFT, PFZ, PCT, PCZ, T, OP_AVG_ADD>), dim3(grid), dim3(256), 0, st,  \
                           uint32_t(n_col), uint32_t(f.nz), f.L, f.inc_ptr, f.inc, f.dir2d, f.top_dir,       \
                           int(c.nz), c.map2d, pit, piz, uc, out);                                             \
      else if (op == OP_AVG_STORE)                                                                             \
        hipLaunchKernelGGL((k_prolong_node<PFT, PFZ, PCT, PCZ, T, OP_AVG_STORE>), dim3(grid), dim3(256), 0,    \
                           st, uint32_t(n_col), uint32_t(f.nz), f.L, f.inc_ptr, f.inc, f.dir2d, f.top_dir,   \
                           int(c.nz), c.map2d, pit, piz, uc, out);                                             \
      else if (op == OP_AVG_RAW)                                                                               \
        hipLaunchKernelGGL((k_prolong_node<PFT, PFZ, PCT, PCZ, T, OP_AVG_RAW>), dim3(grid), dim3(256), 0, st,  \
                           uint32_t(n_col), uint32_t(f.nz), f.L, f.inc_ptr, f.inc, f.dir2d, f.top_dir,       \
                           int(c.nz), c.map2d, pit, piz, uc, out);                                             \
      else                                                                                                     \
        return false;                                                                                          \
      return true;                                                                                             \
    }                                                                                                          \
  }
  PMG_PAIRS(PMG_PRN)
#undef PMG_PRN
  return false;
}
template bool launch_prolong_node<double>(const LevelView&, const LevelView&, const double*, const double*,
                                          const double*, double*, int, hipStream_t);
template bool launch_prolong_node<float>(const LevelView&, const LevelView&, const float*, const float*,
                                         const float*, float*, int, hipStream_t);

template <typename T>
void launch_restrict_elem(const LevelView& f, const LevelView& c, const T* pit, const T* piz, const T* rf,
                          T* Yc, hipStream_t st) {
  const int grid = grid_for(f.n_elem, XFER_NEB, 262144);
#define PMG_RES(PFT, PFZ, PCT, PCZ)                                                                  \
  if (f.P == PFT && f.PZ == PFZ && c.P == PCT && c.PZ == PCZ) {                                       \
    hipLaunchKernelGGL((k_restrict_elem<PFT, PFZ, PCT, PCZ, T>), dim3(grid), dim3(256), 0, st, f.n_elem, f.L, \
                       int(f.nz), f.map2d, f.inc_ptr, f.dir2d, f.top_dir, pit, piz, rf, Yc);        \
    return;                                                                                          \
  }
  PMG_PAIRS(PMG_RES)
#undef PMG_RES
}
template void launch_prolong_elem<double>(const LevelView&, const LevelView&, const double*, const double*, const double*, double*, hipStream_t);
template void launch_prolong_elem<float>(const LevelView&, const LevelView&, const float*, const float*, const float*, float*, hipStream_t);
template void launch_restrict_elem<double>(const LevelView&, const LevelView&, const double*, const double*, const double*, double*, hipStream_t);
template void launch_restrict_elem<float>(const LevelView&, const LevelView&, const float*, const float*, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// coarse exact solve (dense inverse on the free coarse nodes)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gather_idx(int n, const int32_t* __restrict__ idx, const T* __restrict__ x, T* __restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[idx[i]];
}
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_rows(int n, const int32_t* __restrict__ idx,
                                                   const T* __restrict__ A, const T* __restrict__ x,
                                                   T* __restrict__ y) {
  // one wave per row, deterministic lane-strided sum then butterfly
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const T* a = A + size_t(row) * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += double(a[j]) * double(x[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) y[idx[row]] = T(s);
}

template <typename T>
void launch_coarse_dense(int n, const int32_t* idx, const T* Ainv, const T* x, T* y, T* tmp, int64_t n_dof,
                         hipStream_t st) {
  launch_fill<T>(y, T(0), n_dof, st);
  hipLaunchKernelGGL((k_gather_idx<T>), dim3((n + 255) / 256), dim3(256), 0, st, n, idx, x, tmp);
  hipLaunchKernelGGL((k_gemv_rows<T>), dim3((n + 3) / 4), dim3(256), 0, st, n, idx, Ainv, tmp, y);
}
template void launch_coarse_dense<double>(int, const int32_t*, const double*, const double*, double*, double*, int64_t, hipStream_t);
template void launch_coarse_dense<float>(int, const int32_t*, const float*, const float*, float*, float*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// vector kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* x, T v, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) x[i] = v;
}
template <typename T> void launch_fill(T* x, T v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(256), 0, st, x, v, n);
}
template <typename T>
__global__ void k_copy(const T* __restrict__ x, T* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) y[i] = x[i];
}
template <typename T> void launch_copy(const T* x, T* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
}
template <typename T>
__global__ void k_scale_diag(const T* __restrict__ d, const T* __restrict__ x, T* __restrict__ y, T w, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) y[i] = w * d[i] * x[i];
}
template <typename T>
void launch_scale_diag(const T* d, const T* x, T* y, double omega, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_diag<T>), dim3(grid_for(n)), dim3(256), 0, st, d, x, y, T(omega), n);
}
template <typename Ts, typename Td>
__global__ void k_cast(const Ts* __restrict__ x, Td* __restrict__ y, double s, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    y[i] = Td(double(x[i]) * s);
}
template <typename Ts, typename Td>
void launch_cast(const Ts* x, Td* y, double scale, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_cast<Ts, Td>), dim3(grid_for(n)), dim3(256), 0, st, x, y, scale, n);
}
template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
                                             double* __restrict__ partial) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    acc += double(x[i]) * double(y[i]);
  const double b = block_sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}
template <typename T>
void launch_dot(const T* x, const T* y, int64_t n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((k_dot<T>), dim3(RED_BLOCKS), dim3(256), 0, st, x, y, n, partial);
}
template <typename T>
__global__ void k_dinv(int64_t n, int nz, const uint8_t* __restrict__ dir2d, int top_dir,
                       const double* __restrict__ diag, T* __restrict__ dinv) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n; g += int64_t(gridDim.x) * 256) {
    const int64_t g2 = g / nz;
    const int z = int(g - g2 * nz);
    const bool dir = dir2d[g2] || (top_dir && z == nz - 1);
    dinv[g] = dir ? T(0) : T(1.0 / diag[g]);
  }
}
template <typename T>
void launch_dinv(const LevelView& lv, const T*, const double* diag, T* dinv, hipStream_t st) {
  hipLaunchKernelGGL((k_dinv<T>), dim3(grid_for(lv.n_dof)), dim3(256), 0, st, lv.n_dof, int(lv.nz), lv.dir2d,
                     lv.top_dir, diag, dinv);
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partial, double* __restrict__ scal,
                                                  int slot, int op) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) a += partial[i];
  if (op == FIN_BETA_PR)
    for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) b += partial[RED_BLOCKS + i];
  const double sa = block_sum256(a);
  const double sb = block_sum256(b);
  if (threadIdx.x == 0) {
    if (op == FIN_SET) {
      scal[slot] = sa;
    } else if (op == FIN_ALPHA) {
      scal[S_PQ] = sa;
      scal[S_ALPHA] = scal[S_DELTA] / sa;
    } else if (op == FIN_BETA_FR) {
      scal[S_ZR] = sa;
      scal[S_BETA] = sa / scal[S_DELTA];
      scal[S_DELTA] = sa;
    } else if (op == FIN_BETA_PR) {
      // Polak-Ribiere: z.(r_new - r_old) = -alpha z.q, since r_new = r_old - alpha q
      scal[S_ZR] = sa;
      scal[S_BETA] = -scal[S_ALPHA] * sb / scal[S_DELTA];
      scal[S_DELTA] = sa;
    } else if (op == FIN_DELTA) {
      scal[S_DELTA] = sa;
      scal[S_ZR] = sa;
    }
  }
}
void launch_finalize(const double* partial, double* scal, int slot, int op, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partial, scal, slot, op);
}

__global__ __launch_bounds__(256) void k_cg_update(double* __restrict__ u, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   const double* __restrict__ scal, double* __restrict__ partial,
                                                   int64_t n, float* __restrict__ r32) {
  const double alpha = scal[S_ALPHA];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    u[i] += alpha * p[i];
    const double rn = r[i] - alpha * q[i];
    r[i] = rn;
    if (r32) r32[i] = float(rn);
    acc += rn * rn;
  }
  const double b = block_sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}
void launch_cg_update(double* u, double* r, const double* p, const double* q, const double* scal,
                      double* partial, int64_t n, hipStream_t st, float* r32) {
  hipLaunchKernelGGL(k_cg_update, dim3(RED_BLOCKS), dim3(256), 0, st, u, r, p, q, scal, partial, n, r32);
}
template <typename TZ>
__global__ void k_cg_dir(double* __restrict__ p, const TZ* __restrict__ z, const double* __restrict__ scal,
                         int64_t n) {
  const double beta = scal[S_BETA];
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    p[i] = double(z[i]) + beta * p[i];
}
void launch_cg_dir(double* p, const double* z, const double* scal, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_dir<double>, dim3(grid_for(n)), dim3(256), 0, st, p, z, scal, n);
}
void launch_cg_dir(double* p, const float* z, const double* scal, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_dir<float>, dim3(grid_for(n)), dim3(256), 0, st, p, z, scal, n);
}
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) y[i] += a * x[i];
}
void launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, st, y, x, a, n);
}
__global__ __launch_bounds__(256) void k_resid_norm(double* __restrict__ r, const double* __restrict__ f,
                                                    const double* __restrict__ y, double* __restrict__ partial,
                                                    int64_t n) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double v = f[i] - y[i];
    r[i] = v;
    acc += v * v;
  }
  const double b = block_sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}
void launch_resid_norm(double* r, const double* f, const double* y, double* partial, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_resid_norm, dim3(RED_BLOCKS), dim3(256), 0, st, r, f, y, partial, n);
}
__global__ void k_lift(int64_t n, int nz, const uint8_t* __restrict__ dir2d, int top_dir,
                       const double* __restrict__ surf, const double* __restrict__ bc, double* __restrict__ out) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n; g += int64_t(gridDim.x) * 256) {
    const int64_t g2 = g / nz;
    const int z = int(g - g2 * nz);
    const bool top = top_dir && z == nz - 1;
    const bool dir = dir2d[g2] || top;
    double v = 0.0;
    if (dir) v = bc ? bc[g] : (top && surf ? surf[g2] : 0.0);
    out[g] = v;
  }
}
void launch_lift(const LevelView& lv, const double* surf, const double* bc, double* phiD, hipStream_t st) {
  hipLaunchKernelGGL(k_lift, dim3(grid_for(lv.n_dof)), dim3(256), 0, st, lv.n_dof, int(lv.nz), lv.dir2d,
                     lv.top_dir, surf, bc, phiD);
}
__global__ void k_merge_free(int64_t n, int nz, const uint8_t* __restrict__ dir2d, int top_dir,
                             const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n; g += int64_t(gridDim.x) * 256) {
    const int64_t g2 = g / nz;
    const int z = int(g - g2 * nz);
    const bool dir = dir2d[g2] || (top_dir && z == nz - 1);
    out[g] = dir ? (b ? b[g] : 0.0) : a[g];
  }
}
void launch_merge_free(const LevelView& lv, const double* a, const double* b, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_merge_free, dim3(grid_for(lv.n_dof)), dim3(256), 0, st, lv.n_dof, int(lv.nz), lv.dir2d,
                     lv.top_dir, a, b, out);
}
__global__ __launch_bounds__(256) void k_nonfinite(const double* __restrict__ x, int64_t n, double* __restrict__ partial) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    acc += isfinite(x[i]) ? 0.0 : 1.0;
  const double b = block_sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}
void launch_count_nonfinite(const double* x, int64_t n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_nonfinite, dim3(RED_BLOCKS), dim3(256), 0, st, x, n, partial);
}

template void launch_fill<double>(double*, double, int64_t, hipStream_t);
template void launch_fill<float>(float*, float, int64_t, hipStream_t);
template void launch_copy<double>(const double*, double*, int64_t, hipStream_t);
template void launch_copy<float>(const float*, float*, int64_t, hipStream_t);
template void launch_scale_diag<double>(const double*, const double*, double*, double, int64_t, hipStream_t);
template void launch_scale_diag<float>(const float*, const float*, float*, double, int64_t, hipStream_t);
template void launch_cast<double, float>(const double*, float*, double, int64_t, hipStream_t);
template void launch_cast<float, double>(const float*, double*, double, int64_t, hipStream_t);
template void launch_cast<double, double>(const double*, double*, double, int64_t, hipStream_t);
template void launch_dot<double>(const double*, const double*, int64_t, double*, hipStream_t);
template void launch_dot<float>(const float*, const float*, int64_t, double*, hipStream_t);
template void launch_dinv<double>(const LevelView&, const double*, const double*, double*, hipStream_t);
template void launch_dinv<float>(const LevelView&, const float*, const double*, float*, hipStream_t);

}  // namespace pmg

namespace pmg {
template <typename TX>
__global__ __launch_bounds__(256) void k_dot2(const TX* __restrict__ x, const double* __restrict__ y1,
                                              const double* __restrict__ y2, int64_t n,
                                              double* __restrict__ partial) {
  double a = 0.0, b = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double xi = double(x[i]);
    a += xi * y1[i];
    b += xi * y2[i];
  }
  const double sa = block_sum256(a);
  const double sb = block_sum256(b);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = sa;
    partial[RED_BLOCKS + blockIdx.x] = sb;
  }
}
void launch_dot2(const double* x, const double* y1, const double* y2, int64_t n, double* partial,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_dot2<double>, dim3(RED_BLOCKS), dim3(256), 0, st, x, y1, y2, n, partial);
}
void launch_dot2(const float* x, const double* y1, const double* y2, int64_t n, double* partial,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_dot2<float>, dim3(RED_BLOCKS), dim3(256), 0, st, x, y1, y2, n, partial);
}
}  // namespace pmg

namespace pmg {
template <typename T>
__global__ void k_mask(int64_t n, int nz, const uint8_t* __restrict__ dir2d, int top_dir, const T* __restrict__ x,
                       T* __restrict__ out) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n; g += int64_t(gridDim.x) * 256) {
    const int64_t g2 = g / nz;
    const int z = int(g - g2 * nz);
    const bool dir = dir2d[g2] || (top_dir && z == nz - 1);
    out[g] = dir ? T(0) : x[g];
  }
}
template <typename T>
void launch_mask(const LevelView& lv, const T* x, T* out, hipStream_t st) {
  hipLaunchKernelGGL((k_mask<T>), dim3(grid_for(lv.n_dof)), dim3(256), 0, st, lv.n_dof, int(lv.nz), lv.dir2d,
                     lv.top_dir, x, out);
}
template void launch_mask<double>(const LevelView&, const double*, double*, hipStream_t);
template void launch_mask<float>(const LevelView&, const float*, float*, hipStream_t);
}  // namespace pmg

namespace pmg {
__global__ void k_xpay(double* __restrict__ p, const double* __restrict__ z, double beta, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    p[i] = z[i] + beta * p[i];
}
void launch_xpay(double* p, const double* z, double beta, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_xpay, dim3(grid_for(n)), dim3(256), 0, st, p, z, beta, n);
}
}  // namespace pmg

namespace pmg {
template <typename T>
__global__ void k_axpy_t(T* __restrict__ y, const T* __restrict__ x, T a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) y[i] += a * x[i];
}
template <typename T> void launch_axpy_t(T* y, const T* x, double a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_axpy_t<T>), dim3(grid_for(n)), dim3(256), 0, st, y, x, T(a), n);
}
template void launch_axpy_t<double>(double*, const double*, double, int64_t, hipStream_t);
template void launch_axpy_t<float>(float*, const float*, double, int64_t, hipStream_t);
}  // namespace pmg

// ---------------------------------------------------------------------------
// assembled P = 1 operator (coarse Chebyshev solve): element matrices, CSR
// values by an ordered per-entry sum, and the fused Chebyshev step
// ---------------------------------------------------------------------------
namespace pmg {

// Ae[e][i*6+j] = sum_q sum_ab G_ab[q] D_a[q][i] D_b[q][j]; G standard layout
// [e][6][8] (rr, rs, rt, ss, st, tt), Dref[a][q][n] the reference derivatives
__global__ __launch_bounds__(256) void k_p1_elem_mat(int64_t n_elem, const double* __restrict__ G,
                                                     const double* __restrict__ Dref, double* __restrict__ Ae) {
  constexpr int NQ = 8, NPE = 6;
  const int comp[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  for (int64_t id = int64_t(blockIdx.x) * 256 + threadIdx.x; id < n_elem * 36; id += int64_t(gridDim.x) * 256) {
    const int64_t e = id / 36;
    const int ij = int(id - e * 36), i = ij / NPE, j = ij - i * NPE;
    const double* Ge = G + e * 6 * NQ;
    double s = 0.0;
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double da = Dref[(a * NQ + q) * NPE + i];
#pragma unroll
        for (int b = 0; b < 3; ++b) s += Ge[comp[a][b] * NQ + q] * da * Dref[(b * NQ + q) * NPE + j];
      }
    Ae[id] = s;
  }
}
void launch_p1_elem_mat(int64_t n_elem, const double* G, const double* Dref, double* Ae, hipStream_t st) {
  hipLaunchKernelGGL(k_p1_elem_mat, dim3(grid_for(n_elem * 36)), dim3(256), 0, st, n_elem, G, Dref, Ae);
}

// val[k] = sum of the element-matrix entries listed for entry k, in list order
// ELL slot (k, g) holds the k-th nonzero of row g (CSR position rp[g] + k), the
// sum of its element entries in ascending order; slots past the row's end hold 0.
__global__ __launch_bounds__(256) void k_ell_sum(int64_t n, int w, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ cp, const int64_t* __restrict__ cl,
                                                 const double* __restrict__ Ae, double* __restrict__ v64,
                                                 float* __restrict__ v32) {
  const int64_t total = n * w;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < total; i += int64_t(gridDim.x) * 256) {
    const int64_t k = i / n, g = i - k * n;
    const int64_t j = rp[g] + k;
    double s = 0.0;
    if (j < rp[g + 1])
      for (int m = cp[j]; m < cp[j + 1]; ++m) s += Ae[cl[m]];
    v64[i] = s;
    v32[i] = float(s);
  }
}
void launch_ell_sum(int64_t n, int w, const int32_t* rp, const int32_t* cp, const int64_t* cl, const double* Ae,
                    double* v64, float* v32, hipStream_t st) {
  hipLaunchKernelGGL(k_ell_sum, dim3(grid_for(n * w)), dim3(256), 0, st, n, w, rp, cp, cl, Ae, v64, v32);
}

// Chebyshev start from x = 0: r = f, d = D^-1 f / theta, x = d
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_start(int64_t n, const T* __restrict__ f, const T* __restrict__ dinv,
                                                    T* __restrict__ r, T* __restrict__ d, T* __restrict__ x,
                                                    T inv_theta) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n; g += int64_t(gridDim.x) * 256) {
    const T fv = f[g];
    const T dv = inv_theta * dinv[g] * fv;
    r[g] = fv;
    d[g] = dv;
    x[g] = dv;
  }
}
// One Chebyshev step on the assembled free-node matrix in ELL layout (slot
// (k, g) at k n + g, so a wave reads each slot column with unit stride; padding
// slots have column g and value 0; a Dirichlet row has column -1 in slot 0):
// r -= A d_old; d_new = c0 d_old + c1 D^-1 r; x += d_new.
// d is double-buffered because every row reads its neighbours' d_old.
// ELL_LANES lanes share a row (slots k = part, part + ELL_LANES, ...), their
// partial sums joined by shuffles: four times the waves of one lane per row for
// the same rows, which the 83k-row coarse problem needs to hide its latency.
constexpr int ELL_LANES = 4;
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_ell(int64_t n, int w, const int32_t* __restrict__ ci,
                                                  const T* __restrict__ val, const T* __restrict__ dinv,
                                                  const T* __restrict__ d_old, T* __restrict__ d_new,
                                                  T* __restrict__ r, T* __restrict__ x, T c0, T c1) {
  const int part = threadIdx.x % ELL_LANES;
  const int64_t rows_per_grid = int64_t(gridDim.x) * (256 / ELL_LANES);
  // every lane of a row group runs the same trip count (the shuffles need all of them)
  for (int64_t g0 = int64_t(blockIdx.x) * (256 / ELL_LANES); g0 < n; g0 += rows_per_grid) {
    const int64_t g = g0 + threadIdx.x / ELL_LANES;
    const bool row = g < n;
    const bool dir = row && ci[g] < 0;
    T s = 0;
    if (row && !dir)
      for (int k = part; k < w; k += ELL_LANES) {
        const int64_t j = int64_t(k) * n + g;
        s += val[j] * d_old[ci[j]];
      }
#pragma unroll
    for (int o = 1; o < ELL_LANES; o <<= 1) s += __shfl_xor(s, o, ELL_LANES);
    if (!row || part != 0) continue;
    if (dir) {
      d_new[g] = T(0);
      continue;
    }
    const T rn = r[g] - s;
    r[g] = rn;
    const T dn = c0 * d_old[g] + c1 * dinv[g] * rn;
    d_new[g] = dn;
    x[g] += dn;
  }
}
template <typename T>
void launch_cheb_start(int64_t n, const T* f, const T* dinv, T* r, T* d, T* x, double inv_theta, hipStream_t st) {
  hipLaunchKernelGGL((k_cheb_start<T>), dim3(grid_for(n)), dim3(256), 0, st, n, f, dinv, r, d, x, T(inv_theta));
}
template <typename T>
void launch_cheb_ell(int64_t n, int w, const int32_t* ci, const T* val, const T* dinv, const T* d_old, T* d_new,
                     T* r, T* x, double c0, double c1, hipStream_t st) {
  hipLaunchKernelGGL((k_cheb_ell<T>), dim3(grid_for(n * ELL_LANES)), dim3(256), 0, st, n, w, ci, val, dinv, d_old,
                     d_new, r, x, T(c0), T(c1));
}
template void launch_cheb_start<double>(int64_t, const double*, const double*, double*, double*, double*, double, hipStream_t);
template void launch_cheb_start<float>(int64_t, const float*, const float*, float*, float*, float*, double, hipStream_t);
template void launch_cheb_ell<double>(int64_t, int, const int32_t*, const double*, const double*, const double*, double*, double*, double*, double, double, hipStream_t);
template void launch_cheb_ell<float>(int64_t, int, const int32_t*, const float*, const float*, const float*, float*, float*, float*, double, double, hipStream_t);

}  // namespace pmg
