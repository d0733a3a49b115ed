// MFMA element operator for the fine levels (gfx950).
//
// y_e = sum_{a,b in r,s,t} D_a^T diag(G_ab) D_b u_e for 16 prisms per wave:
// the 16 prisms are the 16 columns of every MFMA tile.
//   1. vertical (VALU): W[k][a] = sum_c Bz[k][c] u[c][a],  Wz with Dz
//   2. triangle (MFMA): [ur|us|ut][q] = [Dr|Ds|B][q][a] x [W|W|Wz][a]
//      (A operand = reference matrix tile from LDS, B operand = W in registers)
//   3. pointwise (VALU): (vr, vs, vt) = G (ur, us, ut), G formed in registers
//      from the column factors of the prism's triangle (the sigma-transform
//      shares them along the column; see launch_geom) or streamed from a stored
//      lane-native copy (no padding); the result stays in the MFMA registers
//   4. transposed triangle (MFMA): Yr[a] = sum_q Dr[q][a] vr[q] + Ds[q][a] vs[q],
//      Yt[a] = sum_q B[q][a] vt[q]; the K index of each step is chosen so that
//      the B operand is exactly the register the pointwise stage produced
//   5. vertical transpose (VALU): y[c][a] += Bz[k][c] Yr[k][a] + Dz[k][c] Yt[k][a]
// Output is the E-layout vector [t][a][layer][c] consumed by the atomic-free
// node-centric summation kernel.
//
// Flavours: FP32 (v_mfma_f32_16x16x4f32), FP64 (v_mfma_f64_16x16x4f64), BF16
// operands with FP32 accumulation (v_mfma_f32_16x16x16bf16_1k), and split-BF16
// products on the same BF16 instruction.  Output registers: FP32/BF16 hold
// D[4g+r][j], FP64 holds D[g+4r][j] (g = lane/16, j = lane%16, r = 0..3; see
// row_of).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "epilogue.hpp"
#include "kernels.hpp"
#include "kernels_mfma.hpp"

namespace pmg {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

// PT: triangle order, PZ: vertical order; N1 = PZ + 1 vertical nodes, Gauss points and waves
template <int PT, int PZ> struct MD {
  static constexpr int N1 = PZ + 1, NPT = (PT + 1) * (PT + 2) / 2, NQT = (PT + 1) * (PT + 1), NQ = NQT * N1;
  static constexpr int NT2 = (NQT + 15) / 16;        // q tiles of 16
  static constexpr int NTF = NQT / 16;               // full q tiles
  static constexpr int NQR = NQT - 16 * NTF;         // rows of the remainder tile
  static constexpr int KS = (NPT + 3) / 4;           // K=4 steps over a
  static constexpr int KS16 = (NPT + 15) / 16;       // K=16 steps over a
  static constexpr int NAT = (NPT + 15) / 16;        // a tiles
};

template <bool F64ROW> __device__ __forceinline__ constexpr int row_of(int g, int r) {
  return F64ROW ? g + 4 * r : 4 * g + r;
}
template <int PT, int PZ, bool F64ROW> constexpr int n_steps4() {
  int n = 0;
  for (int t = 0; t < MD<PT, PZ>::NT2; ++t)
    for (int r = 0; r < 4; ++r)
      if (16 * t + (F64ROW ? 4 * r : r) < MD<PT, PZ>::NQT) ++n;
  return n;
}

__device__ __forceinline__ f4_t mfma4(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4_t mfma4(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(s4_t a, s4_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ short f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return short(u >> 16);
}
// Packed rounding to BF16 (nearest even) on the gfx950 conversion unit: one
// v_cvt_pk_bf16_f32 per pair, low half = first value.  Same result as f2bf for
// every finite input; used where the rounding sits in the kernels' inner loops.
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef float fv2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf2(float x0, float x1) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(fv2_t{x0, x1}, bf2_t));
}
__device__ __forceinline__ s4_t bf4(const float (&x)[4]) {
  return __builtin_bit_cast(s4_t, u2_t{bf2(x[0], x[1]), bf2(x[2], x[3])});
}
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi), four values at once
__device__ __forceinline__ void split4(const float (&x)[4], s4_t& hi, s4_t& lo) {
  const uint32_t h01 = bf2(x[0], x[1]), h23 = bf2(x[2], x[3]);
  const float d[4] = {x[0] - __uint_as_float(h01 << 16), x[1] - __uint_as_float(h01 & 0xFFFF0000u),
                      x[2] - __uint_as_float(h23 << 16), x[3] - __uint_as_float(h23 & 0xFFFF0000u)};
  hi = __builtin_bit_cast(s4_t, u2_t{h01, h23});
  lo = bf4(d);
}
template <typename TG> __device__ __forceinline__ float gld(const TG* p, size_t i);
template <> __device__ __forceinline__ float gld<float>(const float* p, size_t i) { return p[i]; }
template <> __device__ __forceinline__ float gld<bf16_t>(const bf16_t* p, size_t i) {
  return __uint_as_float(uint32_t(p[i]) << 16);
}

// XCD-aware block order: consecutive logical blocks land on one XCD (its L2
// then holds the shared nodes of neighbouring prisms).
__device__ __forceinline__ int64_t xcd_block(int nblk) {
  const int b = blockIdx.x;
  const int per = nblk / 8;
  if (per * 8 != nblk) return b;
  return int64_t(b % 8) * per + b / 8;
}

// offset of G for (batch, k, m, lane, r) in the lane-native layout; -1 if q >= NQT
template <int PT, int PZ, bool F64ROW>
__device__ __forceinline__ int64_t gnat_off(int64_t b, int k, int m, int t, int g, int j, int r) {
  using D = MD<PT, PZ>;
  const int64_t blk = ((b * D::N1 + k) * 6 + m) * (16 * D::NQT);
  if (t < D::NTF) return blk + t * 256 + (g * 16 + j) * 4 + r;
  const int row = row_of<F64ROW>(g, r);
  if (row >= D::NQR) return -1;
  return blk + D::NTF * 256 + row * 16 + j;
}

// ---------------------------------------------------------------------------
// Workgroup = N1 waves on one batch of 16 prisms; wave k owns vertical Gauss
// level k.  Phase 0 stages u in LDS; phase 1 (per wave) runs stages 1-4 for
// its k; phase 2 (all threads) does the vertical transpose sum over k from
// LDS and writes the E-layout output with runs of L*(PZ+1) contiguous values.
// ---------------------------------------------------------------------------
template <int PT, int PZ> struct KS_LDS {
  using D = MD<PT, PZ>;
  static constexpr int U_WORDS = D::N1 * D::NPT * 16;           // U[c][a][el]
  static constexpr int S_WORDS = D::N1 * 2 * D::NAT * 16 * 16;  // S[k][h][a][el]
  static constexpr int R_WORDS = U_WORDS > S_WORDS ? U_WORDS : S_WORDS;
};

// (triangle, layer) of prism e = 16 b + j of a batch; te = -1 past the last
// prism.  Every thread with lane % 16 == j stages and writes this slot (the
// workgroup is a multiple of 16 threads), so one 32-bit division per batch
// serves stage_u, geo_lane and vertical_out (pmg_create rejects meshes of
// 2^31 or more prisms).
struct ColSlot {
  int te, layer;
};
__device__ __forceinline__ ColSlot col_slot(int64_t b, int j, int64_t n_elem, int L) {
  const int64_t e = b * 16 + j;
  if (e >= n_elem) return ColSlot{-1, 0};
  const uint32_t eu = uint32_t(e), te = eu / uint32_t(L);
  return ColSlot{int(te), int(eu - te * uint32_t(L))};
}

// Stage the 16 prisms' nodal values: U[c][a][el] = u[map2d[t][a] nz + layer PZ + c].
// One thread per (a, el) pair: one map read, then the PZ+1 vertical values of
// the column issued together (independent loads, a single wait).  cs: the
// thread's column slot (el = lane % 16).
template <int PT, int PZ, typename T>
__device__ __forceinline__ void stage_u(const int32_t* __restrict__ map2d, int nz, ColSlot cs,
                                        const T* __restrict__ u, T* __restrict__ sR) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NTH = 64 * N1;
  static_assert(NTH % 16 == 0, "pr & 15 must be the lane's slot");
  for (int pr = threadIdx.x; pr < 16 * NPT; pr += NTH) {
    const int a = pr >> 4, el = pr & 15;
    T v[N1];
    if (cs.te >= 0) {
      const T* col = u + int64_t(map2d[size_t(cs.te) * NPT + a]) * nz + cs.layer * PZ;
#pragma unroll
      for (int c = 0; c < N1; ++c) v[c] = col[c];
    } else {
#pragma unroll
      for (int c = 0; c < N1; ++c) v[c] = T(0);
    }
#pragma unroll
    for (int c = 0; c < N1; ++c) sR[(c * NPT + a) * 16 + el] = v[c];
  }
}
// Per-use form for the BF16 and split-BF16 kernels: the slot is derived where it
// is used, so it is not held across the batch (at their 128-VGPR cap that costs
// more than the repeated division: 189 -> 208 us for the split kernel on the
// 131,072-prism box at P = 6).
template <int PT, int PZ, typename T>
__device__ __forceinline__ void stage_u(const int32_t* __restrict__ map2d, int L, int nz, int64_t n_elem,
                                        int64_t b, const T* __restrict__ u, T* __restrict__ sR) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NTH = 64 * N1;
  for (int pr = threadIdx.x; pr < 16 * NPT; pr += NTH) {
    const int a = pr >> 4, el = pr & 15;
    const int64_t e = b * 16 + el;
    T v[N1];
    if (e < n_elem) {
      const uint32_t eu = uint32_t(e), tu = eu / uint32_t(L);  // e < 2^31 (pmg_create)
      const int te = int(tu), layer = int(eu - tu * uint32_t(L));
      const T* col = u + int64_t(map2d[size_t(te) * NPT + a]) * nz + layer * PZ;
#pragma unroll
      for (int c = 0; c < N1; ++c) v[c] = col[c];
    } else {
#pragma unroll
      for (int c = 0; c < N1; ++c) v[c] = T(0);
    }
#pragma unroll
    for (int c = 0; c < N1; ++c) sR[(c * NPT + a) * 16 + el] = v[c];
  }
}

// Vertical transpose and output: y[c][a] of prism el = sum_k Bz[k][c] Yr[k][a] +
// Dz[k][c] Yt[k][a], with S[k][h][a][el] in LDS.  One thread per (a, el) pair
// reads its 2(PZ+1) partials once and writes the PZ+1 contiguous outputs of its
// column slot in the E-layout [t][a][layer][c].
template <int PT, int PZ, typename T>
__device__ __forceinline__ void vertical_out(int L, ColSlot cs, const T* __restrict__ sR,
                                             const T* __restrict__ sV, T* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NAT = D::NAT, NTH = 64 * N1;
  if (cs.te < 0) return;
  for (int pr = threadIdx.x; pr < 16 * NPT; pr += NTH) {
    const int a = pr >> 4, el = pr & 15;
    T yr[N1], yt[N1];
#pragma unroll
    for (int kk = 0; kk < N1; ++kk) {
      yr[kk] = sR[((kk * 2 + 0) * NAT * 16 + a) * 16 + el];
      yt[kk] = sR[((kk * 2 + 1) * NAT * 16 + a) * 16 + el];
    }
    T* out = Y + ((size_t(cs.te) * NPT + a) * L + cs.layer) * N1;
    // rolled: the coefficients are LDS broadcasts read per c, not 2(PZ+1)^2 registers
#pragma unroll 1
    for (int c = 0; c < N1; ++c) {
      T y = 0;
#pragma unroll
      for (int kk = 0; kk < N1; ++kk) y += sV[kk * N1 + c] * yr[kk] + sV[N1 * N1 + kk * N1 + c] * yt[kk];
      out[c] = y;
    }
  }
}
template <int PT, int PZ, typename T>
__device__ __forceinline__ void vertical_out(int L, int64_t n_elem, int64_t b, const T* __restrict__ sR,
                                             const T* __restrict__ sV, T* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NAT = D::NAT, NTH = 64 * N1;
  for (int pr = threadIdx.x; pr < 16 * NPT; pr += NTH) {
    const int a = pr >> 4, el = pr & 15;
    const int64_t e = b * 16 + el;
    if (e >= n_elem) continue;
    T yr[N1], yt[N1];
#pragma unroll
    for (int kk = 0; kk < N1; ++kk) {
      yr[kk] = sR[((kk * 2 + 0) * NAT * 16 + a) * 16 + el];
      yt[kk] = sR[((kk * 2 + 1) * NAT * 16 + a) * 16 + el];
    }
    const uint32_t eu = uint32_t(e), tu = eu / uint32_t(L);  // e < 2^31 (pmg_create)
    const int te = int(tu), layer = int(eu - tu * uint32_t(L));
    T* out = Y + ((size_t(te) * NPT + a) * L + layer) * N1;
    // rolled: the coefficients are LDS broadcasts read per c, not 2(PZ+1)^2 registers
#pragma unroll 1
    for (int c = 0; c < N1; ++c) {
      T y = 0;
#pragma unroll
      for (int kk = 0; kk < N1; ++kk) y += sV[kk * N1 + c] * yr[kk] + sV[N1 * N1 + kk * N1 + c] * yt[kk];
      out[c] = y;
    }
  }
}

// vertical_out on the FP32 matrix cores: for node a (wave k takes a = k,
// k + N1, ...) D[c][el] = sum_kappa C[c][kappa] S[kappa][a][el], kappa =
// 2 kk + h, C[c][kappa] = sV[h][kk][c]; M = c (N1 of 16 rows), K = 2 N1 padded
// to a multiple of 4, N = the 16 prisms.  Lane (g, j) holds rows c = 4 g + r of
// prism j (the prism of this lane's column slot).
template <int PT, int PZ>
__device__ __forceinline__ void vertical_out_mfma(int L, ColSlot cs, int k, const float* __restrict__ sR,
                                                  const float* __restrict__ sV, float* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NAT = D::NAT, KS2 = (2 * N1 + 3) / 4;
  static_assert(N1 <= 16, "the outputs of a node fit one 16-row tile");
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  float ca[KS2];
#pragma unroll
  for (int s = 0; s < KS2; ++s) {
    const int kap = 4 * s + g;
    ca[s] = (j < N1 && kap < 2 * N1) ? sV[(kap & 1) * N1 * N1 + (kap >> 1) * N1 + j] : 0.f;
  }
  const float* sb = sR + g * NAT * 256 + j;  // S[kappa = g][a = 0][el = j]
  for (int a = k; a < NPT; a += N1) {
    f4_t acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS2; ++s) {
      const float bv = 4 * s + g < 2 * N1 ? sb[(4 * s * NAT * 16 + a) * 16] : 0.f;
      acc = mfma4(ca[s], bv, acc);
    }
    if (4 * g < N1 && cs.te >= 0) {
      float* out = Y + ((size_t(cs.te) * NPT + a) * L + cs.layer) * N1 + 4 * g;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * g + r < N1) out[r] = acc[r];
    }
  }
}

// vertical_out with S staged one half at a time (S[k][a][el] of Yr, then of
// Yt), for kernels whose LDS cannot hold both; the sums and their order are
// those of vertical_out.  Every thread holds the Yr partials of its (a, el)
// pairs (at most two) across the second staging.
template <int PT, int PZ, typename T, typename ACC, bool F64ROW>
__device__ __forceinline__ void vertical_out_halves(int L, ColSlot cs, int k, const ACC (&yr)[MD<PT, PZ>::NAT],
                                                    const ACC (&yt)[MD<PT, PZ>::NAT], T* __restrict__ sR,
                                                    const T* __restrict__ sV, T* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NAT = D::NAT, NTH = 64 * N1;
  static_assert(16 * NPT <= 2 * NTH, "at most two (node, prism) pairs per thread");
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  T hr[2][N1];
#pragma unroll
  for (int at = 0; at < NAT; ++at)
#pragma unroll
    for (int r = 0; r < 4; ++r) sR[(k * NAT * 16 + 16 * at + row_of<F64ROW>(g, r)) * 16 + j] = yr[at][r];
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int pr = threadIdx.x + p * NTH, a = pr >> 4, el = pr & 15;
#pragma unroll
    for (int kk = 0; kk < N1; ++kk) hr[p][kk] = pr < 16 * NPT ? sR[(kk * NAT * 16 + a) * 16 + el] : T(0);
  }
  __syncthreads();
#pragma unroll
  for (int at = 0; at < NAT; ++at)
#pragma unroll
    for (int r = 0; r < 4; ++r) sR[(k * NAT * 16 + 16 * at + row_of<F64ROW>(g, r)) * 16 + j] = yt[at][r];
  __syncthreads();
  if (cs.te < 0) return;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int pr = threadIdx.x + p * NTH, a = pr >> 4, el = pr & 15;
    if (pr >= 16 * NPT) continue;
    T ht[N1];
#pragma unroll
    for (int kk = 0; kk < N1; ++kk) ht[kk] = sR[(kk * NAT * 16 + a) * 16 + el];
    T* out = Y + ((size_t(cs.te) * NPT + a) * L + cs.layer) * N1;
#pragma unroll 1
    for (int c = 0; c < N1; ++c) {
      T y = 0;
#pragma unroll
      for (int kk = 0; kk < N1; ++kk) y += sV[kk * N1 + c] * hr[p][kk] + sV[N1 * N1 + kk * N1 + c] * ht[kk];
      out[c] = y;
    }
  }
}

// Phase 2 writing column sums (CS; 16 % L == 0, so the batch holds 16/L whole
// columns and prism el + 1 is the layer above el).  Thread (a, el) reads its
// partials from S, then (once every thread holds its own) writes y[c] of prism
// el to LDS as Ycol[el][a][c]; it then writes the column values z = layer PZ +
// c, c = (layer > 0) .. PZ, of its (triangle, node a), the top one adding the
// bottom value of the layer above: for a node inside the triangle to
// Y[(te NINT + rank) nz + z], for a node on the triangle's boundary to
// Y[nt NINT nz + (te 3P + s) nz + z] (layout of launch_col_sum).  Only stores
// leave the workgroup: nothing in this phase waits on global memory.
template <int PT, int PZ, typename T>
__device__ __forceinline__ void vertical_colsum(int te, int layer, int L, int nz, int64_t bnd_off,
                                                T* __restrict__ sR, const T* __restrict__ sV, T* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NAT = D::NAT, NTH = 64 * N1, NINT = (PT - 1) * (PT - 2) / 2;
  static_assert(16 * NPT <= NTH, "one (node, prism) pair per thread");
  static_assert(16 * NPT * N1 <= KS_LDS<PT, PZ>::R_WORDS, "Ycol fits in the staging buffer");
  const int pr = threadIdx.x, a = pr >> 4, el = pr & 15;
  const bool act = pr < 16 * NPT;
  T yr[N1], yt[N1];
  if (act) {
#pragma unroll
    for (int kk = 0; kk < N1; ++kk) {
      yr[kk] = sR[((kk * 2 + 0) * NAT * 16 + a) * 16 + el];
      yt[kk] = sR[((kk * 2 + 1) * NAT * 16 + a) * 16 + el];
    }
  }
  __syncthreads();  // every thread holds its partials; sR becomes Ycol
  T* ycol = sR + (el * NPT + a) * N1;
  if (act) {
#pragma unroll 1
    for (int c = 0; c < N1; ++c) {
      T v = 0;
#pragma unroll
      for (int kk = 0; kk < N1; ++kk) v += sV[kk * N1 + c] * yr[kk] + sV[N1 * N1 + kk * N1 + c] * yt[kk];
      ycol[c] = v;
    }
  }
  __syncthreads();
  if (!act || te < 0) return;
  const bool above = layer + 1 < L;
  const T top = above ? sR[((el + 1) * NPT + a) * N1] : T(0);
  const int code = tri_code<PT>(a);
  T* dst = (code >= 0 ? Y + bnd_off + (size_t(te) * (3 * PT) + code) * nz
                      : Y + (size_t(te) * NINT + (-1 - code)) * nz) + layer * PZ;
#pragma unroll 1
  for (int c = layer > 0 ? 1 : 0; c < N1; ++c) dst[c] = c == PZ && above ? ycol[c] + top : ycol[c];
}

// geometric factors of one full tile (lane-native: 4 contiguous values per lane)
template <typename T, typename TG>
__device__ __forceinline__ void load_full(const TG* __restrict__ G, int64_t blk, int64_t mst, int t, int lane,
                                          T (&gv)[6][4]) {
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) gv[m][r] = T(gld_any(G, blk + m * mst + t * 256 + lane * 4 + r));
}
// geometric factors of the remainder tile (rows < NQR only)
template <typename T, int NTF, int NQR, bool F64ROW, typename TG>
__device__ __forceinline__ void load_rem(const TG* __restrict__ G, int64_t blk, int64_t mst, int g, int j,
                                         T (&gv)[6][4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row_of<F64ROW>(g, r);
#pragma unroll
    for (int m = 0; m < 6; ++m)
      gv[m][r] = row < NQR ? T(gld_any(G, blk + m * mst + NTF * 256 + row * 16 + j)) : T(0);
  }
}
// Geometric factors of q tile t computed from the column factors (see
// launch_geom): lane rows q = 16 t + row(g, r) of triangle tri; p = zw_k,
// ps = zw_k s, ps2 = zw_k s^2 for the lane's layer.  Every load is in bounds
// and unpredicated: rows past the last q read the last row (the operand tables
// are zero there, so those rows of the products are exactly zero), and lanes
// past the last element (tri < 0, p = ps = ps2 = 0) read triangle 0 and get 0.
__device__ __forceinline__ void load8(const double* p, double (&b)[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 v = reinterpret_cast<const double2*>(p)[i];
    b[2 * i] = v.x;
    b[2 * i + 1] = v.y;
  }
}
__device__ __forceinline__ void load8(const float* p, float (&b)[8]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float4 v = reinterpret_cast<const float4*>(p)[i];
    b[4 * i] = v.x;
    b[4 * i + 1] = v.y;
    b[4 * i + 2] = v.z;
    b[4 * i + 3] = v.w;
  }
}
// ONE: the Gauss weight zw_k is carried by the vertical transpose (its rows of
// Bz and Dz scaled by zw_k), so G is formed without it (p = 1).
template <typename T, int PT, int PZ, bool F64ROW, bool ONE = false>
__device__ __forceinline__ void load_geo(const T* __restrict__ geo, int64_t tri, int t, int g, T p, T ps, T ps2,
                                         T (&gv)[6][4]) {
  using D = MD<PT, PZ>;
  const int64_t tc = tri >= 0 ? tri : 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = 16 * t + row_of<F64ROW>(g, r);
    T bq[8];
    load8(geo + (tc * D::NQT + (q < D::NQT ? q : D::NQT - 1)) * 8, bq);
    if constexpr (ONE) {
      gv[0][r] = bq[0];
      gv[1][r] = bq[1];
      gv[3][r] = bq[3];
      gv[5][r] = ps2 * bq[5] + bq[6];
    } else {
      gv[0][r] = p * bq[0];
      gv[1][r] = p * bq[1];
      gv[3][r] = p * bq[3];
      gv[5][r] = ps2 * bq[5] + p * bq[6];
    }
    gv[2][r] = ps * bq[2];
    gv[4][r] = ps * bq[4];
  }
}
// per-lane constants of load_geo for the lane's column slot at vertical Gauss point k
template <typename T>
__device__ __forceinline__ void geo_lane(ColSlot cs, int L, T zw, T zh, int64_t& tri, T& p, T& ps, T& ps2) {
  tri = -1;
  p = ps = ps2 = T(0);
  if (cs.te >= 0) {
    tri = cs.te;
    const T sg = (T(cs.layer) + zh) / T(L);
    p = zw;
    ps = zw * sg;
    ps2 = ps * sg;
  }
}
template <typename T>
__device__ __forceinline__ void geo_lane(int64_t e, int64_t n_elem, int L, T zw, T zh, int64_t& tri, T& p, T& ps,
                                         T& ps2) {
  tri = -1;
  p = ps = ps2 = T(0);
  if (e < n_elem) {
    const uint32_t eu = uint32_t(e), tu = eu / uint32_t(L);  // e < 2^31 (pmg_create)
    tri = tu;
    const T sg = (T(int(eu - tu * uint32_t(L))) + zh) / T(L);
    p = zw;
    ps = zw * sg;
    ps2 = ps * sg;
  }
}

template <typename T, typename ACC>
__device__ __forceinline__ void pointwise(const T (&gv)[6][4], ACC& dr, ACC& ds, ACC& db) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T ur = dr[r], us = ds[r], ut = db[r];
    dr[r] = gv[0][r] * ur + gv[1][r] * us + gv[2][r] * ut;
    ds[r] = gv[1][r] * ur + gv[3][r] * us + gv[4][r] * ut;
    db[r] = gv[2][r] * ur + gv[4][r] * us + gv[5][r] * ut;
  }
}

// FP32 / FP64 flavours (K = 4).  GT (FP64 at P = 8, whose padded operand
// tables and staging buffer do not fit in the LDS together): the three
// reference tables sit in LDS once, unpadded ([m][q][a], 87.5 KB), and serve
// the operands of both contractions by index; the staging buffer holds one
// half of S at a time (Yr, then Yt); one workgroup per CU.
// GEO: G from the column factors (Gnat is then geo[t][q][8] of type T) instead
// of the stored lane-native G.
// CS: phase 2 writes column sums (vertical_colsum) instead of the E-layout output.
template <int PT, int PZ, typename T, typename TG, typename ACC, bool F64ROW, bool GT = false, bool GEO = false,
          bool CS = false>
__global__ __launch_bounds__(64 * (PZ + 1), GT ? 1 : (sizeof(T) == 8 ? 2 : (PZ >= 8 ? 3 : ((GEO && PT <= 3) ? 6 : 4)))) void k_ax_mfma4(const int32_t* __restrict__ map2d, int L, int nz,
                                                         int64_t n_elem, int64_t n_batch,
                                                         const TG* __restrict__ Gnat, const T* __restrict__ tab2,
                                                         const T* __restrict__ tab4, VertMats<T> vm,
                                                         const T* __restrict__ u, T* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NP = NPT * N1, NT2 = D::NT2, KS = D::KS, NAT = D::NAT;
  constexpr int NS4 = n_steps4<PT, PZ, F64ROW>();
  constexpr int NTAB2 = 3 * NT2 * KS * 64, NTAB4 = 3 * NAT * NS4 * 64;
  constexpr int NTH = 64 * N1;
  constexpr int NCT = 3 * D::NQT * NPT;                    // GT: unpadded tables
  constexpr int SH_WORDS = N1 * NAT * 16 * 16;             // GT: one half of S
  constexpr int GT_R = KS_LDS<PT, PZ>::U_WORDS > SH_WORDS ? KS_LDS<PT, PZ>::U_WORDS : SH_WORDS;
  __shared__ T s2buf[GT ? NCT + 8 : NTAB2];
  __shared__ T s4buf[GT ? 1 : NTAB4];
  __shared__ T sR[GT ? GT_R : KS_LDS<PT, PZ>::R_WORDS];
  __shared__ T sV[2 * N1 * N1];
  const T* __restrict__ s2 = s2buf;
  const T* __restrict__ s4 = s4buf;
  if constexpr (GT) {
    for (int i = threadIdx.x; i < NCT + 8; i += NTH) s2buf[i] = i < NCT ? tab2[i] : T(0);
  } else {
    for (int i = threadIdx.x; i < NTAB2; i += NTH) s2buf[i] = tab2[i];
    for (int i = threadIdx.x; i < NTAB4; i += NTH) s4buf[i] = tab4[i];
  }
  // vertical transpose coefficients; with the column factors (GEO) row k carries
  // the Gauss weight zw_k, which G then leaves out
  for (int i = threadIdx.x; i < N1 * N1; i += NTH) {
    const T w = GEO ? vm.zw[i / N1] : T(1);
    sV[i] = vm.Bz[i] * w;
    sV[N1 * N1 + i] = vm.Dz[i] * w;
  }
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  // operand of stage 2 (M_m[16 t + j][4 s + g]) and stage 4 (M_m[q][16 at + j]
  // with q the K row of step st = 4 t + r); with GT read from the unpadded
  // tables, where entries past a = NPT wrap into the next row (multiplied by a
  // zero of w, or landing in output rows past NPT) and q past NQT reads 0
  auto op2 = [&](int m, int t, int s) -> T {
    if constexpr (GT) return s2[(m * D::NQT + 16 * t + j) * NPT + 4 * s + g];
    else return s2[((m * NT2 + t) * KS + s) * 64 + lane];
  };
  auto op4 = [&](int m, int at, int st, int t, int r) -> T {
    if constexpr (GT) {
      const int q = 16 * t + row_of<F64ROW>(g, r);
      return q < D::NQT ? s2[(m * D::NQT + q) * NPT + 16 * at + j] : T(0);
    } else {
      return s4[((m * NAT + at) * NS4 + st) * 64 + lane];
    }
  };
  // wave-uniform vertical level: its Bz/Dz row stays in scalar registers
  const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T bzk[N1], dzk[N1];
#pragma unroll
  for (int c = 0; c < N1; ++c) {
    bzk[c] = vm.Bz[k * N1 + c];
    dzk[c] = vm.Dz[k * N1 + c];
  }
  const int64_t bnd_off = CS ? int64_t(n_elem / L) * ((PT - 1) * (PT - 2) / 2) * nz : 0;
  const int64_t lb = xcd_block(gridDim.x);
  // PF: one (node, prism) pair of the staging per thread; its column values for
  // the next batch are loaded while this batch computes (map entry at the top
  // of the batch, values after stage 1), hiding the gather's two dependent
  // memory latencies
  constexpr bool PF = 16 * NPT <= NTH;
  const int pa = threadIdx.x >> 4;
  T pf[N1];
  int32_t pidx = 0;
  if constexpr (PF) {
    const ColSlot c0 = col_slot(lb, j, n_elem, L);
    if (pa < NPT && lb < n_batch && c0.te >= 0) {
      const T* col = u + int64_t(map2d[size_t(c0.te) * NPT + pa]) * nz + c0.layer * PZ;
#pragma unroll
      for (int c = 0; c < N1; ++c) pf[c] = col[c];
    } else {
#pragma unroll
      for (int c = 0; c < N1; ++c) pf[c] = T(0);
    }
  }
  for (int64_t b = lb; b < n_batch; b += gridDim.x) {
    __syncthreads();  // previous batch's phase 2 done with sR
    // phase 0: U[c][a][el] <- u
    const ColSlot cs = col_slot(b, j, n_elem, L);
    ColSlot cn{-1, 0};
    if constexpr (PF) {
      if (pa < NPT) {
#pragma unroll
        for (int c = 0; c < N1; ++c) sR[(c * NPT + pa) * 16 + j] = pf[c];
      }
      cn = col_slot(b + gridDim.x, j, n_elem, L);
      if (pa < NPT && b + gridDim.x < n_batch && cn.te >= 0) pidx = map2d[size_t(cn.te) * NPT + pa];
    } else {
      stage_u<PT, PZ, T>(map2d, nz, cs, u, sR);
    }
    __syncthreads();
    // phase 1, stage 1: W[k][a], Wz[k][a] for a = 4s + g of element j
    T w[KS], wz[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int a = 4 * s + g;
      T a0 = 0, a1 = 0;
      if (a < NPT) {
#pragma unroll
        for (int c = 0; c < N1; ++c) {
          const T uv = sR[(c * NPT + a) * 16 + j];
          a0 += bzk[c] * uv;
          a1 += dzk[c] * uv;
        }
      }
      w[s] = a0;
      wz[s] = a1;
    }
    if constexpr (PF) {
      if (pa < NPT && b + gridDim.x < n_batch && cn.te >= 0) {
        const T* col = u + int64_t(pidx) * nz + cn.layer * PZ;
#pragma unroll
        for (int c = 0; c < N1; ++c) pf[c] = col[c];
      } else {
#pragma unroll
        for (int c = 0; c < N1; ++c) pf[c] = T(0);
      }
    }
    __syncthreads();  // every wave has read U; sR becomes S
    ACC yr[NAT], yt[NAT];
#pragma unroll
    for (int at = 0; at < NAT; ++at) { yr[at] = ACC{0, 0, 0, 0}; yt[at] = ACC{0, 0, 0, 0}; }
    const int64_t blk = ((b * N1 + k) * 6) * (16 * D::NQT);
    constexpr int64_t MST = 16 * D::NQT;
    int64_t tri;
    T gp, gps, gps2;
    if constexpr (GEO) geo_lane<T>(cs, L, T(1), vm.zh[k], tri, gp, gps, gps2);
    T ga[6][4];
    // FP64: G one row at a time (the next row's loads in flight), pointwise and
    // stage 4 per row: six live factors instead of 24 plus four rows of loads
    // (FP32 measured slower this way at order 6 and keeps the whole tile)
    constexpr bool ROWWISE = sizeof(T) == 8;
    auto g_row = [&](int t, int r, T (&gv)[6]) {
      if constexpr (GEO) {
        const int q = 16 * t + row_of<F64ROW>(g, r);
        const int64_t tc = tri >= 0 ? tri : 0;
        T bq[8];
        load8((const T*)Gnat + (tc * D::NQT + (q < D::NQT ? q : D::NQT - 1)) * 8, bq);
        gv[0] = bq[0];
        gv[1] = bq[1];
        gv[3] = bq[3];
        gv[5] = gps2 * bq[5] + bq[6];
        gv[2] = gps * bq[2];
        gv[4] = gps * bq[4];
      } else {
#pragma unroll
        for (int m = 0; m < 6; ++m) gv[m] = T(gld_any(Gnat, blk + m * MST + t * 256 + lane * 4 + r));
      }
    };
#pragma unroll 1
    for (int t = 0; t < D::NTF; ++t) {
      if constexpr (ROWWISE) {
        T gn[6];
        g_row(t, 0, gn);
        ACC dr = {0, 0, 0, 0}, ds = {0, 0, 0, 0}, db = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          dr = mfma4(op2(0, t, s), w[s], dr);
          ds = mfma4(op2(1, t, s), w[s], ds);
          db = mfma4(op2(2, t, s), wz[s], db);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          T gv[6];
#pragma unroll
          for (int m = 0; m < 6; ++m) gv[m] = gn[m];
          if (r + 1 < 4) g_row(t, r + 1, gn);
          const T ur = dr[r], us = ds[r], ut = db[r];
          const T pr = gv[0] * ur + gv[1] * us + gv[2] * ut;
          const T ps = gv[1] * ur + gv[3] * us + gv[4] * ut;
          const T pt = gv[2] * ur + gv[4] * us + gv[5] * ut;
          const int st = 4 * t + r;
#pragma unroll
          for (int at = 0; at < NAT; ++at) {
            yr[at] = mfma4(op4(0, at, st, t, r), pr, yr[at]);
            yr[at] = mfma4(op4(1, at, st, t, r), ps, yr[at]);
            yt[at] = mfma4(op4(2, at, st, t, r), pt, yt[at]);
          }
        }
        continue;
      }
      if constexpr (GEO) load_geo<T, PT, PZ, F64ROW, true>((const T*)Gnat, tri, t, g, gp, gps, gps2, ga);
      else load_full<T>(Gnat, blk, MST, t, lane, ga);
      ACC dr = {0, 0, 0, 0}, ds = {0, 0, 0, 0}, db = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        dr = mfma4(op2(0, t, s), w[s], dr);
        ds = mfma4(op2(1, t, s), w[s], ds);
        db = mfma4(op2(2, t, s), wz[s], db);
      }
      pointwise<T, ACC>(ga, dr, ds, db);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int st = 4 * t + r;
#pragma unroll
        for (int at = 0; at < NAT; ++at) {
          yr[at] = mfma4(op4(0, at, st, t, r), dr[r], yr[at]);
          yr[at] = mfma4(op4(1, at, st, t, r), ds[r], yr[at]);
          yt[at] = mfma4(op4(2, at, st, t, r), db[r], yt[at]);
        }
      }
    }
    if constexpr (D::NQR > 0) {
      constexpr int t = D::NTF;
      if constexpr (GEO) load_geo<T, PT, PZ, F64ROW, true>((const T*)Gnat, tri, D::NTF, g, gp, gps, gps2, ga);
      else load_rem<T, D::NTF, D::NQR, F64ROW>(Gnat, blk, MST, g, j, ga);
      ACC dr = {0, 0, 0, 0}, ds = {0, 0, 0, 0}, db = {0, 0, 0, 0};
      if constexpr (D::NQR == 1) {
        // one valid row (q = 16 NTF, held by lanes g = 0 in register 0): three dot
        // products over a on VALU instead of 3 KS MFMAs of which 15/16 rows are
        // padding.  Lane (g, j) holds W at a = 4 s + g; the row's coefficients are
        // the table entries of lane 16 g (row 0 of the tile, column 4 s + g).
        T pr = 0, ps = 0, pb = 0;
        auto row0 = [&](int m, int s) -> T {
          if constexpr (GT) return s2[(m * D::NQT + 16 * t) * NPT + 4 * s + g];
          else return s2[((m * NT2 + t) * KS + s) * 64 + 16 * g];
        };
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          pr += row0(0, s) * w[s];
          ps += row0(1, s) * w[s];
          pb += row0(2, s) * wz[s];
        }
#pragma unroll
        for (int o = 16; o < 64; o <<= 1) {
          pr += __shfl_xor(pr, o);
          ps += __shfl_xor(ps, o);
          pb += __shfl_xor(pb, o);
        }
        if (g == 0) {
          dr[0] = pr;
          ds[0] = ps;
          db[0] = pb;
        }
      } else {
        static_assert(!GT || D::NQR == 1, "GT stage 2 reads full rows of the remainder tile");
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          dr = mfma4(op2(0, t, s), w[s], dr);
          ds = mfma4(op2(1, t, s), w[s], ds);
          db = mfma4(op2(2, t, s), wz[s], db);
        }
      }
      pointwise<T, ACC>(ga, dr, ds, db);
      int st = 4 * D::NTF;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (row_of<F64ROW>(0, r) < D::NQR) {
#pragma unroll
          for (int at = 0; at < NAT; ++at) {
            yr[at] = mfma4(op4(0, at, st, t, r), dr[r], yr[at]);
            yr[at] = mfma4(op4(1, at, st, t, r), ds[r], yr[at]);
            yt[at] = mfma4(op4(2, at, st, t, r), db[r], yt[at]);
          }
          ++st;
        }
      }
    }
    if constexpr (GT) {
      static_assert(!CS, "GT keeps the element layout");
      vertical_out_halves<PT, PZ, T, ACC, F64ROW>(L, cs, k, yr, yt, sR, sV, Y);
      continue;
    }
    // S[k][h][a][el]: lane holds a = 16 at + row(g, r) of element j
#pragma unroll
    for (int at = 0; at < NAT; ++at)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * at + row_of<F64ROW>(g, r);
        sR[((k * 2 + 0) * NAT * 16 + a) * 16 + j] = yr[at][r];
        sR[((k * 2 + 1) * NAT * 16 + a) * 16 + j] = yt[at][r];
      }
    __syncthreads();
    // phase 2: y[el][c][a] = sum_k Bz[k][c] Yr[k][a] + Dz[k][c] Yt[k][a]
    if constexpr (CS) vertical_colsum<PT, PZ, T>(cs.te, cs.layer, L, nz, bnd_off, sR, sV, Y);
    else if constexpr (sizeof(T) == 4) vertical_out_mfma<PT, PZ>(L, cs, k, sR, sV, Y);
    else vertical_out<PT, PZ, T>(L, cs, sR, sV, Y);
  }
}

// BF16 G of q tile t for lane (g, j), rows 4g+r (r = 0..3), packed two per word
// (low half = even r): one 8-byte load per factor on full tiles; rows past the
// last q of the remainder tile read as 0.
template <int PT, int PZ>
__device__ __forceinline__ void load_g_bf16(const bf16_t* __restrict__ Gnat, int64_t blk, int64_t mst, int t,
                                            int lane, int g, int j, uint32_t (&gw)[6][2]) {
  using D = MD<PT, PZ>;
  if (t < D::NTF) {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const uint2 v = *reinterpret_cast<const uint2*>(Gnat + blk + m * mst + t * 256 + lane * 4);
      gw[m][0] = v.x;
      gw[m][1] = v.y;
    }
  } else {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      uint32_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * g + r;
        h[r] = row < D::NQR ? uint32_t(Gnat[blk + m * mst + D::NTF * 256 + row * 16 + j]) : 0u;
      }
      gw[m][0] = h[0] | (h[1] << 16);
      gw[m][1] = h[2] | (h[3] << 16);
    }
  }
}

// BF16 operands, FP32 accumulation (K = 16)
template <int PT, int PZ, typename TG, bool CS = false>
__global__ __launch_bounds__(64 * (PZ + 1), PZ >= 8 ? 3 : 4) void k_ax_mfma_bf16(const int32_t* __restrict__ map2d, int L, int nz,
                                                             int64_t n_elem, int64_t n_batch,
                                                             const TG* __restrict__ Gnat,
                                                             const s4_t* __restrict__ tab2,
                                                             const s4_t* __restrict__ tab4, VertMats<float> vm,
                                                             const float* __restrict__ u, float* __restrict__ Y) {
  using D = MD<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NP = NPT * N1, NT2 = D::NT2, KS16 = D::KS16, NAT = D::NAT;
  constexpr int NTAB2 = 3 * NT2 * KS16 * 64, NTAB4 = 3 * NAT * NT2 * 64;
  constexpr int NTH = 64 * N1;
  __shared__ s4_t s2[NTAB2];
  __shared__ s4_t s4[NTAB4];
  __shared__ float sR[KS_LDS<PT, PZ>::R_WORDS];
  __shared__ float sV[2 * N1 * N1];
  for (int i = threadIdx.x; i < NTAB2; i += NTH) s2[i] = tab2[i];
  for (int i = threadIdx.x; i < NTAB4; i += NTH) s4[i] = tab4[i];
  for (int i = threadIdx.x; i < N1 * N1; i += NTH) { sV[i] = vm.Bz[i]; sV[N1 * N1 + i] = vm.Dz[i]; }
  const int lane = threadIdx.x & 63, k = threadIdx.x >> 6, g = lane >> 4, j = lane & 15;
  const int64_t bnd_off = CS ? int64_t(n_elem / L) * ((PT - 1) * (PT - 2) / 2) * nz : 0;
  const int64_t lb = xcd_block(gridDim.x);
  for (int64_t b = lb; b < n_batch; b += gridDim.x) {
    __syncthreads();
    // G of tile t as raw BF16 pairs (PF: one tile ahead, the first under the
    // staging of u and stage 1, as in the split-BF16 kernel; measured faster at
    // P = 6 only: 190 -> 180 us, while the smaller and the P = 8 orders lost)
    constexpr bool PF = PT == 6;
    const int64_t blk = ((b * N1 + k) * 6) * (16 * D::NQT);
    constexpr int64_t mst = 16 * D::NQT;
    uint32_t gw[6][2];
    if constexpr (PF) load_g_bf16<PT, PZ>(Gnat, blk, mst, 0, lane, g, j, gw);
    stage_u<PT, PZ, float>(map2d, L, nz, n_elem, b, u, sR);
    __syncthreads();
    s4_t w[KS16], wz[KS16];
#pragma unroll
    for (int s = 0; s < KS16; ++s) {
      float a0[4], a1[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int a = 16 * s + 4 * g + kk;
        a0[kk] = 0.f;
        a1[kk] = 0.f;
        if (a < NPT) {
#pragma unroll
          for (int c = 0; c < N1; ++c) {
            const float uv = sR[(c * NPT + a) * 16 + j];
            a0[kk] += sV[k * N1 + c] * uv;
            a1[kk] += sV[N1 * N1 + k * N1 + c] * uv;
          }
        }
      }
      w[s] = bf4(a0);
      wz[s] = bf4(a1);
    }
    __syncthreads();
    f4_t yr[NAT], yt[NAT];
#pragma unroll
    for (int at = 0; at < NAT; ++at) { yr[at] = f4_t{0, 0, 0, 0}; yt[at] = f4_t{0, 0, 0, 0}; }
#pragma unroll 1
    for (int t = 0; t < NT2; ++t) {
      uint32_t gc[6][2];
      float gd[6][4];
      if constexpr (PF) {
#pragma unroll
        for (int m = 0; m < 6; ++m) { gc[m][0] = gw[m][0]; gc[m][1] = gw[m][1]; }
        if (t + 1 < NT2) load_g_bf16<PT, PZ>(Gnat, blk, mst, t + 1, lane, g, j, gw);
      } else if (t < D::NTF) {
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) gd[m][r] = gld<TG>(Gnat, blk + m * mst + t * 256 + lane * 4 + r);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * g + r;
#pragma unroll
          for (int m = 0; m < 6; ++m)
            gd[m][r] = row < D::NQR ? gld<TG>(Gnat, blk + m * mst + D::NTF * 256 + row * 16 + j) : 0.f;
        }
      }
      f4_t dr = {0, 0, 0, 0}, ds = {0, 0, 0, 0}, db = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS16; ++s) {
        dr = mfma16(s2[((0 * NT2 + t) * KS16 + s) * 64 + lane], w[s], dr);
        ds = mfma16(s2[((1 * NT2 + t) * KS16 + s) * 64 + lane], w[s], ds);
        db = mfma16(s2[((2 * NT2 + t) * KS16 + s) * 64 + lane], wz[s], db);
      }
      float pr[4], ps[4], pt[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float ur = dr[r], us = ds[r], ut = db[r];
        float gv[6][4];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          if constexpr (PF) {
            const uint32_t wv = gc[m][r >> 1];
            gv[m][r] = __uint_as_float((r & 1) ? (wv & 0xFFFF0000u) : (wv << 16));
          } else {
            gv[m][r] = gd[m][r];
          }
        }
        pr[r] = gv[0][r] * ur + gv[1][r] * us + gv[2][r] * ut;
        ps[r] = gv[1][r] * ur + gv[3][r] * us + gv[4][r] * ut;
        pt[r] = gv[2][r] * ur + gv[4][r] * us + gv[5][r] * ut;
      }
      const s4_t br = bf4(pr), bs = bf4(ps), bt = bf4(pt);
#pragma unroll
      for (int at = 0; at < NAT; ++at) {
        yr[at] = mfma16(s4[((0 * NAT + at) * NT2 + t) * 64 + lane], br, yr[at]);
        yr[at] = mfma16(s4[((1 * NAT + at) * NT2 + t) * 64 + lane], bs, yr[at]);
        yt[at] = mfma16(s4[((2 * NAT + at) * NT2 + t) * 64 + lane], bt, yt[at]);
      }
    }
#pragma unroll
    for (int at = 0; at < NAT; ++at)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * at + 4 * g + r;
        sR[((k * 2 + 0) * NAT * 16 + a) * 16 + j] = yr[at][r];
        sR[((k * 2 + 1) * NAT * 16 + a) * 16 + j] = yt[at][r];
      }
    __syncthreads();
    if constexpr (CS) {
      const int64_t e = b * 16 + (threadIdx.x & 15);
      const uint32_t eu = uint32_t(e), tu = eu / uint32_t(L);  // e < 2^31 (pmg_create)
      vertical_colsum<PT, PZ, float>(e < n_elem ? int(tu) : -1, int(eu - tu * uint32_t(L)), L, nz, bnd_off, sR, sV,
                                     Y);
    } else {
      vertical_out_mfma<PT, PZ>(L, col_slot(b, threadIdx.x & 15, n_elem, L), k, sR, sV, Y);
    }
  }
}

// Split-BF16 products (FP32 accumulation): every operand x = x_hi + x_lo with
// x_hi = bf16(x), x_lo = bf16(x - x_hi).
// LO: a product keeps the three terms a_hi b_hi + a_hi b_lo + a_lo b_hi (about
//   16 significant bits, against 8 for one BF16 product).  Tables: hi and lo
//   copies, both in LDS (79 KB at P = 6, two workgroups per CU within 128
//   VGPRs).
// !LO: the reference tables are rounded to BF16 once (a fixed, symmetric
//   perturbation of the reference matrices, as G's rounding is of the
//   geometry) and only the vectors are split: a_hi b_hi + a_hi b_lo.
// Stage 2 runs on the K = 32 BF16 MFMA of gfx950 (v_mfma_f32_16x16x32_bf16):
// one step covers the 28 triangle nodes of P = 6, half the instructions of two
// K = 16 steps.  K slots: lane group g = lane / 16 holds slots 8g .. 8g+7, and
// slot e of group g is node a = 16 (e / 4) + 4 (e % 4) + g, so that stage 1
// reads 64 consecutive LDS words per instruction.  Stage 4 stays on K = 16 per
// q tile, its B operand being the registers the pointwise stage produced (a
// K = 32 form over q tile pairs halves those instructions too but holds two
// tiles' values at once and measured slower at 128 VGPRs).
// Phase 2 reads the vertical coefficients from the kernel arguments (scalar
// registers), and the partial results from S[k][h][a][el] with rows of 20
// words (conflict-free stores from the MFMA output layout).
// GEO: G in FP32 from the FP32 column factors (Gsrc = geo[t][q][8]) instead of
// the stored lane-native BF16 G (Gsrc = Gnat).
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef short s8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4_t mfma32(s8_t a, s8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), c, 0, 0,
                                                 0);
}
__device__ __forceinline__ void split8(const float (&x)[8], s8_t& hi, s8_t& lo) {
  const float x0[4] = {x[0], x[1], x[2], x[3]}, x1[4] = {x[4], x[5], x[6], x[7]};
  s4_t h0, l0, h1, l1;
  split4(x0, h0, l0);
  split4(x1, h1, l1);
  hi = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
  lo = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
}
template <int PT, int PZ> struct X3 {
  using D = MD<PT, PZ>;
  static constexpr int SROW = 20;                          // words per row of S
  static constexpr int S_WORDS = D::N1 * 2 * D::NPT * SROW;
  static constexpr int U_WORDS = D::N1 * D::NPT * 16;
  static constexpr int C_WORDS = 16 * D::NPT * D::N1;      // Ycol of the column-sum phase 2
  static constexpr int R_WORDS = S_WORDS > U_WORDS ? (S_WORDS > C_WORDS ? S_WORDS : C_WORDS)
                                                   : (U_WORDS > C_WORDS ? U_WORDS : C_WORDS);
  static constexpr int NTAB2 = 3 * D::NT2 * 64, NTAB4 = 3 * D::NAT * D::NT2 * 64;
};
__device__ __forceinline__ int x3_srow(int k, int h, int a, int NPT) { return ((k * 2 + h) * NPT + a) * 20; }

template <int PT, int PZ, bool LO, bool GEO = false, bool CS = false>
__global__ __launch_bounds__(64 * (PZ + 1), (LO && PZ >= 8) ? 2 : 4) void k_ax_mfma_bf16x3(const int32_t* __restrict__ map2d, int L,
                                                                     int nz, int64_t n_elem, int64_t n_batch,
                                                                     const void* __restrict__ Gsrc,
                                                                     const s8_t* __restrict__ tab2,
                                                                     const s4_t* __restrict__ tab4,
                                                                     const s8_t* __restrict__ tab2lo,
                                                                     const s4_t* __restrict__ tab4lo,
                                                                     VertMats<float> vm, const float* __restrict__ u,
                                                                     float* __restrict__ Y) {
  using D = MD<PT, PZ>;
  using XS = X3<PT, PZ>;
  constexpr int N1 = D::N1, NPT = D::NPT, NT2 = D::NT2, NAT = D::NAT;
  constexpr int NTAB2 = XS::NTAB2, NTAB4 = XS::NTAB4, NTH = 64 * N1;
  static_assert(NPT <= 32, "one K = 32 step over the triangle nodes");
  __shared__ s8_t s2[NTAB2];
  __shared__ s8_t s2l[LO ? NTAB2 : 1];
  __shared__ s4_t s4[NTAB4];
  __shared__ s4_t s4l[LO ? NTAB4 : 1];
  __shared__ float sR[XS::R_WORDS];
  __shared__ float sC[CS ? 1 : 2 * N1 * N1];  // phase-2 coefficients [h][kk][c]
  for (int i = threadIdx.x; i < NTAB2; i += NTH) {
    s2[i] = tab2[i];
    if constexpr (LO) s2l[i] = tab2lo[i];
  }
  for (int i = threadIdx.x; i < NTAB4; i += NTH) {
    s4[i] = tab4[i];
    if constexpr (LO) s4l[i] = tab4lo[i];
  }
  // wave-uniform Gauss level: the stage-1 coefficients are scalar loads
  const int k = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const bf16_t* __restrict__ Gnat = static_cast<const bf16_t*>(Gsrc);
  const float* __restrict__ geo = static_cast<const float*>(Gsrc);
  // vertical transpose coefficients (kernel arguments, uniform index: scalar
  // loads); with GEO the Gauss weight zw_k rides on them (rows of Bz and Dz
  // scaled by zw_k) and G is formed without it
  auto vB = [&](int i) {
    if constexpr (GEO) return vm.Bzw[i]; else return vm.Bz[i];
  };
  auto vD = [&](int i) {
    if constexpr (GEO) return vm.Dzw[i]; else return vm.Dz[i];
  };
  if constexpr (!CS) {
    // one lane copies the coefficients (uniform indices: scalar loads); the
    // first batch's barrier publishes them
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < N1 * N1; ++i) {
        sC[i] = vB(i);
        sC[N1 * N1 + i] = vD(i);
      }
    }
  }
  const int64_t bnd_off = CS ? int64_t(n_elem / L) * ((PT - 1) * (PT - 2) / 2) * nz : 0;
  const int64_t lb = xcd_block(gridDim.x);
  for (int64_t b = lb; b < n_batch; b += gridDim.x) {
    __syncthreads();
    const int64_t blk = ((b * N1 + k) * 6) * (16 * D::NQT);
    constexpr int64_t mst = 16 * D::NQT;
    uint32_t gw[6][2];
    int64_t tri;
    float gp, gps, gps2;
    if constexpr (GEO) geo_lane<float>(b * 16 + j, n_elem, L, 1.0f, vm.zh[k], tri, gp, gps, gps2);
    else load_g_bf16<PT, PZ>(Gnat, blk, mst, 0, lane, g, j, gw);
    stage_u<PT, PZ, float>(map2d, L, nz, n_elem, b, u, sR);
    __syncthreads();
    // stage 1: the lane's eight node slots a = 16 s + 4 kk + g
    s8_t wh, wl, zh, zl;
    {
      float w0[8], w1[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int a = 16 * (e >> 2) + 4 * (e & 3) + g;
        w0[e] = 0.f;
        w1[e] = 0.f;
        if (a < NPT) {
#pragma unroll
          for (int c = 0; c < N1; ++c) {
            const float uv = sR[(c * NPT + a) * 16 + j];
            w0[e] = __builtin_fmaf(vm.Bz[k * N1 + c], uv, w0[e]);
            w1[e] = __builtin_fmaf(vm.Dz[k * N1 + c], uv, w1[e]);
          }
        }
      }
      split8(w0, wh, wl);
      split8(w1, zh, zl);
    }
    __syncthreads();
    f4_t yr[NAT], yt[NAT];
#pragma unroll
    for (int at = 0; at < NAT; ++at) { yr[at] = f4_t{0, 0, 0, 0}; yt[at] = f4_t{0, 0, 0, 0}; }
#pragma unroll 1
    for (int t = 0; t < NT2; ++t) {
      uint32_t gc[6][2];
      float gg[6][4];
      if constexpr (GEO) {
        load_geo<float, PT, PZ, false, true>(geo, tri, t, g, gp, gps, gps2, gg);
      } else {
#pragma unroll
        for (int m = 0; m < 6; ++m) { gc[m][0] = gw[m][0]; gc[m][1] = gw[m][1]; }
        if (t + 1 < NT2) load_g_bf16<PT, PZ>(Gnat, blk, mst, t + 1, lane, g, j, gw);
      }
      const int i0 = (0 * NT2 + t) * 64 + lane, i1 = (1 * NT2 + t) * 64 + lane, i2 = (2 * NT2 + t) * 64 + lane;
      f4_t dr = mfma32(s2[i0], wh, f4_t{0, 0, 0, 0});
      f4_t ds = mfma32(s2[i1], wh, f4_t{0, 0, 0, 0});
      f4_t db = mfma32(s2[i2], zh, f4_t{0, 0, 0, 0});
      dr = mfma32(s2[i0], wl, dr);
      ds = mfma32(s2[i1], wl, ds);
      db = mfma32(s2[i2], zl, db);
      if constexpr (LO) {
        dr = mfma32(s2l[i0], wh, dr);
        ds = mfma32(s2l[i1], wh, ds);
        db = mfma32(s2l[i2], zh, db);
      }
      float pr[4], ps[4], pt[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float ur = dr[r], us = ds[r], ut = db[r];
        float gv[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          if constexpr (GEO) {
            gv[m] = gg[m][r];
          } else {
            const uint32_t wv = gc[m][r >> 1];
            gv[m] = __uint_as_float((r & 1) ? (wv & 0xFFFF0000u) : (wv << 16));
          }
        }
        pr[r] = gv[0] * ur + gv[1] * us + gv[2] * ut;
        ps[r] = gv[1] * ur + gv[3] * us + gv[4] * ut;
        pt[r] = gv[2] * ur + gv[4] * us + gv[5] * ut;
      }
      s4_t rh, rl, sh, sl, th, tl;
      split4(pr, rh, rl);
      split4(ps, sh, sl);
      split4(pt, th, tl);
#pragma unroll
      for (int at = 0; at < NAT; ++at) {
        const int k0 = ((0 * NAT + at) * NT2 + t) * 64 + lane, k1 = ((1 * NAT + at) * NT2 + t) * 64 + lane,
                  k2 = ((2 * NAT + at) * NT2 + t) * 64 + lane;
        yr[at] = mfma16(s4[k0], rh, yr[at]);
        yr[at] = mfma16(s4[k1], sh, yr[at]);
        yt[at] = mfma16(s4[k2], th, yt[at]);
        yr[at] = mfma16(s4[k0], rl, yr[at]);
        yr[at] = mfma16(s4[k1], sl, yr[at]);
        yt[at] = mfma16(s4[k2], tl, yt[at]);
        if constexpr (LO) {
          yr[at] = mfma16(s4l[k0], rh, yr[at]);
          yr[at] = mfma16(s4l[k1], sh, yr[at]);
          yt[at] = mfma16(s4l[k2], th, yt[at]);
        }
      }
    }
    // partials to S[k][h][a][el] (rows a >= NPT hold no node)
#pragma unroll
    for (int at = 0; at < NAT; ++at)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * at + 4 * g + r;
        if (a < NPT) {
          sR[x3_srow(k, 0, a, NPT) + j] = yr[at][r];
          sR[x3_srow(k, 1, a, NPT) + j] = yt[at][r];
        }
      }
    __syncthreads();
    // phase 2: y[c] of (node a, prism el) = sum over the Gauss levels kk of
    // vB[kk][c] Yr[kk][a][el] + vD[kk][c] Yt[kk][a][el]
    static_assert(16 * NPT <= NTH, "one (node, prism) pair per thread");
    const int pr2 = threadIdx.x, a2 = pr2 >> 4, el = pr2 & 15;
    const bool act = pr2 < 16 * NPT;
    const int64_t e = b * 16 + el;
    const uint32_t eu = uint32_t(e), tu = eu / uint32_t(L);  // e < 2^31 (pmg_create)
    const int te = e < n_elem ? int(tu) : -1, layer = int(eu - tu * uint32_t(L));
    if constexpr (CS) {
      // thread (a, el) sums over the Gauss levels for its PZ+1 outputs
      float yv[N1], zv[N1];
      if (act) {
#pragma unroll
        for (int kk = 0; kk < N1; ++kk) {
          yv[kk] = sR[x3_srow(kk, 0, a2, NPT) + el];
          zv[kk] = sR[x3_srow(kk, 1, a2, NPT) + el];
        }
      }
      // column sums (16 % L == 0: whole columns per batch, prism el + 1 is the
      // layer above el): y[c] of prism el to Ycol[el][a][c], then the column
      // values z = layer PZ + c, c = (layer > 0) .. PZ, of (triangle, node a),
      // the top one adding the bottom value of the layer above, to the layout
      // of launch_col_sum
      constexpr int NINT = (PT - 1) * (PT - 2) / 2;
      __syncthreads();  // every thread holds its partials; sR becomes Ycol
      float* ycol = sR + (el * NPT + a2) * N1;
      if (act) {
#pragma unroll 1
        for (int c = 0; c < N1; ++c) {
          float y = 0.f;
#pragma unroll
          for (int kk = 0; kk < N1; ++kk) {
            y = __builtin_fmaf(vB(kk * N1 + c), yv[kk], y);
            y = __builtin_fmaf(vD(kk * N1 + c), zv[kk], y);
          }
          ycol[c] = y;
        }
      }
      __syncthreads();
      if (act && te >= 0) {
        const bool above = layer + 1 < L;
        const float top = above ? sR[((el + 1) * NPT + a2) * N1] : 0.f;
        const int code = tri_code<PT>(a2);
        float* dst = (code >= 0 ? Y + bnd_off + (size_t(te) * (3 * PT) + code) * nz
                                : Y + (size_t(te) * NINT + (-1 - code)) * nz) + layer * PZ;
#pragma unroll 1
        for (int c = layer > 0 ? 1 : 0; c < N1; ++c) dst[c] = c == PZ && above ? ycol[c] + top : ycol[c];
      }
    } else {
      // on the FP32 matrix cores: per node a (wave k takes a = k, k + N1, ...),
      // D[c][el] = sum_kappa C[c][kappa] S[kappa][a][el] with kappa = 2 kk + h,
      // C[c][2 kk + h] = (h ? vD : vB)[kk][c]; M = c (N1 of 16 rows), K = 2 N1
      // (padded to 4 KS2), N = the 16 prisms.  Lane (g, j) holds rows
      // c = 4 g + r of prism j, the prism of this thread's te and layer.
      constexpr int KS2 = (2 * N1 + 3) / 4;
      float ca[KS2];
#pragma unroll
      for (int s = 0; s < KS2; ++s) {
        const int kap = 4 * s + g;
        ca[s] = (j < N1 && kap < 2 * N1) ? sC[(kap & 1) * N1 * N1 + (kap >> 1) * N1 + j] : 0.f;
      }
      for (int a = k; a < NPT; a += N1) {
        f4_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS2; ++s) {
          const int kap = 4 * s + g;
          const float bv = kap < 2 * N1 ? sR[x3_srow(kap >> 1, kap & 1, a, NPT) + j] : 0.f;
          acc = mfma4(ca[s], bv, acc);
        }
        if (4 * g < N1 && te >= 0) {
          float* out = Y + ((size_t(te) * NPT + a) * L + layer) * N1 + 4 * g;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (4 * g + r < N1) out[r] = acc[r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// G re-layout: standard [e][m][k*NQT+q] (FP64) -> lane-native order of a flavour
// ---------------------------------------------------------------------------
// COL: G formed from the column factors geo[t][q][8] (L layers, vertical Gauss
// points zq, weights zw; see launch_geom) instead of read from the standard G.
template <int PT, int PZ, typename TO, bool F64ROW, bool COL = false>
__global__ __launch_bounds__(256) void k_g_native(int64_t n_elem, int64_t n_batch, const double* __restrict__ G,
                                                  TO* __restrict__ out, int L, const double* __restrict__ geo,
                                                  const double* __restrict__ zq, const double* __restrict__ zw) {
  using D = MD<PT, PZ>;
  // one thread per (batch, k, slot w of a factor's 16 NQT block) writes all six
  // factors of its cubature point (they are 16 NQT apart)
  constexpr int64_t MST = int64_t(16) * D::NQT;
  const int64_t per_batch = D::N1 * MST;
  const int64_t total = n_batch * per_batch;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < total; i += int64_t(gridDim.x) * 256) {
    const int64_t b = i / per_batch;
    const int64_t rem = i - b * per_batch;
    const int k = int(rem / MST);
    int w = int(rem - int64_t(k) * MST);
    const int64_t o = (b * D::N1 + k) * 6 * MST + w;
    int q, jj;
    if (w < D::NTF * 256) {
      const int t = w / 256;
      const int l = (w % 256) / 4, r = w % 4;
      jj = l & 15;
      q = 16 * t + row_of<F64ROW>(l >> 4, r);
    } else {
      w -= D::NTF * 256;
      q = 16 * D::NTF + w / 16;
      jj = w % 16;
    }
    const int64_t e = b * 16 + jj;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (e < n_elem) {
      if constexpr (COL) {
        const int64_t tri = e / L;
        const double sg = (double(e - tri * L) + 0.5 * (1.0 + zq[k])) / L, wk = zw[k];
        const double* bq = geo + (tri * D::NQT + q) * 8;
        v[0] = wk * bq[0];
        v[1] = wk * bq[1];
        v[2] = wk * (sg * bq[2]);
        v[3] = wk * bq[3];
        v[4] = wk * (sg * bq[4]);
        v[5] = wk * (sg * sg * bq[5] + bq[6]);
      } else {
#pragma unroll
        for (int m = 0; m < 6; ++m) v[m] = G[(e * 6 + m) * D::NQ + int64_t(k) * D::NQT + q];
      }
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) out[o + m * MST] = cvt_out<TO>(v[m]);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// One resident wave of workgroups: every workgroup stays on its CU and walks
// batches b, b + grid, ... (the LDS reference tables are loaded once per
// workgroup).  Occupancy comes from the runtime for the kernel's own LDS and
// register use; the grid is a multiple of the XCD count.
static int grid_batches(int64_t n_batch, const void* kernel, int threads) {
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
      n_cu = 256;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int64_t blocks = std::min<int64_t>(n_batch, int64_t(per_cu) * n_cu);
  blocks = ((blocks + 7) / 8) * 8;
  return int(blocks < 8 ? 8 : blocks);
}



template <int PT, int PZ>
static void relayout_p(int64_t n_elem, const double* G, void* out, int flavour, hipStream_t st, const double* geo,
                       int L, const double* zq, const double* zw) {
  const int64_t nb = (n_elem + 15) / 16;
  const int64_t total = nb * 16 * MD<PT, PZ>::NQ;
  int64_t grid = (total + 255) / 256;
  if (grid > 65535 * 4) grid = 65535 * 4;
#define PMG_GN(TO, ROW)                                                                                    \
  if (geo)                                                                                                 \
    hipLaunchKernelGGL((k_g_native<PT, PZ, TO, ROW, true>), dim3(grid), dim3(256), 0, st, n_elem, nb, G,    \
                       (TO*)out, L, geo, zq, zw);                                                          \
  else                                                                                                     \
    hipLaunchKernelGGL((k_g_native<PT, PZ, TO, ROW, false>), dim3(grid), dim3(256), 0, st, n_elem, nb, G,   \
                       (TO*)out, L, geo, zq, zw)
  if (flavour == MF_F64) PMG_GN(double, true);
  else if (flavour == MF_F32) PMG_GN(float, false);
  else PMG_GN(bf16_t, false);
#undef PMG_GN
}

// orders with MFMA kernels: (3,3), (6,6), (3,6), (4,8), (2,8) [the in-plane-
// coarsened levels of P = 6 and P = 8] and (8,8) (its FP64 kernel with
// unpadded LDS tables); split-BF16 kernels at in-plane order 6 only
#define PMG_MFMA_ORDERS(X) X(3, 3) X(6, 6) X(3, 6) X(8, 8) X(4, 8) X(2, 8)

void launch_g_native(int PT, int PZ, int64_t n_elem, const double* G, void* out, int flavour, hipStream_t st,
                     const double* geo, int L, const double* zq, const double* zw) {
#define PMG_REL(PTV, PZV) \
  if (PT == PTV && PZ == PZV) return relayout_p<PTV, PZV>(n_elem, G, out, flavour, st, geo, L, zq, zw);
  PMG_MFMA_ORDERS(PMG_REL)
#undef PMG_REL
}

// one launch of kernel kern over the batches, its resident-grid size cached per
// instantiation (KEY)
template <typename KEY, typename K, typename... A>
static void launch_batches(K kern, int NT, int64_t need, hipStream_t st, A... args) {
  static const int grid = grid_batches(1 << 30, (const void*)kern, NT);
  hipLaunchKernelGGL(kern, dim3(std::min<int64_t>(grid, need)), dim3(NT), 0, st, args...);
}
template <int PT, int PZ, int FL, bool GEO, bool CS = false> struct KeyOf {};

template <int PT, int PZ>
static bool ax_mfma_p(const LevelView& lv, const void* Gnat, int flavour, const void* tab2, const void* tab4,
                      const void* vmats, const void* u, void* Y, hipStream_t st, const void* tab2lo,
                      const void* tab4lo, const void* geo, bool colsum) {
  const int64_t nb = (lv.n_elem + 15) / 16;
  const int64_t need = ((nb + 7) / 8) * 8;
  constexpr int NT = 64 * (PZ + 1);
  // the column-sum phase 2 keeps one (node, prism) pair per thread
  constexpr bool CSOK = 16 * MD<PT, PZ>::NPT <= NT;
  if (colsum && (!CSOK || !lv.colsum)) return false;
  const VertMats<double>& v64 = *(const VertMats<double>*)vmats;
  const VertMats<float>& v32 = *(const VertMats<float>*)vmats;
#define PMG_ARGS(TG, TT, VM) lv.map2d, lv.L, int(lv.nz), lv.n_elem, nb, (const TG*)G, (const TT*)tab2, \
    (const TT*)tab4, VM, (const TT*)u, (TT*)Y
// launch with column sums (C = true) or the element layout
#define PMG_CSW(LAUNCH)                  \
  if (colsum) {                          \
    if constexpr (CSOK) LAUNCH(true);    \
  } else {                               \
    LAUNCH(false);                       \
  }                                      \
  return true;
  if (flavour == MF_F64) {
    const void* G = geo ? geo : Gnat;
    if (geo) {
#define PMG_L(C)                                                                                              \
  launch_batches<KeyOf<PT, PZ, MF_F64, true, C>>(k_ax_mfma4<PT, PZ, double, double, d4_t, true, PT == 8, true, C>, \
                                                 NT, need, st, PMG_ARGS(double, double, v64))
      PMG_CSW(PMG_L)
#undef PMG_L
    }
    if (colsum) return false;
    launch_batches<KeyOf<PT, PZ, MF_F64, false>>(k_ax_mfma4<PT, PZ, double, double, d4_t, true, PT == 8>, NT,
                                                 need, st, PMG_ARGS(double, double, v64));
    return true;
  } else if (flavour == MF_F32) {
    const void* G = geo ? geo : Gnat;
    if (geo) {
#define PMG_L(C)                                                                                             \
  launch_batches<KeyOf<PT, PZ, MF_F32, true, C>>(k_ax_mfma4<PT, PZ, float, float, f4_t, false, false, true, C>, \
                                                 NT, need, st, PMG_ARGS(float, float, v32))
      PMG_CSW(PMG_L)
#undef PMG_L
    }
    if (colsum) return false;
    launch_batches<KeyOf<PT, PZ, MF_F32, false>>(k_ax_mfma4<PT, PZ, float, float, f4_t, false>, NT, need, st,
                                                 PMG_ARGS(float, float, v32));
    return true;
  } else if (flavour == MF_F32G16) {
    const void* G = Gnat;
#define PMG_L(C)                                                                                              \
  launch_batches<KeyOf<PT, PZ, MF_F32G16, false, C>>(                                                         \
      k_ax_mfma4<PT, PZ, float, bf16_t, f4_t, false, false, false, C>, NT, need, st, PMG_ARGS(bf16_t, float, v32))
    PMG_CSW(PMG_L)
#undef PMG_L
  } else if (flavour == MF_BF16X3 || flavour == MF_BF16X2) {
    if constexpr (PT == 6) {
      const void* G = geo ? geo : Gnat;
      const void* lo2 = flavour == MF_BF16X3 ? tab2lo : nullptr;
      const void* lo4 = flavour == MF_BF16X3 ? tab4lo : nullptr;
#define PMG_X(LO, GE, C)                                                                                      \
  launch_batches<KeyOf<PT, PZ, LO ? MF_BF16X3 : MF_BF16X2, GE, C>>(                                           \
      k_ax_mfma_bf16x3<PT, PZ, LO, GE, C>, NT, need, st, lv.map2d, lv.L, int(lv.nz), lv.n_elem, nb, G,        \
      (const s8_t*)tab2, (const s4_t*)tab4, (const s8_t*)lo2, (const s4_t*)lo4, v32, (const float*)u,         \
      (float*)Y)
      if (flavour == MF_BF16X3 && geo) {
#define PMG_L(C) PMG_X(true, true, C)
        PMG_CSW(PMG_L)
#undef PMG_L
      }
      if (colsum) return false;
      if (flavour == MF_BF16X3) {
        PMG_X(true, false, false);
      } else {
        if (geo) PMG_X(false, true, false); else PMG_X(false, false, false);
      }
#undef PMG_X
      return true;
    }
    return false;
  } else {
#define PMG_L(C)                                                                                              \
  launch_batches<KeyOf<PT, PZ, MF_BF16, false, C>>(                                                           \
      k_ax_mfma_bf16<PT, PZ, bf16_t, C>, NT, need, st, lv.map2d, lv.L, int(lv.nz), lv.n_elem, nb,             \
      (const bf16_t*)Gnat, (const s4_t*)tab2, (const s4_t*)tab4, v32, (const float*)u, (float*)Y)
    PMG_CSW(PMG_L)
#undef PMG_L
  }
#undef PMG_CSW
#undef PMG_ARGS
  return false;
}

bool launch_ax_mfma(const LevelView& lv, const void* Gnat, int flavour, const void* tab2, const void* tab4,
                    const void* vmats, const void* u, void* Y, hipStream_t st, const void* tab2lo,
                    const void* tab4lo, const void* geo, bool colsum) {
#define PMG_AXM(PTV, PZV)                                                                                      \
  if (lv.P == PTV && lv.PZ == PZV)                                                                             \
    return ax_mfma_p<PTV, PZV>(lv, Gnat, flavour, tab2, tab4, vmats, u, Y, st, tab2lo, tab4lo, geo, colsum);
  PMG_MFMA_ORDERS(PMG_AXM)
#undef PMG_AXM
  return false;
}

}  // namespace pmg
