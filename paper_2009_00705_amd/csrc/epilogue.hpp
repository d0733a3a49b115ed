// Node epilogues of the direct-stiffness sum (Sec. 3.1: the global operator is
// the sum over elements of the element contributions at each global node).
// One definition serves the node-centric summation kernel (k_assemble) and the
// node kernel of the column-sum layout (k_col_sum), so both apply the same
// arithmetic to a node's sum s.  The vectors an epilogue reads are loaded by
// node_in before the node's gather starts (their reads are then in flight
// together with it); node_epilogue computes and stores.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace pmg {

// y = node value of A x; dir = Dirichlet node (corrections there are zero).
//   OP_RAW       out = s
//   OP_STORE     out = mask s
//   OP_RESID     out = mask (a1 - s)
//   OP_JACOBI    out += omega a2 (a1 - s)              (a2 = masked D^-1)
//   OP_STORE_DOT out = mask s; acc += a1 out
//   OP_CHEB0     a4 = r = mask (a1 - s); a3 = d = c1 a2 r; out += d
//   OP_CHEB      r = a1 (in/out): r -= s; d = a3 = omega d + c1 a2 r; out += d
template <typename T> struct NodeIn {
  T a1, a2, a3, o;
};
template <typename T, int OP>
__device__ __forceinline__ NodeIn<T> node_in(uint64_t g, const T* __restrict__ out, const T* __restrict__ a1,
                                             const T* __restrict__ a2, const T* __restrict__ a3) {
  NodeIn<T> v{T(0), T(0), T(0), T(0)};
  if constexpr (OP == OP_RESID || OP == OP_STORE_DOT || OP == OP_JACOBI || OP == OP_CHEB0 || OP == OP_CHEB)
    v.a1 = a1[g];
  if constexpr (OP == OP_JACOBI || OP == OP_CHEB0 || OP == OP_CHEB) v.a2 = a2[g];
  if constexpr (OP == OP_JACOBI || OP == OP_CHEB0 || OP == OP_CHEB || OP == OP_AVG_ADD) v.o = out[g];
  if constexpr (OP == OP_CHEB) v.a3 = a3[g];
  return v;
}
template <typename T, int OP>
__device__ __forceinline__ void node_epilogue(uint64_t g, bool dir, T s, const NodeIn<T>& in, T* __restrict__ out,
                                              T* __restrict__ r, T* __restrict__ a3, T* __restrict__ a4, T omega,
                                              T c1, double& acc) {
  if constexpr (OP == OP_RAW) {
    out[g] = s;
  } else if constexpr (OP == OP_STORE) {
    out[g] = dir ? T(0) : s;
  } else if constexpr (OP == OP_RESID) {
    out[g] = dir ? T(0) : in.a1 - s;
  } else if constexpr (OP == OP_JACOBI) {
    if (!dir) out[g] = in.o + omega * in.a2 * (in.a1 - s);
  } else if constexpr (OP == OP_STORE_DOT) {
    const T v = dir ? T(0) : s;
    out[g] = v;
    acc += double(in.a1) * double(v);
  } else if constexpr (OP == OP_CHEB0) {
    const T rn = dir ? T(0) : in.a1 - s;
    a4[g] = rn;
    const T dn = c1 * in.a2 * rn;
    a3[g] = dn;
    out[g] = in.o + dn;
  } else if constexpr (OP == OP_CHEB) {
    if (!dir) {
      const T rn = in.a1 - s;
      r[g] = rn;
      const T dn = omega * in.a3 + c1 * in.a2 * rn;
      a3[g] = dn;
      out[g] = in.o + dn;
    }
  }
}

// Shared slot of local triangle node a (Blyth-Pozrikidis order: j outer
// 0..P, i inner 0..P-j) on the triangle's boundary: 0..P along j = 0, P+1..2P
// along i + j = P (j = 1..P), 2P+1..3P-1 along i = 0 (j = P-1..1); -1 for
// nodes inside the triangle, which no other triangle holds.
__host__ __device__ inline int tri_slot_of(int a, int P) {
  int j = 0, rem = a;
  while (rem > P - j) {
    rem -= P - j + 1;
    ++j;
  }
  const int i = rem;
  if (j == 0) return i;
  if (i + j == P) return P + j;
  if (i == 0) return 3 * P - j;
  return -1;
}
template <int P>
__device__ __forceinline__ int tri_slot(int a) {
  int j = 0, rem = a;
#pragma unroll
  for (int jj = 0; jj < P; ++jj)
    if (rem > P - j) {
      rem -= P - j + 1;
      ++j;
    }
  const int i = rem;
  if (j == 0) return i;
  if (i + j == P) return P + j;
  if (i == 0) return 3 * P - j;
  return -1;
}

// Column-sum code of local node a: its boundary slot s >= 0 (tri_slot), or
// -1 - rank for a node inside the triangle, rank = its index among the interior
// nodes in the same (j outer, i inner) order, which is the order of the global
// numbering of triangle-interior nodes.
__host__ __device__ inline int tri_code_of(int a, int P) {
  const int s = tri_slot_of(a, P);
  if (s >= 0) return s;
  int j = 0, rem = a;
  while (rem > P - j) {
    rem -= P - j + 1;
    ++j;
  }
  // rows 1 .. j-1 hold P - j' - 1 interior nodes each; node i of row j is the (i-1)-th
  const int before = (j - 1) * (P - 1) - (j - 1) * j / 2;
  return -1 - (before + rem - 1);
}
template <int P>
__device__ __forceinline__ int tri_code(int a) {
  return tri_code_of(a, P);
}

}  // namespace pmg
