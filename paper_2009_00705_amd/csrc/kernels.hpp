// Launchers of the device kernels (gfx950).  Every pointer is device memory
// unless stated; every launch is enqueued on the given stream.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace pmg {

typedef uint16_t bf16_t;  // bfloat16 storage (upper half of an IEEE float)

enum GStore { G_F64 = 0, G_F32 = 1, G_BF16 = 2 };

// Reduction buffer: fixed grid so the summation order never changes.
constexpr int RED_BLOCKS = 4096;

// Scalar slots of the Krylov loop (device double array of size N_SCAL).
enum Scal {
  S_DELTA = 0, S_PQ, S_ALPHA, S_RR, S_ZR, S_BETA, S_FF, S_TMP0, S_TMP1, S_ZRO, S_NF, N_SCAL = 16
};

// (triangle order, vertical order) of the levels the library builds: the
// isotropic orders, the in-plane-first chains (P, P) -> (P/2, P) -> ... ->
// (1, P) -> (1, P/2) -> ... -> (1, 1) of every fine order up to 8, and the
// anisotropic finest levels of the equal-order chains (4,2), (5,3), (6,4)
#define PMG_ORDERS(X)                                                                                \
  X(1, 1) X(2, 2) X(3, 3) X(4, 4) X(5, 5) X(6, 6) X(7, 7) X(8, 8) X(1, 2) X(1, 3) X(1, 4) X(1, 5) \
  X(1, 6) X(1, 7) X(1, 8) X(2, 4) X(2, 5) X(2, 8) X(3, 6) X(3, 7) X(4, 8) X(4, 2) X(5, 3) X(6, 4)
// consecutive level pairs (fine PT, PZ, coarse PT, PZ) of the coarsening sequences:
// all directions, in-plane first, and equal-order (semi-coarsening of the
// higher order until the two agree, then both)
#define PMG_PAIRS(X)                                                                                 \
  X(2, 2, 1, 1) X(3, 3, 1, 1) X(4, 4, 2, 2) X(5, 5, 2, 2) X(6, 6, 3, 3) X(7, 7, 3, 3) X(8, 8, 4, 4) \
  X(2, 2, 1, 2) X(1, 2, 1, 1) X(3, 3, 1, 3) X(1, 3, 1, 1) X(4, 4, 2, 4) X(2, 4, 1, 4) X(1, 4, 1, 2) \
  X(5, 5, 2, 5) X(2, 5, 1, 5) X(1, 5, 1, 2) X(6, 6, 3, 6) X(3, 6, 1, 6) X(1, 6, 1, 3) X(7, 7, 3, 7) \
  X(3, 7, 1, 7) X(1, 7, 1, 3) X(8, 8, 4, 8) X(4, 8, 2, 8) X(2, 8, 1, 8) X(1, 8, 1, 4)               \
  X(4, 2, 2, 2) X(5, 3, 3, 3) X(6, 4, 4, 4) X(2, 4, 2, 2) X(3, 6, 3, 3) X(4, 8, 4, 4)

// whether the element kernels exist for a level order / the transfers for a pair
bool order_supported(int PT, int PZ);
bool pair_supported(int PFT, int PFZ, int PCT, int PCZ);

// ---- direct-stiffness sum of an E-layout vector (atomic-free, node-centric)
enum AsmOp {
  OP_STORE = 0,     // out = mask * sum
  OP_AVG_ADD = 1,   // out += mask * sum / multiplicity
  OP_RESID = 2,     // out = mask * (a1 - sum)
  OP_JACOBI = 3,    // out += omega * a2 * (a1 - sum)      (a2 = masked D^-1)
  OP_STORE_DOT = 4, // out = mask * sum; partial += a1 . out
  OP_AVG_STORE = 5, // out = mask * sum / multiplicity
  OP_CHEB = 6,      // Chebyshev step on (x=out, r=a1, d=a3): r -= sum; x += d_new ...
  OP_RAW = 7,       // out = sum (no mask)
  OP_AVG_RAW = 8,   // out = sum / multiplicity (no mask)
  OP_CHEB0 = 9      // first Chebyshev step from x = out: a4 = r = mask (a1 - sum), a3 = d = c1 a2 r, x += d
};

// Per-level device description.
struct LevelView {
  int P, PZ, L, nt;        // P: triangle order, PZ: vertical order
  int np_tri, np, nq;
  int64_t n2d, nz, n_dof, n_elem;
  const int32_t* map2d;    // [nt][np_tri]
  const int32_t* inc_ptr;  // [n2d+1]
  const int32_t* inc;      // [nnz] = t*np_tri + a
  const uint8_t* dir2d;    // [n2d] lateral Dirichlet columns
  int top_dir;             // surface nodes are Dirichlet
  // Column-sum layout (launch_col_sum): 2D ids below n_bnd are vertices and
  // edge nodes (on triangle boundaries), those from n_bnd on are triangle
  // interiors, nint per triangle in triangle order.  sh_ptr/sh_idx: for every
  // 2D node below n_bnd the boundary slots t*3P + s of the triangles holding
  // it, in ascending triangle order.  colsum: this level's numbering has that
  // form and L divides 16 (the MFMA operators can write column sums).
  int64_t n_bnd;
  int nint;
  const int32_t* sh_ptr;   // [n_bnd+1]
  const int32_t* sh_idx;   // [sh_ptr[n_bnd]] = t*3P + s
  int colsum;
  // Coloured direct-stiffness sum (launch_dss): the triangles grouped by
  // colour (no two of one colour share a vertex), ascending within a colour.
  const int32_t* tcol_list;  // [nt]
};

// Coloured direct-stiffness sum (alternative to launch_assemble, same ops and
// arguments): S (an L-vector of zeros) += the element values of every
// triangle column, one launch per triangle colour (ranges tcol_ptr of
// lv.tcol_list, host), thread per (triangle, node a, z) with z fastest: no two
// triangles of a colour share a node, so the adds need no atomics and every
// node sums its triangles in colour order.  Then one pass per node applies
// the epilogue op to S and puts the zeros back.
template <typename T>
void launch_dss(const LevelView& lv, const std::vector<int64_t>& tcol_ptr, int op, const T* Y, T* S, T* out,
                const T* a1, const T* a2, T* a3, double omega, double c1, double* partial, hipStream_t st,
                T* a4 = nullptr);

// Direct-stiffness sum from column sums.  A batch of 16 prisms holds 16/L whole
// triangle columns (L divides 16), so the element operator sums each column's
// layers itself and writes one value per (triangle, local node, z): at the
// nint interior nodes of triangle t to cv[(t nint + rank) nz + z] (the 2D node
// n_bnd + t nint + rank, so this part of cv is in global-vector order), at the
// 3P boundary nodes to cv[nt nint nz + (t 3P + s) nz + z] (s: tri_slot).  The
// node kernel then reads an interior node's value directly and sums a boundary
// node's slots over the triangles holding it (ascending triangle order), and
// applies the node epilogue op.  No atomics; every sum has a fixed order.
template <typename T>
void launch_col_sum(const LevelView& lv, int op, const T* cv, T* out, const T* a1, const T* a2, T* a3,
                    double omega, double c1, double* partial, hipStream_t st, T* a4 = nullptr);

// ---- element operator: Y_E = blockdiag(A_e) Q u (E-layout [t][a][layer][c])
template <typename T>
void launch_ax(const LevelView& lv, const T* mats, const void* G, int gstore, const T* u, T* Y,
               hipStream_t st);

template <typename T>
void launch_assemble(const LevelView& lv, int op, const T* Y, T* out, const T* a1, const T* a2,
                     T* a3, double omega, double c1, double* partial, hipStream_t st, T* a4 = nullptr);

// ---- geometric factors at level cubature from the fine isoparametric map
// G64/G32/G16: G[e][m][k*nqt+q] (any may be null).  geo64/geo32 (may be null):
// the column factors geo[t][q][0..7] of the sigma-transformed prism, from
// which G at vertical Gauss point k of layer l follows as
//   G = zw_k (B0, B1, s B2, B3, s B4, s^2 B5 + B6),  s = (l + (1+zq_k)/2) / L
// (slot 7 is zero).
void launch_geom(const LevelView& fine, const LevelView& lvl, double depth, const double* xyt,
                 const double* eta, const double* gmats, const double* wq, const double* zq,
                 const double* zw, double* G64, float* G32, bf16_t* G16, int* bad, hipStream_t st,
                 double* geo64 = nullptr, float* geo32 = nullptr);

// ---- diagonal of the element matrices (E-layout), FP64: from the standard G, or
// from the column factors of launch_geom (zq, zw: vertical Gauss rule)
void launch_diag(const LevelView& lv, const double* mats, const double* G64, double* Y, hipStream_t st);
void launch_diag_col(const LevelView& lv, const double* mats, const double* zq, const double* zw, const double* geo,
                     double* Y, hipStream_t st);

// ---- transfers between level f and the next coarser level c (E-layout output)
template <typename T>
void launch_prolong_elem(const LevelView& f, const LevelView& c, const T* pit, const T* piz,
                         const T* uc, T* Yf, hipStream_t st);
template <typename T>
void launch_restrict_elem(const LevelView& f, const LevelView& c, const T* pit, const T* piz,
                          const T* rf, T* Yc, hipStream_t st);
// Node-wise prolongation straight to the fine nodes (op: OP_AVG_ADD, OP_AVG_STORE
// or OP_AVG_RAW on the prolongated value) for level pairs where the triangle or
// the vertical order is kept; returns false, launching nothing, otherwise.
template <typename T>
bool launch_prolong_node(const LevelView& f, const LevelView& c, const T* pit, const T* piz, const T* uc, T* out,
                         int op, hipStream_t st);

// ---- coarse exact solve: y[idx[i]] = sum_j Ainv[i][j] x[idx[j]], y zero elsewhere
template <typename T>
void launch_coarse_dense(int n, const int32_t* idx, const T* Ainv, const T* x, T* y, T* tmp,
                         int64_t n_dof, hipStream_t st);

// assembled P = 1 operator for the coarse Chebyshev solve
void launch_p1_elem_mat(int64_t n_elem, const double* G, const double* Dref, double* Ae, hipStream_t st);
// ELL values (n rows, w slots, slot-major) of the CSR pattern rp whose nonzero j
// sums the element entries Ae[cl[cp[j] .. cp[j+1])]
void launch_ell_sum(int64_t n, int w, const int32_t* rp, const int32_t* cp, const int64_t* cl, const double* Ae,
                    double* v64, float* v32, hipStream_t st);
template <typename T>
void launch_cheb_start(int64_t n, const T* f, const T* dinv, T* r, T* d, T* x, double inv_theta, hipStream_t st);
template <typename T>
void launch_cheb_ell(int64_t n, int w, const int32_t* ci, const T* val, const T* dinv, const T* d_old, T* d_new,
                     T* r, T* x, double c0, double c1, hipStream_t st);

// ---- vector kernels
template <typename T> void launch_fill(T* x, T v, int64_t n, hipStream_t st);
template <typename T> void launch_copy(const T* x, T* y, int64_t n, hipStream_t st);
template <typename T>  // y = omega * d .* x
void launch_scale_diag(const T* d, const T* x, T* y, double omega, int64_t n, hipStream_t st);
template <typename Ts, typename Td>  // y = (Td)(x * scale)
void launch_cast(const Ts* x, Td* y, double scale, int64_t n, hipStream_t st);
template <typename T>  // partial[b] = sum x.y
void launch_dot(const T* x, const T* y, int64_t n, double* partial, hipStream_t st);
template <typename T>
void launch_dinv(const LevelView& lv, const T* diag_src_unused, const double* diag, T* dinv,
                 hipStream_t st);

// finalize: reduce partial into scal[slot] (optionally sets derived scalars)
enum FinOp { FIN_SET = 0, FIN_ALPHA = 1, FIN_BETA_FR = 2, FIN_BETA_PR = 3, FIN_DELTA = 4 };
void launch_finalize(const double* partial, double* scal, int slot, int op, hipStream_t st);

// PCG vector updates (FP64)
// u += alpha p; r -= alpha q; partial = ||r||^2    (alpha = scal[S_ALPHA]);
// r32 (optional) = float(r), the input of a low-precision V-cycle
void launch_cg_update(double* u, double* r, const double* p, const double* q, const double* scal,
                      double* partial, int64_t n, hipStream_t st, float* r32 = nullptr);
// p = z + beta p (beta = scal[S_BETA]); z FP64 or the FP32 V-cycle output
void launch_cg_dir(double* p, const double* z, const double* scal, int64_t n, hipStream_t st);
void launch_cg_dir(double* p, const float* z, const double* scal, int64_t n, hipStream_t st);
// u += z ; partial of nothing
void launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st);
// r = f - y (masked by a2 != 0 when mask given) ; partial ||r||^2
void launch_resid_norm(double* r, const double* f, const double* y, double* partial, int64_t n,
                       hipStream_t st);
// Dirichlet lifting: phiD at Dirichlet nodes from surf (per 2D node) or bc (full), zero elsewhere
void launch_lift(const LevelView& lv, const double* surf, const double* bc, double* phiD,
                 hipStream_t st);
// out = where(free, a, b)
void launch_merge_free(const LevelView& lv, const double* a, const double* b, double* out,
                       hipStream_t st);
// partial[0..RED_BLOCKS) = x.y1, partial[RED_BLOCKS..) = x.y2 (x FP64 or FP32, in FP64)
void launch_dot2(const double* x, const double* y1, const double* y2, int64_t n, double* partial,
                 hipStream_t st);
void launch_dot2(const float* x, const double* y1, const double* y2, int64_t n, double* partial,
                 hipStream_t st);
// y += a x
template <typename T> void launch_axpy_t(T* y, const T* x, double a, int64_t n, hipStream_t st);
// p = z + beta p (beta from the host)
void launch_xpay(double* p, const double* z, double beta, int64_t n, hipStream_t st);
// out = x on free nodes, 0 on Dirichlet nodes
template <typename T> void launch_mask(const LevelView& lv, const T* x, T* out, hipStream_t st);
// non-finite count into partial (as double)
void launch_count_nonfinite(const double* x, int64_t n, double* partial, hipStream_t st);

}  // namespace pmg
