// Reference prism of order P (host, FP64): 1D rules, triangle nodes,
// orthonormal triangle basis, collapsed cubature and the nodal
// interpolation/derivative matrices used by the device kernels.
//
// Sec. 3.1 of the paper: V^p is spanned by a cardinal nodal basis; LGL nodes
// sit on element edges (Fig. pcoarse).  Local node n = c*Np_tri + a pairs the
// vertical LGL node c with triangle node a; cubature point k*Nq_tri + q pairs
// a vertical Gauss point with a collapsed triangle point q = j*(P+1) + i.
#pragma once
#include <vector>

namespace pmg {

// Dense row-major matrix helper.
struct Mat {
  int rows = 0, cols = 0;
  std::vector<double> v;
  Mat() = default;
  Mat(int r, int c) : rows(r), cols(c), v(size_t(r) * c, 0.0) {}
  double& operator()(int i, int j) { return v[size_t(i) * cols + j]; }
  double operator()(int i, int j) const { return v[size_t(i) * cols + j]; }
};

Mat matmul(const Mat& a, const Mat& b);
Mat inverse(const Mat& a);  // Gauss-Jordan with partial pivoting

// 1D rules on [-1, 1]
std::vector<double> lgl_nodes(int P);                       // P+1 nodes
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void gauss_jacobi10(int n, std::vector<double>& x, std::vector<double>& w);  // weight (1-x)

// Orthonormal Legendre (1D) and PKD (triangle) bases at given points.
void legendre_basis(int P, const std::vector<double>& x, Mat& V, Mat& Vx);
void pkd_basis(int P, const std::vector<double>& r, const std::vector<double>& s,
               Mat& V, Mat& Vr, Mat& Vs);

// Lattice (i,j,k) of local triangle node a, order j outer, i inner.
struct Ijk { int i, j, k; };
std::vector<Ijk> tri_lattice(int P);

// Order P on the triangle and PZ (default P) along the extrusion: n1 = PZ + 1
// vertical nodes and Gauss points, (P+1)^2 triangle cubature points.
struct RefElem {
  int P = 0, PZ = 0, n1 = 0, np_tri = 0, np = 0, nq_tri = 0, nq = 0;
  std::vector<double> r, s, t;      // triangle nodes (r,s), vertical LGL t
  std::vector<double> cr, cs, cw;   // triangle cubature points / weights
  std::vector<double> zq, zw;       // vertical Gauss points / weights
  Mat Vinv, V1inv;                  // inverse Vandermonde matrices
  Mat B, Dr, Ds;                    // Nq_tri x Np_tri at own cubature
  Mat Bz, Dz;                       // n1 x n1 at own Gauss points
  explicit RefElem(int P, int PZ = -1);
  // Order-P nodal triangle basis (and r,s-derivatives) at arbitrary points.
  void tri_eval(const std::vector<double>& pr, const std::vector<double>& ps,
                Mat& Bo, Mat& Dro, Mat& Dso) const;
  // Order-PZ nodal 1D basis (and derivative) at arbitrary points.
  void line_eval(const std::vector<double>& pt, Mat& Bo, Mat& Do) const;
};

}  // namespace pmg
