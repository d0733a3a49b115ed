// Reference prism (host, FP64).  See refelem.hpp.
#include "refelem.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace pmg {

Mat matmul(const Mat& a, const Mat& b) {
  if (a.cols != b.rows) throw std::runtime_error("matmul: shape");
  Mat c(a.rows, b.cols);
  for (int i = 0; i < a.rows; ++i)
    for (int k = 0; k < a.cols; ++k) {
      const double aik = a(i, k);
      if (aik == 0.0) continue;
      for (int j = 0; j < b.cols; ++j) c(i, j) += aik * b(k, j);
    }
  return c;
}

Mat inverse(const Mat& a) {
  const int n = a.rows;
  if (a.cols != n) throw std::runtime_error("inverse: not square");
  Mat m = a, inv(n, n);
  for (int i = 0; i < n; ++i) inv(i, i) = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(m(r, col)) > std::fabs(m(piv, col))) piv = r;
    if (m(piv, col) == 0.0) throw std::runtime_error("inverse: singular");
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(m(piv, j), m(col, j));
        std::swap(inv(piv, j), inv(col, j));
      }
    const double d = 1.0 / m(col, col);
    for (int j = 0; j < n; ++j) { m(col, j) *= d; inv(col, j) *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = m(r, col);
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { m(r, j) -= f * m(col, j); inv(r, j) -= f * inv(col, j); }
    }
  }
  return inv;
}

// ---------------------------------------------------------------------------
// Jacobi polynomials P_n^(al,be) by the three-term recurrence.
// ---------------------------------------------------------------------------
static double jacobi(int n, double al, double be, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * (al - be) + 0.5 * (al + be + 2.0) * x;
  for (int m = 2; m <= n; ++m) {
    const double s = 2.0 * m + al + be;
    const double a1 = 2.0 * m * (m + al + be) * (s - 2.0);
    const double a2 = (s - 1.0) * (al * al - be * be);
    const double a3 = (s - 2.0) * (s - 1.0) * s;
    const double a4 = 2.0 * (m + al - 1.0) * (m + be - 1.0) * s;
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}
static double jacobi_d(int n, double al, double be, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + al + be + 1.0) * jacobi(n - 1, al + 1.0, be + 1.0, x);
}
// squared norm of P_n^(al,be) under its weight
static double jacobi_norm2(int n, double al, double be) {
  return std::pow(2.0, al + be + 1.0) / (2.0 * n + al + be + 1.0) * std::tgamma(n + al + 1.0) *
         std::tgamma(n + be + 1.0) / (std::tgamma(n + al + be + 1.0) * std::tgamma(n + 1.0));
}

// Roots of P_n^(al,be) by Newton with deflation from Chebyshev guesses.
static std::vector<double> jacobi_roots(int n, double al, double be) {
  std::vector<double> x(n);
  for (int i = 0; i < n; ++i) {
    double z = -std::cos((2.0 * i + 1.0) * M_PI / (2.0 * n));
    if (i > 0) z = 0.5 * (z + x[i - 1]);
    for (int it = 0; it < 100; ++it) {
      double defl = 0.0;
      for (int j = 0; j < i; ++j) defl += 1.0 / (z - x[j]);
      const double f = jacobi(n, al, be, z), fd = jacobi_d(n, al, be, z);
      const double dz = f / (fd - f * defl);
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  std::sort(x.begin(), x.end());
  // final polish without deflation
  for (double& z : x)
    for (int it = 0; it < 3; ++it) {
      const double fd = jacobi_d(n, al, be, z);
      if (fd != 0.0) z -= jacobi(n, al, be, z) / fd;
    }
  return x;
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x = jacobi_roots(n, 0.0, 0.0);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    const double d = jacobi_d(n, 0.0, 0.0, x[i]);
    w[i] = 2.0 / ((1.0 - x[i] * x[i]) * d * d);
  }
}

void gauss_jacobi10(int n, std::vector<double>& x, std::vector<double>& w) {
  x = jacobi_roots(n, 1.0, 0.0);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    const double d = jacobi_d(n, 1.0, 0.0, x[i]);
    w[i] = 4.0 / ((1.0 - x[i] * x[i]) * d * d);
  }
}

std::vector<double> lgl_nodes(int P) {
  std::vector<double> x(P + 1);
  if (P == 0) { x[0] = 0.0; return x; }
  x[0] = -1.0;
  x[P] = 1.0;
  if (P >= 2) {
    // interior LGL nodes are the roots of P_P' ~ P_{P-1}^(1,1)
    std::vector<double> in = jacobi_roots(P - 1, 1.0, 1.0);
    for (int i = 1; i < P; ++i) x[i] = in[i - 1];
  }
  return x;
}

void legendre_basis(int P, const std::vector<double>& x, Mat& V, Mat& Vx) {
  const int m = int(x.size());
  V = Mat(m, P + 1);
  Vx = Mat(m, P + 1);
  for (int n = 0; n <= P; ++n) {
    const double s = 1.0 / std::sqrt(jacobi_norm2(n, 0.0, 0.0));
    for (int i = 0; i < m; ++i) {
      V(i, n) = jacobi(n, 0.0, 0.0, x[i]) * s;
      Vx(i, n) = jacobi_d(n, 0.0, 0.0, x[i]) * s;
    }
  }
}

void pkd_basis(int P, const std::vector<double>& r, const std::vector<double>& s, Mat& V,
               Mat& Vr, Mat& Vs) {
  const int m = int(r.size());
  const int nm = (P + 1) * (P + 2) / 2;
  V = Mat(m, nm);
  Vr = Mat(m, nm);
  Vs = Mat(m, nm);
  for (int p = 0; p < m; ++p) {
    const double om = 1.0 - s[p];
    const bool top = std::fabs(om) < 1e-14;
    const double a = top ? -1.0 : 2.0 * (1.0 + r[p]) / om - 1.0;
    const double b = s[p];
    int col = 0;
    for (int i = 0; i <= P; ++i) {
      const double ni = 1.0 / std::sqrt(jacobi_norm2(i, 0.0, 0.0));
      const double f = jacobi(i, 0.0, 0.0, a) * ni;
      const double fd = jacobi_d(i, 0.0, 0.0, a) * ni;
      const double pw = std::pow(1.0 - b, i);
      const double pwm1 = i >= 1 ? std::pow(1.0 - b, i - 1) : 0.0;
      for (int j = 0; j + i <= P; ++j) {
        const double al = 2.0 * i + 1.0;
        const double nj = 1.0 / std::sqrt(jacobi_norm2(j, al, 0.0));
        const double g = jacobi(j, al, 0.0, b) * nj;
        const double gd = jacobi_d(j, al, 0.0, b) * nj;
        V(p, col) = M_SQRT2 * f * g * pw;
        Vr(p, col) = M_SQRT2 * 2.0 * fd * g * pwm1;
        Vs(p, col) = M_SQRT2 * (fd * (1.0 + a) * g * pwm1 + f * gd * pw - i * f * g * pwm1);
        ++col;
      }
    }
  }
}

std::vector<Ijk> tri_lattice(int P) {
  std::vector<Ijk> out;
  for (int j = 0; j <= P; ++j)
    for (int i = 0; i + j <= P; ++i) out.push_back({i, j, P - i - j});
  return out;
}

RefElem::RefElem(int P_, int PZ_) : P(P_), PZ(PZ_ < 0 ? P_ : PZ_) {
  if (P < 1 || P > 8 || PZ < 1 || PZ > 8) throw std::runtime_error("order must be in [1, 8]");
  const int m1 = P + 1;  // 1D points of the triangle order
  n1 = PZ + 1;
  np_tri = (P + 1) * (P + 2) / 2;
  np = np_tri * n1;
  nq_tri = m1 * m1;
  nq = nq_tri * n1;
  // triangle nodes from the LGL nodes (closed form of Blyth & Pozrikidis)
  const std::vector<double> tl = lgl_nodes(P);
  std::vector<double> v(m1);
  for (int i = 0; i < m1; ++i) v[i] = 0.5 * (1.0 + tl[i]);
  for (const Ijk& l : tri_lattice(P)) {
    const double x = (1.0 + 2.0 * v[l.i] - v[l.j] - v[l.k]) / 3.0;
    const double y = (1.0 + 2.0 * v[l.j] - v[l.i] - v[l.k]) / 3.0;
    r.push_back(2.0 * x - 1.0);
    s.push_back(2.0 * y - 1.0);
  }
  Mat V, Vr, Vs;
  pkd_basis(P, r, s, V, Vr, Vs);
  Vinv = inverse(V);
  // vertical LGL nodes of order PZ
  t = lgl_nodes(PZ);
  Mat V1, V1x;
  legendre_basis(PZ, t, V1, V1x);
  V1inv = inverse(V1);
  // collapsed cubature: GL in a, GJ(1,0) in b
  std::vector<double> a, wa, b, wb;
  gauss_legendre(m1, a, wa);
  gauss_jacobi10(m1, b, wb);
  for (int j = 0; j < m1; ++j)
    for (int i = 0; i < m1; ++i) {
      cr.push_back(0.5 * (1.0 + a[i]) * (1.0 - b[j]) - 1.0);
      cs.push_back(b[j]);
      cw.push_back(0.5 * wa[i] * wb[j]);
    }
  gauss_legendre(n1, zq, zw);
  tri_eval(cr, cs, B, Dr, Ds);
  line_eval(zq, Bz, Dz);
}

void RefElem::tri_eval(const std::vector<double>& pr, const std::vector<double>& ps, Mat& Bo,
                       Mat& Dro, Mat& Dso) const {
  Mat V, Vr, Vs;
  pkd_basis(P, pr, ps, V, Vr, Vs);
  Bo = matmul(V, Vinv);
  Dro = matmul(Vr, Vinv);
  Dso = matmul(Vs, Vinv);
}

void RefElem::line_eval(const std::vector<double>& pt, Mat& Bo, Mat& Do) const {
  Mat V, Vx;
  legendre_basis(PZ, pt, V, Vx);
  Bo = matmul(V, V1inv);
  Do = matmul(Vx, V1inv);
}

}  // namespace pmg
