// Free-surface time stepping of the FNPF equations (eq. FSeta, eq. FSphi)
// around the Laplace solve: surface gradients, the vertical velocity w~ at
// the surface, the pointwise right-hand side and the Runge-Kutta stage
// combinations (all FP64, device memory, enqueued on the given stream).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmg {

// E2[t][a][2] = (df/dx, df/dy) at node a of triangle t: derivatives of the
// order-P interpolant (Dr, Ds: npt x npt nodal differentiation matrices)
// through the isoparametric map of the triangle nodes xyt[t][a][2].
void launch_surf_grad_elem(int nt, int npt, const int32_t* map2d, const double* Dr, const double* Ds,
                           const double* xyt, const double* f, double* E2, hipStream_t st);
// fx[g], fy[g]: average of E2 over the incidences (t*npt + a) of 2D node g.
void launch_surf_avg(int64_t n2d, const int32_t* inc_ptr, const int32_t* inc, const double* E2, double* fx,
                     double* fy, hipStream_t st);
// w[g] = (sum_c dtop[c] phi[g*nz + (L-1)*PZ + c]) * 2L / (eta[g] + depth).
void launch_surf_w(int64_t n2d, int64_t nz, int L, int PZ, double depth, const double* dtop, const double* phi,
                   const double* eta, double* w, hipStream_t st);
// eq. FSeta and eq. FSphi pointwise.
void launch_fnpf_rhs(int64_t n2d, double g, const double* eta, const double* ex, const double* ey, const double* px,
                     const double* py, const double* w, double* deta, double* dphis, hipStream_t st);
// out = 2 a - b (n entries; out may be a or b).
void launch_lin_extrap(int64_t n, const double* a, const double* b, double* out, hipStream_t st);
// ys = y0 + a k; acc = (first ? 0 : acc) + b k (n entries).
void launch_rk_stage(int64_t n, const double* y0, const double* k, double a, double* ys, double b, bool first,
                     double* acc, hipStream_t st);

}  // namespace pmg
