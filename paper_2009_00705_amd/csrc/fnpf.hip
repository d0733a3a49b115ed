// Free-surface kernels (see fnpf.hpp).  All streams of n2d-sized vectors;
// the time step is dominated by the Laplace solve.
#include "fnpf.hpp"

namespace pmg {

namespace {
int blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return int(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}
}  // namespace

__global__ __launch_bounds__(256) void k_surf_grad_elem(int nt, int npt, const int32_t* __restrict__ map2d,
                                                        const double* __restrict__ Dr,
                                                        const double* __restrict__ Ds,
                                                        const double* __restrict__ xyt,
                                                        const double* __restrict__ f, double* __restrict__ E2) {
  const int64_t n = int64_t(nt) * npt;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int t = int(i / npt), a = int(i - int64_t(t) * npt);
    const int32_t* m = map2d + size_t(t) * npt;
    const double* X = xyt + size_t(t) * npt * 2;
    double fr = 0, fs = 0, xr = 0, xs = 0, yr = 0, ys = 0;
    for (int b = 0; b < npt; ++b) {
      const double dr = Dr[a * npt + b], ds = Ds[a * npt + b];
      const double fb = f[m[b]], xb = X[2 * b], yb = X[2 * b + 1];
      fr += dr * fb;
      fs += ds * fb;
      xr += dr * xb;
      xs += ds * xb;
      yr += dr * yb;
      ys += ds * yb;
    }
    const double det = xr * ys - xs * yr;
    // (r_x, r_y, s_x, s_y) = (y_s, -x_s, -y_r, x_r) / det
    E2[2 * i] = (fr * ys - fs * yr) / det;
    E2[2 * i + 1] = (-fr * xs + fs * xr) / det;
  }
}

void launch_surf_grad_elem(int nt, int npt, const int32_t* map2d, const double* Dr, const double* Ds,
                           const double* xyt, const double* f, double* E2, hipStream_t st) {
  hipLaunchKernelGGL(k_surf_grad_elem, dim3(blocks(int64_t(nt) * npt)), dim3(256), 0, st, nt, npt, map2d, Dr, Ds,
                     xyt, f, E2);
}

__global__ __launch_bounds__(256) void k_surf_avg(int64_t n2d, const int32_t* __restrict__ inc_ptr,
                                                  const int32_t* __restrict__ inc, const double* __restrict__ E2,
                                                  double* __restrict__ fx, double* __restrict__ fy) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n2d; g += int64_t(gridDim.x) * 256) {
    double sx = 0, sy = 0;
    const int32_t p0 = inc_ptr[g], p1 = inc_ptr[g + 1];
    for (int32_t p = p0; p < p1; ++p) {
      const int64_t e = inc[p];
      sx += E2[2 * e];
      sy += E2[2 * e + 1];
    }
    const double inv = 1.0 / double(p1 - p0);
    fx[g] = sx * inv;
    fy[g] = sy * inv;
  }
}

void launch_surf_avg(int64_t n2d, const int32_t* inc_ptr, const int32_t* inc, const double* E2, double* fx,
                     double* fy, hipStream_t st) {
  hipLaunchKernelGGL(k_surf_avg, dim3(blocks(n2d)), dim3(256), 0, st, n2d, inc_ptr, inc, E2, fx, fy);
}

__global__ __launch_bounds__(256) void k_surf_w(int64_t n2d, int64_t nz, int L, int PZ, double depth,
                                                const double* __restrict__ dtop, const double* __restrict__ phi,
                                                const double* __restrict__ eta, double* __restrict__ w) {
  for (int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x; g < n2d; g += int64_t(gridDim.x) * 256) {
    const double* col = phi + g * nz + int64_t(L - 1) * PZ;
    double d = 0;
    for (int c = 0; c <= PZ; ++c) d += dtop[c] * col[c];
    w[g] = d * (2.0 * L) / (eta[g] + depth);
  }
}

void launch_surf_w(int64_t n2d, int64_t nz, int L, int PZ, double depth, const double* dtop, const double* phi,
                   const double* eta, double* w, hipStream_t st) {
  hipLaunchKernelGGL(k_surf_w, dim3(blocks(n2d)), dim3(256), 0, st, n2d, nz, L, PZ, depth, dtop, phi, eta, w);
}

__global__ __launch_bounds__(256) void k_fnpf_rhs(int64_t n2d, double g, const double* __restrict__ eta,
                                                  const double* __restrict__ ex, const double* __restrict__ ey,
                                                  const double* __restrict__ px, const double* __restrict__ py,
                                                  const double* __restrict__ w, double* __restrict__ deta,
                                                  double* __restrict__ dphis) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n2d; i += int64_t(gridDim.x) * 256) {
    const double s = 1.0 + ex[i] * ex[i] + ey[i] * ey[i];
    const double wi = w[i];
    deta[i] = -(ex[i] * px[i] + ey[i] * py[i]) + wi * s;
    dphis[i] = -g * eta[i] - 0.5 * ((px[i] * px[i] + py[i] * py[i]) - wi * wi * s);
  }
}

void launch_fnpf_rhs(int64_t n2d, double g, const double* eta, const double* ex, const double* ey, const double* px,
                     const double* py, const double* w, double* deta, double* dphis, hipStream_t st) {
  hipLaunchKernelGGL(k_fnpf_rhs, dim3(blocks(n2d)), dim3(256), 0, st, n2d, g, eta, ex, ey, px, py, w, deta, dphis);
}

__global__ __launch_bounds__(256) void k_lin_extrap(int64_t n, const double* a, const double* b, double* out) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double v = 2.0 * a[i] - b[i];
    out[i] = v;
  }
}

void launch_lin_extrap(int64_t n, const double* a, const double* b, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_lin_extrap, dim3(blocks(n)), dim3(256), 0, st, n, a, b, out);
}

__global__ __launch_bounds__(256) void k_rk_stage(int64_t n, const double* __restrict__ y0,
                                                  const double* __restrict__ k, double a, double* __restrict__ ys,
                                                  double b, int first, double* __restrict__ acc) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double ki = k[i];
    if (ys) ys[i] = y0[i] + a * ki;
    acc[i] = (first ? 0.0 : acc[i]) + b * ki;
  }
}

void launch_rk_stage(int64_t n, const double* y0, const double* k, double a, double* ys, double b, bool first,
                     double* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_rk_stage, dim3(blocks(n)), dim3(256), 0, st, n, y0, k, a, ys, b, int(first), acc);
}

}  // namespace pmg
