// libpmg: host orchestration and C-ABI (see include/pmg.h).
//
// The context owns, per level l (order P_l = P, floor(P/2), ..., 1 on one
// mesh, Sec. 5): numbering and incidence lists, reference matrices, the
// geometric factors G_l (FP64 plus FP32 and BF16 copies for the mixed
// preconditioner), the Jacobi diagonal, the transfer matrices to level l+1,
// and work vectors.  The V-cycle follows Alg. 1; the outer iterations follow
// Alg. 2 and Alg. 3 of the paper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <fstream>
#include <cmath>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "kernels_mfma.hpp"
#include "mlp.hpp"
#include "mesh.hpp"
#include "pmg.h"
#include "refelem.hpp"
#include "schwarz.hpp"
#include "epilogue.hpp"
#include "fnpf.hpp"

namespace pmg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      throw Error(e_ == hipErrorOutOfMemory ? PMG_ENOMEM : PMG_EDEVICE,                        \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                          \
  } while (0)

template <typename T>
static T* dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  HIPCHK(hipMalloc(&p, n * sizeof(T)));
  return static_cast<T*>(p);
}
template <typename T>
static T* dupload(const std::vector<T>& h) {
  T* p = dalloc<T>(h.size());
  if (!h.empty()) HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}
static std::vector<float> to_f32(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

// splitmix64 counter generator: unit(i) = top 53 bits of splitmix64(seed + (i+1)*golden)
static double splitmix_unit(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return double(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Level {
  int P = 0, PZ = 0;  // triangle and vertical order
  std::unique_ptr<RefElem> re;
  Numbering num;
  std::vector<uint8_t> dir2d_h;
  int64_t n_free = 0;
  int top_dir = 1;
  // device
  int32_t *map2d = nullptr, *inc_ptr = nullptr, *inc = nullptr;
  int32_t *sh_ptr = nullptr, *sh_idx = nullptr;  // boundary nodes of the column-sum path
  std::vector<int64_t> tcol_ptr;                  // coloured sum: colour ranges of tcol_list (host)
  int32_t* tcol_list = nullptr;                   // triangles grouped by colour (device)
  int64_t n_bnd = 0;
  int nint = 0, colsum = 0;
  uint8_t* dir2d = nullptr;
  double* mats64 = nullptr;
  float* mats32 = nullptr;
  double *gmats = nullptr, *wq = nullptr, *zq = nullptr, *zw = nullptr;
  double* G64 = nullptr;
  float* G32 = nullptr;
  bf16_t* G16 = nullptr;
  double *diag = nullptr, *dinv64 = nullptr;
  float* dinv32 = nullptr;
  double *f64 = nullptr, *u64 = nullptr, *r64 = nullptr, *d64 = nullptr;
  float *f32 = nullptr, *u32 = nullptr, *r32 = nullptr, *d32 = nullptr;
  double *pit64 = nullptr, *piz64 = nullptr;  // transfer to the next coarser level
  float *pit32 = nullptr, *piz32 = nullptr;
  double omega = 0.0;
  double omega_user = 0.0;
  LevelView view{};
  // MFMA element operator (per flavour MF_F64, MF_F32, MF_BF16)
  bool mf[3] = {false, false, false};
  void* gnat[3] = {nullptr, nullptr, nullptr};
  // gnat[f] no longer matches the level's geometry: rebuilt before its next use
  bool nat_stale[3] = {false, false, false};
  void* tab2[3] = {nullptr, nullptr, nullptr};
  void* tab4[3] = {nullptr, nullptr, nullptr};
  // lo parts of the BF16 tables (split-BF16 products, MF_BF16X3)
  void *tab2x = nullptr, *tab4x = nullptr, *tab2lo = nullptr, *tab4lo = nullptr;  // split-BF16 tables
  bool mfx3 = false;
  // column factors geo[t][q][8] of the MFMA operators (PMG_GEOM_COLUMN)
  double* geo64 = nullptr;
  float* geo32 = nullptr;
  VertMats<double> vm64{};
  VertMats<float> vm32{};
  // overlapping Schwarz smoother: host plan, device view, local inverses
  // (FP64 and the FP32 / BF16 copies), weights, subdomain vectors
  bool has_sz = false;
  SchwarzPlan sz;
  SchwarzView szv{};
  double* sz_inv64 = nullptr;
  float* sz_inv32 = nullptr;
  bf16_t* sz_inv16 = nullptr;
  double *sz_w64 = nullptr, *sz_z64 = nullptr;
  float *sz_w32 = nullptr, *sz_z32 = nullptr;
  template <typename T> T* szw();
  template <typename T> T* szz();

  template <typename T> T* f();
  template <typename T> T* u();
  template <typename T> T* r();
  template <typename T> T* dinv();
  template <typename T> T* d();
  template <typename T> T* mats();
  template <typename T> T* pit();
  template <typename T> T* piz();
};
template <> double* Level::f<double>() { return f64; }
template <> float* Level::f<float>() { return f32; }
template <> double* Level::u<double>() { return u64; }
template <> float* Level::u<float>() { return u32; }
template <> double* Level::r<double>() { return r64; }
template <> float* Level::r<float>() { return r32; }
template <> double* Level::d<double>() { return d64; }
template <> float* Level::d<float>() { return d32; }
template <> double* Level::dinv<double>() { return dinv64; }
template <> float* Level::dinv<float>() { return dinv32; }
template <> double* Level::mats<double>() { return mats64; }
template <> float* Level::mats<float>() { return mats32; }
template <> double* Level::pit<double>() { return pit64; }
template <> float* Level::pit<float>() { return pit32; }
template <> double* Level::piz<double>() { return piz64; }
template <> float* Level::piz<float>() { return piz32; }
template <> double* Level::szw<double>() { return sz_w64; }
template <> float* Level::szw<float>() { return sz_w32; }
template <> double* Level::szz<double>() { return sz_z64; }
template <> float* Level::szz<float>() { return sz_z32; }

}  // namespace pmg

struct pmg_ctx {
  std::string err;
  pmg::MeshIn mesh;
  pmg_options opt{};
  int nl = 0;
  int device = 0;
  bool host_only = false;
  std::vector<pmg::Level> lv;
  std::vector<double> xyt_h;  // fine triangle-node xy [nt][NPT][2]
  std::vector<double> eta_h;  // current surface (host copy)
  double* xyt = nullptr;
  double* eta = nullptr;
  int* bad = nullptr;
  double* Y = nullptr;        // E-layout work buffer (bytes for max E*Np doubles)
  double* partial = nullptr;  // 2*RED_BLOCKS
  double* scal = nullptr;     // N_SCAL
  double* scal_h = nullptr;   // pinned mirror
  // coarse solve
  int nc = 0;
  int32_t* cidx = nullptr;
  double* cinv64 = nullptr;
  float* cinv32 = nullptr;
  double* ctmp64 = nullptr;
  float* ctmp32 = nullptr;
  // assembled free-node P = 1 matrix (coarse Chebyshev): CSR pattern and the
  // element entries summed into each nonzero; the ELL copy (ell_w slots per row)
  // the Chebyshev steps read, with values per precision; second d buffer
  int32_t *csr_rp = nullptr, *csr_cp = nullptr;
  int64_t* csr_cl = nullptr;
  int ell_w = 0;
  int32_t* ell_ci = nullptr;
  double* ell_v64 = nullptr;
  float* ell_v32 = nullptr;
  double* p1_dref = nullptr;
  double* cd64 = nullptr;
  float* cd32 = nullptr;
  double cheb_lmin = 0, cheb_lmax = 0;
  int cheb_k = 0;
  bool coarse_exact = true;
  // solve work (finest level)
  double *s_phiD = nullptr, *s_f = nullptr, *s_u = nullptr, *s_r = nullptr, *s_p = nullptr, *s_q = nullptr,
         *s_z = nullptr, *s_y = nullptr;
  float *s_r32 = nullptr, *s_z32 = nullptr;
  float* feat_cst = nullptr; // [n1][4] constant features of the coarsest nodes
  int lowp = pmg::G_F32;      // G storage of the float V-cycle
  bool bf16_ops = false;      // BF16 MFMA operands (PMG_MIXED_BF16) rather than FP32 arithmetic
  bool bf16x3 = false;        // split-BF16 MFMA products (PMG_MIXED_BF16X3)
  bool bf16x2 = false;        // split vectors on BF16 tables (PMG_MIXED_BF16X2)
  int n_vcycles = 0, n_fine_applies = 0, n_graph_vcycles = 0;
  // free-surface time stepping: nodal triangle derivatives, top-node column
  // derivative, stage buffers ([eta | phi~] pairs), gradients and w~
  double *fn_Dr = nullptr, *fn_Ds = nullptr, *fn_dtop = nullptr;
  double *fn_y0 = nullptr, *fn_ys = nullptr, *fn_acc = nullptr, *fn_k = nullptr, *fn_gr = nullptr,
         *fn_w = nullptr;
  // stage solutions kept for the stage predictor: t_n (stage 1), t_n + dt/2
  // (stage 3) and the previous step's t_n - dt/2; fn_dt: that step's dt (0: none)
  double *fn_p1 = nullptr, *fn_p3 = nullptr, *fn_p3prev = nullptr;
  double fn_dt = 0.0;
  // operator reuse across surfaces (pmg_reuse); eta_flat: zeros for the LIN levels
  int reuse = PMG_REUSE_NONE;
  double* eta_flat = nullptr;
  std::vector<void*> allocs;
  double* dss_s = nullptr;  // accumulator of the coloured direct-stiffness sum (pmg_options.dss)

  template <typename T> T* A(size_t n) {
    T* p = pmg::dalloc<T>(n);
    allocs.push_back(p);
    return p;
  }
  template <typename T> T* U(const std::vector<T>& h) {
    T* p = pmg::dupload<T>(h);
    allocs.push_back(p);
    return p;
  }
  // V-cycle graphs (pmg_options.graphs), one per V-cycle precision (0: FP64, 1: low):
  // gen counts changes of the context; a graph is valid for the gen, stream and
  // low-precision mode it was captured at; warm: gen of the last eager V-cycle
  uint64_t gen = 1;
  struct VGraph {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0, warm = 0;
    hipStream_t st = nullptr;
    int lowp = -1;
  } vg[2];
  ~pmg_ctx() {
    for (auto& g : vg)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (void* p : allocs) (void)hipFree(p);
    if (scal_h) (void)hipHostFree(scal_h);
  }
};

struct pmg_net {
  std::string err;
  int device = 0;
  int din = pmg::NET_DIN, width = 0, depth = 0;
  int64_t np = 0;
  std::vector<int> fin, fout;
  std::vector<int64_t> woff, boff;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  int t = 0;
  std::vector<float> mean_h, istd_h;
  double tscale = 1.0;
  float *mean = nullptr, *istd = nullptr;
  int bmax = 0;
  float *Xb = nullptr, *Tb = nullptr, *dy = nullptr, *dzA = nullptr, *dzB = nullptr, *X1 = nullptr, *Xn = nullptr,
        *y1 = nullptr;
  int64_t n1cap = 0;
  std::vector<float*> Z, H;
  double *partial = nullptr, *scal = nullptr, *losses = nullptr;
  int nloss = 0;
  float* scratch = nullptr;  // this GPU's activation array of the allocation-free forward
  std::vector<void*> allocs;
  template <typename T> T* A(size_t n) {
    T* p = pmg::dalloc<T>(n);
    allocs.push_back(p);
    return p;
  }
  ~pmg_net() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace pmg {

static thread_local std::string g_err;

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
static std::vector<double> pack_mats(const RefElem& re) {
  std::vector<double> m;
  m.insert(m.end(), re.Dr.v.begin(), re.Dr.v.end());
  m.insert(m.end(), re.Ds.v.begin(), re.Ds.v.end());
  m.insert(m.end(), re.B.v.begin(), re.B.v.end());
  m.insert(m.end(), re.Bz.v.begin(), re.Bz.v.end());
  m.insert(m.end(), re.Dz.v.begin(), re.Dz.v.end());
  return m;
}

// Orders of the levels, finest first, from the finest (P, PZ); a coarsening
// step takes an order p to max(1, floor(p/2)) (Sec. 5).  BOTH: both orders
// together.  XY_FIRST: the triangle order first with the vertical order kept,
// then the vertical order: (P,PZ) -> ... -> (1,PZ) -> (1,PZ/2) -> ... -> (1,1).
// EQUAL: the higher order alone, to max(lower, floor(higher/2)), until the two
// agree, then both (Sec. 6.2, Table BTcoarse3D: (5,3) -> (3,3) -> (1,1)).
static std::vector<std::pair<int, int>> level_orders(int P, int PZ, int coarsening) {
  auto half = [](int p) { return std::max(1, p / 2); };
  std::vector<std::pair<int, int>> out{{P, PZ}};
  if (coarsening == PMG_COARSEN_XY_FIRST) {
    for (int pt = P; pt > 1;) out.emplace_back(pt = half(pt), PZ);
    for (int pz = PZ; pz > 1;) out.emplace_back(1, pz = half(pz));
  } else if (coarsening == PMG_COARSEN_EQUAL) {
    int pt = P, pz = PZ;
    while (pt != pz) {
      if (pt > pz) pt = std::max(pz, half(pt)); else pz = std::max(pt, half(pz));
      out.emplace_back(pt, pz);
    }
    while (pt > 1) { pt = pz = half(pt); out.emplace_back(pt, pz); }
  } else {
    int pt = P, pz = PZ;
    while (pt > 1 || pz > 1) { pt = half(pt); pz = half(pz); out.emplace_back(pt, pz); }
  }
  return out;
}

static void build_levels(pmg_ctx* c) {
  const pmg_options& o = c->opt;
  const std::vector<std::pair<int, int>> orders = level_orders(o.P, o.PZ > 0 ? o.PZ : o.P, o.coarsening);
  for (size_t i = 0; i < orders.size(); ++i) {
    const auto& a = orders[i];
    if (!order_supported(a.first, a.second) ||
        (i + 1 < orders.size() && !pair_supported(a.first, a.second, orders[i + 1].first, orders[i + 1].second)))
      throw Error(PMG_EINVAL, "level orders (" + std::to_string(a.first) + "," + std::to_string(a.second) +
                                  ") of this coarsening sequence are not built by the library");
  }
  c->nl = int(orders.size());
  c->lv.resize(c->nl);
  for (int i = 0; i < c->nl; ++i) {
    Level& L = c->lv[i];
    L.P = orders[i].first;
    L.PZ = orders[i].second;
    L.re.reset(new RefElem(L.P, L.PZ));
    L.num.build(c->mesh, L.P, L.PZ);
    // node kernels index a level's nodes with 32-bit integers
    if (L.num.n_dof >= (int64_t(1) << 32)) throw Error(PMG_EINVAL, "a level with 2^32 or more nodes");
    L.dir2d_h = lateral_dirichlet(c->mesh, L.num, o.dirichlet_tags);
    L.top_dir = o.top_neumann ? 0 : 1;
    int64_t nd = 0;
    for (int64_t g2 = 0; g2 < L.num.n2d; ++g2)
      nd += L.dir2d_h[g2] ? L.num.nz : (L.top_dir ? 1 : 0);
    L.n_free = L.num.n_dof - nd;
    L.omega_user = (i < 8) ? o.omega[i] : 0.0;
  }
  if (o.smoother == PMG_SMOOTH_SCHWARZ) {
    const int nth = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    for (int i = 0; i + 1 < c->nl; ++i) {
      Level& L = c->lv[i];
      const int dt = o.overlap < 0 ? (L.P + 2) / 2 : o.overlap;
      const int dz = o.overlap < 0 ? (L.PZ + 2) / 2 : o.overlap;
      try {
        build_schwarz(c->mesh, L.num, L.dir2d_h, L.top_dir, dt, dz, nth, L.sz);
      } catch (const std::runtime_error& e) {
        throw Error(PMG_EINVAL, e.what());
      }
      int mmax = 0;
      for (int32_t m : L.sz.msz) mmax = std::max(mmax, m);
      if (mmax > 8192) throw Error(PMG_EINVAL, "Schwarz subdomain larger than 8192 nodes");
      L.has_sz = true;
    }
  }
  const RefElem& rf = *c->lv[0].re;
  c->xyt_h = triangle_node_xy(c->mesh, rf, c->lv[0].num);
  // check straight/curved triangles are not inverted (flat surface)
  for (int t = 0; t < c->mesh.nt; ++t) {
    const int* tv = &c->mesh.tri[3 * t];
    const double* p0 = &c->mesh.xy[2 * tv[0]];
    const double* p1 = &c->mesh.xy[2 * tv[1]];
    const double* p2 = &c->mesh.xy[2 * tv[2]];
    const double a2 = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p1[1] - p0[1]) * (p2[0] - p0[0]);
    if (!(a2 > 0)) throw Error(PMG_EMESH, "triangle " + std::to_string(t) + " is not counter-clockwise");
  }
  c->eta_h.assign(size_t(c->lv[0].num.n2d), 0.0);
}

// MFMA operand tables of one order (see kernels_mfma.hip): row map of the
// output registers is 4g+r (FP32, BF16) or g+4r (FP64), g = lane/16, j = lane%16.
static void mfma_tables(const RefElem& re, int flavour, std::vector<double>& t2, std::vector<double>& t4,
                        std::vector<uint16_t>& b2, std::vector<uint16_t>& b4) {
  const int NPT = re.np_tri, NQT = re.nq_tri;
  const int NT2 = (NQT + 15) / 16, KS = (NPT + 3) / 4, KS16 = (NPT + 15) / 16, NAT = (NPT + 15) / 16;
  const Mat* M[3] = {&re.Dr, &re.Ds, &re.B};
  auto at = [&](int mt, int q, int a) { return (q < NQT && a < NPT) ? (*M[mt])(q, a) : 0.0; };
  auto bf = [](double v) {
    float f = float(v);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
  };
  t2.clear(); t4.clear(); b2.clear(); b4.clear();
  if (flavour == MF_BF16) {
    for (int mt = 0; mt < 3; ++mt)
      for (int t = 0; t < NT2; ++t)
        for (int s = 0; s < KS16; ++s)
          for (int l = 0; l < 64; ++l)
            for (int kk = 0; kk < 4; ++kk) b2.push_back(bf(at(mt, 16 * t + (l & 15), 16 * s + 4 * (l >> 4) + kk)));
    for (int mt = 0; mt < 3; ++mt)
      for (int a = 0; a < NAT; ++a)
        for (int t = 0; t < NT2; ++t)
          for (int l = 0; l < 64; ++l)
            for (int kk = 0; kk < 4; ++kk) b4.push_back(bf(at(mt, 16 * t + 4 * (l >> 4) + kk, 16 * a + (l & 15))));
    return;
  }
  const bool f64row = flavour == MF_F64;
  auto row = [&](int g, int r) { return f64row ? g + 4 * r : 4 * g + r; };
  for (int mt = 0; mt < 3; ++mt)
    for (int t = 0; t < NT2; ++t)
      for (int s = 0; s < KS; ++s)
        for (int l = 0; l < 64; ++l) t2.push_back(at(mt, 16 * t + (l & 15), 4 * s + (l >> 4)));
  for (int mt = 0; mt < 3; ++mt)
    for (int a = 0; a < NAT; ++a)
      for (int t = 0; t < NT2; ++t)
        for (int r = 0; r < 4; ++r) {
          if (16 * t + row(0, r) >= NQT) continue;
          for (int l = 0; l < 64; ++l) t4.push_back(at(mt, 16 * t + row(l >> 4, r), 16 * a + (l & 15)));
        }
}

// Operand tables of the split-BF16 operator (see kernels_mfma.hip), hi =
// bf16(v) and lo = bf16(v - hi) copies: stage 2 (K = 32, 8 values per lane)
// [m][q tile t][lane][e] = M_m[16 t + lane % 16][a], a = 16 (e / 4) + 4 (e % 4)
// + lane / 16; stage 4 (K = 16, 4 values per lane) [m][a tile][t][lane][kk] =
// M_m[16 t + 4 (lane / 16) + kk][16 a_tile + lane % 16]; zero outside the
// NQT x NPT matrices.
static void split_tables(const RefElem& re, std::vector<uint16_t>& h2, std::vector<uint16_t>& h4,
                         std::vector<uint16_t>& l2, std::vector<uint16_t>& l4) {
  const int NPT = re.np_tri, NQT = re.nq_tri;
  const int NT2 = (NQT + 15) / 16, NAT = (NPT + 15) / 16;
  const Mat* M[3] = {&re.Dr, &re.Ds, &re.B};
  auto at = [&](int mt, int q, int a) { return (q < NQT && a < NPT) ? (*M[mt])(q, a) : 0.0; };
  auto bf = [](float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
  };
  auto push = [&](double v, std::vector<uint16_t>& hi, std::vector<uint16_t>& lo) {
    const float f = float(v);
    const uint16_t h = bf(f);
    const uint32_t hb = uint32_t(h) << 16;
    float hf;
    std::memcpy(&hf, &hb, 4);
    hi.push_back(h);
    lo.push_back(bf(f - hf));
  };
  h2.clear(); h4.clear(); l2.clear(); l4.clear();
  for (int mt = 0; mt < 3; ++mt)
    for (int t = 0; t < NT2; ++t)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e)
          push(at(mt, 16 * t + (l & 15), 16 * (e >> 2) + 4 * (e & 3) + (l >> 4)), h2, l2);
  for (int mt = 0; mt < 3; ++mt)
    for (int a = 0; a < NAT; ++a)
      for (int t = 0; t < NT2; ++t)
        for (int l = 0; l < 64; ++l)
          for (int kk = 0; kk < 4; ++kk) push(at(mt, 16 * t + 4 * (l >> 4) + kk, 16 * a + (l & 15)), h4, l4);
}

static void upload_mfma(pmg_ctx* c, Level& L) {
  const RefElem& re = *L.re;
  for (int i = 0; i < re.n1 * re.n1; ++i) {
    L.vm64.Bz[i] = re.Bz.v[i];
    L.vm64.Dz[i] = re.Dz.v[i];
    L.vm32.Bz[i] = float(re.Bz.v[i]);
    L.vm32.Dz[i] = float(re.Dz.v[i]);
  }
  for (int i = 0; i < re.n1 * re.n1; ++i) {
    const double w = re.zw[i / re.n1];
    L.vm64.Bzw[i] = re.Bz.v[i] * w;
    L.vm64.Dzw[i] = re.Dz.v[i] * w;
    L.vm32.Bzw[i] = float(L.vm64.Bzw[i]);
    L.vm32.Dzw[i] = float(L.vm64.Dzw[i]);
  }
  for (int k = 0; k < re.n1; ++k) {
    L.vm64.zw[k] = re.zw[k];
    L.vm64.zh[k] = 0.5 * (1.0 + re.zq[k]);
    L.vm32.zw[k] = float(L.vm64.zw[k]);
    L.vm32.zh[k] = float(L.vm64.zh[k]);
  }
  const int64_t nb = (L.num.n_elem + 15) / 16;
  const size_t ng = size_t(nb) * 16 * 6 * re.nq;
  // with column factors the FP64 and FP32 kernels read no stored G: no native copy
  const bool col = c->opt.geometry == PMG_GEOM_COLUMN;
  for (int f = 0; f < 3; ++f) {
    if (!mfma_available(L.P, L.PZ, f)) continue;
    std::vector<double> t2, t4;
    std::vector<uint16_t> b2, b4;
    mfma_tables(re, f, t2, t4, b2, b4);
    if (f == MF_BF16 && mfma_available(L.P, L.PZ, MF_BF16X3)) {
      std::vector<uint16_t> h2, h4, l2, l4;
      split_tables(re, h2, h4, l2, l4);
      L.tab2x = c->U(h2);
      L.tab4x = c->U(h4);
      L.tab2lo = c->U(l2);
      L.tab4lo = c->U(l4);
      L.mfx3 = true;
    }
    if (f == MF_F64 && L.P == 8) {
      // the in-plane order 8 FP64 kernel reads the unpadded tables [m][q][a]
      std::vector<double> m3;
      for (const Mat* M : {&re.Dr, &re.Ds, &re.B}) m3.insert(m3.end(), M->v.begin(), M->v.end());
      L.tab2[f] = c->U(m3);
      L.tab4[f] = L.tab2[f];
      if (!col) L.gnat[f] = c->A<double>(ng);
    } else if (f == MF_F64) {
      L.tab2[f] = c->U(t2);
      L.tab4[f] = c->U(t4);
      if (!col) L.gnat[f] = c->A<double>(ng);
    } else if (f == MF_F32) {
      L.tab2[f] = c->U(to_f32(t2));
      L.tab4[f] = c->U(to_f32(t4));
      if (!col) L.gnat[f] = c->A<float>(ng);
    } else {
      L.tab2[f] = c->U(b2);
      L.tab4[f] = c->U(b4);
      L.gnat[f] = c->A<bf16_t>(ng);
    }
    L.mf[f] = true;
  }
}

static void upload_levels(pmg_ctx* c) {
  const RefElem& rf = *c->lv[0].re;
  int64_t maxE = 0;
  for (int i = 0; i < c->nl; ++i) {
    Level& L = c->lv[i];
    const RefElem& re = *L.re;
    L.map2d = c->U(L.num.map2d);
    L.inc_ptr = c->U(L.num.inc_ptr);
    L.inc = c->U(L.num.inc);
    L.dir2d = c->U(L.dir2d_h);
    std::vector<double> m = pack_mats(re);
    L.mats64 = c->U(m);
    L.mats32 = c->U(to_f32(m));
    // fine basis at this level's cubature (geometry of every level uses the fine map)
    Mat Bf, Drf, Dsf;
    rf.tri_eval(re.cr, re.cs, Bf, Drf, Dsf);
    std::vector<double> gm;
    gm.insert(gm.end(), Bf.v.begin(), Bf.v.end());
    gm.insert(gm.end(), Drf.v.begin(), Drf.v.end());
    gm.insert(gm.end(), Dsf.v.begin(), Dsf.v.end());
    L.gmats = c->U(gm);
    L.wq = c->U(re.cw);
    L.zq = c->U(re.zq);
    L.zw = c->U(re.zw);
    const int64_t E = L.num.n_elem, N = L.num.n_dof;
    // stored G: every level without an MFMA operator on column factors, and every
    // level under the Schwarz smoother (its element matrices read G)
    const bool col_only = c->opt.geometry == PMG_GEOM_COLUMN && c->opt.kernel_variant == 0 &&
                          c->opt.smoother != PMG_SMOOTH_SCHWARZ && mfma_available(L.P, L.PZ, MF_F64);
    if (!col_only) {
      L.G64 = c->A<double>(size_t(E) * 6 * re.nq);
      L.G32 = c->A<float>(size_t(E) * 6 * re.nq);
      L.G16 = c->A<bf16_t>(size_t(E) * 6 * re.nq);
    }
    // column factors of every level (the MFMA operators and the diagonal read them)
    if (c->opt.geometry == PMG_GEOM_COLUMN) {
      const size_t n = size_t(c->mesh.nt) * re.nq_tri * 8;
      // padded with 16 zero records: the MFMA operators read whole 16-row tiles of
      // cubature points, past a triangle's last point into the next one's
      L.geo64 = c->A<double>(n + 128);
      L.geo32 = c->A<float>(n + 128);
      HIPCHK(hipMemset(L.geo64 + n, 0, 128 * sizeof(double)));
      HIPCHK(hipMemset(L.geo32 + n, 0, 128 * sizeof(float)));
    }
    L.diag = c->A<double>(N);
    L.dinv64 = c->A<double>(N);
    L.dinv32 = c->A<float>(N);
    L.r64 = c->A<double>(N);
    L.r32 = c->A<float>(N);
    if (i + 1 < c->nl) {
      L.d64 = c->A<double>(N);
      L.d32 = c->A<float>(N);
    }
    if (i > 0) {
      L.f64 = c->A<double>(N);
      L.u64 = c->A<double>(N);
      L.f32 = c->A<float>(N);
      L.u32 = c->A<float>(N);
    }
    maxE = std::max(maxE, E * re.np);
    if (c->opt.kernel_variant == 0) upload_mfma(c, L);
    if (L.has_sz) {
      const SchwarzPlan& P = L.sz;
      SchwarzView& v = L.szv;
      v.n_sub = P.n_sub;
      v.max_n = P.max_n;
      v.max_m = 0;
      for (int32_t m : P.msz) v.max_m = std::max(v.max_m, int(m));
      v.sd_ptr = c->U(P.sd_ptr);
      v.sd_node = c->U(P.sd_node);
      v.msz = c->U(P.msz);
      v.inv_off = c->U(P.inv_off);
      v.tile_off = c->U(P.tile_off);
      v.blk_ptr = c->U(P.blk_ptr);
      v.blk_elem = c->U(P.blk_elem);
      v.blk_ent = c->U(P.blk_ent);
      v.ent = c->U(P.ent);
      v.node_ptr = c->U(P.node_ptr);
      v.node_pos = c->U(P.node_pos);
      L.sz_w64 = c->U(P.w);
      L.sz_w32 = c->U(to_f32(P.w));
      const size_t ninv = size_t(P.tile_off.back());
      const int keep = c->opt.schwarz_store == 0 ? 7 : c->opt.schwarz_store;
      int lds_max = 0;
      HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
      const size_t lds = sd_apply_lds(P.max_n, (keep & 1) ? 8 : 4);
      if (lds > size_t(lds_max))
        throw Error(PMG_EINVAL, "Schwarz subdomains too large for the local solve (" + std::to_string(P.max_n) +
                                    " nodes)");
      if (keep & 1) L.sz_inv64 = c->A<double>(ninv);
      if (keep & 2) L.sz_inv32 = c->A<float>(ninv);
      if (keep & 4) L.sz_inv16 = c->A<bf16_t>(ninv);
      L.sz_z64 = c->A<double>(size_t(std::max<int64_t>(1, P.total)));
      L.sz_z32 = c->A<float>(size_t(std::max<int64_t>(1, P.total)));
    }
    {
      // column-sum layout: 2D ids below n_bnd are the vertices and edge nodes,
      // then nint interior nodes per triangle in triangle order; the boundary
      // slots t*3P + s of every node below n_bnd, in ascending triangle order
      const int P3 = 3 * L.P, npt = L.num.np_tri;
      L.nint = (L.P - 1) * (L.P - 2) / 2;
      L.n_bnd = int64_t(L.num.nv) + int64_t(L.num.ne) * (L.P - 1);
      bool ok = L.n_bnd + int64_t(L.num.nt) * L.nint == L.num.n2d && 16 % L.num.L == 0 &&
                L.num.n_dof < (int64_t(1) << 32);
      std::vector<int32_t> ptr(size_t(L.n_bnd) + 1, 0);
      for (int t = 0; t < L.num.nt && ok; ++t)
        for (int a = 0; a < npt; ++a) {
          const int code = tri_code_of(a, L.P);
          const int64_t n = L.num.map2d[size_t(t) * npt + a];
          if (code >= 0) {
            if (n >= L.n_bnd) ok = false; else ptr[size_t(n) + 1]++;
          } else if (n != L.n_bnd + int64_t(t) * L.nint + (-1 - code)) {
            ok = false;
          }
        }
      if (ok) {
        for (size_t n = 0; n < size_t(L.n_bnd); ++n) ptr[n + 1] += ptr[n];
        std::vector<int32_t> idx(size_t(ptr.back())), fill(ptr.begin(), ptr.end() - 1);
        for (int t = 0; t < L.num.nt; ++t)
          for (int a = 0; a < npt; ++a) {
            const int code = tri_code_of(a, L.P);
            if (code >= 0) idx[size_t(fill[size_t(L.num.map2d[size_t(t) * npt + a])]++)] = t * P3 + code;
          }
        L.sh_ptr = c->U(ptr);
        L.sh_idx = c->U(idx);
      }
      L.colsum = ok ? 1 : 0;
    }
    if (c->opt.dss == 1) {
      // triangles grouped by colour, ascending within a colour (32-bit item ids per colour)
      if (int64_t(L.num.nt) * L.num.np_tri * L.num.nz >= (int64_t(1) << 32))
        throw Error(PMG_EINVAL, "coloured sum: 2^32 or more (triangle, node, z) items on a level");
      const std::vector<int32_t> col = L.num.tri_colours();
      const int ncol = col.empty() ? 0 : 1 + *std::max_element(col.begin(), col.end());
      L.tcol_ptr.assign(size_t(ncol) + 1, 0);
      for (int32_t v : col) L.tcol_ptr[size_t(v) + 1]++;
      for (int k = 0; k < ncol; ++k) L.tcol_ptr[size_t(k) + 1] += L.tcol_ptr[size_t(k)];
      std::vector<int32_t> list(col.size());
      std::vector<int64_t> fill(L.tcol_ptr.begin(), L.tcol_ptr.end() - 1);
      for (int t = 0; t < int(col.size()); ++t) list[size_t(fill[size_t(col[size_t(t)])]++)] = t;
      L.tcol_list = c->U(list);
    }
    L.view = LevelView{L.P, L.PZ, L.num.L, L.num.nt, re.np_tri, re.np, re.nq, L.num.n2d, L.num.nz, N, E,
                       L.map2d, L.inc_ptr, L.inc, L.dir2d, L.top_dir, L.n_bnd, L.nint, L.sh_ptr, L.sh_idx,
                       L.colsum, L.tcol_list};
    if (i + 1 < c->nl) {
      const RefElem& rc = *c->lv[i + 1].re;
      // coarse nodal basis at the fine nodes
      Mat Bt, d1, d2;
      rc.tri_eval(re.r, re.s, Bt, d1, d2);
      Mat Bz1, dz1;
      rc.line_eval(re.t, Bz1, dz1);
      L.pit64 = c->U(Bt.v);
      L.piz64 = c->U(Bz1.v);
      L.pit32 = c->U(to_f32(Bt.v));
      L.piz32 = c->U(to_f32(Bz1.v));
    }
  }
  // also holds the 6x6 element matrices of the P = 1 level (coarse CSR values) and
  // the boundary column sums [nt][3P][nz] of the fused summation
  maxE = std::max<int64_t>(maxE, c->lv[c->nl - 1].num.n_elem * 36);
  for (int i = 0; i < c->nl; ++i)
    maxE = std::max<int64_t>(maxE, int64_t(c->lv[i].num.nt) * c->lv[i].num.np_tri * c->lv[i].num.nz);
  c->Y = c->A<double>(size_t(maxE));
  if (c->opt.dss == 1) {
    // L-vector accumulator of the coloured sum: zero here, put back to zero by every sum
    c->dss_s = c->A<double>(size_t(c->lv[0].num.n_dof));
    HIPCHK(hipMemset(c->dss_s, 0, size_t(c->lv[0].num.n_dof) * sizeof(double)));
  }
  c->partial = c->A<double>(2 * RED_BLOCKS);
  c->scal = c->A<double>(N_SCAL);
  HIPCHK(hipHostMalloc((void**)&c->scal_h, N_SCAL * sizeof(double), hipHostMallocDefault));
  c->bad = c->A<int>(1);
  c->xyt = c->U(c->xyt_h);
  c->eta = c->A<double>(size_t(c->lv[0].num.n2d));
  HIPCHK(hipMemset(c->eta, 0, sizeof(double) * c->lv[0].num.n2d));
  const int64_t N = c->lv[0].num.n_dof;
  c->s_phiD = c->A<double>(N);
  c->s_f = c->A<double>(N);
  c->s_u = c->A<double>(N);
  c->s_r = c->A<double>(N);
  c->s_p = c->A<double>(N);
  c->s_q = c->A<double>(N);
  c->s_z = c->A<double>(N);
  c->s_y = c->A<double>(N);
  c->s_r32 = c->A<float>(N);
  c->s_z32 = c->A<float>(N);
}

// ---------------------------------------------------------------------------
// operator building blocks
// ---------------------------------------------------------------------------
// precision of the float V-cycle: G storage and MFMA operand type
static void set_lowp(pmg_ctx* c, int precision) {
  c->lowp = (precision == PMG_MIXED_BF16 || precision == PMG_MIXED_BF16G || precision == PMG_MIXED_BF16X3 ||
             precision == PMG_MIXED_BF16X2)
                ? G_BF16
                : G_F32;
  c->bf16_ops = precision == PMG_MIXED_BF16;
  c->bf16x3 = precision == PMG_MIXED_BF16X3;
  c->bf16x2 = precision == PMG_MIXED_BF16X2;
}

template <typename T> static const void* gptr(pmg_ctx* c, Level& L, int& gstore);
template <> const void* gptr<double>(pmg_ctx*, Level& L, int& gs) { gs = G_F64; return L.G64; }
template <> const void* gptr<float>(pmg_ctx* c, Level& L, int& gs) {
  gs = c->lowp;
  return c->lowp == G_BF16 ? (const void*)L.G16 : (const void*)L.G32;
}

// Lane-native copy of G for flavour f: from the stored G64, or formed from the
// FP64 column factors when the level keeps no stored G.  The copies are built
// lazily: a surface change marks them stale, and a kernel that reads one
// rebuilds it first (paths that never read a flavour never pay for it).
static void native_g(pmg_ctx* c, Level& L, int f, hipStream_t st) {
  launch_g_native(L.P, L.PZ, L.num.n_elem, L.G64, L.gnat[f], f, st, L.G64 ? nullptr : L.geo64, L.view.L, L.zq,
                  L.zw);
}
static void ensure_native(pmg_ctx* c, Level& L, int f, hipStream_t st) {
  if (!L.nat_stale[f]) return;
  native_g(c, L, f, st);
  L.nat_stale[f] = false;
}

// Element operator of level i on x into c->Y: the element layout (for the
// node-centric sum), or with colsum the column sums of launch_col_sum; returns
// false, launching nothing, where the level has no column-sum kernel.
template <typename T>
static bool ax_elem(pmg_ctx* c, int i, const T* x, hipStream_t st, bool colsum = false) {
  Level& L = c->lv[i];
  int gs;
  const void* G = gptr<T>(c, L, gs);
  const int f = sizeof(T) == 8 ? MF_F64 : (gs == G_BF16 ? MF_BF16 : MF_F32);
  bool ok = false;
  if (L.mf[f]) {
    const void* vm = sizeof(T) == 8 ? (const void*)&L.vm64 : (const void*)&L.vm32;
    // column factors in the precision of the kernel's arithmetic (not for BF16 operands)
    const bool col = c->opt.geometry == PMG_GEOM_COLUMN && L.geo64;
    const void* geo = !col ? nullptr : (sizeof(T) == 8 ? (const void*)L.geo64 : (const void*)L.geo32);
    if (f == MF_BF16 && c->bf16x3 && L.mfx3) {
      if (!geo) ensure_native(c, L, MF_BF16, st);
      ok = launch_ax_mfma(L.view, L.gnat[MF_BF16], MF_BF16X3, L.tab2x, L.tab4x, vm, x, c->Y, st, L.tab2lo,
                          L.tab4lo, geo, colsum);
    } else if (f == MF_BF16 && c->bf16x2 && L.mfx3) {
      if (!geo) ensure_native(c, L, MF_BF16, st);
      ok = launch_ax_mfma(L.view, L.gnat[MF_BF16], MF_BF16X2, L.tab2x, L.tab4x, vm, x, c->Y, st, nullptr, nullptr,
                          geo, colsum);
    } else if (f == MF_BF16 && !c->bf16_ops && L.mf[MF_F32]) {
      // FP32 arithmetic on the stored BF16 copy of G (FP32 tables); at in-plane
      // order 3 this is faster than forming G from the column factors, whose
      // kernel holds more registers
      ensure_native(c, L, MF_BF16, st);
      ok = launch_ax_mfma(L.view, L.gnat[MF_BF16], MF_F32G16, L.tab2[MF_F32], L.tab4[MF_F32], vm, x, c->Y, st,
                          nullptr, nullptr, nullptr, colsum);
    } else {
      if (f == MF_BF16 || !geo) ensure_native(c, L, f, st);
      ok = launch_ax_mfma(L.view, L.gnat[f], f, L.tab2[f], L.tab4[f], vm, x, c->Y, st, nullptr, nullptr,
                          f == MF_BF16 ? nullptr : geo, colsum);
    }
  } else if (!colsum) {
    launch_ax<T>(L.view, L.mats<T>(), G, gs, x, reinterpret_cast<T*>(c->Y), st);
    ok = true;
  }
  if (ok && i == 0 && sizeof(T) == 8) c->n_fine_applies++;
  return ok;
}

// Direct-stiffness sum of the element layout in c->Y with epilogue op: the
// node-centric kernel, or the coloured passes (pmg_options.dss = 1).
template <typename T>
static void dss_sum(pmg_ctx* c, int i, int op, T* out, const T* a1, const T* a2, T* a3, double w, double c1,
                    hipStream_t st, T* a4 = nullptr) {
  const Level& L = c->lv[i];
  const T* Y = reinterpret_cast<const T*>(c->Y);
  if (c->opt.dss == 1)
    launch_dss<T>(L.view, L.tcol_ptr, op, Y, reinterpret_cast<T*>(c->dss_s), out, a1, a2, a3, w, c1, c->partial, st,
                  a4);
  else
    launch_assemble<T>(L.view, op, Y, out, a1, a2, a3, w, c1, c->partial, st, a4);
}

template <typename T>
static void assemble(pmg_ctx* c, int i, int op, T* out, const T* a1, const T* a2, T* a3, double w, double c1,
                     hipStream_t st) {
  dss_sum<T>(c, i, op, out, a1, a2, a3, w, c1, st);
}

// Prolongation from level i+1 to level i, then op (OP_AVG_ADD, OP_AVG_STORE or
// OP_AVG_RAW) at the fine nodes: node-wise where one factor of the transfer is
// the identity, else element-wise with the averaging sum.
template <typename T>
static void prolong_add(pmg_ctx* c, int i, const T* uc, T* out, int op, hipStream_t st) {
  Level& L = c->lv[i];
  Level& C = c->lv[i + 1];
  if (launch_prolong_node<T>(L.view, C.view, L.pit<T>(), L.piz<T>(), uc, out, op, st)) return;
  launch_prolong_elem<T>(L.view, C.view, L.pit<T>(), L.piz<T>(), uc, reinterpret_cast<T*>(c->Y), st);
  assemble<T>(c, i, op, out, nullptr, nullptr, nullptr, 0, 0, st);
}

// out (+)= epilogue op of (A x) on level i (see AsmOp): where the level's MFMA
// operator writes column sums (16 % L == 0), the operator and the node kernel
// of launch_col_sum; otherwise the element layout and the node-centric sum.
// Both add every node's contributions in a fixed order without atomics.
template <typename T>
static void apply_op(pmg_ctx* c, int i, const T* x, int op, T* out, const T* a1, const T* a2, T* a3, double w,
                     double c1, hipStream_t st, T* a4 = nullptr) {
  Level& L = c->lv[i];
  const bool avg = op == OP_AVG_ADD || op == OP_AVG_STORE || op == OP_AVG_RAW;
  if (c->opt.fused_sum && !avg && ax_elem<T>(c, i, x, st, true)) {
    launch_col_sum<T>(L.view, op, reinterpret_cast<const T*>(c->Y), out, a1, a2, a3, w, c1, c->partial, st, a4);
    return;
  }
  ax_elem<T>(c, i, x, st);
  dss_sum<T>(c, i, op, out, a1, a2, a3, w, c1, st, a4);
}

template <typename T>
static void jacobi_sweep(pmg_ctx* c, int i, const T* f, T* u, hipStream_t st) {
  Level& L = c->lv[i];
  apply_op<T>(c, i, u, OP_JACOBI, u, f, L.dinv<T>(), nullptr, L.omega, 0.0, st);
}

// Chebyshev-accelerated Jacobi smoothing (k >= 1 steps) of the defect f - A u on
// [lambda/ratio, lambda], lambda = 4/(3 omega); from u = 0 when zero_guess.
template <typename T>
static void cheb_smooth(pmg_ctx* c, int i, const T* f, T* u, bool zero_guess, int k, hipStream_t st) {
  Level& L = c->lv[i];
  const int64_t N = L.num.n_dof;
  const double lmax = 4.0 / (3.0 * L.omega), lmin = lmax / c->opt.smooth_ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  T* r = L.r<T>();
  T* d = L.d<T>();
  if (zero_guess) {
    launch_cheb_start<T>(N, f, L.dinv<T>(), r, d, u, 1.0 / theta, st);  // r = f, d = D^-1 f / theta, u = d
  } else {
    // r = f - A u, d = D^-1 r / theta, u += d (one fused summation)
    apply_op<T>(c, i, u, OP_CHEB0, u, f, L.dinv<T>(), d, 0.0, 1.0 / theta, st, r);
  }
  double rho = 1.0 / sigma;
  for (int j = 1; j < k; ++j) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    apply_op<T>(c, i, d, OP_CHEB, u, r, L.dinv<T>(), d, rho_new * rho, 2.0 * rho_new / delta, st);
    rho = rho_new;
  }
}

// inverse storage of a Schwarz application in the V-cycle precision; EINVAL if not kept
static void need_sz(const Level& L, bool f64, int lowp) {
  const bool ok = f64 ? L.sz_inv64 != nullptr : (lowp == G_BF16 ? L.sz_inv16 != nullptr : L.sz_inv32 != nullptr);
  if (!ok)
    throw Error(PMG_EINVAL, std::string("Schwarz inverses not kept in ") +
                                (f64 ? "FP64" : (lowp == G_BF16 ? "BF16" : "FP32")) + " (options.schwarz_store)");
}

// k sweeps of the Schwarz smoother u <- u + omega S^-1 (f - A u), from u = 0
// when zero_guess; post: the transpose sum_k R_k^T A_k^-1 R_k W.
template <typename T>
static void schwarz_smooth(pmg_ctx* c, int i, const T* f, T* u, bool zero_guess, bool post, int k, hipStream_t st) {
  Level& L = c->lv[i];
  T* r = L.r<T>();
  T* z = L.szz<T>();
  const T* w = L.szw<T>();
  need_sz(L, sizeof(T) == 8, c->lowp);
  for (int s = 0; s < k; ++s) {
    const bool first = zero_guess && s == 0;
    const T* x = f;
    if (!first) {
      apply_op<T>(c, i, u, OP_RESID, r, f, nullptr, nullptr, 0, 0, st);
      x = r;
    }
    if (sizeof(T) == 8)
      launch_sd_apply<double, double>(L.szv, L.sz_inv64, (const double*)x, (const double*)(post ? w : nullptr),
                                      (double*)z, st);
    else if (c->lowp == G_BF16)
      launch_sd_apply<float, bf16_t>(L.szv, L.sz_inv16, (const float*)x, (const float*)(post ? w : nullptr),
                                     (float*)z, st);
    else
      launch_sd_apply<float, float>(L.szv, L.sz_inv32, (const float*)x, (const float*)(post ? w : nullptr),
                                    (float*)z, st);
    launch_sd_sum<T>(L.szv, L.num.n_dof, z, post ? nullptr : w, T(L.omega), !first, u, st);
  }
}

static double read_scal(pmg_ctx* c, int slot, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(c->scal_h, c->scal, N_SCAL * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return c->scal_h[slot];
}

static double dot_host(pmg_ctx* c, const double* x, const double* y, int64_t n, hipStream_t st) {
  launch_dot<double>(x, y, n, c->partial, st);
  launch_finalize(c->partial, c->scal, S_TMP0, FIN_SET, st);
  return read_scal(c, S_TMP0, st);
}

// ---------------------------------------------------------------------------
// coarse solve
// ---------------------------------------------------------------------------
template <typename T> static T* cinv(pmg_ctx* c);
template <> double* cinv<double>(pmg_ctx* c) { return c->cinv64; }
template <> float* cinv<float>(pmg_ctx* c) { return c->cinv32; }
template <typename T> static T* ctmp(pmg_ctx* c);
template <> double* ctmp<double>(pmg_ctx* c) { return c->ctmp64; }
template <> float* ctmp<float>(pmg_ctx* c) { return c->ctmp32; }
template <typename T> T* cdbuf(pmg_ctx* c);
template <> double* cdbuf<double>(pmg_ctx* c) { return c->cd64; }
template <> float* cdbuf<float>(pmg_ctx* c) { return c->cd32; }
template <typename T> const T* ell_val(pmg_ctx* c);
template <> const double* ell_val<double>(pmg_ctx* c) { return c->ell_v64; }
template <> const float* ell_val<float>(pmg_ctx* c) { return c->ell_v32; }

template <typename T>
static void coarse_solve(pmg_ctx* c, const T* f, T* u, hipStream_t st) {
  const int i = c->nl - 1;
  Level& L = c->lv[i];
  if (c->coarse_exact) {
    launch_coarse_dense<T>(c->nc, c->cidx, cinv<T>(c), f, u, ctmp<T>(c), L.num.n_dof, st);
    return;
  }
  // Jacobi-preconditioned Chebyshev iteration from zero (three-term recurrence)
  const int k = std::max(1, c->cheb_k > 0 ? c->cheb_k : c->opt.cheb_degree);
  const double lmin = c->cheb_lmin, lmax = c->cheb_lmax;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  T* r = L.r<T>();
  T* d = ctmp<T>(c);
  T* d2 = cdbuf<T>(c);
  const int64_t N = L.num.n_dof;
  launch_cheb_start<T>(N, f, L.dinv<T>(), r, d, u, 1.0 / theta, st);  // r = f, d0 = D^-1 r / theta, x1 = d0
  double rho = 1.0 / sigma;
  for (int j = 1; j < k; ++j) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    // r -= A d; d' = rho_new rho d + 2 rho_new/delta D^-1 r; x += d' (one fused kernel)
    launch_cheb_ell<T>(N, c->ell_w, c->ell_ci, ell_val<T>(c), L.dinv<T>(), d, d2, r, u, rho_new * rho,
                       2.0 * rho_new / delta, st);
    std::swap(d, d2);
    rho = rho_new;
  }
}

// power estimate of lambda_max(D^-1 A) on level i (free nodes), 1.05 x Rayleigh quotient
static double lambda_max(pmg_ctx* c, int i, hipStream_t st) {
  Level& L = c->lv[i];
  const int64_t N = L.num.n_dof;
  std::vector<double> x0(N);
  for (int64_t g = 0; g < N; ++g) x0[g] = splitmix_unit(c->opt.seed, uint64_t(g));
  double* x = L.r64;
  double* y = c->s_y;  // finest-size scratch >= N
  HIPCHK(hipMemcpyAsync(y, x0.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // x0 is a temporary host buffer
  launch_mask<double>(L.view, y, x, st);
  for (int it = 0; it < 30; ++it) {
    ax_elem<double>(c, i, x, st);
    assemble<double>(c, i, OP_STORE, y, nullptr, nullptr, nullptr, 0, 0, st);
    launch_scale_diag<double>(L.dinv64, y, y, 1.0, N, st);
    const double nrm = std::sqrt(dot_host(c, y, y, N, st));
    if (!(nrm > 0)) throw Error(PMG_EBREAKDOWN, "power iteration collapsed");
    launch_cast<double, double>(y, x, 1.0 / nrm, N, st);
  }
  ax_elem<double>(c, i, x, st);
  assemble<double>(c, i, OP_STORE, y, nullptr, nullptr, nullptr, 0, 0, st);
  const double xax = dot_host(c, x, y, N, st);
  launch_scale_diag<double>(L.diag, x, y, 1.0, N, st);
  const double xdx = dot_host(c, x, y, N, st);
  return 1.05 * xax / xdx;
}

// Spectral radius of S^-1 A for the Schwarz preconditioner S^-1 of level i:
// 30 power steps x <- S^-1 A x / ||S^-1 A x|| from the masked counter-based
// vector, then 1.05 ||S^-1 A x||.  Vectors in T; the inverse copy is the one
// a V-cycle in T reads.
template <typename T>
static double schwarz_rho_t(pmg_ctx* c, int i, hipStream_t st) {
  Level& L = c->lv[i];
  const int64_t N = L.num.n_dof;
  std::vector<double> x0(N);
  for (int64_t g = 0; g < N; ++g) x0[g] = splitmix_unit(c->opt.seed, uint64_t(g));
  T* x = L.r<T>();
  T* y = L.d<T>();
  HIPCHK(hipMemcpyAsync(c->s_y, x0.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // x0 is a temporary host buffer
  launch_cast<double, T>(c->s_y, y, 1.0, N, st);
  launch_mask<T>(L.view, y, x, st);
  auto step = [&](T* out) {  // out = S^-1 A x
    ax_elem<T>(c, i, x, st);
    assemble<T>(c, i, OP_STORE, y, nullptr, nullptr, nullptr, 0, 0, st);
    if (sizeof(T) == 8)
      launch_sd_apply<double, double>(L.szv, L.sz_inv64, (const double*)y, nullptr, (double*)L.szz<T>(), st);
    else if (c->lowp == G_BF16)
      launch_sd_apply<float, bf16_t>(L.szv, L.sz_inv16, (const float*)y, nullptr, (float*)L.szz<T>(), st);
    else
      launch_sd_apply<float, float>(L.szv, L.sz_inv32, (const float*)y, nullptr, (float*)L.szz<T>(), st);
    launch_sd_sum<T>(L.szv, N, L.szz<T>(), L.szw<T>(), T(1), false, out, st);
  };
  auto norm = [&](const T* v) {
    launch_dot<T>(v, v, N, c->partial, st);
    launch_finalize(c->partial, c->scal, S_TMP0, FIN_SET, st);
    return std::sqrt(read_scal(c, S_TMP0, st));
  };
  for (int it = 0; it < 30; ++it) {
    step(x);
    const double nrm = norm(x);
    if (!(nrm > 0)) throw Error(PMG_EBREAKDOWN, "power iteration collapsed");
    launch_sd_scale<T>(x, 1.0 / nrm, N, st);
  }
  step(y);
  return 1.05 * norm(y);
}

static double schwarz_rho(pmg_ctx* c, int i, hipStream_t st) {
  Level& L = c->lv[i];
  if (L.sz_inv64) return schwarz_rho_t<double>(c, i, st);
  const int lowp = c->lowp;
  const bool ops = c->bf16_ops;
  set_lowp(c, L.sz_inv32 ? PMG_MIXED_FP32 : PMG_MIXED_BF16G);
  const double rho = schwarz_rho_t<float>(c, i, st);
  c->lowp = lowp;
  c->bf16_ops = ops;
  return rho;
}

// smallest / largest eigenvalue of a symmetric tridiagonal matrix (Sturm bisection)
static void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double& lo, double& hi) {
  const int m = int(d.size());
  double a = d[0], b = d[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
    a = std::min(a, d[i] - r);
    b = std::max(b, d[i] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int k) {  // k-th smallest (0-based)
    double l = a, h = b;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + h);
      if (count_below(mid) > k) h = mid; else l = mid;
    }
    return 0.5 * (l + h);
  };
  lo = kth(0);
  hi = kth(m - 1);
}

// extreme eigenvalues of D^-1 A on level i from m steps of Jacobi-preconditioned
// CG (Lanczos coefficients), started from the counter-based vector
static void lanczos_bounds(pmg_ctx* c, int i, int m, double& lmin, double& lmax, hipStream_t st) {
  Level& L = c->lv[i];
  const int64_t N = L.num.n_dof;
  m = int(std::min<int64_t>(m, std::max<int64_t>(L.n_free, 1)));
  std::vector<double> x0(N);
  for (int64_t g = 0; g < N; ++g) x0[g] = splitmix_unit(c->opt.seed + 1, uint64_t(g)) - 0.5;
  double* r = L.r64;
  double* p = c->s_p;
  double* z = c->s_z;
  double* q = c->s_y;
  HIPCHK(hipMemcpyAsync(q, x0.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  launch_mask<double>(L.view, q, r, st);
  launch_scale_diag<double>(L.dinv64, r, z, 1.0, N, st);
  launch_copy<double>(z, p, N, st);
  double rz = dot_host(c, r, z, N, st);
  const double rz0 = rz;
  std::vector<double> al, be;
  for (int it = 0; it < m; ++it) {
    ax_elem<double>(c, i, p, st);
    assemble<double>(c, i, OP_STORE_DOT, q, p, nullptr, nullptr, 0, 0, st);
    launch_finalize(c->partial, c->scal, S_TMP0, FIN_SET, st);
    const double pq = read_scal(c, S_TMP0, st);
    if (!(pq > 0)) break;
    const double alpha = rz / pq;
    launch_axpy(r, q, -alpha, N, st);
    launch_scale_diag<double>(L.dinv64, r, z, 1.0, N, st);
    const double rzn = dot_host(c, r, z, N, st);
    const double beta = rzn / rz;
    al.push_back(alpha);
    be.push_back(beta);
    rz = rzn;
    if (!(rz > 1e-28 * rz0)) break;
    launch_xpay(p, z, beta, N, st);
  }
  if (al.empty()) throw Error(PMG_EBREAKDOWN, "Lanczos estimate failed on the coarse level");
  const int k = int(al.size());
  std::vector<double> d(k), e(std::max(k - 1, 1), 0.0);
  for (int t = 0; t < k; ++t) {
    d[t] = 1.0 / al[t] + (t > 0 ? be[t - 1] / al[t - 1] : 0.0);
    if (t + 1 < k) e[t] = std::sqrt(be[t]) / al[t];
  }
  tridiag_extremes(d, e, lmin, lmax);
}

// CSR pattern of the free-node P = 1 matrix and, per nonzero, the element-matrix
// entries (e*36 + i*6 + j) that sum into it, in ascending order; rows of
// Dirichlet nodes stay empty and Dirichlet columns are left out.  Also uploads
// the reference derivative matrices D_a[q][n] of the P = 1 prism.
static void coarse_csr_pattern(pmg_ctx* c) {
  Level& L = c->lv[c->nl - 1];
  if (L.P != 1 || L.PZ != 1) throw Error(PMG_EINVAL, "coarsest level is not of order 1");
  const RefElem& re = *L.re;
  const int64_t E = L.num.n_elem, N = L.num.n_dof;
  const int np = re.np, nq = re.nq, npt = re.np_tri, nqt = re.nq_tri, n1 = re.n1;
  std::vector<uint8_t> dir(N);
  for (int64_t g = 0; g < N; ++g) {
    const int64_t g2 = g / L.num.nz;
    const int z = int(g - g2 * L.num.nz);
    dir[g] = L.dir2d_h[g2] || (L.top_dir && z == L.num.nz - 1);
  }
  std::vector<int32_t> map(size_t(E) * np);
  L.num.gather_map(map.data());
  // bucket the contributions by row (counting sort), then order each row by column
  std::vector<int64_t> rcount(N + 1, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int i = 0; i < np; ++i) {
      const int32_t g = map[e * np + i];
      if (dir[g]) continue;
      for (int j = 0; j < np; ++j)
        if (!dir[map[e * np + j]]) rcount[g + 1]++;
    }
  for (int64_t g = 0; g < N; ++g) rcount[g + 1] += rcount[g];
  std::vector<std::pair<int32_t, int64_t>> items(rcount[N]);  // (column, entry id)
  std::vector<int64_t> fill(rcount.begin(), rcount.end() - 1);
  for (int64_t e = 0; e < E; ++e)
    for (int i = 0; i < np; ++i) {
      const int32_t g = map[e * np + i];
      if (dir[g]) continue;
      for (int j = 0; j < np; ++j) {
        const int32_t h = map[e * np + j];
        if (!dir[h]) items[fill[g]++] = {h, e * 36 + i * np + j};
      }
    }
  std::vector<int32_t> rp(N + 1, 0), ci, cp{0};
  std::vector<int64_t> cl;
  cl.reserve(items.size());
  for (int64_t g = 0; g < N; ++g) {
    std::sort(items.begin() + rcount[g], items.begin() + rcount[g + 1]);
    for (int64_t m = rcount[g]; m < rcount[g + 1]; ++m) {
      if (m == rcount[g] || items[m].first != items[m - 1].first) {
        ci.push_back(items[m].first);
        cp.push_back(cp.back());
      }
      cl.push_back(items[m].second);
      cp.back()++;
    }
    rp[g + 1] = int32_t(ci.size());
  }
  if (cl.size() > size_t(INT32_MAX)) throw Error(PMG_EINVAL, "coarse matrix too large");
  // ELL columns: slot-major, padding slots point at the row itself, Dirichlet rows
  // carry -1 in slot 0
  int w = 1;
  for (int64_t g = 0; g < N; ++g) w = std::max(w, rp[g + 1] - rp[g]);
  std::vector<int32_t> eci(size_t(w) * N);
  for (int64_t g = 0; g < N; ++g) {
    const int len = rp[g + 1] - rp[g];
    for (int k = 0; k < w; ++k) eci[size_t(k) * N + g] = k < len ? ci[rp[g] + k] : int32_t(g);
    if (len == 0) eci[g] = -1;
  }
  c->ell_w = w;
  c->csr_rp = c->A<int32_t>(N + 1);
  c->csr_cp = c->A<int32_t>(cp.size());
  c->csr_cl = c->A<int64_t>(cl.size());
  c->ell_ci = c->A<int32_t>(eci.size());
  c->ell_v64 = c->A<double>(eci.size());
  c->ell_v32 = c->A<float>(eci.size());
  HIPCHK(hipMemcpy(c->csr_rp, rp.data(), rp.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->ell_ci, eci.data(), eci.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->csr_cp, cp.data(), cp.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->csr_cl, cl.data(), cl.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  std::vector<double> Dp(size_t(3) * nq * np);
  for (int k = 0; k < n1; ++k)
    for (int q = 0; q < nqt; ++q)
      for (int cc = 0; cc < n1; ++cc)
        for (int aa = 0; aa < npt; ++aa) {
          const size_t o = size_t(k * nqt + q) * np + cc * npt + aa;
          Dp[0 * nq * np + o] = re.Bz(k, cc) * re.Dr(q, aa);
          Dp[1 * nq * np + o] = re.Bz(k, cc) * re.Ds(q, aa);
          Dp[2 * nq * np + o] = re.Dz(k, cc) * re.B(q, aa);
        }
  c->p1_dref = c->A<double>(Dp.size());
  HIPCHK(hipMemcpy(c->p1_dref, Dp.data(), Dp.size() * sizeof(double), hipMemcpyHostToDevice));
}

// dense inverse of the free-node P=1 matrix (host, from the device G of the level)
static void coarse_exact_setup(pmg_ctx* c, hipStream_t st) {
  Level& L = c->lv[c->nl - 1];
  const RefElem& re = *L.re;
  const int64_t E = L.num.n_elem, N = L.num.n_dof;
  const int np = re.np, nq = re.nq, npt = re.np_tri, nqt = re.nq_tri, n1 = re.n1;
  std::vector<double> G(size_t(E) * 6 * nq);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(G.data(), L.G64, G.size() * sizeof(double), hipMemcpyDeviceToHost));
  // free-node index
  std::vector<int32_t> fidx(N, -1), idx;
  for (int64_t g = 0; g < N; ++g) {
    const int64_t g2 = g / L.num.nz;
    const int z = int(g - g2 * L.num.nz);
    const bool dir = L.dir2d_h[g2] || (L.top_dir && z == L.num.nz - 1);
    if (!dir) { fidx[g] = int32_t(idx.size()); idx.push_back(int32_t(g)); }
  }
  const int n = int(idx.size());
  c->nc = n;
  // reference derivative matrices of the prism (nq x np)
  std::vector<double> Dp[3];
  for (int a = 0; a < 3; ++a) Dp[a].assign(size_t(nq) * np, 0.0);
  for (int k = 0; k < n1; ++k)
    for (int q = 0; q < nqt; ++q)
      for (int cc = 0; cc < n1; ++cc)
        for (int aa = 0; aa < npt; ++aa) {
          const size_t o = size_t(k * nqt + q) * np + cc * npt + aa;
          Dp[0][o] = re.Bz(k, cc) * re.Dr(q, aa);
          Dp[1][o] = re.Bz(k, cc) * re.Ds(q, aa);
          Dp[2][o] = re.Dz(k, cc) * re.B(q, aa);
        }
  std::vector<int32_t> map(size_t(E) * np);
  L.num.gather_map(map.data());
  // bandwidth of the free ordering
  int bw = 0;
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        const int fa = fidx[map[e * np + a]], fb = fidx[map[e * np + b]];
        if (fa >= 0 && fb >= 0) bw = std::max(bw, std::abs(fa - fb));
      }
  const int W = bw + 1;
  std::vector<double> band(size_t(n) * W, 0.0);  // band[i*W + (i-j)] = A(i, j), j <= i
  const int comp[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  std::vector<double> Ae(size_t(np) * np);
  for (int64_t e = 0; e < E; ++e) {
    std::fill(Ae.begin(), Ae.end(), 0.0);
    const double* Ge = &G[size_t(e) * 6 * nq];
    for (int p = 0; p < nq; ++p)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double gab = Ge[comp[a][b] * nq + p];
          for (int x = 0; x < np; ++x) {
            const double da = Dp[a][size_t(p) * np + x] * gab;
            if (da == 0.0) continue;
            for (int y = 0; y < np; ++y) Ae[x * np + y] += da * Dp[b][size_t(p) * np + y];
          }
        }
    for (int x = 0; x < np; ++x) {
      const int fi = fidx[map[e * np + x]];
      if (fi < 0) continue;
      for (int y = 0; y < np; ++y) {
        const int fj = fidx[map[e * np + y]];
        if (fj < 0 || fj > fi) continue;
        band[size_t(fi) * W + (fi - fj)] += Ae[x * np + y];
      }
    }
  }
  // banded Cholesky A = L L^T (in place)
  for (int i = 0; i < n; ++i) {
    const int j0 = std::max(0, i - bw);
    for (int j = j0; j <= i; ++j) {
      double s = band[size_t(i) * W + (i - j)];
      const int k0 = std::max(j0, j - bw);
      for (int k = k0; k < j; ++k) s -= band[size_t(i) * W + (i - k)] * band[size_t(j) * W + (j - k)];
      if (j == i) {
        if (!(s > 0)) throw Error(PMG_EBREAKDOWN, "coarse matrix not positive definite");
        band[size_t(i) * W] = std::sqrt(s);
      } else {
        band[size_t(i) * W + (i - j)] = s / band[size_t(j) * W];
      }
    }
  }
  // inverse columns by forward/backward substitution, in parallel
  std::vector<double> inv(size_t(n) * n, 0.0);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned tid = 0; tid < nth; ++tid)
    th.emplace_back([&, tid]() {
      std::vector<double> y(n);
      for (int col = int(tid); col < n; col += int(nth)) {
        std::fill(y.begin(), y.end(), 0.0);
        for (int i = col; i < n; ++i) {  // L y = e_col
          double s = (i == col) ? 1.0 : 0.0;
          const int k0 = std::max(col, i - bw);
          for (int k = k0; k < i; ++k) s -= band[size_t(i) * W + (i - k)] * y[k];
          y[i] = s / band[size_t(i) * W];
        }
        for (int i = n - 1; i >= 0; --i) {  // L^T x = y
          double s = y[i];
          const int k1 = std::min(n - 1, i + bw);
          for (int k = i + 1; k <= k1; ++k) s -= band[size_t(k) * W + (k - i)] * y[k];
          y[i] = s / band[size_t(i) * W];
        }
        for (int i = 0; i < n; ++i) inv[size_t(i) * n + col] = y[i];
      }
    });
  for (auto& t : th) t.join();
  // (re)upload
  if (!c->cidx) {
    c->cidx = c->U(idx);
    c->cinv64 = c->A<double>(size_t(n) * n);
    c->cinv32 = c->A<float>(size_t(n) * n);
    c->ctmp64 = c->A<double>(std::max<int64_t>(n, N));
    c->ctmp32 = c->A<float>(std::max<int64_t>(n, N));
  }
  HIPCHK(hipMemcpy(c->cinv64, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<float> inv32(inv.begin(), inv.end());
  HIPCHK(hipMemcpy(c->cinv32, inv32.data(), inv32.size() * sizeof(float), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------------------
// Schwarz smoother: local matrices R_k A R_k^T from the element matrices of the
// current geometry, inverted in place (FP64), with FP32 / BF16 copies.  The
// element matrices live in a scratch buffer freed afterwards.
// ---------------------------------------------------------------------------
// The blocks are built and inverted in FP64 in chunks of at most
// options.schwarz_chunk entries (one block at least), then written to the kept
// copies as packed tiles.
static void schwarz_setup(pmg_ctx* c, hipStream_t st, int i0 = 0) {
  for (int i = i0; i + 1 < c->nl; ++i) {
    Level& L = c->lv[i];
    if (!L.has_sz) continue;
    const size_t nK = size_t(L.num.n_elem) * L.re->np * L.re->np;
    double *K = nullptr, *W = nullptr;
    const std::vector<int64_t>& off = L.sz.inv_off;
    const int64_t E = L.sz.n_sub;
    if (hipMalloc((void**)&K, nK * sizeof(double)) != hipSuccess)
      throw Error(PMG_ENOMEM, "no device memory for the Schwarz element matrices");
    const int64_t chunk = c->opt.schwarz_chunk > 0 ? c->opt.schwarz_chunk : (int64_t(1) << 29);
    int64_t blk_max = 0;
    for (int64_t k = 0; k < E; ++k) blk_max = std::max(blk_max, off[k + 1] - off[k]);
    {
      const int64_t nw = std::min<int64_t>(off.back(), std::max<int64_t>(chunk, blk_max));
      if (hipMalloc((void**)&W, size_t(nw) * sizeof(double)) != hipSuccess) {
        (void)hipFree(K);
        throw Error(PMG_ENOMEM, "no device memory for the Schwarz set-up");
      }
    }
    HIPCHK(hipMemsetAsync(c->bad, 0, sizeof(int), st));
    launch_elem_mats(L.view, L.mats64, L.G64, K, st);
    for (int64_t k0 = 0; k0 < E;) {
      int64_t k1 = k0 + 1;
      while (k1 < E && off[k1 + 1] - off[k0] <= chunk) ++k1;
      const int64_t base = off[k0];
      launch_sd_assemble(L.szv, k0, k1, base, L.re->np, K, W, st);
      launch_sd_invert(L.szv, k0, k1, base, W, L.sz_inv64, L.sz_inv32, L.sz_inv16, c->bad, st);
      k0 = k1;
    }
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(K));
    if (W) HIPCHK(hipFree(W));
    if (bad) throw Error(PMG_EBREAKDOWN, "Schwarz local matrix with a non-positive pivot (singular subdomain?)");
  }
}


// ---------------------------------------------------------------------------
// surface / geometry
// ---------------------------------------------------------------------------
static void set_surface_all(pmg_ctx* c, const double* eta, hipStream_t st);

// Diagonal (and its inverses) of one level from its column factors, or from its
// stored G64 without them.
static void level_diag(pmg_ctx* c, Level& L, hipStream_t st) {
  if (L.geo64) launch_diag_col(L.view, L.mats64, L.zq, L.zw, L.geo64, c->Y, st);
  else launch_diag(L.view, L.mats64, L.G64, c->Y, st);
  launch_assemble<double>(L.view, OP_RAW, c->Y, L.diag, nullptr, nullptr, nullptr, 0, 0, nullptr, st);
  launch_dinv<double>(L.view, nullptr, L.diag, L.dinv64, st);
  launch_dinv<float>(L.view, nullptr, L.diag, L.dinv32, st);
}

// Geometry of level i for surface eta (G64, and the FP32/BF16 copies when
// lowp), with the native copies of the flavours listed in `flavours` (bitmask).
// Returns nonzero if an element is inverted.
static int level_geom(pmg_ctx* c, int i, const double* eta, bool lowp, int flavours, hipStream_t st) {
  Level& F = c->lv[0];
  Level& L = c->lv[i];
  HIPCHK(hipMemsetAsync(c->bad, 0, sizeof(int), st));
  launch_geom(F.view, L.view, c->mesh.depth, c->xyt, eta, L.gmats, L.wq, L.zq, L.zw, L.G64, lowp ? L.G32 : nullptr,
              lowp ? L.G16 : nullptr, c->bad, st, L.geo64, lowp ? L.geo32 : nullptr);
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) return bad;
  for (int f = 0; f < 3; ++f)
    if (L.mf[f] && L.gnat[f] && ((flavours >> f) & 1)) L.nat_stale[f] = true;
  return 0;
}

// Under a reuse mode only the finest level follows the surface: its G64 (the
// operator of the outer iteration) always; under LIN also its low-precision
// copies, diagonals and Schwarz inverses.
static void set_surface(pmg_ctx* c, const double* eta, hipStream_t st) {
  c->gen++;  // V-cycle graphs of the previous state are stale
  if (c->reuse == PMG_REUSE_NONE) {
    set_surface_all(c, eta, st);
    return;
  }
  const bool lin = c->reuse == PMG_REUSE_LIN;
  const int64_t n2 = c->lv[0].num.n2d;
  if (level_geom(c, 0, eta, lin, lin ? 7 : 1 << MF_F64, st)) {
    (void)level_geom(c, 0, c->eta, lin, lin ? 7 : 1 << MF_F64, st);  // restore the previous surface
    throw Error(PMG_EMESH, "non-positive Jacobian for the given surface (eta <= -depth?)");
  }
  if (eta != c->eta) HIPCHK(hipMemcpyAsync(c->eta, eta, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(c->eta_h.data(), c->eta, n2 * sizeof(double), hipMemcpyDeviceToHost, st));
  if (lin) {
    level_diag(c, c->lv[0], st);
    if (c->lv[0].has_sz) {
      // Schwarz inverses of the finest level only
      std::vector<bool> keep(size_t(c->nl));
      for (int i = 1; i < c->nl; ++i) {
        keep[size_t(i)] = c->lv[i].has_sz;
        c->lv[i].has_sz = false;
      }
      schwarz_setup(c, st);
      for (int i = 1; i < c->nl; ++i) c->lv[i].has_sz = keep[size_t(i)];
    }
  }
  HIPCHK(hipStreamSynchronize(st));
}

static void coarse_setup(pmg_ctx* c, hipStream_t st);

static void set_surface_all(pmg_ctx* c, const double* eta, hipStream_t st) {
  Level& F = c->lv[0];
  const int64_t n2 = F.num.n2d;
  HIPCHK(hipMemsetAsync(c->bad, 0, sizeof(int), st));
  for (int i = 0; i < c->nl; ++i) {
    Level& L = c->lv[i];
    launch_geom(F.view, L.view, c->mesh.depth, c->xyt, eta, L.gmats, L.wq, L.zq, L.zw, L.G64, L.G32, L.G16,
                c->bad, st, L.geo64, L.geo32);
  }
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) {
    // restore the previous surface
    HIPCHK(hipMemcpyAsync(c->eta, c->eta_h.data(), n2 * sizeof(double), hipMemcpyHostToDevice, st));
    for (int i = 0; i < c->nl; ++i) {
      Level& L = c->lv[i];
      launch_geom(F.view, L.view, c->mesh.depth, c->xyt, c->eta, L.gmats, L.wq, L.zq, L.zw, L.G64, L.G32,
                  L.G16, c->bad, st, L.geo64, L.geo32);
    }
    HIPCHK(hipStreamSynchronize(st));
    throw Error(PMG_EMESH, "non-positive Jacobian for the given surface (eta <= -depth?)");
  }
  if (eta != c->eta) HIPCHK(hipMemcpyAsync(c->eta, eta, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(c->eta_h.data(), c->eta, n2 * sizeof(double), hipMemcpyDeviceToHost, st));
  // lane-native copies of G for the MFMA element operator
  for (int i = 0; i < c->nl; ++i) {
    Level& L = c->lv[i];
    for (int f = 0; f < 3; ++f)
      if (L.mf[f] && L.gnat[f]) L.nat_stale[f] = true;
  }
  // Jacobi diagonals
  for (int i = 0; i < c->nl; ++i) level_diag(c, c->lv[i], st);
  schwarz_setup(c, st);
  for (int i = 0; i + 1 < c->nl; ++i) {
    Level& L = c->lv[i];
    const bool sz = c->opt.smoother == PMG_SMOOTH_SCHWARZ;
    L.omega = L.omega_user > 0 ? L.omega_user : 4.0 / (3.0 * (sz ? schwarz_rho(c, i, st) : lambda_max(c, i, st)));
  }
  coarse_setup(c, st);
  HIPCHK(hipStreamSynchronize(st));
}

// coarse solver of the current coarsest-level operator
static void coarse_setup(pmg_ctx* c, hipStream_t st) {
  Level& C = c->lv[c->nl - 1];
  c->coarse_exact = c->opt.coarse == PMG_COARSE_EXACT;
  if (c->coarse_exact && C.n_free > c->opt.exact_max)
    throw Error(PMG_EINVAL, "free coarse size " + std::to_string(C.n_free) + " exceeds exact_max; use the "
                            "Chebyshev coarse solve");
  if (c->coarse_exact) {
    coarse_exact_setup(c, st);
  } else {
    if (!c->ctmp64) {
      c->ctmp64 = c->A<double>(C.num.n_dof);
      c->ctmp32 = c->A<float>(C.num.n_dof);
    }
    if (!c->cd64) {
      c->cd64 = c->A<double>(C.num.n_dof);
      c->cd32 = c->A<float>(C.num.n_dof);
    }
    if (!c->csr_rp) coarse_csr_pattern(c);
    launch_p1_elem_mat(C.num.n_elem, C.G64, c->p1_dref, c->Y, st);
    launch_ell_sum(C.num.n_dof, c->ell_w, c->csr_rp, c->csr_cp, c->csr_cl, c->Y, c->ell_v64, c->ell_v32, st);
    if (c->opt.cheb_lmax > 0 && c->opt.cheb_lmin > 0) {
      c->cheb_lmax = c->opt.cheb_lmax;
      c->cheb_lmin = c->opt.cheb_lmin;
    } else if (c->opt.cheb_ratio > 0) {
      c->cheb_lmax = c->opt.cheb_lmax > 0 ? c->opt.cheb_lmax : lambda_max(c, c->nl - 1, st);
      c->cheb_lmin = c->cheb_lmax / std::max(1.0001, c->opt.cheb_ratio);
    } else {
      double lo, hi;
      lanczos_bounds(c, c->nl - 1, 120, lo, hi, st);
      c->cheb_lmax = c->opt.cheb_lmax > 0 ? c->opt.cheb_lmax : 1.05 * hi;
      c->cheb_lmin = c->opt.cheb_lmin > 0 ? c->opt.cheb_lmin : 0.9 * lo;
    }
    // degree for a 0.1 error reduction over [lmin, lmax] unless given
    c->cheb_k = c->opt.cheb_degree > 0
                    ? c->opt.cheb_degree
                    : std::max(4, std::min(400, int(std::ceil(0.5 * std::sqrt(c->cheb_lmax / c->cheb_lmin) *
                                                              std::log(20.0)))));
  }
  HIPCHK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// V-cycle (Alg. 1) with zero initial guess
// ---------------------------------------------------------------------------
// Pre/post sweeps of level i: nu1, nu2 on the finest level, and on the levels
// below it unless nu1_coarse / nu2_coarse (>= 0) override them.
static int sweeps_pre(const pmg_ctx* c, int i) {
  return i > 0 && c->opt.nu1_coarse >= 0 ? c->opt.nu1_coarse : c->opt.nu1;
}
static int sweeps_post(const pmg_ctx* c, int i) {
  return i > 0 && c->opt.nu2_coarse >= 0 ? c->opt.nu2_coarse : c->opt.nu2;
}

template <typename T>
static void vcycle(pmg_ctx* c, int i, const T* f, T* u, hipStream_t st) {
  if (i == c->nl - 1) {
    coarse_solve<T>(c, f, u, st);
    return;
  }
  Level& L = c->lv[i];
  Level& C = c->lv[i + 1];
  const int64_t N = L.num.n_dof;
  const bool cheb = c->opt.smoother == PMG_SMOOTH_CHEBYSHEV;
  const bool asm_ = c->opt.smoother == PMG_SMOOTH_SCHWARZ;
  const int nu1 = sweeps_pre(c, i), nu2 = sweeps_post(c, i);
  if (nu1 >= 1 && asm_) {
    schwarz_smooth<T>(c, i, f, u, true, false, nu1, st);
  } else if (nu1 >= 1 && cheb) {
    cheb_smooth<T>(c, i, f, u, true, nu1, st);
  } else if (nu1 >= 1) {
    launch_scale_diag<T>(L.dinv<T>(), f, u, L.omega, N, st);
    for (int m = 1; m < nu1; ++m) jacobi_sweep<T>(c, i, f, u, st);
  } else {
    launch_fill<T>(u, T(0), N, st);
  }
  T* r = L.r<T>();
  apply_op<T>(c, i, u, OP_RESID, r, f, nullptr, nullptr, 0, 0, st);
  launch_restrict_elem<T>(L.view, C.view, L.pit<T>(), L.piz<T>(), r, reinterpret_cast<T*>(c->Y), st);
  assemble<T>(c, i + 1, OP_STORE, C.f<T>(), nullptr, nullptr, nullptr, 0, 0, st);
  vcycle<T>(c, i + 1, C.f<T>(), C.u<T>(), st);
  prolong_add<T>(c, i, C.u<T>(), u, OP_AVG_ADD, st);
  if (asm_) {
    schwarz_smooth<T>(c, i, f, u, false, true, nu2, st);
  } else if (cheb) {
    if (nu2 >= 1) cheb_smooth<T>(c, i, f, u, false, nu2, st);
  } else {
    for (int m = 0; m < nu2; ++m) jacobi_sweep<T>(c, i, f, u, st);
  }
}

// One finest-level V-cycle of the solve, f -> u, replayed from a captured HIP
// graph where pmg_options.graphs allows: the kernels and their arguments of a
// V-cycle depend only on the context's state and the (fixed) vectors, so a
// graph captured after one eager V-cycle at the current state (lazily built
// operand copies then exist) reproduces it exactly.  Captures never run on
// the null stream.
template <typename T>
static void solve_vcycle(pmg_ctx* c, const T* f, T* u, hipStream_t st) {
  pmg_ctx::VGraph& g = c->vg[sizeof(T) == 8 ? 0 : 1];
  const int lowp = sizeof(T) == 8 ? -1 : c->lowp;
  if (!c->opt.graphs || st == nullptr) {
    vcycle<T>(c, 0, f, u, st);
    return;
  }
  if (g.exec && g.gen == c->gen && g.st == st && g.lowp == lowp) {
    HIPCHK(hipGraphLaunch(g.exec, st));
    c->n_graph_vcycles++;
    return;
  }
  if (g.warm != c->gen) {
    vcycle<T>(c, 0, f, u, st);
    g.warm = c->gen;
    return;
  }
  if (g.exec) {
    HIPCHK(hipGraphExecDestroy(g.exec));
    g.exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    vcycle<T>(c, 0, f, u, st);
  } catch (...) {  // leave the caller's stream out of capture mode
    hipGraph_t partial = nullptr;
    (void)hipStreamEndCapture(st, &partial);
    if (partial) (void)hipGraphDestroy(partial);
    throw;
  }
  HIPCHK(hipStreamEndCapture(st, &graph));
  const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(e);
  g.gen = c->gen;
  g.st = st;
  g.lowp = lowp;
  HIPCHK(hipGraphLaunch(g.exec, st));
  c->n_graph_vcycles++;
}

// z = M^-1 r at the finest level in the context's precision (r, z FP64: the
// solve's own vectors, fixed for the context, so its V-cycle may be a graph)
static void precond(pmg_ctx* c, const double* r, double* z, hipStream_t st) {
  c->n_vcycles++;
  const int64_t N = c->lv[0].num.n_dof;
  if (c->opt.precision == PMG_FP64) {
    solve_vcycle<double>(c, r, z, st);
    return;
  }
  set_lowp(c, c->opt.precision);
  launch_cast<double, float>(r, c->s_r32, 1.0, N, st);
  solve_vcycle<float>(c, c->s_r32, c->s_z32, st);
  launch_cast<float, double>(c->s_z32, z, 1.0, N, st);
}

// y = A_FF x (FP64, finest), partial of p.y when dot_with != nullptr
static void fine_apply(pmg_ctx* c, const double* x, double* y, const double* dot_with, hipStream_t st) {
  if (dot_with)
    apply_op<double>(c, 0, x, OP_STORE_DOT, y, dot_with, nullptr, nullptr, 0, 0, st);
  else
    apply_op<double>(c, 0, x, OP_STORE, y, nullptr, nullptr, nullptr, 0, 0, st);
}

// ---------------------------------------------------------------------------
// warm-start network
// ---------------------------------------------------------------------------
static void net_reserve(pmg_net* n, int B) {
  if (B <= n->bmax) return;
  n->bmax = B;
  n->Xb = n->A<float>(size_t(B) * n->din);
  n->Tb = n->A<float>(B);
  n->dy = n->A<float>(B);
  n->dzA = n->A<float>(size_t(B) * n->width);
  n->dzB = n->A<float>(size_t(B) * n->width);
  n->Z.assign(n->fin.size(), nullptr);
  n->H.assign(n->fin.size(), nullptr);
  for (size_t l = 0; l < n->fin.size(); ++l) {
    n->Z[l] = n->A<float>(size_t(B) * n->fout[l]);
    n->H[l] = n->A<float>(size_t(B) * n->fout[l]);
  }
}

// forward of B rows of X (device, row-major [B][din]); output n->H.back() [B]
static void net_forward(pmg_net* n, const float* X, int B, hipStream_t st) {
  net_reserve(n, B);
  const float* h = X;
  const int L = int(n->fin.size());
  for (int l = 0; l < L; ++l) {
    launch_gemm(B, n->fout[l], n->fin[l], h, n->fin[l], 1, n->theta + n->woff[l], n->fout[l], 1,
                n->theta + n->boff[l], n->Z[l], n->H[l], n->fout[l], l + 1 < L, st);
    h = n->H[l];
  }
}

// loss and gradient (into n->grad) of B rows; loss sum of squares -> *slot
static void net_backward(pmg_net* n, const float* X, const float* T, int B, double* loss_slot, hipStream_t st) {
  net_forward(n, X, B, st);
  const int L = int(n->fin.size());
  launch_mse(n->H[L - 1], T, n->dy, B, n->partial, st);
  launch_red_final(n->partial, MLP_RED, loss_slot, st);
  const float* dz = n->dy;
  for (int l = L - 1; l >= 0; --l) {
    const float* hin = l == 0 ? X : n->H[l - 1];
    launch_gemm(n->fin[l], n->fout[l], B, hin, 1, n->fin[l], dz, n->fout[l], 1, nullptr, nullptr,
                n->grad + n->woff[l], n->fout[l], false, st);
    launch_colsum(dz, B, n->fout[l], n->grad + n->boff[l], st);
    if (l > 0) {
      launch_gemm(B, n->fin[l], n->fout[l], dz, n->fout[l], 1, n->theta + n->woff[l], 1, n->fout[l], nullptr,
                  nullptr, n->dzA, n->fin[l], false, st);
      launch_silu_back(n->dzA, n->Z[l - 1], n->dzB, int64_t(B) * n->fin[l], st);
      dz = n->dzB;
    }
  }
}

// Level of the learned correction: the coarsest one (order (1,1); its 2D nodes
// are the mesh vertices).  A network on the (1,P) level of the in-plane-first
// sequence (every vertical node kept) was measured too: five times the rows, no
// fewer iterations.
static int net_level(const pmg_ctx* c) { return c->nl - 1; }

// constant features of the network level's nodes: sigma, x and y in [-1,1], distance to the nearest circle
static void build_feat_cst(pmg_ctx* c) {
  if (c->feat_cst) return;
  Level& C = c->lv[net_level(c)];
  const int64_t n1 = C.num.n_dof;
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int v = 0; v < c->mesh.nv; ++v) {
    xmin = std::min(xmin, c->mesh.xy[2 * v]);
    xmax = std::max(xmax, c->mesh.xy[2 * v]);
    ymin = std::min(ymin, c->mesh.xy[2 * v + 1]);
    ymax = std::max(ymax, c->mesh.xy[2 * v + 1]);
  }
  std::vector<float> f(size_t(n1) * 4);
  for (int64_t g = 0; g < n1; ++g) {
    const int64_t v = g / C.num.nz;
    const int z = int(g - v * C.num.nz);
    const double x = c->mesh.xy[2 * v], y = c->mesh.xy[2 * v + 1];
    double dist = 0.0;
    for (size_t k = 0; k * 3 < c->mesh.circle.size(); ++k) {
      const double d = std::hypot(x - c->mesh.circle[3 * k], y - c->mesh.circle[3 * k + 1]) - c->mesh.circle[3 * k + 2];
      dist = (k == 0) ? d : std::min(dist, d);
    }
    f[4 * g + 0] = float(double(z) / double(C.num.nz - 1));
    f[4 * g + 1] = float(2.0 * (x - xmin) / std::max(xmax - xmin, 1e-300) - 1.0);
    f[4 * g + 2] = float(2.0 * (y - ymin) / std::max(ymax - ymin, 1e-300) - 1.0);
    f[4 * g + 3] = float(dist);
  }
  c->feat_cst = c->U(f);
}

static void features(pmg_ctx* c, const double* surf, const double* p1, const double* p2, const double* p3,
                     const double* pnow, float* X, float* T, hipStream_t st) {
  build_feat_cst(c);
  Level& C = c->lv[net_level(c)];
  Level& F = c->lv[0];
  launch_features(C.num.n_dof, int(C.num.nz), int(F.num.nz), F.PZ / C.PZ, c->feat_cst, surf, p1, p2, p3, pnow, X,
                  T, st);
}

// learned correction of the extrapolation, prolongated to the finest level: out (free nodes)
static void learned_guess(pmg_ctx* c, pmg_net* n, const double* surf, const double* p1, const double* p2,
                          const double* p3, double* out, hipStream_t st) {
  const int NL = net_level(c);
  Level& C = c->lv[NL];
  const int64_t n1 = C.num.n_dof;
  if (n->n1cap < n1) {
    n->X1 = n->A<float>(size_t(n1) * n->din);
    n->Xn = n->A<float>(size_t(n1) * n->din);
    n->y1 = n->A<float>(n1);
    n->n1cap = n1;
  }
  features(c, surf, p1, p2, p3, nullptr, n->X1, nullptr, st);
  launch_normalize(n->X1, n1, n->din, n->mean, n->istd, n->Xn, st);
  const int L = int(n->fin.size());
  const int chunk = 65536;  // one or two chunks on the benchmark meshes: fewer, larger GEMMs
  for (int64_t r0 = 0; r0 < n1; r0 += chunk) {
    const int B = int(std::min<int64_t>(chunk, n1 - r0));
    net_forward(n, n->Xn + r0 * n->din, B, st);
    launch_copy<float>(n->H[L - 1], n->y1 + r0, B, st);
  }
  // coarsest correction: predicted inside, exact at the surface nodes (new surface data minus its
  // extrapolation), prolongated level by level without masking, in FP32 (it is a starting
  // guess; its residual is formed in FP64 by the caller, who keeps the free part)
  double* c64 = NL > 0 ? C.u64 : out;
  launch_scale_out(n->y1, n->tscale, n1, c64, st);
  launch_corr_surface(n1, int(C.num.nz), int(c->lv[0].num.nz), surf, p1, p2, p3, c64, st);
  if (NL == 0) return;
  launch_cast<double, float>(c64, C.u32, 1.0, n1, st);
  const float* cur = C.u32;
  for (int i = NL - 1; i >= 0; --i) {
    float* dst = i == 0 ? c->s_z32 : c->lv[i].u32;
    prolong_add<float>(c, i, cur, dst, OP_AVG_RAW, st);
    cur = dst;
  }
  launch_cast<float, double>(c->s_z32, out, 1.0, c->lv[0].num.n_dof, st);
}

static int solve(pmg_ctx* c, const double* surf, const double* bc, double* phi, int guess, pmg_net* net,
                 const double* const* hist, double rtol, double atol, int imax, pmg_stats* stats, hipStream_t st) {
  Level& F = c->lv[0];
  const int64_t N = F.num.n_dof;
  int fallback = 0;
  if (!surf && !bc) throw Error(PMG_EINVAL, "no Dirichlet data (phi_surf and phi_bc are NULL)");
  if (!bc && c->opt.dirichlet_tags) throw Error(PMG_EINVAL, "lateral Dirichlet tags need phi_bc");
  if (!phi) throw Error(PMG_EINVAL, "phi is NULL");
  if (!(rtol >= 0) || !(atol >= 0) || imax < 0) throw Error(PMG_EINVAL, "bad tolerance");
  if (guess < PMG_GUESS_GIVEN || guess > PMG_GUESS_LEARNED3) throw Error(PMG_EINVAL, "unknown guess mode");
  const bool third = guess == PMG_GUESS_EXTRAP3 || guess == PMG_GUESS_LEARNED3;
  const bool learned = guess == PMG_GUESS_LEARNED || guess == PMG_GUESS_LEARNED3;
  const bool hist_based = learned || guess == PMG_GUESS_EXTRAP || guess == PMG_GUESS_EXTRAP3;
  if (hist_based && (!hist || !hist[0] || !hist[1] || (third && !hist[2])))
    throw Error(PMG_EINVAL, third ? "this guess needs the three previous solutions"
                                  : "the learned and extrapolated guesses need the two previous solutions");
  if (learned && !net) throw Error(PMG_EINVAL, "learned guess without a network");
  if (learned && !surf) throw Error(PMG_EINVAL, "learned guess needs phi_surf");
  hipEvent_t ev0, ev1;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev0, st));
  c->n_vcycles = 0;
  c->n_fine_applies = 0;
  c->n_graph_vcycles = 0;
  // non-finite boundary data
  launch_count_nonfinite(bc ? bc : surf, bc ? N : F.num.n2d, c->partial, st);
  launch_finalize(c->partial, c->scal, S_TMP1, FIN_SET, st);
  if (read_scal(c, S_TMP1, st) != 0.0) throw Error(PMG_ENONFINITE, "non-finite Dirichlet data");
  // lifting: f = -A phi_D on free nodes
  launch_lift(F.view, surf, bc, c->s_phiD, st);
  fine_apply(c, c->s_phiD, c->s_y, nullptr, st);
  launch_cast<double, double>(c->s_y, c->s_f, -1.0, N, st);
  const double nf = std::sqrt(dot_host(c, c->s_f, c->s_f, N, st));
  // initial guess
  double rr0 = -1.0;  // ||f - A u||^2 of the chosen guess once known
  if (guess == PMG_GUESS_GIVEN) {
    launch_count_nonfinite(phi, N, c->partial, st);
    launch_finalize(c->partial, c->scal, S_TMP1, FIN_SET, st);
    if (read_scal(c, S_TMP1, st) != 0.0) throw Error(PMG_ENONFINITE, "non-finite initial guess");
    launch_merge_free(F.view, phi, nullptr, c->s_u, st);
  } else if (hist_based) {
    const double* p3 = third ? hist[2] : nullptr;
    launch_extrap(hist[0], hist[1], p3, c->s_y, N, st);
    launch_mask<double>(F.view, c->s_y, c->s_u, st);
    if (learned) {
      // candidate = extrapolation + learned correction delta, kept only if its residual
      // is smaller: r_ex = f - A u_ex and r_ln = r_ex - A delta (one fine apply each,
      // both norms read with one synchronisation); the chosen residual seeds the loop
      learned_guess(c, net, surf, hist[0], hist[1], p3, c->s_q, st);
      launch_mask<double>(F.view, c->s_q, c->s_q, st);
      apply_op<double>(c, 0, c->s_u, OP_RESID, c->s_r, c->s_f, nullptr, nullptr, 0, 0, st);
      apply_op<double>(c, 0, c->s_q, OP_RESID, c->s_y, c->s_r, nullptr, nullptr, 0, 0, st);
      launch_dot<double>(c->s_r, c->s_r, N, c->partial, st);
      launch_finalize(c->partial, c->scal, S_TMP0, FIN_SET, st);
      launch_dot<double>(c->s_y, c->s_y, N, c->partial, st);
      launch_finalize(c->partial, c->scal, S_TMP1, FIN_SET, st);
      const double r_ex = read_scal(c, S_TMP0, st), r_ln = c->scal_h[S_TMP1];
      if (std::isfinite(r_ln) && r_ln < r_ex) {
        launch_axpy(c->s_u, c->s_q, 1.0, N, st);
        launch_copy<double>(c->s_y, c->s_r, N, st);
        rr0 = r_ln;
      } else {
        fallback = 1;
        rr0 = r_ex;
      }
    }
  } else {
    launch_fill<double>(c->s_u, 0.0, N, st);
  }
  HIPCHK(hipEventRecord(ev1, st));
  HIPCHK(hipEventSynchronize(ev1));
  float tg = 0;
  HIPCHK(hipEventElapsedTime(&tg, ev0, ev1));
  // r = f - A u (already at hand for the learned guess)
  if (rr0 < 0.0) {
    apply_op<double>(c, 0, c->s_u, OP_RESID, c->s_r, c->s_f, nullptr, nullptr, 0, 0, st);
    rr0 = dot_host(c, c->s_r, c->s_r, N, st);
  }
  std::vector<double> hist_r{std::sqrt(rr0)};
  const double tol = rtol * nf + atol;
  int it = 0;
  int status = PMG_OK;
  const int kry = c->opt.krylov;
  if (kry == PMG_PCG || kry == PMG_FPCG) {
    if (hist_r.back() > tol && imax > 0) {
      precond(c, c->s_r, c->s_z, st);
      launch_copy<double>(c->s_z, c->s_p, N, st);
      launch_dot<double>(c->s_z, c->s_r, N, c->partial, st);
      launch_finalize(c->partial, c->scal, 0, FIN_DELTA, st);
    }
    // low-precision V-cycle: the update also writes r in FP32 (the V-cycle input)
    // and the beta dot and the direction read its FP32 output directly
    const bool lowp = c->opt.precision != PMG_FP64;
    while (it < imax && hist_r.back() > tol) {
      fine_apply(c, c->s_p, c->s_q, c->s_p, st);
      launch_finalize(c->partial, c->scal, 0, FIN_ALPHA, st);
      launch_cg_update(c->s_u, c->s_r, c->s_p, c->s_q, c->scal, c->partial, N, st, lowp ? c->s_r32 : nullptr);
      launch_finalize(c->partial, c->scal, S_RR, FIN_SET, st);
      HIPCHK(hipMemcpyAsync(c->scal_h, c->scal, N_SCAL * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const double pq = c->scal_h[S_PQ], delta = c->scal_h[S_DELTA], rr = c->scal_h[S_RR];
      if (!(pq > 0) || !(delta > 0)) { status = PMG_EBREAKDOWN; break; }
      if (!std::isfinite(rr)) { status = PMG_ENONFINITE; break; }
      hist_r.push_back(std::sqrt(rr));
      ++it;
      if (hist_r.back() <= tol || it >= imax) break;
      if (lowp) {
        // z = M r with r already in FP32; z stays FP32 (widened where read)
        c->n_vcycles++;
        set_lowp(c, c->opt.precision);
        solve_vcycle<float>(c, c->s_r32, c->s_z32, st);
        launch_dot2(c->s_z32, c->s_r, c->s_q, N, c->partial, st);
        launch_finalize(c->partial, c->scal, 0, kry == PMG_PCG ? FIN_BETA_FR : FIN_BETA_PR, st);
        launch_cg_dir(c->s_p, c->s_z32, c->scal, N, st);
        continue;
      }
      precond(c, c->s_r, c->s_z, st);
      if (kry == PMG_PCG) {
        launch_dot<double>(c->s_z, c->s_r, N, c->partial, st);
        launch_finalize(c->partial, c->scal, 0, FIN_BETA_FR, st);
      } else {
        launch_dot2(c->s_z, c->s_r, c->s_q, N, c->partial, st);
        launch_finalize(c->partial, c->scal, 0, FIN_BETA_PR, st);
      }
      launch_cg_dir(c->s_p, c->s_z, c->scal, N, st);
    }
  } else if (kry == PMG_PDC || kry == PMG_MG) {
    while (it < imax && hist_r.back() > tol) {
      precond(c, c->s_r, c->s_z, st);
      launch_axpy(c->s_u, c->s_z, 1.0, N, st);
      apply_op<double>(c, 0, c->s_u, OP_RESID, c->s_r, c->s_f, nullptr, nullptr, 0, 0, st);
      const double rr = dot_host(c, c->s_r, c->s_r, N, st);
      if (!std::isfinite(rr)) { status = PMG_ENONFINITE; break; }
      hist_r.push_back(std::sqrt(rr));
      ++it;
    }
  } else {
    throw Error(PMG_EINVAL, "unknown krylov method");
  }
  // phi = phi_D + u; true relative residual in FP64
  launch_merge_free(F.view, c->s_u, c->s_phiD, phi, st);
  apply_op<double>(c, 0, c->s_u, OP_RESID, c->s_y, c->s_f, nullptr, nullptr, 0, 0, st);
  const double rtrue = std::sqrt(dot_host(c, c->s_y, c->s_y, N, st));
  HIPCHK(hipEventRecord(ev1, st));
  HIPCHK(hipEventSynchronize(ev1));
  float tms = 0;
  HIPCHK(hipEventElapsedTime(&tms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (status == PMG_OK && hist_r.back() > tol) status = PMG_NOT_CONVERGED;
  if (status == PMG_OK && fallback) status = PMG_FALLBACK_USED;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = it;
    stats->n_hist = int(std::min<size_t>(hist_r.size(), 512));
    for (int k = 0; k < stats->n_hist; ++k) stats->res_hist[k] = hist_r[k];
    stats->rel_res = nf > 0 ? rtrue / nf : 0.0;
    stats->norm_f = nf;
    stats->t_solve_ms = tms;
    stats->t_guess_ms = tg;
    stats->n_vcycles = c->n_vcycles;
    stats->n_fine_applies = c->n_fine_applies;
    stats->n_graph_vcycles = c->n_graph_vcycles;
    stats->fallback = fallback;
  }
  if (status < 0) throw Error(status, status == PMG_EBREAKDOWN ? "breakdown: p^T A p <= 0 or z^T r <= 0"
                                                               : "non-finite iterate");
  return status;
}

// host xyz of level nodes under the current surface (fine isoparametric map)
static void node_xyz(pmg_ctx* c, int level, double* xyz) {
  Level& F = c->lv[0];
  Level& L = c->lv[level];
  const RefElem& rf = *F.re;
  const RefElem& rl = *L.re;
  Mat Bf, d1, d2;
  rf.tri_eval(rl.r, rl.s, Bf, d1, d2);  // fine basis at level nodes
  const int nptf = rf.np_tri, nptl = rl.np_tri;
  std::vector<double> xy2(size_t(L.num.n2d) * 2), eta2(size_t(L.num.n2d));
  for (int t = 0; t < L.num.nt; ++t)
    for (int a = 0; a < nptl; ++a) {
      double x = 0, y = 0, h = 0;
      for (int b = 0; b < nptf; ++b) {
        const double w = Bf(a, b);
        x += w * c->xyt_h[(size_t(t) * nptf + b) * 2];
        y += w * c->xyt_h[(size_t(t) * nptf + b) * 2 + 1];
        h += w * c->eta_h[F.num.map2d[size_t(t) * nptf + b]];
      }
      const int32_t g2 = L.num.map2d[size_t(t) * nptl + a];
      if (level == 0) {
        x = c->xyt_h[(size_t(t) * nptf + a) * 2];
        y = c->xyt_h[(size_t(t) * nptf + a) * 2 + 1];
        h = c->eta_h[g2];
      }
      xy2[2 * g2] = x;
      xy2[2 * g2 + 1] = y;
      eta2[g2] = h;
    }
  const double hd = c->mesh.depth;
  const int Lr = L.num.L, PZ = L.PZ;
  for (int64_t g2 = 0; g2 < L.num.n2d; ++g2)
    for (int z = 0; z < L.num.nz; ++z) {
      const int layer = std::min(z / PZ, Lr - 1);
      const int cc = z - layer * PZ;
      const double sig = (layer + 0.5 * (1.0 + rl.t[cc])) / Lr;
      const size_t g = size_t(g2) * L.num.nz + z;
      xyz[3 * g] = xy2[2 * g2];
      xyz[3 * g + 1] = xy2[2 * g2 + 1];
      xyz[3 * g + 2] = -hd + sig * (eta2[g2] + hd);
    }
}

}  // namespace pmg

// ===========================================================================
// C-ABI
// ===========================================================================
using namespace pmg;

#define PMG_TRY(ctx, ...)                                    \
  try {                                                      \
    __VA_ARGS__;                                             \
  } catch (const Error& e) {                                 \
    if (ctx) (ctx)->err = e.what();                          \
    g_err = e.what();                                        \
    return e.code;                                           \
  } catch (const std::exception& e) {                        \
    if (ctx) (ctx)->err = e.what();                          \
    g_err = e.what();                                        \
    return PMG_EINVAL;                                       \
  }

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static void need_device(pmg_ctx* c) {
  if (c->host_only) throw Error(PMG_ESTATE, "context was created host-only");
  HIPCHK(hipSetDevice(c->device));
}
static void check_level(const pmg_ctx* c, int level) {
  if (level < 0 || level >= c->nl) throw Error(PMG_EINVAL, "level out of range");
}

template <typename T>
static void smooth_t(pmg_ctx* c, int level, int sweeps, const T* f, T* u, hipStream_t st) {
  if (c->opt.smoother == PMG_SMOOTH_SCHWARZ) {
    schwarz_smooth<T>(c, level, f, u, false, false, sweeps, st);
    return;
  }
  if (c->opt.smoother == PMG_SMOOTH_CHEBYSHEV) {
    if (sweeps >= 1) cheb_smooth<T>(c, level, f, u, false, sweeps, st);
    return;
  }
  for (int m = 0; m < sweeps; ++m) jacobi_sweep<T>(c, level, f, u, st);
}

template <typename T>
static void transfer_t(pmg_ctx* c, int level, bool prolong, const T* x, T* y, hipStream_t st) {
  Level& L = c->lv[level];
  Level& C = c->lv[level + 1];
  if (prolong) {
    prolong_add<T>(c, level, x, y, OP_AVG_STORE, st);
  } else {
    launch_restrict_elem<T>(L.view, C.view, L.pit<T>(), L.piz<T>(), x, reinterpret_cast<T*>(c->Y), st);
    assemble<T>(c, level + 1, OP_STORE, y, nullptr, nullptr, nullptr, 0, 0, st);
  }
}

extern "C" {

void pmg_options_default(pmg_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->P = 6;
  o->nu1 = 2;
  o->nu2 = 2;
  o->precision = PMG_FP64;
  o->krylov = PMG_PCG;
  o->coarse = PMG_COARSE_EXACT;
  o->cheb_degree = 0;
  o->cheb_ratio = 0.0;
  o->exact_max = 12000;
  o->smoother = PMG_SMOOTH_JACOBI;
  o->smooth_ratio = 15.0;
  o->coarsening = PMG_COARSEN_BOTH;
  o->overlap = 1;
  o->seed = 0;
  o->geometry = PMG_GEOM_COLUMN;
  o->PZ = 0;
  o->fused_sum = 0;
  o->dss = 0;
  o->graphs = 0;
  o->nu1_coarse = -1;
  o->nu2_coarse = -1;
}

int pmg_abi_version(void) { return PMG_ABI_VERSION; }
const char* pmg_global_error(void) { return g_err.c_str(); }
const char* pmg_last_error(const pmg_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int pmg_create(const pmg_mesh* m, const pmg_options* o, pmg_ctx** out) {
  pmg_ctx* c = nullptr;
  try {
    if (!m || !o || !out) throw Error(PMG_EINVAL, "NULL argument");
    *out = nullptr;
    if (o->P < 1 || o->P > 8) throw Error(PMG_EINVAL, "P must be in 1..8");
    if (m->nv < 3 || m->nt < 1 || !m->xy || !m->tri || m->n_layers < 1 || !(m->depth > 0))
      throw Error(PMG_EINVAL, "bad mesh sizes");
    if (int64_t(m->nt) * m->n_layers >= (int64_t(1) << 31)) throw Error(PMG_EINVAL, "2^31 or more prisms");
    if (o->nu1 < 0 || o->nu2 < 0) throw Error(PMG_EINVAL, "negative sweep count");
    if (o->precision < 0 || o->precision > 5) throw Error(PMG_EINVAL, "bad precision");
    if (o->krylov < 0 || o->krylov > 3) throw Error(PMG_EINVAL, "bad krylov method");
    if (o->smoother < 0 || o->smoother > 2) throw Error(PMG_EINVAL, "bad smoother");
    if (o->smoother == PMG_SMOOTH_SCHWARZ && o->overlap < -1) throw Error(PMG_EINVAL, "bad Schwarz overlap");
    if (o->schwarz_store < 0 || o->schwarz_store > 7) throw Error(PMG_EINVAL, "bad schwarz_store mask");
    if (o->coarsening < 0 || o->coarsening > 2) throw Error(PMG_EINVAL, "bad coarsening");
    if (o->PZ > 8) throw Error(PMG_EINVAL, "PZ must be in 1..8 (or <= 0 for P)");
    if (o->geometry < 0 || o->geometry > 1) throw Error(PMG_EINVAL, "bad geometry mode");
    if (o->dss < 0 || o->dss > 1) throw Error(PMG_EINVAL, "bad dss mode");
    if (o->smoother == PMG_SMOOTH_CHEBYSHEV && !(o->smooth_ratio > 1.0))
      throw Error(PMG_EINVAL, "smooth_ratio must exceed 1");
    c = new pmg_ctx();
    c->opt = *o;
    c->host_only = o->host_only != 0;
    MeshIn& mi = c->mesh;
    mi.nv = m->nv;
    mi.nt = m->nt;
    mi.L = m->n_layers;
    mi.depth = m->depth;
    mi.xy.assign(m->xy, m->xy + 2 * size_t(m->nv));
    mi.tri.assign(m->tri, m->tri + 3 * size_t(m->nt));
    if (m->edge_tag) mi.edge_tag.assign(m->edge_tag, m->edge_tag + 3 * size_t(m->nt));
    else mi.edge_tag.assign(3 * size_t(m->nt), 0);
    for (int32_t v : mi.tri)
      if (v < 0 || v >= m->nv) throw Error(PMG_EINVAL, "triangle vertex id out of range");
    if (m->ncurved > 0) {
      if (!m->curved_edge || !m->circle) throw Error(PMG_EINVAL, "curved edges without circle data");
      mi.curved.assign(m->curved_edge, m->curved_edge + 2 * size_t(m->ncurved));
      mi.circle.assign(m->circle, m->circle + 3 * size_t(m->ncurved));
    }
    build_levels(c);
    if (!c->host_only) {
      HIPCHK(hipGetDevice(&c->device));
      upload_levels(c);
      set_surface(c, c->eta, nullptr);
    }
    *out = c;
    return PMG_OK;
  } catch (const Error& e) {
    g_err = e.what();
    delete c;
    return e.code;
  } catch (const std::exception& e) {
    g_err = e.what();
    delete c;
    return PMG_EINVAL;
  }
}

void pmg_destroy(pmg_ctx* c) {
  if (!c) return;
  if (!c->host_only) (void)hipSetDevice(c->device);
  delete c;
}

int pmg_n_levels(const pmg_ctx* c) { return c ? c->nl : PMG_EINVAL; }

int pmg_level_info_get(const pmg_ctx* c, int level, pmg_level_info* info) {
  if (!c || !info) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    const Level& L = c->lv[level];
    info->order = L.P;
    info->order_z = L.PZ;
    info->np = L.re->np;
    info->nq = L.re->nq;
    info->n_dof = L.num.n_dof;
    info->n_free = L.n_free;
    info->n_elem = L.num.n_elem;
    info->n_surface = L.num.n2d;
    std::vector<int32_t> col = L.num.colours();
    info->n_colours = col.empty() ? 0 : 1 + *std::max_element(col.begin(), col.end());
  });
  return PMG_OK;
}

int pmg_gather_map(const pmg_ctx* c, int level, int32_t* map) {
  if (!c || !map) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    c->lv[level].num.gather_map(map);
  });
  return PMG_OK;
}

int pmg_dss_colours(const pmg_ctx* c, int level, int32_t* colour) {
  if (!c || !colour) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    const std::vector<int32_t> col = c->lv[level].num.tri_colours();
    std::copy(col.begin(), col.end(), colour);
  });
  return PMG_OK;
}

int pmg_colours(const pmg_ctx* c, int level, int32_t* colour) {
  if (!c || !colour) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    std::vector<int32_t> col = c->lv[level].num.colours();
    std::copy(col.begin(), col.end(), colour);
  });
  return PMG_OK;
}

int pmg_surface_xy(const pmg_ctx* c, double* xy) {
  if (!c || !xy) return PMG_EINVAL;
  const Level& F = c->lv[0];
  const int npt = F.re->np_tri;
  for (int t = 0; t < F.num.nt; ++t)
    for (int a = 0; a < npt; ++a) {
      const int32_t g2 = F.num.map2d[size_t(t) * npt + a];
      xy[2 * size_t(g2)] = c->xyt_h[(size_t(t) * npt + a) * 2];
      xy[2 * size_t(g2) + 1] = c->xyt_h[(size_t(t) * npt + a) * 2 + 1];
    }
  return PMG_OK;
}

int pmg_dirichlet_mask(const pmg_ctx* c, int level, uint8_t* mask) {
  if (!c || !mask) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    const Level& L = c->lv[level];
    for (int64_t g2 = 0; g2 < L.num.n2d; ++g2)
      for (int z = 0; z < L.num.nz; ++z)
        mask[g2 * L.num.nz + z] = (L.dir2d_h[g2] || (L.top_dir && z == L.num.nz - 1)) ? 1 : 0;
  });
  return PMG_OK;
}

int pmg_set_surface(pmg_ctx* c, const double* eta, void* stream) {
  if (!c || !eta) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    set_surface(c, eta, S(stream));
  });
  return PMG_OK;
}

int pmg_node_xyz(pmg_ctx* c, int level, double* xyz) {
  if (!c || !xyz) return PMG_EINVAL;
  PMG_TRY(c, {
    check_level(c, level);
    node_xyz(c, level, xyz);
  });
  return PMG_OK;
}

int pmg_apply(pmg_ctx* c, int level, int precision, int flags, const void* x, void* y, void* stream) {
  if (!c || !x || !y) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    check_level(c, level);
    hipStream_t st = S(stream);
    Level& L = c->lv[level];
    if (precision == PMG_FP64) {
      const double* xin = (const double*)x;
      if (flags & 1) { launch_mask<double>(L.view, xin, L.r64, st); xin = L.r64; }
      apply_op<double>(c, level, xin, (flags & 1) ? OP_STORE : OP_RAW, (double*)y, nullptr, nullptr, nullptr, 0, 0,
                       st);
    } else if (precision == PMG_MIXED_FP32 || precision == PMG_MIXED_BF16 || precision == PMG_MIXED_BF16G ||
               precision == PMG_MIXED_BF16X3 || precision == PMG_MIXED_BF16X2) {
      set_lowp(c, precision);
      const float* xin = (const float*)x;
      if (flags & 1) { launch_mask<float>(L.view, xin, L.r32, st); xin = L.r32; }
      apply_op<float>(c, level, xin, (flags & 1) ? OP_STORE : OP_RAW, (float*)y, nullptr, nullptr, nullptr, 0, 0,
                      st);
    } else {
      throw Error(PMG_EINVAL, "bad precision");
    }
  });
  return PMG_OK;
}

int pmg_diagonal(pmg_ctx* c, int level, double* d, void* stream) {
  if (!c || !d) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    check_level(c, level);
    launch_copy<double>(c->lv[level].diag, d, c->lv[level].num.n_dof, S(stream));
  });
  return PMG_OK;
}

int pmg_smooth(pmg_ctx* c, int level, int precision, int sweeps, const void* f, void* u, void* stream) {
  if (!c || !f || !u || sweeps < 0) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    check_level(c, level);
    if (level == c->nl - 1) throw Error(PMG_EINVAL, "no smoother on the coarsest level");
    if (precision == PMG_FP64) smooth_t<double>(c, level, sweeps, (const double*)f, (double*)u, S(stream));
    else {
      set_lowp(c, precision);
      smooth_t<float>(c, level, sweeps, (const float*)f, (float*)u, S(stream));
    }
  });
  return PMG_OK;
}

int pmg_prolong(pmg_ctx* c, int level, int precision, const void* xc, void* yf, void* stream) {
  if (!c || !xc || !yf) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    if (level < 0 || level + 1 >= c->nl) throw Error(PMG_EINVAL, "level out of range");
    if (precision == PMG_FP64) transfer_t<double>(c, level, true, (const double*)xc, (double*)yf, S(stream));
    else transfer_t<float>(c, level, true, (const float*)xc, (float*)yf, S(stream));
  });
  return PMG_OK;
}

int pmg_restrict(pmg_ctx* c, int level, int precision, const void* xf, void* yc, void* stream) {
  if (!c || !xf || !yc) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    if (level < 0 || level + 1 >= c->nl) throw Error(PMG_EINVAL, "level out of range");
    if (precision == PMG_FP64) transfer_t<double>(c, level, false, (const double*)xf, (double*)yc, S(stream));
    else transfer_t<float>(c, level, false, (const float*)xf, (float*)yc, S(stream));
  });
  return PMG_OK;
}

int pmg_coarse_solve(pmg_ctx* c, int precision, const void* f, void* u, void* stream) {
  if (!c || !f || !u) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    if (precision == PMG_FP64) coarse_solve<double>(c, (const double*)f, (double*)u, S(stream));
    else {
      set_lowp(c, precision);
      coarse_solve<float>(c, (const float*)f, (float*)u, S(stream));
    }
  });
  return PMG_OK;
}

int pmg_vcycle(pmg_ctx* c, int precision, const void* r, void* z, void* stream) {
  if (!c || !r || !z) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    if (precision == PMG_FP64) vcycle<double>(c, 0, (const double*)r, (double*)z, S(stream));
    else {
      set_lowp(c, precision);
      vcycle<float>(c, 0, (const float*)r, (float*)z, S(stream));
    }
  });
  return PMG_OK;
}

int pmg_schwarz_info_get(const pmg_ctx* c, int level, pmg_schwarz_info* info) {
  if (!c || !info) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    const Level& L = c->lv[level];
    if (!L.has_sz) throw Error(PMG_EINVAL, "no Schwarz smoother on this level");
    info->dt = L.sz.dt;
    info->dz = L.sz.dz;
    info->n_sub = L.sz.n_sub;
    info->max_size = L.sz.max_n;
    info->total = L.sz.total;
    info->inv_entries = L.sz.tile_off.back();
  });
  return PMG_OK;
}

int pmg_schwarz_nodes(const pmg_ctx* c, int level, int32_t* ptr, int32_t* nodes) {
  if (!c || !ptr || !nodes) return PMG_EINVAL;
  PMG_TRY(const_cast<pmg_ctx*>(c), {
    check_level(c, level);
    const Level& L = c->lv[level];
    if (!L.has_sz) throw Error(PMG_EINVAL, "no Schwarz smoother on this level");
    std::memcpy(ptr, L.sz.sd_ptr.data(), L.sz.sd_ptr.size() * sizeof(int32_t));
    std::memcpy(nodes, L.sz.sd_node.data(), L.sz.sd_node.size() * sizeof(int32_t));
  });
  return PMG_OK;
}

int pmg_coarse_info(const pmg_ctx* c, int* mode, int* degree, double* lmin, double* lmax, int64_t* n_free) {
  if (!c) return PMG_EINVAL;
  if (mode) *mode = c->coarse_exact ? PMG_COARSE_EXACT : PMG_COARSE_CHEBYSHEV;
  if (degree) *degree = c->coarse_exact ? 0 : c->cheb_k;
  if (lmin) *lmin = c->cheb_lmin;
  if (lmax) *lmax = c->cheb_lmax;
  if (n_free) *n_free = c->lv[c->nl - 1].n_free;
  return PMG_OK;
}

int pmg_get_params(const pmg_ctx* c, double* omega, double* lmin, double* lmax) {
  if (!c) return PMG_EINVAL;
  if (omega)
    for (int i = 0; i < c->nl; ++i) omega[i] = c->lv[i].omega;
  if (lmin) *lmin = c->cheb_lmin;
  if (lmax) *lmax = c->cheb_lmax;
  return PMG_OK;
}

int pmg_set_params(pmg_ctx* c, const double* omega, double lmin, double lmax) {
  if (!c) return PMG_EINVAL;
  c->gen++;
  if (omega)
    for (int i = 0; i + 1 < c->nl; ++i) {
      if (!(omega[i] > 0)) return PMG_EINVAL;
      c->lv[i].omega = omega[i];
      c->lv[i].omega_user = omega[i];
    }
  // kept by later pmg_set_surface calls (operators of t = 0 reused, as in the paper's strategy I)
  if (lmax > 0) c->cheb_lmax = c->opt.cheb_lmax = lmax;
  if (lmin > 0) c->cheb_lmin = c->opt.cheb_lmin = lmin;
  if (lmin > 0 && lmax > 0 && c->opt.cheb_degree <= 0) c->opt.cheb_degree = c->cheb_k;
  return PMG_OK;
}

// ---------------------------------------------------------------------------
// free-surface time stepping (eq. FSeta, eq. FSphi) around the Laplace solve
// ---------------------------------------------------------------------------
static void fnpf_alloc(pmg_ctx* c) {
  if (c->fn_Dr) return;
  const RefElem& re = *c->lv[0].re;
  Mat B, Dr, Ds, B1, D1;
  re.tri_eval(re.r, re.s, B, Dr, Ds);
  re.line_eval(re.t, B1, D1);
  std::vector<double> dtop(size_t(re.n1));
  for (int k = 0; k < re.n1; ++k) dtop[size_t(k)] = D1(re.n1 - 1, k);
  c->fn_Dr = c->U(Dr.v);
  c->fn_Ds = c->U(Ds.v);
  c->fn_dtop = c->U(dtop);
  const size_t n2 = size_t(c->lv[0].num.n2d);
  c->fn_y0 = c->A<double>(2 * n2);
  c->fn_ys = c->A<double>(2 * n2);
  c->fn_acc = c->A<double>(2 * n2);
  c->fn_k = c->A<double>(2 * n2);
  c->fn_gr = c->A<double>(4 * n2);
  c->fn_w = c->A<double>(n2);
  const size_t N = size_t(c->lv[0].num.n_dof);
  c->fn_p1 = c->A<double>(N);
  c->fn_p3 = c->A<double>(N);
  c->fn_p3prev = c->A<double>(N);
}

// (fx, fy) of a surface field: element derivatives averaged over triangles
static void surface_grad(pmg_ctx* c, const double* f, double* fx, double* fy, hipStream_t st) {
  const Level& F = c->lv[0];
  launch_surf_grad_elem(F.num.nt, F.re->np_tri, F.map2d, c->fn_Dr, c->fn_Ds, c->xyt, f, c->Y, st);
  launch_surf_avg(F.num.n2d, F.inc_ptr, F.inc, c->Y, fx, fy, st);
}

static void surface_w(pmg_ctx* c, const double* phi, const double* eta, double* w, hipStream_t st) {
  const Level& F = c->lv[0];
  launch_surf_w(F.num.n2d, F.num.nz, F.num.L, F.PZ, c->mesh.depth, c->fn_dtop, phi, eta, w, st);
}

// The smoothing weights and the coarse interval and degree keep their current
// values for later surfaces (the parameter part of strategy I of Sec. 6).
static void fnpf_freeze(pmg_ctx* c) {
  for (int i = 0; i + 1 < c->nl; ++i)
    if (!(c->lv[i].omega_user > 0)) c->lv[i].omega_user = c->lv[i].omega;
  if (!c->coarse_exact) {
    if (!(c->opt.cheb_lmax > 0)) c->opt.cheb_lmax = c->cheb_lmax;
    if (!(c->opt.cheb_lmin > 0)) c->opt.cheb_lmin = c->cheb_lmin;
    if (c->opt.cheb_degree <= 0) c->opt.cheb_degree = c->cheb_k;
  }
}

// deta, dphis at the state (eta, phis): surface geometry, Laplace solve (from
// phi when warm, else from zero), w~, gradients, eq. FSeta / eq. FSphi.
static int fnpf_rhs(pmg_ctx* c, const double* eta, const double* phis, double g, double* phi, bool warm,
                    double rtol, double atol, int imax, double* deta, double* dphis, pmg_stats* stats,
                    hipStream_t st) {
  const int64_t n2 = c->lv[0].num.n2d;
  set_surface(c, eta, st);
  pmg_stats local;
  const int rc = solve(c, phis, nullptr, phi, warm ? PMG_GUESS_GIVEN : PMG_GUESS_ZERO, nullptr, nullptr, rtol, atol,
                       imax, stats ? stats : &local, st);
  if (rc != PMG_OK && rc != PMG_NOT_CONVERGED) return rc;
  double* ex = c->fn_gr;
  double* ey = ex + n2;
  double* px = ey + n2;
  double* py = px + n2;
  surface_w(c, phi, eta, c->fn_w, st);
  surface_grad(c, eta, ex, ey, st);
  surface_grad(c, phis, px, py, st);
  launch_fnpf_rhs(n2, g, eta, ex, ey, px, py, c->fn_w, deta, dphis, st);
  return rc;
}

int pmg_surface_grad(pmg_ctx* c, const double* f, double* fx, double* fy, void* stream) {
  if (!c || !f || !fx || !fy) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    fnpf_alloc(c);
    surface_grad(c, f, fx, fy, S(stream));
  });
  return PMG_OK;
}

int pmg_surface_w(pmg_ctx* c, const double* phi, double* w, void* stream) {
  if (!c || !phi || !w) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    fnpf_alloc(c);
    surface_w(c, phi, c->eta, w, S(stream));
  });
  return PMG_OK;
}

int pmg_fnpf_rhs(pmg_ctx* c, const double* eta, const double* phis, double g, double* phi, int32_t warm,
                 double rtol, double atol, int32_t imax, double* deta, double* dphis, pmg_stats* stats,
                 void* stream) {
  if (!c || !eta || !phis || !phi || !deta || !dphis) return PMG_EINVAL;
  int rc = PMG_OK;
  PMG_TRY(c, {
    need_device(c);
    fnpf_alloc(c);
    fnpf_freeze(c);
    rc = fnpf_rhs(c, eta, phis, g, phi, warm != 0, rtol, atol, imax, deta, dphis, stats, S(stream));
  });
  return rc;
}

int pmg_fnpf_erk4(pmg_ctx* c, double* eta, double* phis, double dt, double g, double* phi, int32_t warm,
                  double rtol, double atol, int32_t imax, pmg_fnpf_stats* fs, void* stream) {
  if (!c || !eta || !phis || !phi || !(dt > 0)) return PMG_EINVAL;
  int rc = PMG_OK;
  PMG_TRY(c, {
    need_device(c);
    fnpf_alloc(c);
    fnpf_freeze(c);
    hipStream_t st = S(stream);
    const int64_t n2 = c->lv[0].num.n2d;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    HIPCHK(hipMemcpyAsync(c->fn_y0, eta, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c->fn_y0 + n2, phis, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    // classical Runge-Kutta: stage s evaluates at y0 + a_s dt k_{s-1}; weights b = (1, 2, 2, 1)/6
    const double a[4] = {0.0, 0.5, 0.5, 1.0}, b[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
    const int64_t N = c->lv[0].num.n_dof;
    const bool have_prev = warm != 0 && c->fn_dt == dt;
    pmg_fnpf_stats loc{};
    for (int s = 0; s < 4 && rc >= 0; ++s) {
      const double* y = s == 0 ? c->fn_y0 : c->fn_ys;
      // stage predictor (linear in time over steps of dt/2): stage 2 (t + dt/2)
      // from t and t - dt/2, stage 4 (t + dt) from t + dt/2 and t; stage 3 (t +
      // dt/2) starts from stage 2's solution, stage 1 from phi
      if (s == 1 && have_prev) launch_lin_extrap(N, c->fn_p1, c->fn_p3prev, phi, st);
      if (s == 3) launch_lin_extrap(N, c->fn_p3, c->fn_p1, phi, st);
      pmg_stats ps;
      const int r = fnpf_rhs(c, y, y + n2, g, phi, warm != 0 || s > 0, rtol, atol, imax, c->fn_k, c->fn_k + n2,
                             &ps, st);
      if (r < 0) { rc = r; break; }
      if (r != PMG_OK) rc = r;
      if (s == 0) launch_copy<double>(phi, c->fn_p1, N, st);
      if (s == 2) launch_copy<double>(phi, c->fn_p3, N, st);
      loc.iters[s] = ps.iters;
      loc.rel_res[s] = ps.rel_res;
      loc.t_solve_ms += ps.t_solve_ms;
      // next stage state (unused after the last stage) and the weighted sum
      launch_rk_stage(2 * n2, c->fn_y0, c->fn_k, s < 3 ? a[s + 1] * dt : 0.0, s < 3 ? c->fn_ys : nullptr, b[s] * dt,
                      s == 0, c->fn_acc, st);
    }
    if (rc >= 0) {
      std::swap(c->fn_p3, c->fn_p3prev);
      c->fn_dt = dt;
      launch_rk_stage(2 * n2, c->fn_y0, c->fn_acc, 1.0, c->fn_ys, 0.0, false, c->fn_k, st);
      HIPCHK(hipMemcpyAsync(eta, c->fn_ys, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(phis, c->fn_ys + n2, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    loc.t_step_ms = ms;
    loc.status = rc;
    if (fs) *fs = loc;
  });
  return rc;
}

int pmg_set_reuse(pmg_ctx* c, int mode, void* stream) {
  if (!c || mode < PMG_REUSE_NONE || mode > PMG_REUSE_LIN) return PMG_EINVAL;
  c->gen++;
  PMG_TRY(c, {
    need_device(c);
    hipStream_t st = S(stream);
    if (mode != PMG_REUSE_NONE) {
      fnpf_freeze(c);
      // the kept preconditioner includes the native copies of the current surface
      for (int i = 0; i < c->nl; ++i)
        for (int f = 0; f < 3; ++f) ensure_native(c, c->lv[i], f, st);
      if (mode == PMG_REUSE_LIN) {
        const int64_t n2 = c->lv[0].num.n2d;
        if (!c->eta_flat) {
          c->eta_flat = c->A<double>(size_t(n2));
          HIPCHK(hipMemsetAsync(c->eta_flat, 0, n2 * sizeof(double), st));
        }
        for (int i = 1; i < c->nl; ++i) {
          if (level_geom(c, i, c->eta_flat, true, 7, st)) throw Error(PMG_EMESH, "inverted element at eta = 0");
          level_diag(c, c->lv[i], st);
        }
        schwarz_setup(c, st, 1);
        coarse_setup(c, st);
        HIPCHK(hipStreamSynchronize(st));
      }
    }
    c->reuse = mode;
  });
  return PMG_OK;
}

int pmg_solve(pmg_ctx* c, const double* phi_surf, const double* phi_bc, double* phi, int guess_mode,
              const pmg_net* net, const double* const* hist_phi, double rtol, double atol, int32_t imax,
              pmg_stats* stats, void* stream) {
  if (!c) return PMG_EINVAL;
  int rc = PMG_OK;
  PMG_TRY(c, {
    need_device(c);
    rc = solve(c, phi_surf, phi_bc, phi, guess_mode, const_cast<pmg_net*>(net), hist_phi, rtol, atol, imax, stats,
               S(stream));
  });
  return rc;
}

int pmg_set_solver(pmg_ctx* c, int precision, int krylov) {
  if (!c || precision < 0 || precision > 5 || krylov < 0 || krylov > 3) return PMG_EINVAL;
  c->gen++;
  c->opt.precision = precision;
  c->opt.krylov = krylov;
  return PMG_OK;
}

int pmg_time_kernel(pmg_ctx* c, int kernel, int level, int precision, int reps, double* ms, void* stream) {
  if (!c || !ms || reps < 1) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    check_level(c, level);
    hipStream_t st = S(stream);
    Level& L = c->lv[level];
    const bool f64 = precision == PMG_FP64;
    set_lowp(c, precision);
    if ((kernel == PMG_K_RESTRICT || kernel == PMG_K_PROLONG) && level + 1 >= c->nl)
      throw Error(PMG_EINVAL, "no coarser level");
    if (kernel == PMG_K_SCHWARZ && !L.has_sz) throw Error(PMG_EINVAL, "no Schwarz smoother on this level");
    if (kernel == PMG_K_SCHWARZ) need_sz(L, f64, c->lowp);
    launch_fill<double>(L.r64, 1.0, L.num.n_dof, st);
    launch_fill<float>(L.r32, 1.0f, L.num.n_dof, st);
    auto one = [&]() {
      switch (kernel) {
        case PMG_K_ELEMENT_OP:
          if (f64) ax_elem<double>(c, level, L.r64, st); else ax_elem<float>(c, level, L.r32, st);
          break;
        case PMG_K_ASSEMBLE:
          if (f64) assemble<double>(c, level, OP_STORE, c->s_y, nullptr, nullptr, nullptr, 0, 0, st);
          else assemble<float>(c, level, OP_STORE, c->s_z32, nullptr, nullptr, nullptr, 0, 0, st);
          break;
        case PMG_K_GEOMETRY:
          launch_geom(c->lv[0].view, L.view, c->mesh.depth, c->xyt, c->eta, L.gmats, L.wq, L.zq, L.zw, L.G64,
                      L.G32, L.G16, c->bad, st, L.geo64, L.geo32);
          break;
        case PMG_K_RESTRICT:
          if (f64) launch_restrict_elem<double>(L.view, c->lv[level + 1].view, L.pit64, L.piz64, L.r64, c->Y, st);
          else launch_restrict_elem<float>(L.view, c->lv[level + 1].view, L.pit32, L.piz32, L.r32,
                                           reinterpret_cast<float*>(c->Y), st);
          break;
        case PMG_K_PROLONG: {
          Level& C = c->lv[level + 1];
          if (f64) prolong_add<double>(c, level, C.r64, c->s_y, OP_AVG_STORE, st);
          else prolong_add<float>(c, level, C.r32, reinterpret_cast<float*>(c->s_y), OP_AVG_STORE, st);
          break;
        }
        case PMG_K_COPY: launch_copy<double>(L.r64, c->s_y, L.num.n_dof, st); break;
        case PMG_K_COLSUM_OP: {
          const bool ok = f64 ? ax_elem<double>(c, level, L.r64, st, true) : ax_elem<float>(c, level, L.r32, st, true);
          if (!ok) throw Error(PMG_EINVAL, "no column-sum element operator on this level");
          break;
        }
        case PMG_K_COL_SUM_STORE: case PMG_K_COL_SUM_CHEB: {
          // x = s_y / s_z32, r = r, d = the level's direction vector (column sums read from c->Y)
          if (!L.colsum) throw Error(PMG_EINVAL, "no column-sum layout on this level");
          const int op = kernel == PMG_K_COL_SUM_STORE ? OP_STORE : OP_CHEB;
          if (f64)
            launch_col_sum<double>(L.view, op, c->Y, c->s_y, L.r64, L.dinv64, L.d64 ? L.d64 : c->s_q, 0.5, 0.1,
                                   c->partial, st);
          else
            launch_col_sum<float>(L.view, op, reinterpret_cast<const float*>(c->Y), c->s_z32, L.r32, L.dinv32,
                                  L.d32 ? L.d32 : L.r32, 0.5, 0.1, c->partial, st);
          break;
        }
        case PMG_K_SCHWARZ:
          if (f64) launch_sd_apply<double, double>(L.szv, L.sz_inv64, L.r64, nullptr, L.sz_z64, st);
          else if (c->lowp == G_BF16) launch_sd_apply<float, bf16_t>(L.szv, L.sz_inv16, L.r32, nullptr, L.sz_z32, st);
          else launch_sd_apply<float, float>(L.szv, L.sz_inv32, L.r32, nullptr, L.sz_z32, st);
          break;
        default: throw Error(PMG_EINVAL, "unknown kernel");
      }
    };
    one();  // warm
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int k = 0; k < reps; ++k) one();
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = double(t) / reps;
  });
  return PMG_OK;
}

int pmg_net_level(const pmg_ctx* c) { return c ? net_level(c) : PMG_EINVAL; }

int pmg_features(pmg_ctx* c, const double* surf, const double* p1, const double* p2, const double* p3,
                 const double* pnow, float* X,
                 float* T, void* stream) {
  if (!c || !surf || !p1 || !p2 || !X || (T && !pnow)) return PMG_EINVAL;
  PMG_TRY(c, {
    need_device(c);
    features(c, surf, p1, p2, p3, pnow, X, T, S(stream));
  });
  return PMG_OK;
}

int pmg_net_create(const pmg_ctx* c, int32_t width, int32_t depth, uint64_t seed, pmg_net** out) {
  if (!c || !out || width < 1 || width > 1024 || depth < 0 || depth > 8) return PMG_EINVAL;
  pmg_net* n = nullptr;
  try {
    if (c->host_only) throw Error(PMG_ESTATE, "host-only context");
    HIPCHK(hipSetDevice(c->device));
    n = new pmg_net();
    n->device = c->device;
    n->width = width;
    n->depth = depth;
    std::vector<int> dims{n->din};
    for (int l = 0; l < depth; ++l) dims.push_back(width);
    dims.push_back(1);
    int64_t o = 0;
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
      n->fin.push_back(dims[l]);
      n->fout.push_back(dims[l + 1]);
      n->woff.push_back(o);
      o += int64_t(dims[l]) * dims[l + 1];
      n->boff.push_back(o);
      o += dims[l + 1];
    }
    n->np = o;
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights from the counter generator, zero biases
    std::vector<float> th(n->np, 0.0f);
    for (size_t l = 0; l < n->fin.size(); ++l) {
      const double s = 1.0 / std::sqrt(double(n->fin[l]));
      for (int64_t k = 0; k < int64_t(n->fin[l]) * n->fout[l]; ++k)
        th[n->woff[l] + k] = float((2.0 * splitmix_unit(seed, uint64_t(n->woff[l] + k)) - 1.0) * s);
    }
    n->theta = n->A<float>(n->np);
    n->grad = n->A<float>(n->np);
    n->m = n->A<float>(n->np);
    n->v = n->A<float>(n->np);
    HIPCHK(hipMemcpy(n->theta, th.data(), n->np * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(n->m, 0, n->np * sizeof(float)));
    HIPCHK(hipMemset(n->v, 0, n->np * sizeof(float)));
    n->mean_h.assign(n->din, 0.0f);
    n->istd_h.assign(n->din, 1.0f);
    n->mean = n->A<float>(n->din);
    n->istd = n->A<float>(n->din);
    HIPCHK(hipMemcpy(n->mean, n->mean_h.data(), n->din * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(n->istd, n->istd_h.data(), n->din * sizeof(float), hipMemcpyHostToDevice));
    n->partial = n->A<double>(MLP_RED);
    n->scal = n->A<double>(64);
    net_reserve(n, 1024);
    hipError_t se;
    n->scratch = net_scratch_ptr(n->device, &se);
    if (!n->scratch) throw Error(PMG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(se));
    *out = n;
    return PMG_OK;
  } catch (const Error& e) {
    g_err = e.what();
    delete n;
    return e.code;
  } catch (const std::exception& e) {
    g_err = e.what();
    delete n;
    return PMG_EINVAL;
  }
}

void pmg_net_destroy(pmg_net* n) {
  if (!n) return;
  (void)hipSetDevice(n->device);
  delete n;
}

int pmg_net_size(const pmg_net* n, int64_t* n_params, int32_t* d_in, int32_t* width, int32_t* depth) {
  if (!n) return PMG_EINVAL;
  if (n_params) *n_params = n->np;
  if (d_in) *d_in = n->din;
  if (width) *width = n->width;
  if (depth) *depth = n->depth;
  return PMG_OK;
}

int pmg_net_get_params(const pmg_net* n, float* theta, float* mean, float* inv_std, double* tscale) {
  if (!n) return PMG_EINVAL;
  try {
    HIPCHK(hipSetDevice(n->device));
    HIPCHK(hipDeviceSynchronize());
    if (theta) HIPCHK(hipMemcpy(theta, n->theta, n->np * sizeof(float), hipMemcpyDeviceToHost));
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  }
  if (mean) std::copy(n->mean_h.begin(), n->mean_h.end(), mean);
  if (inv_std) std::copy(n->istd_h.begin(), n->istd_h.end(), inv_std);
  if (tscale) *tscale = n->tscale;
  return PMG_OK;
}

int pmg_net_set_params(pmg_net* n, const float* theta, const float* mean, const float* inv_std, double tscale) {
  if (!n) return PMG_EINVAL;
  try {
    HIPCHK(hipSetDevice(n->device));
    if (theta) HIPCHK(hipMemcpy(n->theta, theta, n->np * sizeof(float), hipMemcpyHostToDevice));
    if (mean) n->mean_h.assign(mean, mean + n->din);
    if (inv_std) n->istd_h.assign(inv_std, inv_std + n->din);
    if (tscale > 0) n->tscale = tscale;
    HIPCHK(hipMemcpy(n->mean, n->mean_h.data(), n->din * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(n->istd, n->istd_h.data(), n->din * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(n->m, 0, n->np * sizeof(float)));
    HIPCHK(hipMemset(n->v, 0, n->np * sizeof(float)));
    n->t = 0;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  }
  return PMG_OK;
}

int pmg_net_forward(pmg_net* n, const float* X, int64_t rows, float* y, void* stream) {
  if (!n || !X || !y || rows < 0) return PMG_EINVAL;
  PMG_TRY(n, {
    HIPCHK(hipSetDevice(n->device));
    const int L = int(n->fin.size());
    for (int64_t r0 = 0; r0 < rows; r0 += 16384) {
      const int B = int(std::min<int64_t>(16384, rows - r0));
      net_forward(n, X + r0 * n->din, B, S(stream));
      launch_copy<float>(n->H[L - 1], y + r0, B, S(stream));
    }
  });
  return PMG_OK;
}

int pmg_net_forward_noalloc(pmg_net* n, const float* X, int64_t rows, float* y, void* stream) {
  if (!n || rows < 0) return PMG_EINVAL;
  if (rows == 0) return PMG_OK;
  if (!X || !y) return PMG_EINVAL;
  PMG_TRY(n, {
    HIPCHK(hipSetDevice(n->device));
    if (n->width > NET_NOALLOC_WIDTH)
      throw Error(PMG_EINVAL, "pmg_net_forward_noalloc: hidden width " + std::to_string(n->width) +
                                  " exceeds the allocation-free limit of " + std::to_string(NET_NOALLOC_WIDTH));
    if (!n->scratch) throw Error(PMG_ESTATE, "pmg_net_forward_noalloc: activation array not set up");
    hipStream_t st = S(stream);
    const int L = int(n->fin.size());
    float* half[2] = {n->scratch, n->scratch + size_t(NET_NOALLOC_ROWS) * NET_NOALLOC_WIDTH};
    for (int64_t r0 = 0; r0 < rows; r0 += NET_NOALLOC_ROWS) {
      const int B = int(std::min<int64_t>(NET_NOALLOC_ROWS, rows - r0));
      const float* h = X + r0 * n->din;
      for (int l = 0; l < L; ++l) {
        // hidden layers write alternate halves; the scalar output layer writes y directly
        float* out = l + 1 < L ? half[l & 1] : y + r0;
        launch_gemm(B, n->fout[l], n->fin[l], h, n->fin[l], 1, n->theta + n->woff[l], n->fout[l], 1,
                    n->theta + n->boff[l], nullptr, out, n->fout[l], l + 1 < L, st);
        h = out;
      }
    }
  });
  return PMG_OK;
}

int pmg_net_loss_grad(pmg_net* n, const float* X, const float* T, int32_t rows, double* loss, float* grad,
                      void* stream) {
  if (!n || !X || !T || rows < 1) return PMG_EINVAL;
  PMG_TRY(n, {
    HIPCHK(hipSetDevice(n->device));
    hipStream_t st = S(stream);
    net_backward(n, X, T, rows, n->scal, st);
    double l = 0;
    HIPCHK(hipMemcpyAsync(&l, n->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad) HIPCHK(hipMemcpyAsync(grad, n->grad, n->np * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (loss) *loss = l / rows;
  });
  return PMG_OK;
}

int pmg_net_adam_step(pmg_net* n, double lr, void* stream) {
  if (!n || !(lr > 0)) return PMG_EINVAL;
  PMG_TRY(n, {
    HIPCHK(hipSetDevice(n->device));
    n->t += 1;
    launch_adam(n->theta, n->grad, n->m, n->v, n->np, lr, n->t, S(stream));
  });
  return PMG_OK;
}

int pmg_net_train(pmg_net* n, const float* X, const float* T, int64_t rows, int32_t steps, int32_t batch,
                  double lr, uint64_t seed, double* final_loss, void* stream) {
  if (!n || !X || !T || rows < 1 || steps < 1 || batch < 1 || !(lr > 0)) return PMG_EINVAL;
  PMG_TRY(n, {
    HIPCHK(hipSetDevice(n->device));
    hipStream_t st = S(stream);
    // normalisation from the training set: inputs to zero mean / unit variance, targets by their rms
    double* stats = n->scal + 8;
    launch_colstats(X, rows, n->din, stats, st);
    launch_colstats(T, rows, 1, stats + 2 * n->din, st);
    std::vector<double> h(2 * n->din + 2);
    HIPCHK(hipMemcpyAsync(h.data(), stats, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int cc = 0; cc < n->din; ++cc) {
      const double mu = h[2 * cc], var = std::max(h[2 * cc + 1] - mu * mu, 0.0);
      n->mean_h[cc] = float(mu);
      n->istd_h[cc] = float(var > 1e-30 ? 1.0 / std::sqrt(var) : 1.0);
    }
    n->tscale = std::sqrt(std::max(h[2 * n->din + 1], 1e-300));
    HIPCHK(hipMemcpy(n->mean, n->mean_h.data(), n->din * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(n->istd, n->istd_h.data(), n->din * sizeof(float), hipMemcpyHostToDevice));
    net_reserve(n, batch);
    if (n->nloss < steps) {
      n->losses = n->A<double>(steps);
      n->nloss = steps;
    }
    for (int s = 0; s < steps; ++s) {
      launch_gather_batch(X, T, rows, n->din, batch, seed, uint64_t(s), n->mean, n->istd, float(1.0 / n->tscale),
                          n->Xb, n->Tb, st);
      net_backward(n, n->Xb, n->Tb, batch, n->losses + s, st);
      n->t += 1;
      launch_adam(n->theta, n->grad, n->m, n->v, n->np, lr, n->t, st);
    }
    std::vector<double> ls(steps);
    HIPCHK(hipMemcpyAsync(ls.data(), n->losses, steps * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int tail = std::min(20, steps);
    double acc = 0;
    for (int s = steps - tail; s < steps; ++s) acc += ls[s] / batch;
    if (final_loss) *final_loss = acc / tail;
  });
  return PMG_OK;
}

// file: "PMGNET01", din, width, depth, np, theta[np] (f32), mean[din], inv_std[din], tscale (f64), FNV-1a of all
int pmg_net_save(const pmg_net* n, const char* path) {
  if (!n || !path) return PMG_EINVAL;
  std::vector<float> th(n->np);
  if (pmg_net_get_params(n, th.data(), nullptr, nullptr, nullptr) != PMG_OK) return PMG_EDEVICE;
  std::string buf("PMGNET01");
  auto put = [&](const void* p, size_t k) { buf.append(static_cast<const char*>(p), k); };
  const int32_t hdr[3] = {n->din, n->width, n->depth};
  put(hdr, sizeof(hdr));
  put(&n->np, sizeof(n->np));
  put(th.data(), th.size() * sizeof(float));
  put(n->mean_h.data(), n->din * sizeof(float));
  put(n->istd_h.data(), n->din * sizeof(float));
  put(&n->tscale, sizeof(double));
  uint64_t hsh = 1469598103934665603ull;
  for (unsigned char ch : buf) hsh = (hsh ^ ch) * 1099511628211ull;
  put(&hsh, sizeof(hsh));
  std::ofstream f(path, std::ios::binary);
  if (!f) { g_err = "cannot open file"; return PMG_EINVAL; }
  f.write(buf.data(), std::streamsize(buf.size()));
  return f ? PMG_OK : PMG_EINVAL;
}

int pmg_net_load(pmg_net* n, const char* path) {
  if (!n || !path) return PMG_EINVAL;
  std::ifstream f(path, std::ios::binary);
  if (!f) { g_err = "cannot open file"; return PMG_EINVAL; }
  std::string buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  const size_t need = 8 + 12 + 8 + n->np * 4 + 2 * size_t(n->din) * 4 + 8 + 8;
  if (buf.size() != need || buf.compare(0, 8, "PMGNET01") != 0) { g_err = "not a matching network file"; return PMG_EINVAL; }
  uint64_t hsh = 1469598103934665603ull;
  for (size_t k = 0; k + 8 < buf.size(); ++k) hsh = (hsh ^ (unsigned char)buf[k]) * 1099511628211ull;
  uint64_t stored;
  std::memcpy(&stored, buf.data() + buf.size() - 8, 8);
  if (stored != hsh) { g_err = "network file checksum mismatch"; return PMG_EINVAL; }
  int32_t hdr[3];
  int64_t np;
  std::memcpy(hdr, buf.data() + 8, 12);
  std::memcpy(&np, buf.data() + 20, 8);
  if (hdr[0] != n->din || hdr[1] != n->width || hdr[2] != n->depth || np != n->np) {
    g_err = "network shape mismatch";
    return PMG_EINVAL;
  }
  const char* p = buf.data() + 28;
  std::vector<float> th(np), mean(n->din), istd(n->din);
  std::memcpy(th.data(), p, np * 4);
  p += np * 4;
  std::memcpy(mean.data(), p, n->din * 4);
  p += n->din * 4;
  std::memcpy(istd.data(), p, n->din * 4);
  p += n->din * 4;
  double ts;
  std::memcpy(&ts, p, 8);
  return pmg_net_set_params(n, th.data(), mean.data(), istd.data(), ts);
}

}  // extern "C"
