// Overlapping additive Schwarz smoother (Sec. 5.2, eq. Mass, eq. weights):
// S^-1 = W sum_k R_k^T (R_k A R_k^T)^-1 R_k, W = (sum_k R_k R_k^T)^-1, one
// subdomain per prism.  Subdomain k holds prism k's nodes and, in every prism
// that touches it, the nodes within dt lattice steps (in the triangle) and dz
// steps (along the extrusion) of the entity the two prisms share; Dirichlet
// nodes are left out.  The local matrices are principal submatrices of the
// assembled operator, inverted once per surface; an application streams the
// inverses (a batched dense matrix-vector product) and sums the local
// corrections node by node.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "mesh.hpp"

namespace pmg {

// The kept local inverses are symmetric: each is stored as the SZ_TS x SZ_TS
// tiles (I, J), I <= J, of its upper block triangle, tile J(J+1)/2 + I at
// SZ_TS^2 (J(J+1)/2 + I); entries past the subdomain size are zero.  About
// 58% of the full square for subdomains of 428 nodes (the mean of the finest
// level of the 131,072-prism box at P = 6, overlap 1).
constexpr int SZ_TS = 32;
inline int64_t sz_tiles(int n) {
  const int64_t t = (n + SZ_TS - 1) / SZ_TS;
  return t * (t + 1) / 2 * SZ_TS * SZ_TS;
}
// Position of entry (r, c) inside a tile whose entries take es bytes: the
// tile is 64 strips (row r, columns 16 h .. 16 h + 15, strip 32 h + r) of
// 16-byte chunks of ec = 16 / es entries; chunk q of strip s sits at 64 q + s.
__host__ __device__ inline int sz_tile_pos(int r, int c, int es) {
  const int ec = 16 / es;
  return ((((c & 15) / ec) * 64) + (c >> 4) * 32 + r) * ec + c % ec;
}

// LDS bytes of the local solve on subdomains of up to max_n nodes, for
// compute values of ts bytes: x, four wave accumulators of z and four column
// reduction buffers of 16 x SD_RED values.
constexpr int SD_RED = 65;
inline size_t sd_apply_lds(int max_n, size_t ts) {
  const size_t ntm = size_t(max_n + SZ_TS - 1) / SZ_TS;
  return ts * (5 * ntm * SZ_TS + 4 * 16 * SD_RED);
}

// Host plan of one level's subdomains.
struct SchwarzPlan {
  int dt = 0, dz = 0;
  int64_t n_sub = 0;
  int max_n = 0;                 // largest subdomain
  int64_t total = 0;             // sum of the subdomain sizes
  std::vector<int32_t> sd_ptr;   // [n_sub+1] into sd_node
  std::vector<int32_t> sd_node;  // sorted free global nodes of every subdomain
  std::vector<int32_t> msz;      // padded size of every local matrix (multiple of 32)
  std::vector<int64_t> inv_off;  // [n_sub+1] entry offsets of the padded msz x msz blocks (set-up work)
  std::vector<int64_t> tile_off; // [n_sub+1] entry offsets of the kept inverses (packed tiles, sz_tiles)
  std::vector<int32_t> blk_ptr;  // [n_sub+1] element blocks of every subdomain
  std::vector<int32_t> blk_elem; // prism of every block
  std::vector<int32_t> blk_ent;  // [n_blk+1] into ent
  std::vector<int32_t> ent;      // local node * 65536 + position in the subdomain
  std::vector<int32_t> node_ptr; // [n_dof+1] positions of every node in the subdomain vector
  std::vector<int32_t> node_pos;
  std::vector<double> w;         // [n_dof] 1 / (subdomains holding the node); 0 if none
};

// Subdomains of a level with numbering `num` (lateral Dirichlet columns
// `dir2d`, Dirichlet surface when top_dir); threads > 1 splits the work.
void build_schwarz(const MeshIn& m, const Numbering& num, const std::vector<uint8_t>& dir2d, int top_dir,
                   int dt, int dz, int threads, SchwarzPlan& out);

// Device arrays of a plan.
struct SchwarzView {
  int64_t n_sub = 0;
  int max_n = 0, max_m = 0;
  const int32_t *sd_ptr = nullptr, *sd_node = nullptr, *msz = nullptr;
  const int64_t *inv_off = nullptr, *tile_off = nullptr;
  const int32_t *blk_ptr = nullptr, *blk_elem = nullptr, *blk_ent = nullptr, *ent = nullptr;
  const int32_t *node_ptr = nullptr, *node_pos = nullptr;
};

// K[e][i][j]: dense element stiffness matrices (FP64), local nodes c*np_tri + a.
void launch_elem_mats(const LevelView& lv, const double* mats, const double* G64, double* K, hipStream_t st);
// A_k = R_k A R_k^T, k in [k0, k1), into the padded blocks of the work array A
// (block k at inv_off[k] - base; identity on the padding).
void launch_sd_assemble(const SchwarzView& sv, int64_t k0, int64_t k1, int64_t base, int np, const double* K,
                        double* A, hipStream_t st);
// In-place inversion of the work blocks k in [k0, k1) (blocked Gauss-Jordan,
// no pivoting: the blocks are SPD), then (A + A^T)/2 written as packed tiles
// to the kept copies A64 / A32 / A16 (nullable; at tile_off[k]).  *bad is set
// when a pivot is not positive.
void launch_sd_invert(const SchwarzView& sv, int64_t k0, int64_t k1, int64_t base, double* A, double* A64,
                      float* A32, bf16_t* A16, int* bad, hipStream_t st);
// zS[sd_ptr[k] + i] = sum_j inv_k[i][j] x_j, x_j = r[node_j] (times w[node_j] when w is given),
// inv_k the packed tiles at tile_off[k].
template <typename T, typename TI>
void launch_sd_apply(const SchwarzView& sv, const TI* inv, const T* r, const T* w, T* zS, hipStream_t st);
// x *= s (n entries).
template <typename T>
void launch_sd_scale(T* x, double s, int64_t n, hipStream_t st);
// u[g] (+)= omega * (w[g] if given) * sum of zS over the positions of g.
template <typename T>
void launch_sd_sum(const SchwarzView& sv, int64_t n_dof, const T* zS, const T* w, T omega, bool accumulate, T* u,
                   hipStream_t st);

}  // namespace pmg
