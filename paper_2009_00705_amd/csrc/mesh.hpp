// Extruded prism mesh: numbering of the nodal space V^p, colouring, node
// placement and the incidence lists of the atomic-free summation (host).
//
// Numbering (Sec. 3.1: one global unknown per shared node of the continuous
// space):
//   edges  = every (min, max) vertex pair, sorted lexicographically;
//   2D id  = vertex v -> v; edge-interior node m (1..P-1, counted from the
//            lower-id vertex) -> nv + e*(P-1) + m-1; triangle-interior node
//            of rank k -> nv + ne*(P-1) + t*(P-1)(P-2)/2 + k;
//   global = id2d*(L*P+1) + layer*P + c (vertical columns contiguous);
//   element e = t*L + layer, local node n = c*Np_tri + a.
#pragma once
#include <cstdint>
#include <vector>

#include "refelem.hpp"

namespace pmg {

struct MeshIn {
  int nv = 0, nt = 0, L = 0;
  double depth = 1.0;
  std::vector<double> xy;        // nv*2
  std::vector<int32_t> tri;      // nt*3 (counter-clockwise)
  std::vector<int32_t> edge_tag; // nt*3, tag of edge (tri[i], tri[(i+1)%3])
  std::vector<int32_t> curved;   // ncurved*2 vertex pairs
  std::vector<double> circle;    // ncurved*3 (cx, cy, R)
};

struct Numbering {
  int P = 0, PZ = 0, L = 0, nv = 0, nt = 0, ne = 0, nint = 0, np_tri = 0, np = 0;  // P: triangle, PZ: vertical
  int64_t n2d = 0, nz = 0, n_dof = 0, n_elem = 0;
  std::vector<int32_t> edges;     // ne*2 sorted (min,max)
  std::vector<int32_t> tri_edge;  // nt*3 edge id of (tri[i], tri[(i+1)%3])
  std::vector<int32_t> map2d;     // nt*np_tri local triangle node -> 2D id
  std::vector<int32_t> inc_ptr;   // n2d+1: incidences of each 2D node
  std::vector<int32_t> inc;       // t*np_tri + a, ascending
  void build(const MeshIn& m, int P, int PZ = -1);
  void gather_map(int32_t* out) const;       // [n_elem][np]
  std::vector<int32_t> colours() const;      // greedy, ascending element order
  std::vector<int32_t> tri_colours() const;  // [nt] greedy over vertex-sharing triangles, ascending
};

// xy of the order-P triangle nodes of every triangle, [nt][np_tri][2]: affine
// vertex map plus, on triangles with a listed curved edge, the blended
// displacement of that edge onto its circle.
std::vector<double> triangle_node_xy(const MeshIn& m, const RefElem& re, const Numbering& num);

// 1 for 2D nodes lying on an edge whose tag bit is set in tag_mask.
std::vector<uint8_t> lateral_dirichlet(const MeshIn& m, const Numbering& num, uint32_t tag_mask);

}  // namespace pmg
