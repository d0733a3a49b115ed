// Numbering, colouring and node placement (host).  See mesh.hpp.
#include "mesh.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <utility>

namespace pmg {

void Numbering::build(const MeshIn& m, int P_, int PZ_) {
  P = P_;
  PZ = PZ_ < 0 ? P_ : PZ_;
  L = m.L;
  nv = m.nv;
  nt = m.nt;
  np_tri = (P + 1) * (P + 2) / 2;
  np = np_tri * (PZ + 1);
  nint = P >= 3 ? (P - 1) * (P - 2) / 2 : 0;
  // unique sorted edges
  std::vector<std::pair<int32_t, int32_t>> ev;
  ev.reserve(size_t(nt) * 3);
  for (int t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) {
      const int32_t a = m.tri[3 * t + i], b = m.tri[3 * t + (i + 1) % 3];
      ev.emplace_back(std::min(a, b), std::max(a, b));
    }
  std::vector<std::pair<int32_t, int32_t>> uniq = ev;
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  ne = int(uniq.size());
  edges.resize(size_t(ne) * 2);
  for (int e = 0; e < ne; ++e) { edges[2 * e] = uniq[e].first; edges[2 * e + 1] = uniq[e].second; }
  tri_edge.resize(size_t(nt) * 3);
  for (size_t k = 0; k < ev.size(); ++k)
    tri_edge[k] = int32_t(std::lower_bound(uniq.begin(), uniq.end(), ev[k]) - uniq.begin());
  n2d = int64_t(nv) + int64_t(ne) * std::max(P - 1, 0) + int64_t(nt) * nint;
  nz = int64_t(L) * PZ + 1;
  n_dof = n2d * nz;
  n_elem = int64_t(nt) * L;
  if (n_dof >= (int64_t(1) << 31) || n_elem * np >= (int64_t(1) << 31))
    throw std::runtime_error("mesh too large for 32-bit indices");
  // local triangle node -> 2D id
  const std::vector<Ijk> lat = tri_lattice(P);
  map2d.assign(size_t(nt) * np_tri, -1);
  auto edge_node = [&](int t, int le, int pos_from_first) -> int32_t {
    const int32_t va = m.tri[3 * t + le], vb = m.tri[3 * t + (le + 1) % 3];
    const int mg = va < vb ? pos_from_first : P - pos_from_first;
    return int32_t(nv + int64_t(tri_edge[3 * t + le]) * (P - 1) + mg - 1);
  };
  for (int t = 0; t < nt; ++t) {
    int rank = 0;
    for (int a = 0; a < np_tri; ++a) {
      const Ijk l = lat[a];
      int32_t g;
      if (l.i == 0 && l.j == 0) g = m.tri[3 * t + 0];
      else if (l.i == P && l.j == 0) g = m.tri[3 * t + 1];
      else if (l.i == 0 && l.j == P) g = m.tri[3 * t + 2];
      else if (l.j == 0) g = edge_node(t, 0, l.i);          // v0 -> v1
      else if (l.k == 0) g = edge_node(t, 1, l.j);          // v1 -> v2
      else if (l.i == 0) g = edge_node(t, 2, P - l.j);      // v2 -> v0
      else g = int32_t(nv + int64_t(ne) * (P - 1) + int64_t(t) * nint + rank++);
      map2d[size_t(t) * np_tri + a] = g;
    }
  }
  // incidence lists (2D node -> (t, a)), ascending in t*np_tri + a
  inc_ptr.assign(size_t(n2d) + 1, 0);
  for (int32_t g : map2d) inc_ptr[size_t(g) + 1]++;
  for (int64_t g = 0; g < n2d; ++g) inc_ptr[g + 1] += inc_ptr[g];
  inc.resize(map2d.size());
  std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
  for (size_t k = 0; k < map2d.size(); ++k) inc[fill[map2d[k]]++] = int32_t(k);
}

void Numbering::gather_map(int32_t* out) const {
  for (int t = 0; t < nt; ++t)
    for (int layer = 0; layer < L; ++layer) {
      int32_t* row = out + (size_t(t) * L + layer) * np;
      for (int c = 0; c <= PZ; ++c)
        for (int a = 0; a < np_tri; ++a)
          row[c * np_tri + a] = int32_t(int64_t(map2d[size_t(t) * np_tri + a]) * nz + layer * PZ + c);
    }
}

std::vector<int32_t> Numbering::tri_colours() const {
  // triangles t and t' share a 2D node iff they share a vertex; ascending
  // triangles take the smallest colour no lower vertex neighbour holds
  const std::vector<Ijk> lat = tri_lattice(P);
  int corner[3] = {-1, -1, -1};
  for (int a = 0; a < np_tri; ++a) {
    if (lat[a].i == 0 && lat[a].j == 0) corner[0] = a;
    if (lat[a].i == P && lat[a].j == 0) corner[1] = a;
    if (lat[a].i == 0 && lat[a].j == P) corner[2] = a;
  }
  std::vector<std::vector<int32_t>> vtri(nv);
  for (int t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) vtri[map2d[size_t(t) * np_tri + corner[i]]].push_back(t);
  std::vector<int32_t> col(size_t(nt), -1);
  std::vector<char> used;
  for (int t = 0; t < nt; ++t) {
    used.assign(64, 0);
    for (int i = 0; i < 3; ++i)
      for (int32_t u : vtri[map2d[size_t(t) * np_tri + corner[i]]])
        if (u < t) {
          if (col[u] >= int32_t(used.size())) used.resize(size_t(col[u]) + 1, 0);
          used[size_t(col[u])] = 1;
        }
    int32_t c = 0;
    while (c < int32_t(used.size()) && used[size_t(c)]) ++c;
    col[size_t(t)] = c;
  }
  return col;
}

std::vector<int32_t> Numbering::colours() const {
  // elements (t, layer) and (t', layer') share a node iff t and t' share a
  // vertex and |layer - layer'| <= 1
  std::vector<std::vector<int32_t>> vtri(nv);
  // vertex ids are the 2D ids of the three corner nodes
  const std::vector<Ijk> lat = tri_lattice(P);
  int corner[3] = {-1, -1, -1};
  for (int a = 0; a < np_tri; ++a) {
    if (lat[a].i == 0 && lat[a].j == 0) corner[0] = a;
    if (lat[a].i == P && lat[a].j == 0) corner[1] = a;
    if (lat[a].i == 0 && lat[a].j == P) corner[2] = a;
  }
  for (int t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) vtri[map2d[size_t(t) * np_tri + corner[i]]].push_back(t);
  std::vector<int32_t> col(size_t(n_elem), -1);
  std::vector<int32_t> nbr;
  std::vector<char> used;
  for (int t = 0; t < nt; ++t) {
    nbr.clear();
    for (int i = 0; i < 3; ++i)
      for (int32_t u : vtri[map2d[size_t(t) * np_tri + corner[i]]]) nbr.push_back(u);
    std::sort(nbr.begin(), nbr.end());
    nbr.erase(std::unique(nbr.begin(), nbr.end()), nbr.end());
    for (int layer = 0; layer < L; ++layer) {
      const int64_t e = int64_t(t) * L + layer;
      used.assign(64, 0);
      for (int32_t u : nbr)
        for (int dl = -1; dl <= 1; ++dl) {
          const int l2 = layer + dl;
          if (l2 < 0 || l2 >= L) continue;
          const int64_t f = int64_t(u) * L + l2;
          if (f < e) {
            const int32_t c = col[f];
            if (c >= int32_t(used.size())) used.resize(c + 1, 0);
            used[c] = 1;
          }
        }
      int32_t c = 0;
      while (c < int32_t(used.size()) && used[c]) ++c;
      col[e] = c;
    }
  }
  return col;
}

std::vector<double> triangle_node_xy(const MeshIn& m, const RefElem& re, const Numbering& num) {
  const int npt = re.np_tri;
  std::vector<double> X(size_t(m.nt) * npt * 2);
  std::map<std::pair<int, int>, int> curved;
  for (size_t k = 0; k * 2 < m.curved.size(); ++k) {
    const int a = m.curved[2 * k], b = m.curved[2 * k + 1];
    curved[{std::min(a, b), std::max(a, b)}] = int(k);
  }
  for (int t = 0; t < m.nt; ++t) {
    double vx[3], vy[3];
    for (int i = 0; i < 3; ++i) {
      vx[i] = m.xy[2 * m.tri[3 * t + i]];
      vy[i] = m.xy[2 * m.tri[3 * t + i] + 1];
    }
    for (int a = 0; a < npt; ++a) {
      const double lam[3] = {-(re.r[a] + re.s[a]) / 2, (1 + re.r[a]) / 2, (1 + re.s[a]) / 2};
      double x = lam[0] * vx[0] + lam[1] * vx[1] + lam[2] * vx[2];
      double y = lam[0] * vy[0] + lam[1] * vy[1] + lam[2] * vy[2];
      for (int le = 0; le < 3 && !curved.empty(); ++le) {
        const int va = m.tri[3 * t + le], vb = m.tri[3 * t + (le + 1) % 3];
        auto it = curved.find({std::min(va, vb), std::max(va, vb)});
        if (it == curved.end()) continue;
        const double cx = m.circle[3 * it->second], cy = m.circle[3 * it->second + 1],
                     R = m.circle[3 * it->second + 2];
        const int ia = le, ib = (le + 1) % 3;
        const double thA = std::atan2(vy[ia] - cy, vx[ia] - cx);
        const double thB = std::atan2(vy[ib] - cy, vx[ib] - cx);
        double d = thB - thA + M_PI;
        d = d - 2 * M_PI * std::floor(d / (2 * M_PI)) - M_PI;  // short arc, in [-pi, pi)
        const double sum = lam[ia] + lam[ib];
        if (sum < 1e-14) continue;
        const double sp = lam[ib] / sum;
        const double ax = cx + R * std::cos(thA + sp * d), ay = cy + R * std::sin(thA + sp * d);
        const double chx = (1 - sp) * vx[ia] + sp * vx[ib], chy = (1 - sp) * vy[ia] + sp * vy[ib];
        x += sum * (ax - chx);
        y += sum * (ay - chy);
      }
      X[(size_t(t) * npt + a) * 2] = x;
      X[(size_t(t) * npt + a) * 2 + 1] = y;
    }
  }
  (void)num;
  return X;
}

std::vector<uint8_t> lateral_dirichlet(const MeshIn& m, const Numbering& num, uint32_t tag_mask) {
  std::vector<uint8_t> out(size_t(num.n2d), 0);
  if (!tag_mask) return out;
  const std::vector<Ijk> lat = tri_lattice(num.P);
  for (int t = 0; t < m.nt; ++t)
    for (int le = 0; le < 3; ++le) {
      const int tg = m.edge_tag[3 * t + le];
      if (tg <= 0 || tg >= 32 || !((tag_mask >> tg) & 1u)) continue;
      for (int a = 0; a < num.np_tri; ++a) {
        const Ijk l = lat[a];
        const bool on = (le == 0 && l.j == 0) || (le == 1 && l.k == 0) || (le == 2 && l.i == 0);
        if (on) out[num.map2d[size_t(t) * num.np_tri + a]] = 1;
      }
    }
  return out;
}

}  // namespace pmg
