// Host plan of the overlapping Schwarz subdomains (see schwarz.hpp).
//
// Two prisms that touch share a product entity: a triangle vertex, edge or
// the whole triangle, times one z level (adjacent layers) or the whole
// vertical range (same layer).  The lattice distance of a node (a, c) of the
// touching prism to that entity therefore splits: in the triangle it is
// lambda_r(a) to an edge whose opposite vertex is r, P - lambda_p(a) to a
// vertex p, 0 to the whole triangle (lambda = barycentric lattice indices);
// along the extrusion it is c to the prism's bottom face, PZ - c to its top
// face, 0 in the same layer.
#include "schwarz.hpp"

#include <algorithm>
#include <stdexcept>
#include <string>
#include <thread>

namespace pmg {

namespace {

struct SubOut {
  std::vector<int32_t> nodes;
  std::vector<int32_t> blk_elem, blk_cnt, ent;
};

void one_subdomain(const Numbering& num, const std::vector<std::vector<int32_t>>& vtris,
                   const std::vector<int32_t>& tri, const std::vector<uint8_t>& dir2d, int top_dir, int dt, int dz,
                   const std::vector<int>& lam, int64_t k, SubOut& o) {
  const int P = num.P, PZ = num.PZ, L = num.L, npt = num.np_tri;
  const int64_t nz = num.nz;
  const int t = int(k / L), layer = int(k - int64_t(t) * L);
  const int32_t* tv = &tri[3 * size_t(t)];
  // triangles touching t (sharing a vertex), ascending
  std::vector<int32_t> tt;
  for (int q = 0; q < 3; ++q) tt.insert(tt.end(), vtris[tv[q]].begin(), vtris[tv[q]].end());
  std::sort(tt.begin(), tt.end());
  tt.erase(std::unique(tt.begin(), tt.end()), tt.end());
  o.nodes.clear();
  for (int32_t t2 : tt) {
    const int32_t* uv = &tri[3 * size_t(t2)];
    int nsh = 0, sh = -1, nosh = -1;
    for (int q = 0; q < 3; ++q) {
      const bool s = uv[q] == tv[0] || uv[q] == tv[1] || uv[q] == tv[2];
      if (s) { ++nsh; sh = q; } else nosh = q;
    }
    for (int dl = -1; dl <= 1; ++dl) {
      const int l2 = layer + dl;
      if (l2 < 0 || l2 >= L) continue;
      for (int a = 0; a < npt; ++a) {
        const int dp = nsh == 3 ? 0 : (nsh == 2 ? lam[3 * a + nosh] : P - lam[3 * a + sh]);
        if (dp > dt) continue;
        const int64_t g2 = num.map2d[size_t(t2) * npt + a];
        if (dir2d[g2]) continue;
        for (int c = 0; c <= PZ; ++c) {
          const int dv = dl == 0 ? 0 : (dl == 1 ? c : PZ - c);
          if (dv > dz) continue;
          const int64_t z = int64_t(l2) * PZ + c;
          if (top_dir && z == nz - 1) continue;
          o.nodes.push_back(int32_t(g2 * nz + z));
        }
      }
    }
  }
  std::sort(o.nodes.begin(), o.nodes.end());
  o.nodes.erase(std::unique(o.nodes.begin(), o.nodes.end()), o.nodes.end());
  if (o.nodes.size() >= 65536) throw std::runtime_error("Schwarz subdomain larger than 65535 nodes");
  // every prism holding a subdomain node: (prism, local node, position)
  std::vector<int64_t> trip;
  for (size_t p = 0; p < o.nodes.size(); ++p) {
    const int64_t g = o.nodes[p];
    const int64_t g2 = g / nz;
    const int z = int(g - g2 * nz);
    int lay[2], cc[2], nl = 0;
    const int lz = z / PZ;
    if (z % PZ == 0) {
      if (lz - 1 >= 0) { lay[nl] = lz - 1; cc[nl++] = PZ; }
      if (lz < L) { lay[nl] = lz; cc[nl++] = 0; }
    } else {
      lay[nl] = lz; cc[nl++] = z - lz * PZ;
    }
    for (int32_t j = num.inc_ptr[g2]; j < num.inc_ptr[g2 + 1]; ++j) {
      const int32_t ta = num.inc[j];
      const int t2 = ta / npt, a = ta - t2 * npt;
      for (int s = 0; s < nl; ++s) {
        const int64_t e = int64_t(t2) * L + lay[s];
        const int64_t n = int64_t(cc[s]) * npt + a;
        trip.push_back((e << 32) | (n << 16) | int64_t(p));
      }
    }
  }
  std::sort(trip.begin(), trip.end());
  o.blk_elem.clear();
  o.blk_cnt.clear();
  o.ent.clear();
  for (size_t i = 0; i < trip.size(); ++i) {
    const int32_t e = int32_t(trip[i] >> 32);
    if (o.blk_elem.empty() || o.blk_elem.back() != e) {
      o.blk_elem.push_back(e);
      o.blk_cnt.push_back(0);
    }
    o.blk_cnt.back()++;
    o.ent.push_back(int32_t(trip[i] & 0xFFFFFFFFll));
  }
}

}  // namespace

void build_schwarz(const MeshIn& m, const Numbering& num, const std::vector<uint8_t>& dir2d, int top_dir, int dt,
                   int dz, int threads, SchwarzPlan& out) {
  if (num.np >= 32768) throw std::runtime_error("element too large for the Schwarz plan");
  const int64_t E = num.n_elem;
  std::vector<std::vector<int32_t>> vtris(size_t(m.nv));
  for (int t = 0; t < m.nt; ++t)
    for (int q = 0; q < 3; ++q) vtris[m.tri[3 * size_t(t) + q]].push_back(t);
  // barycentric lattice indices (lambda_0, lambda_1, lambda_2) = (P-i-j, i, j) of the local triangle nodes
  std::vector<int> lam;
  for (int j = 0; j <= num.P; ++j)
    for (int i = 0; i + j <= num.P; ++i) {
      lam.push_back(num.P - i - j);
      lam.push_back(i);
      lam.push_back(j);
    }
  std::vector<SubOut> subs(static_cast<size_t>(E));
  const int nth = std::max(1, std::min<int>(threads, int(std::max<int64_t>(1, E / 64))));
  std::vector<std::thread> pool;
  std::vector<std::string> errs(static_cast<size_t>(nth));
  for (int th = 0; th < nth; ++th)
    pool.emplace_back([&, th]() {
      try {
        for (int64_t k = th; k < E; k += nth)
          one_subdomain(num, vtris, m.tri, dir2d, top_dir, dt, dz, lam, k, subs[size_t(k)]);
      } catch (const std::exception& e) {
        errs[size_t(th)] = e.what();
      }
    });
  for (auto& p : pool) p.join();
  for (auto& e : errs)
    if (!e.empty()) throw std::runtime_error(e);

  SchwarzPlan& o = out;
  o = SchwarzPlan();
  o.dt = dt;
  o.dz = dz;
  o.n_sub = E;
  o.sd_ptr.assign(size_t(E) + 1, 0);
  o.msz.assign(size_t(E), 0);
  o.inv_off.assign(size_t(E) + 1, 0);
  o.tile_off.assign(size_t(E) + 1, 0);
  o.blk_ptr.assign(size_t(E) + 1, 0);
  int64_t tot = 0, nblk = 0, nent = 0;
  for (int64_t k = 0; k < E; ++k) {
    const SubOut& s = subs[size_t(k)];
    const int n = int(s.nodes.size());
    tot += n;
    nblk += int64_t(s.blk_elem.size());
    nent += int64_t(s.ent.size());
    if (tot >= (int64_t(1) << 31) || nent >= (int64_t(1) << 31))
      throw std::runtime_error("Schwarz plan exceeds 2^31 entries");
    o.sd_ptr[size_t(k) + 1] = int32_t(tot);
    o.max_n = std::max(o.max_n, n);
    const int ms = (n + 31) & ~31;
    o.msz[size_t(k)] = ms;
    o.inv_off[size_t(k) + 1] = o.inv_off[size_t(k)] + int64_t(ms) * ms;
    o.tile_off[size_t(k) + 1] = o.tile_off[size_t(k)] + sz_tiles(n);
    o.blk_ptr[size_t(k) + 1] = int32_t(nblk);
  }
  o.total = tot;
  o.sd_node.reserve(size_t(tot));
  o.blk_elem.reserve(size_t(nblk));
  o.blk_ent.assign(1, 0);
  o.ent.reserve(size_t(nent));
  for (int64_t k = 0; k < E; ++k) {
    const SubOut& s = subs[size_t(k)];
    o.sd_node.insert(o.sd_node.end(), s.nodes.begin(), s.nodes.end());
    o.blk_elem.insert(o.blk_elem.end(), s.blk_elem.begin(), s.blk_elem.end());
    for (int32_t c : s.blk_cnt) o.blk_ent.push_back(o.blk_ent.back() + c);
    o.ent.insert(o.ent.end(), s.ent.begin(), s.ent.end());
  }
  // node -> positions (ascending subdomain) and weights
  const int64_t N = num.n_dof;
  o.node_ptr.assign(size_t(N) + 1, 0);
  for (int32_t g : o.sd_node) o.node_ptr[size_t(g) + 1]++;
  for (int64_t g = 0; g < N; ++g) o.node_ptr[size_t(g) + 1] += o.node_ptr[size_t(g)];
  o.node_pos.assign(size_t(tot), 0);
  std::vector<int32_t> fill(o.node_ptr.begin(), o.node_ptr.end() - 1);
  for (int64_t p = 0; p < tot; ++p) o.node_pos[size_t(fill[size_t(o.sd_node[size_t(p)])]++)] = int32_t(p);
  o.w.assign(size_t(N), 0.0);
  for (int64_t g = 0; g < N; ++g) {
    const int c = o.node_ptr[size_t(g) + 1] - o.node_ptr[size_t(g)];
    if (c > 0) o.w[size_t(g)] = 1.0 / double(c);
  }
}

}  // namespace pmg
