// Host-side mesh analysis: validation, per-side geometry, side pairing,
// reverse Cuthill-McKee renumbering and the CSR pattern.
//
// Geometry (Sec. 3.2.2, eq. cs1_discr): the two-point flux across side j uses
// d_{e,ep}, the signed distance between the circumcenters of e and ep.  Since
// the segment joining two circumcenters is the perpendicular bisector of the
// shared side, d = (l/2)(cot t_e + cot t_ep), t being the angle opposite the
// side, so T = l/d = 2/(cot t_e + cot t_ep); a boundary side's
// circumcenter-to-midpoint distance gives T_b = 2/cot t.  The Delaunay property
// (Sec. 3.1) is exactly cot t_e + cot t_ep > 0, which makes the corrector
// matrices M-matrices; it is checked, never clamped.
//
// This file is compiled with -ffp-contract=off: every floating-point
// expression is evaluated as written, operation by operation.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pm_internal.h"

namespace pm {

namespace {

inline bool finite(double v) { return std::isfinite(v); }

// Breadth-first level structure from root.  Vertices are appended to `queue`
// in visiting order; level_start[l] is where level l begins.  Returns the
// number of levels.
int bfs_levels(int32_t root, const int32_t* nbr, std::vector<int32_t>& stamp, int32_t mark,
               std::vector<int32_t>& queue, std::vector<int32_t>& level_start) {
  queue.clear();
  level_start.clear();
  queue.push_back(root);
  stamp[root] = mark;
  size_t head = 0;
  while (head < queue.size()) {
    level_start.push_back(static_cast<int32_t>(head));
    size_t end = queue.size();
    for (; head < end; ++head) {
      int32_t v = queue[head];
      for (int j = 0; j < 3; ++j) {
        int32_t u = nbr[3 * (size_t)v + j];
        if (u >= 0 && stamp[u] != mark) {
          stamp[u] = mark;
          queue.push_back(u);
        }
      }
    }
  }
  return static_cast<int>(level_start.size());
}

inline bool deg_less(int32_t a, int32_t b, const std::vector<int8_t>& deg) {
  return deg[a] < deg[b] || (deg[a] == deg[b] && a < b);
}

}  // namespace

int build_structure(int32_t n_nodes, const double* xy, int32_t n_cells, const int32_t* tri,
                    const int8_t* side_tag, HostStructure& hs, std::string& err) {
  if (n_nodes <= 0 || n_cells <= 0 || !xy || !tri || !side_tag) {
    err = "empty mesh or null pointer";
    return PM_INVALID_ARG;
  }
  const size_t n = static_cast<size_t>(n_cells);
  for (size_t k = 0; k < 3 * n; ++k)
    if (tri[k] < 0 || tri[k] >= n_nodes) {
      err = "node index out of range";
      return PM_INVALID_ARG;
    }
  for (size_t k = 0; k < 3 * n; ++k)
    if (side_tag[k] < 0 || side_tag[k] > 3) {
      err = "side tag outside 0..3";
      return PM_INVALID_ARG;
    }
  for (size_t k = 0; k < 2 * (size_t)n_nodes; ++k)
    if (!finite(xy[k])) {
      err = "non-finite node coordinates";
      return PM_NONFINITE;
    }
  for (size_t e = 0; e < n; ++e) {
    const int32_t* t = tri + 3 * e;
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) {
      err = "repeated node in a triangle";
      return PM_BAD_MESH;
    }
  }

  hs.n_nodes = n_nodes;
  hs.n = n_cells;
  hs.cot.assign(3 * n, 0.0);
  hs.tx.assign(3 * n, 0.0);
  hs.ty.assign(3 * n, 0.0);
  hs.area.assign(n, 0.0);
  bool bad_area = false;
  for (size_t e = 0; e < n; ++e) {
    for (int j = 0; j < 3; ++j) {
      const double* a = xy + 2 * (size_t)tri[3 * e + j];
      const double* b = xy + 2 * (size_t)tri[3 * e + (j + 1) % 3];
      const double* c = xy + 2 * (size_t)tri[3 * e + (j + 2) % 3];
      double ux = b[0] - a[0], uy = b[1] - a[1];
      double vx = c[0] - a[0], vy = c[1] - a[1];
      double dot = ux * vx + uy * vy;
      double cr = ux * vy - uy * vx;
      if (!(cr > 0.0)) bad_area = true;
      hs.cot[3 * e + j] = dot / cr;
      hs.tx[3 * e + j] = c[0] - b[0];
      hs.ty[3 * e + j] = c[1] - b[1];
      if (j == 0) hs.area[e] = 0.5 * cr;
    }
  }
  if (bad_area) {
    err = "triangle with non-positive area (clockwise or degenerate)";
    return PM_BAD_MESH;
  }

  // Side pairing: bucket sides by their smaller node, then match the larger.
  hs.nbr.assign(3 * n, -1);
  hs.nbr_side.assign(3 * n, -1);
  {
    std::vector<int64_t> start((size_t)n_nodes + 1, 0);
    for (size_t s = 0; s < 3 * n; ++s) {
      size_t e = s / 3;
      int j = static_cast<int>(s % 3);
      int32_t a = tri[3 * e + (j + 1) % 3], b = tri[3 * e + (j + 2) % 3];
      start[(size_t)std::min(a, b) + 1]++;
    }
    for (size_t v = 0; v < (size_t)n_nodes; ++v) start[v + 1] += start[v];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    std::vector<int32_t> bucket(3 * n);
    for (size_t s = 0; s < 3 * n; ++s) {
      size_t e = s / 3;
      int j = static_cast<int>(s % 3);
      int32_t a = tri[3 * e + (j + 1) % 3], b = tri[3 * e + (j + 2) % 3];
      bucket[fill[std::min(a, b)]++] = static_cast<int32_t>(s);
    }
    auto hi_of = [&](int32_t s) {
      size_t e = (size_t)s / 3;
      int j = s % 3;
      return std::max(tri[3 * e + (j + 1) % 3], tri[3 * e + (j + 2) % 3]);
    };
    for (size_t v = 0; v < (size_t)n_nodes; ++v) {
      int32_t* bb = bucket.data() + start[v];
      int64_t len = start[v + 1] - start[v];
      std::sort(bb, bb + len, [&](int32_t x, int32_t y) {
        int32_t hx = hi_of(x), hy = hi_of(y);
        return hx < hy || (hx == hy && x < y);
      });
      for (int64_t i = 0; i < len;) {
        int64_t k = i + 1;
        while (k < len && hi_of(bb[k]) == hi_of(bb[i])) ++k;
        if (k - i > 2) {
          err = "a side is shared by more than two triangles";
          return PM_BAD_MESH;
        }
        if (k - i == 2) {
          int32_t s0 = bb[i], s1 = bb[i + 1];
          int32_t a0 = tri[3 * (s0 / 3) + (s0 % 3 + 1) % 3];
          int32_t a1 = tri[3 * (s1 / 3) + (s1 % 3 + 1) % 3];
          if (a0 == a1) {
            err = "two triangles traverse a shared side in the same direction";
            return PM_BAD_MESH;
          }
          hs.nbr[s0] = s1 / 3;
          hs.nbr_side[s0] = s1 % 3;
          hs.nbr[s1] = s0 / 3;
          hs.nbr_side[s1] = s0 % 3;
        }
        i = k;
      }
    }
  }

  // Transmissibilities and Delaunay checks.
  hs.T.assign(3 * n, 0.0);
  hs.tag.assign(3 * n, 0);
  double max_T = 0.0, min_cs = INFINITY;
  int32_t n_int_half = 0, n_bnd = 0;
  for (size_t s = 0; s < 3 * n; ++s) {
    int32_t o = hs.nbr[s];
    if (o >= 0) {
      double cs = hs.cot[s] + hs.cot[3 * (size_t)o + hs.nbr_side[s]];
      if (!(cs > 0.0)) {
        err = "interior side with non-positive circumcenter distance";
        return PM_NOT_DELAUNAY;
      }
      hs.T[s] = 2.0 / cs;
      min_cs = std::min(min_cs, cs);
      ++n_int_half;
    } else {
      ++n_bnd;
    }
  }
  for (size_t s = 0; s < 3 * n; ++s) {
    if (hs.nbr[s] >= 0) continue;
    hs.tag[s] = side_tag[s];
    if (side_tag[s] != 0 && !(hs.cot[s] > 0.0)) {
      err = "Dirichlet side with non-positive circumcenter-to-side distance";
      return PM_NOT_DELAUNAY;
    }
    hs.T[s] = hs.cot[s] > 0.0 ? 2.0 / hs.cot[s] : 0.0;
  }
  for (size_t s = 0; s < 3 * n; ++s) max_T = std::max(max_T, hs.T[s]);

  // Reverse Cuthill-McKee (specification: minimum-degree start with
  // smaller-index ties, George-Liu pseudo-peripheral iteration, neighbours
  // appended by (degree, index), components by smallest cell index, the
  // whole list reversed).
  std::vector<int8_t> deg(n, 0);
  for (size_t e = 0; e < n; ++e)
    for (int j = 0; j < 3; ++j) deg[e] += hs.nbr[3 * e + j] >= 0;
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<uint8_t> visited(n, 0);
  std::vector<int32_t> stamp(n, -1), queue, lstart, queue2, lstart2;
  hs.comp.assign(n, -1);
  hs.comp_bits.clear();
  int32_t mark = 0;
  for (size_t s = 0; s < n; ++s) {
    if (visited[s]) continue;
    bfs_levels(static_cast<int32_t>(s), hs.nbr.data(), stamp, mark++, queue, lstart);
    int32_t r = queue[0];
    for (int32_t v : queue)
      if (deg_less(v, r, deg)) r = v;
    int nl = bfs_levels(r, hs.nbr.data(), stamp, mark++, queue, lstart);
    for (;;) {
      int32_t x = queue[lstart[nl - 1]];
      for (size_t k = lstart[nl - 1]; k < queue.size(); ++k)
        if (deg_less(queue[k], x, deg)) x = queue[k];
      int nlx = bfs_levels(x, hs.nbr.data(), stamp, mark++, queue2, lstart2);
      if (nlx > nl) {
        r = x;
        nl = nlx;
        queue.swap(queue2);
        lstart.swap(lstart2);
      } else {
        break;
      }
    }
    const int32_t cid = static_cast<int32_t>(hs.comp_bits.size());
    uint8_t bits = 0;
    size_t head = order.size();
    visited[r] = 1;
    order.push_back(r);
    while (head < order.size()) {
      int32_t v = order[head++];
      hs.comp[v] = cid;
      for (int j = 0; j < 3; ++j)
        if (hs.nbr[3 * (size_t)v + j] < 0) bits |= static_cast<uint8_t>(hs.tag[3 * (size_t)v + j]);
      int32_t cand[3];
      int nc = 0;
      for (int j = 0; j < 3; ++j) {
        int32_t u = hs.nbr[3 * (size_t)v + j];
        if (u >= 0 && !visited[u]) cand[nc++] = u;
      }
      for (int a = 1; a < nc; ++a)
        for (int b = a; b > 0 && deg_less(cand[b], cand[b - 1], deg); --b) std::swap(cand[b], cand[b - 1]);
      for (int a = 0; a < nc; ++a) {
        visited[cand[a]] = 1;
        order.push_back(cand[a]);
      }
    }
    hs.comp_bits.push_back(bits);
  }
  std::reverse(order.begin(), order.end());
  hs.perm = order;
  hs.inv.assign(n, 0);
  for (size_t i = 0; i < n; ++i) hs.inv[hs.perm[i]] = static_cast<int32_t>(i);

  // CSR pattern in the new order: diagonal included, ascending columns.
  hs.row_ptr.assign(n + 1, 0);
  hs.col.clear();
  hs.col.reserve(n + (size_t)n_int_half);
  int32_t bw = 0;
  for (size_t i = 0; i < n; ++i) {
    int32_t c[4];
    int nc = 0;
    c[nc++] = static_cast<int32_t>(i);
    size_t old = hs.perm[i];
    for (int j = 0; j < 3; ++j) {
      int32_t u = hs.nbr[3 * old + j];
      if (u >= 0) c[nc++] = hs.inv[u];
    }
    std::sort(c, c + nc);
    for (int a = 0; a < nc; ++a) {
      hs.col.push_back(c[a]);
      bw = std::max(bw, std::abs(c[a] - static_cast<int32_t>(i)));
    }
    hs.row_ptr[i + 1] = static_cast<int32_t>(hs.col.size());
  }

  pm_mesh_stats& st = hs.stats;
  st.n_cells = n_cells;
  st.n_nodes = n_nodes;
  st.nnz = static_cast<int32_t>(hs.col.size());
  st.n_interior_sides = n_int_half / 2;
  st.n_boundary_sides = n_bnd;
  st.bandwidth = bw;
  st.n_components = static_cast<int32_t>(hs.comp_bits.size());
  st.index_bits = bw <= 32767 ? 16 : 32;
  st.max_T = max_T;
  st.min_cot_sum = n_int_half ? min_cs : 0.0;
  return PM_OK;
}

}  // namespace pm
