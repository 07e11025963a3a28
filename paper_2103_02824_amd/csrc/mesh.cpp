// Host-side mesh preparation (once per mesh pair): the fine nodes (P1: the
// vertices; P2: the vertices and edge midpoints), interior DoF numbering,
// locality ordering, element geometry, CSR pattern, row adjacency for the
// row-wise assembly kernel, the prolongation P (coarse hat functions at the
// fine vertices: the spaces are nested, Section 3.2) and the grouping of fine
// tets by their coarse parent tet.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "mlc_internal.h"

namespace mlc {

namespace {

uint64_t spread3(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}

uint64_t morton(const double* p, const double lo[3], const double hi[3]) {
  uint64_t c[3];
  for (int k = 0; k < 3; ++k) {
    double v = (p[k] - lo[k]) * ((double)((1u << 21) - 1) / (hi[k] - lo[k]));
    v = v < 0 ? 0 : (v > (double)((1u << 21) - 1) ? (double)((1u << 21) - 1) : v);
    c[k] = (uint64_t)v;
  }
  return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
}

// Jacobian J = [x1-x0, x2-x0, x3-x0] (columns); returns det and J^{-1}.
double tet_inverse(const double* x0, const double* x1, const double* x2, const double* x3, double Ji[9]) {
  double J[9];
  for (int r = 0; r < 3; ++r) {
    J[3 * r + 0] = x1[r] - x0[r];
    J[3 * r + 1] = x2[r] - x0[r];
    J[3 * r + 2] = x3[r] - x0[r];
  }
  double c00 = J[4] * J[8] - J[5] * J[7];
  double c01 = J[5] * J[6] - J[3] * J[8];
  double c02 = J[3] * J[7] - J[4] * J[6];
  double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  double id = 1.0 / det;
  Ji[0] = c00 * id;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) * id;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) * id;
  Ji[3] = c01 * id;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) * id;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) * id;
  Ji[6] = c02 * id;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) * id;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) * id;
  return det;
}

struct Locator {
  // uniform bucket grid over the coarse tets' bounding boxes
  int nb = 1;
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  std::vector<int32_t> ptr, ids;
  const std::vector<double>* cgeo = nullptr;
  void build(const mlc_ctx* c) {
    nb = std::max(1, (int)std::cbrt((double)c->cnt / 4.0));
    for (int k = 0; k < 3; ++k) {
      lo[k] = c->lo[k];
      hi[k] = c->hi[k];
      h[k] = (hi[k] - lo[k]) / nb;
    }
    std::vector<int32_t> cnt((size_t)nb * nb * nb + 1, 0);
    auto cells = [&](int64_t t, int r[6]) {
      double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
      for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) {
          double v = c->cxyz[3 * (int64_t)c->ctets[4 * t + a] + k];
          mn[k] = std::min(mn[k], v);
          mx[k] = std::max(mx[k], v);
        }
      for (int k = 0; k < 3; ++k) {
        double e = 1e-9 * (hi[k] - lo[k]);
        r[2 * k] = std::max(0, std::min(nb - 1, (int)std::floor((mn[k] - e - lo[k]) / h[k])));
        r[2 * k + 1] = std::max(0, std::min(nb - 1, (int)std::floor((mx[k] + e - lo[k]) / h[k])));
      }
    };
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        ptr.assign(cnt.size(), 0);
        for (size_t i = 1; i < cnt.size(); ++i) ptr[i] = ptr[i - 1] + cnt[i - 1];
        ids.assign(ptr.back(), 0);
        std::fill(cnt.begin(), cnt.end(), 0);
      }
      for (int64_t t = 0; t < c->cnt; ++t) {
        int r[6];
        cells(t, r);
        for (int z = r[4]; z <= r[5]; ++z)
          for (int y = r[2]; y <= r[3]; ++y)
            for (int x = r[0]; x <= r[1]; ++x) {
              size_t cell = ((size_t)z * nb + y) * nb + x;
              if (pass == 1) ids[ptr[cell] + cnt[cell]] = (int32_t)t;
              cnt[cell]++;
            }
      }
    }
  }
  // coarse tet with the largest minimal barycentric coordinate; returns it in b
  int64_t find(const mlc_ctx* c, const double* p, double b[4], double* best_min) const {
    int ix[3];
    for (int k = 0; k < 3; ++k) ix[k] = std::max(0, std::min(nb - 1, (int)std::floor((p[k] - lo[k]) / h[k])));
    size_t cell = ((size_t)ix[2] * nb + ix[1]) * nb + ix[0];
    int64_t best = -1;
    double bm = -1e300;
    for (int32_t e = ptr[cell]; e < ptr[cell + 1]; ++e) {
      int64_t t = ids[e];
      const double* g = c->cgeo.data() + 12 * t;
      double dx = p[0] - g[0], dy = p[1] - g[1], dz = p[2] - g[2];
      double l1 = g[3] * dx + g[4] * dy + g[5] * dz;
      double l2 = g[6] * dx + g[7] * dy + g[8] * dz;
      double l3 = g[9] * dx + g[10] * dy + g[11] * dz;
      double l0 = 1.0 - l1 - l2 - l3;
      double m = std::min(std::min(l0, l1), std::min(l2, l3));
      if (m > bm) {
        bm = m;
        best = t;
        b[0] = l0;
        b[1] = l1;
        b[2] = l2;
        b[3] = l3;
      }
    }
    *best_min = bm;
    return best;
  }
};

std::vector<char> boundary_flags(const std::vector<double>& xyz, const double lo[3], const double hi[3]) {
  int64_t nv = (int64_t)xyz.size() / 3;
  std::vector<char> on(nv, 0);
  for (int64_t v = 0; v < nv; ++v)
    for (int k = 0; k < 3; ++k) {
      double tol = 1e-12 * std::max(1.0, std::max(std::fabs(lo[k]), std::fabs(hi[k])));
      double x = xyz[3 * v + k];
      if (std::fabs(x - lo[k]) <= tol || std::fabs(x - hi[k]) <= tol) on[v] = 1;
    }
  return on;
}

}  // namespace

mlc_status build_mesh(mlc_ctx* c, const mlc_mesh* fine, const mlc_mesh* coarse) {
  // ---- copy and validate ------------------------------------------------------
  c->order = fine->order;
  c->ne = c->order == 2 ? P2_NE : 4;
  c->nq = c->order == 2 ? P2_NQ : 4;
  const int NEL = c->ne;
  c->nvert = fine->n_vertices;
  c->nt = fine->n_tets;
  c->cnv = coarse->n_vertices;
  c->cnt = coarse->n_tets;
  if (c->nvert < 4 || c->nt < 1 || c->cnv < 4 || c->cnt < 1) return fail(c, MLC_ERR_MESH, "empty mesh");
  if (c->nvert >= (1LL << 31) || c->nt * NEL * NEL >= (1LL << 31))
    return fail(c, MLC_ERR_MESH, "mesh too large for int32 indices");
  c->xyz.assign(fine->xyz, fine->xyz + 3 * c->nvert);
  c->cxyz.assign(coarse->xyz, coarse->xyz + 3 * c->cnv);
  std::vector<int32_t> tin(fine->tets, fine->tets + 4 * c->nt);
  c->ctets.assign(coarse->tets, coarse->tets + 4 * c->cnt);
  for (int64_t i = 0; i < 4 * c->nt; ++i)
    if (tin[i] < 0 || tin[i] >= c->nvert) return fail(c, MLC_ERR_MESH, "fine tet index out of range");
  for (int64_t i = 0; i < 4 * c->cnt; ++i)
    if (c->ctets[i] < 0 || c->ctets[i] >= c->cnv) return fail(c, MLC_ERR_MESH, "coarse tet index out of range");
  for (int64_t i = 0; i < 3 * c->nvert; ++i)
    if (!std::isfinite(c->xyz[i])) return fail(c, MLC_ERR_MESH, "non-finite fine coordinate");

  // ---- fine nodes: the vertices, and for P2 one node per edge at its midpoint,
  // edges in increasing (lo, hi) vertex order; element node lists in caller tet order
  std::vector<int32_t> tel;
  if (c->order == 2) {
    static const int EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    const uint64_t NV = (uint64_t)c->nvert;
    std::vector<uint64_t> ek(6 * c->nt);
    for (int64_t t = 0; t < c->nt; ++t)
      for (int e = 0; e < 6; ++e) {
        const uint64_t a = (uint64_t)tin[4 * t + EDGE[e][0]], b = (uint64_t)tin[4 * t + EDGE[e][1]];
        ek[6 * t + e] = std::min(a, b) * NV + std::max(a, b);
      }
    std::vector<uint64_t> edges(ek);
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    if (c->nvert + (int64_t)edges.size() >= (1LL << 31)) return fail(c, MLC_ERR_MESH, "mesh too large for int32 indices");
    for (uint64_t k : edges) {
      const int64_t a = (int64_t)(k / NV), b = (int64_t)(k % NV);
      for (int x = 0; x < 3; ++x) c->xyz.push_back(0.5 * (c->xyz[3 * a + x] + c->xyz[3 * b + x]));
    }
    tel.resize(P2_NE * c->nt);
    for (int64_t t = 0; t < c->nt; ++t) {
      for (int a = 0; a < 4; ++a) tel[P2_NE * t + a] = tin[4 * t + a];
      for (int e = 0; e < 6; ++e)
        tel[P2_NE * t + 4 + e] =
            (int32_t)(c->nvert + (std::lower_bound(edges.begin(), edges.end(), ek[6 * t + e]) - edges.begin()));
    }
    p2_tables(c->qtab);
  } else {
    tel = tin;
  }
  c->nv = (int64_t)c->xyz.size() / 3;

  // ---- fine tets: locality order by Morton code of the centroid -------------
  std::vector<uint64_t> key(c->nt);
  for (int64_t t = 0; t < c->nt; ++t) {
    double p[3] = {0, 0, 0};
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) p[k] += 0.25 * c->xyz[3 * (int64_t)tin[4 * t + a] + k];
    key[t] = morton(p, c->lo, c->hi);
  }
  std::vector<int64_t> tord(c->nt);
  std::iota(tord.begin(), tord.end(), 0);
  if (c->opt.reorder) std::stable_sort(tord.begin(), tord.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  c->tets.resize(NEL * c->nt);
  for (int64_t t = 0; t < c->nt; ++t)
    for (int a = 0; a < NEL; ++a) c->tets[NEL * t + a] = tel[NEL * tord[t] + a];
  if (c->opt.estimator && c->order == 1) {
    // the caller's tet order, and for each face (opposite vertex a) the tet
    // on its other side: faces sorted by their vertex triple, equal triples
    // adjacent
    c->tord.resize(c->nt);
    for (int64_t t = 0; t < c->nt; ++t) c->tord[t] = (int32_t)tord[t];
    struct Face {
      int32_t v[3];
      int32_t id;  // 4 t + a
    };
    std::vector<Face> fs(4 * c->nt);
    for (int64_t t = 0; t < c->nt; ++t)
      for (int a = 0; a < 4; ++a) {
        Face& f = fs[4 * t + a];
        int k = 0;
        for (int b = 0; b < 4; ++b)
          if (b != a) f.v[k++] = c->tets[4 * t + b];
        std::sort(f.v, f.v + 3);
        f.id = (int32_t)(4 * t + a);
      }
    std::sort(fs.begin(), fs.end(), [](const Face& x, const Face& y) {
      if (x.v[0] != y.v[0]) return x.v[0] < y.v[0];
      if (x.v[1] != y.v[1]) return x.v[1] < y.v[1];
      if (x.v[2] != y.v[2]) return x.v[2] < y.v[2];
      return x.id < y.id;
    });
    c->nbr.assign(4 * c->nt, -1);
    for (size_t i = 0; i + 1 < fs.size(); ++i) {
      const Face &x = fs[i], &y = fs[i + 1];
      if (x.v[0] == y.v[0] && x.v[1] == y.v[1] && x.v[2] == y.v[2]) {
        if (i + 2 < fs.size() && fs[i + 2].v[0] == x.v[0] && fs[i + 2].v[1] == x.v[1] && fs[i + 2].v[2] == x.v[2])
          return fail(c, MLC_ERR_MESH, "a face is shared by more than two fine tets");
        c->nbr[x.id] = y.id / 4;
        c->nbr[y.id] = x.id / 4;
        ++i;
      }
    }
  }

  // ---- geometry ---------------------------------------------------------------
  c->geo.assign(16 * c->nt, 0.0);
  for (int64_t t = 0; t < c->nt; ++t) {
    const double* x[4];
    for (int a = 0; a < 4; ++a) x[a] = &c->xyz[3 * (int64_t)c->tets[NEL * t + a]];
    double Ji[9];
    double det = tet_inverse(x[0], x[1], x[2], x[3], Ji);
    double vol = std::fabs(det) / 6.0;
    if (!(vol > 1e-300) || !std::isfinite(vol)) return fail(c, MLC_ERR_MESH, "degenerate fine tet");
    double* G = &c->geo[16 * t];
    G[0] = vol;
    for (int k = 0; k < 3; ++k) {  // grad lambda_{1..3} = rows of J^{-1}
      G[1 + 3 * 1 + k] = Ji[0 * 3 + k];
      G[1 + 3 * 2 + k] = Ji[1 * 3 + k];
      G[1 + 3 * 3 + k] = Ji[2 * 3 + k];
      G[1 + k] = -(Ji[k] + Ji[3 + k] + Ji[6 + k]);
    }
  }

  // ---- interior DoFs ------------------------------------------------------------
  std::vector<char> on = boundary_flags(c->xyz, c->lo, c->hi);
  std::vector<int32_t> interior;
  for (int64_t v = 0; v < c->nv; ++v)
    if (!on[v]) interior.push_back((int32_t)v);
    else c->bverts.push_back((int32_t)v);
  c->n = (int64_t)interior.size();
  if (c->n == 0) return fail(c, MLC_ERR_MESH, "fine mesh has no interior node");
  std::vector<int64_t> dord(c->n);
  std::iota(dord.begin(), dord.end(), 0);
  if (c->opt.reorder) {
    std::vector<uint64_t> vk(c->n);
    for (int64_t i = 0; i < c->n; ++i) vk[i] = morton(&c->xyz[3 * (int64_t)interior[i]], c->lo, c->hi);
    std::stable_sort(dord.begin(), dord.end(), [&](int64_t a, int64_t b) { return vk[a] < vk[b]; });
  }
  c->v2d.assign(c->nv, -1);
  c->d2v.resize(c->n);
  c->dof_user.resize(c->n);
  for (int64_t d = 0; d < c->n; ++d) {
    int32_t v = interior[dord[d]];
    c->d2v[d] = v;
    c->v2d[v] = (int32_t)d;
    c->dof_user[d] = (int32_t)dord[d];
  }

  // ---- node -> tets, CSR pattern, assembly adjacency ------------------------------
  std::vector<int32_t> vt_ptr(c->nv + 1, 0), vt(NEL * c->nt);
  for (int64_t i = 0; i < NEL * c->nt; ++i) vt_ptr[c->tets[i] + 1]++;
  for (int64_t v = 0; v < c->nv; ++v) vt_ptr[v + 1] += vt_ptr[v];
  {
    std::vector<int32_t> fill(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int64_t t = 0; t < c->nt; ++t)
      for (int a = 0; a < NEL; ++a) vt[fill[c->tets[NEL * t + a]]++] = (int32_t)t;
  }
  c->rowptr.assign(c->n + 1, 0);
  c->col.clear();
  c->adj_ptr.assign(c->n + 1, 0);
  c->adj_tet.clear();
  c->adj_loc.clear();
  std::vector<int32_t> nbr;
  for (int64_t d = 0; d < c->n; ++d) {
    int32_t v = c->d2v[d];
    nbr.clear();
    for (int32_t e = vt_ptr[v]; e < vt_ptr[v + 1]; ++e) {
      int64_t t = vt[e];
      for (int a = 0; a < NEL; ++a) {
        int32_t dd = c->v2d[c->tets[NEL * t + a]];
        if (dd >= 0) nbr.push_back(dd);
      }
    }
    std::sort(nbr.begin(), nbr.end());
    nbr.erase(std::unique(nbr.begin(), nbr.end()), nbr.end());
    c->col.insert(c->col.end(), nbr.begin(), nbr.end());
    c->rowptr[d + 1] = (int32_t)c->col.size();
    for (int32_t e = vt_ptr[v]; e < vt_ptr[v + 1]; ++e) {
      int64_t t = vt[e];
      int la = -1;
      for (int a = 0; a < NEL; ++a)
        if (c->tets[NEL * t + a] == v) la = a;
      c->adj_tet.push_back((int32_t)t);
      c->adj_loc.push_back((int8_t)la);
    }
    c->adj_ptr[d + 1] = (int32_t)c->adj_tet.size();
  }
  if ((int64_t)c->col.size() >= (1LL << 31)) return fail(c, MLC_ERR_MESH, "too many nonzeros");
  // For every CSR slot (a, b): the element entries (tet t, local pair) that
  // add into it, in increasing tet order; slot_of[ne^2 t + ne a + b] is the
  // position of entry (a, b) of tet t in that order (-1 when a or b is a
  // boundary node). Assembly writes every element entry to its position and
  // then sums each slot's contiguous run, in this fixed order.
  {
    const int64_t nnz = (int64_t)c->col.size();
    std::vector<int32_t> cnt(nnz + 1, 0);
    c->diag_slot.assign(c->n, -1);
    c->slot_of.assign((int64_t)NEL * NEL * c->nt, -1);
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        c->slot_ptr.assign(nnz + 1, 0);
        for (int64_t j = 0; j < nnz; ++j) {
          if ((int64_t)c->slot_ptr[j] + cnt[j] >= (1LL << 31)) return fail(c, MLC_ERR_MESH, "too many element entries");
          c->slot_ptr[j + 1] = c->slot_ptr[j] + cnt[j];
        }
        std::fill(cnt.begin(), cnt.end(), 0);
      }
      for (int64_t t = 0; t < c->nt; ++t) {
        int32_t dd[P2_NE];
        for (int a = 0; a < NEL; ++a) dd[a] = c->v2d[c->tets[NEL * t + a]];
        for (int a = 0; a < NEL; ++a) {
          if (dd[a] < 0) continue;
          const int32_t* rb = &c->col[c->rowptr[dd[a]]];
          const int32_t* re = &c->col[c->rowptr[dd[a] + 1]];
          for (int b = 0; b < NEL; ++b) {
            if (dd[b] < 0) continue;
            int64_t slot = c->rowptr[dd[a]] + (std::lower_bound(rb, re, dd[b]) - rb);
            if (pass == 1) c->slot_of[(int64_t)NEL * NEL * t + NEL * a + b] = c->slot_ptr[slot] + cnt[slot];
            cnt[slot]++;
            if (a == b) c->diag_slot[dd[a]] = (int32_t)slot;
          }
        }
      }
    }
  }

  // ---- coarse mesh --------------------------------------------------------------
  std::vector<char> con = boundary_flags(c->cxyz, c->lo, c->hi);
  c->cv2d.assign(c->cnv, -1);
  c->cd2v.clear();
  for (int64_t v = 0; v < c->cnv; ++v)
    if (!con[v]) {
      c->cv2d[v] = (int32_t)c->cd2v.size();
      c->cd2v.push_back((int32_t)v);
    }
  c->nH = (int64_t)c->cd2v.size();
  if (c->nH == 0) return fail(c, MLC_ERR_MESH, "coarse mesh has no interior vertex");
  c->cgeo.assign(12 * c->cnt, 0.0);
  c->cvol.assign(c->cnt, 0.0);
  for (int64_t t = 0; t < c->cnt; ++t) {
    const double* x[4];
    for (int a = 0; a < 4; ++a) x[a] = &c->cxyz[3 * (int64_t)c->ctets[4 * t + a]];
    double Ji[9];
    double det = tet_inverse(x[0], x[1], x[2], x[3], Ji);
    if (!(std::fabs(det) > 1e-300)) return fail(c, MLC_ERR_MESH, "degenerate coarse tet");
    c->cvol[t] = std::fabs(det) / 6.0;
    double* g = &c->cgeo[12 * t];
    for (int k = 0; k < 3; ++k) g[k] = x[0][k];
    for (int k = 0; k < 9; ++k) g[3 + k] = Ji[k];
  }

  // ---- point location: prolongation and coarse parents ---------------------------
  Locator loc;
  loc.build(c);
  c->Pfull_k.assign(4 * c->nv, -1);
  c->Pfull_w.assign(4 * c->nv, 0.0);
  for (int64_t v = 0; v < c->nv; ++v) {
    double b[4], bm;
    int64_t t = loc.find(c, &c->xyz[3 * v], b, &bm);
    if (t < 0 || bm < -1e-9) return fail(c, MLC_ERR_NOT_NESTED, "fine node outside the coarse mesh");
    for (int a = 0; a < 4; ++a) {
      double w = std::fabs(b[a]) < 1e-13 ? 0.0 : b[a];
      c->Pfull_k[4 * v + a] = w != 0.0 ? c->ctets[4 * t + a] : -1;
      c->Pfull_w[4 * v + a] = w;
    }
  }
  c->Pk.assign(4 * c->n, -1);
  c->Pw.assign(4 * c->n, 0.0);
  std::vector<int32_t> ptc(c->nH + 1, 0);
  for (int64_t d = 0; d < c->n; ++d) {
    int32_t v = c->d2v[d];
    int s = 0;
    for (int a = 0; a < 4; ++a) {
      int32_t cv = c->Pfull_k[4 * (int64_t)v + a];
      if (cv < 0) continue;
      int32_t k = c->cv2d[cv];
      if (k < 0) continue;
      c->Pk[4 * d + s] = k;
      c->Pw[4 * d + s] = c->Pfull_w[4 * (int64_t)v + a];
      ptc[k + 1]++;
      ++s;
    }
  }
  c->PTptr.assign(c->nH + 1, 0);
  for (int64_t k = 0; k < c->nH; ++k) c->PTptr[k + 1] = c->PTptr[k] + ptc[k + 1];
  c->PTidx.assign(c->PTptr.back(), 0);
  c->PTw.assign(c->PTptr.back(), 0.0);
  {
    std::vector<int32_t> fill(c->PTptr.begin(), c->PTptr.end() - 1);
    for (int64_t d = 0; d < c->n; ++d)
      for (int s = 0; s < 4; ++s) {
        int32_t k = c->Pk[4 * d + s];
        if (k < 0) continue;
        c->PTidx[fill[k]] = (int32_t)d;
        c->PTw[fill[k]] = c->Pw[4 * d + s];
        fill[k]++;
      }
  }
  {
    // chunks of RESTRICT_CHUNK consecutive fine rows; in each, the entries
    // (row, coarse DoF, weight) of its rows sorted by coarse DoF, then row
    const int64_t RC = RESTRICT_CHUNK;
    const int64_t nch = (c->n + RC - 1) / RC;
    c->rch_seg.assign(nch + 1, 0);
    c->rseg_ptr.assign(1, 0);
    c->rent_row.clear();
    c->rent_w.clear();
    std::vector<int32_t> seg_k;
    std::vector<std::pair<int32_t, int32_t>> ent;  // (coarse DoF, slot 4 d + s)
    for (int64_t b = 0; b < nch; ++b) {
      ent.clear();
      for (int64_t d = b * RC; d < std::min<int64_t>(c->n, (b + 1) * RC); ++d)
        for (int s = 0; s < 4; ++s)
          if (c->Pk[4 * d + s] >= 0) ent.emplace_back(c->Pk[4 * d + s], (int32_t)(4 * d + s));
      std::sort(ent.begin(), ent.end());
      for (size_t e = 0; e < ent.size(); ++e) {
        if (e == 0 || ent[e].first != ent[e - 1].first) {
          if (e > 0) c->rseg_ptr.push_back((int32_t)c->rent_row.size());
          seg_k.push_back(ent[e].first);
        }
        c->rent_row.push_back((int32_t)(ent[e].second / 4 - b * RC));
        c->rent_w.push_back(c->Pw[ent[e].second]);
      }
      if (!ent.empty()) c->rseg_ptr.push_back((int32_t)c->rent_row.size());
      c->rch_seg[b + 1] = (int32_t)seg_k.size();
    }
    // segments of each coarse DoF, in chunk order
    c->kseg_ptr.assign(c->nH + 1, 0);
    for (int32_t k : seg_k) c->kseg_ptr[k + 1]++;
    for (int64_t k = 0; k < c->nH; ++k) c->kseg_ptr[k + 1] += c->kseg_ptr[k];
    c->kseg.assign(seg_k.size(), 0);
    std::vector<int32_t> fill(c->kseg_ptr.begin(), c->kseg_ptr.end() - 1);
    for (size_t g = 0; g < seg_k.size(); ++g) c->kseg[fill[seg_k[g]]++] = (int32_t)g;
  }
  c->parent.assign(c->nt, -1);
  std::vector<int32_t> gc(c->cnt + 1, 0);
  for (int64_t t = 0; t < c->nt; ++t) {
    double p[3] = {0, 0, 0};
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) p[k] += 0.25 * c->xyz[3 * (int64_t)c->tets[NEL * t + a] + k];
    double b[4], bm;
    int64_t C = loc.find(c, p, b, &bm);
    if (C < 0 || bm < -1e-9) return fail(c, MLC_ERR_NOT_NESTED, "fine tet outside the coarse mesh");
    // every vertex of the fine tet must lie in the parent (nested refinement)
    const double* g = &c->cgeo[12 * C];
    for (int a = 0; a < 4; ++a) {
      const double* x = &c->xyz[3 * (int64_t)c->tets[NEL * t + a]];
      double dx = x[0] - g[0], dy = x[1] - g[1], dz = x[2] - g[2];
      double l1 = g[3] * dx + g[4] * dy + g[5] * dz, l2 = g[6] * dx + g[7] * dy + g[8] * dz;
      double l3 = g[9] * dx + g[10] * dy + g[11] * dz;
      double m = std::min(std::min(1.0 - l1 - l2 - l3, l1), std::min(l2, l3));
      if (m < -1e-9) return fail(c, MLC_ERR_NOT_NESTED, "fine tet crosses a coarse tet");
    }
    c->parent[t] = (int32_t)C;
    gc[C + 1]++;
  }
  c->cgrp_ptr.assign(c->cnt + 1, 0);
  for (int64_t C = 0; C < c->cnt; ++C) c->cgrp_ptr[C + 1] = c->cgrp_ptr[C] + gc[C + 1];
  c->cgrp_tet.assign(c->nt, 0);
  {
    std::vector<int32_t> fill(c->cgrp_ptr.begin(), c->cgrp_ptr.end() - 1);
    for (int64_t t = 0; t < c->nt; ++t) c->cgrp_tet[fill[c->parent[t]]++] = (int32_t)t;
  }
  // the interior DoFs of every fine tet's nodes in coarse-group order (-1: boundary)
  c->cgrp_dof.assign((int64_t)NEL * c->nt, -1);
  for (int64_t e = 0; e < c->nt; ++e)
    for (int a = 0; a < NEL; ++a) c->cgrp_dof[NEL * e + a] = c->v2d[c->tets[NEL * (int64_t)c->cgrp_tet[e] + a]];
  return MLC_OK;
}

}  // namespace mlc
