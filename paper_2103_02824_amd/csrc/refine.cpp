// Adaptive loop on the host: Doerfler marking and conforming refinement by
// tagged (Maubach) bisection (Algorithm 1 steps 2-3; Section 2, the AFEM
// loop). The refinement reproduces a fixed order: bisected tets leave the list
// (the others keep their order), their first children follow in the order of
// the bisected tets, then their second children; the vertices a bisection
// creates are numbered in increasing order of their edge key (lo * 2^31 + hi).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "mlc.h"

namespace {

struct Refiner {
  std::vector<double> xyz;
  std::vector<int32_t> tets;
  std::vector<int8_t> tags;
  std::unordered_map<uint64_t, int64_t> mids;  // edge key -> midpoint vertex
  std::vector<int64_t> parents;                // 2 per created vertex
  std::vector<int64_t> batch_ptr{0};

  static uint64_t key(int64_t a, int64_t b) {
    const uint64_t lo = (uint64_t)std::min(a, b), hi = (uint64_t)std::max(a, b);
    return (lo << 31) + hi;
  }
  int64_t nv() const { return (int64_t)xyz.size() / 3; }
  int64_t nt() const { return (int64_t)tets.size() / 4; }

  // Bisect the tets whose mask entry is set; returns their number.
  int64_t bisect(const std::vector<uint8_t>& mask) {
    std::vector<int64_t> idx;
    for (int64_t t = 0; t < nt(); ++t)
      if (mask[t]) idx.push_back(t);
    if (idx.empty()) return 0;
    const int64_t m = (int64_t)idx.size();
    std::vector<uint64_t> keys(m);
    for (int64_t i = 0; i < m; ++i) {
      const int32_t* T = &tets[4 * idx[i]];
      keys[i] = key(T[0], T[tags[idx[i]]]);
    }
    // the missing midpoints, created in increasing key order
    std::vector<uint64_t> fresh;
    for (uint64_t k : keys)
      if (!mids.count(k)) fresh.push_back(k);
    std::sort(fresh.begin(), fresh.end());
    fresh.erase(std::unique(fresh.begin(), fresh.end()), fresh.end());
    for (uint64_t k : fresh) {
      const int64_t lo = (int64_t)(k >> 31), hi = (int64_t)(k & ((1ull << 31) - 1));
      const int64_t v = nv();
      for (int c = 0; c < 3; ++c) xyz.push_back(0.5 * (xyz[3 * lo + c] + xyz[3 * hi + c]));
      mids[k] = v;
      parents.push_back(lo);
      parents.push_back(hi);
    }
    if (!fresh.empty()) batch_ptr.push_back((int64_t)parents.size() / 2);
    std::vector<int32_t> c1(4 * m), c2(4 * m);
    std::vector<int8_t> nt_tag(m);
    for (int64_t i = 0; i < m; ++i) {
      const int32_t* T = &tets[4 * idx[i]];
      const int k = tags[idx[i]];
      const int32_t z = (int32_t)mids[keys[i]];
      // first child (x0..x_{k-1}, z, x_{k+1}..x3), second (x1..x_k, z, x_{k+1}..x3)
      for (int a = 0; a < 4; ++a) c1[4 * i + a] = T[a];
      c1[4 * i + k] = z;
      for (int a = 0; a < k; ++a) c2[4 * i + a] = T[a + 1];
      c2[4 * i + k] = z;
      for (int a = k + 1; a < 4; ++a) c2[4 * i + a] = T[a];
      nt_tag[i] = (int8_t)(k > 1 ? k - 1 : 3);
    }
    std::vector<int32_t> nt4;
    std::vector<int8_t> ntg;
    nt4.reserve(tets.size() + 4 * m);
    ntg.reserve(tags.size() + m);
    for (int64_t t = 0; t < nt(); ++t)
      if (!mask[t]) {
        nt4.insert(nt4.end(), &tets[4 * t], &tets[4 * t] + 4);
        ntg.push_back(tags[t]);
      }
    nt4.insert(nt4.end(), c1.begin(), c1.end());
    ntg.insert(ntg.end(), nt_tag.begin(), nt_tag.end());
    nt4.insert(nt4.end(), c2.begin(), c2.end());
    ntg.insert(ntg.end(), nt_tag.begin(), nt_tag.end());
    tets.swap(nt4);
    tags.swap(ntg);
    return m;
  }

  // Tets with an edge whose midpoint exists (a hanging vertex on that edge).
  std::vector<uint8_t> hanging(bool* any) const {
    static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    std::vector<uint8_t> h(nt(), 0);
    *any = false;
    for (int64_t t = 0; t < nt(); ++t)
      for (auto& e : E)
        if (mids.count(key(tets[4 * t + e[0]], tets[4 * t + e[1]]))) {
          h[t] = 1;
          *any = true;
          break;
        }
    return h;
  }
};

struct RefineOut {
  Refiner r;
};

}  // namespace

extern "C" mlc_status mlc_mark_dorfler(const double* eta2, int64_t nt, double theta, uint8_t* marked,
                                       int64_t* count) {
  if (!eta2 || !marked || nt < 1 || !(theta > 0.0 && theta <= 1.0)) return MLC_ERR_ARG;
  for (int64_t t = 0; t < nt; ++t)
    if (!(eta2[t] >= 0.0) || !std::isfinite(eta2[t])) return MLC_ERR_ARG;
  std::vector<int64_t> ord(nt);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return eta2[a] > eta2[b]; });
  double total = 0.0;  // summed in the sorted order, as the partial sums below
  for (int64_t k = 0; k < nt; ++k) total += eta2[ord[k]];
  std::fill(marked, marked + nt, (uint8_t)0);
  double acc = 0.0;
  int64_t k = 0;
  while (k < nt) {
    acc += eta2[ord[k]];
    marked[ord[k]] = 1;
    ++k;
    if (acc >= theta * total) break;
  }
  if (count) *count = k;
  return MLC_OK;
}

extern "C" mlc_status mlc_refine(int64_t nv, const double* xyz, int64_t nt, const int32_t* tets, const int8_t* tags,
                                 const uint8_t* marked, mlc_refine_result* out) {
  if (!out || !xyz || !tets || !tags || !marked || nv < 4 || nt < 1 || nv >= (int64_t)1 << 31) return MLC_ERR_ARG;
  *out = mlc_refine_result{};
  for (int64_t i = 0; i < 4 * nt; ++i)
    if (tets[i] < 0 || tets[i] >= nv) return MLC_ERR_MESH;
  for (int64_t t = 0; t < nt; ++t)
    if (tags[t] < 1 || tags[t] > 3) return MLC_ERR_ARG;
  auto* o = new RefineOut;
  Refiner& r = o->r;
  r.xyz.assign(xyz, xyz + 3 * nv);
  r.tets.assign(tets, tets + 4 * nt);
  r.tags.assign(tags, tags + nt);
  // the existing mesh is conforming: no midpoints yet
  std::vector<uint8_t> mask(marked, marked + nt);
  r.bisect(mask);
  for (int round = 0;; ++round) {
    if (round > 10000) {
      delete o;
      return MLC_ERR_MESH;  // closure did not terminate
    }
    bool any = false;
    std::vector<uint8_t> h = r.hanging(&any);
    if (!any) break;
    r.bisect(h);
  }
  out->nv = r.nv();
  out->nt = r.nt();
  out->xyz = r.xyz.data();
  out->tets = r.tets.data();
  out->tags = r.tags.data();
  out->n_new = r.nv() - nv;
  out->parents = r.parents.data();
  out->nbatch = (int32_t)r.batch_ptr.size() - 1;
  out->batch_ptr = r.batch_ptr.data();
  out->internal = o;
  return MLC_OK;
}

extern "C" void mlc_refine_free(mlc_refine_result* r) {
  if (!r) return;
  delete static_cast<RefineOut*>(r->internal);
  *r = mlc_refine_result{};
}
