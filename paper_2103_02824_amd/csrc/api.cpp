// The extern "C" entry points of include/mlc.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "inner.h"
#include "dense.h"
#include "mlc_internal.h"

namespace mlc {

int64_t small_len(int64_t nH, int N);

mlc_status fail(mlc_ctx* c, mlc_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

mlc_status hip_fail(mlc_ctx* c, hipError_t e, const char* what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return MLC_ERR_HIP;
}

namespace {

struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    return p;
  }
};

}  // namespace

size_t workspace_layout(mlc_ctx* c, char* base, Dev* d) {
  Carver w{base};
  const int64_t n = c->n, nt = c->nt, nv = c->nv, nH = c->nH, N = c->N, cnt = c->cnt;
  const int64_t nnz = (int64_t)c->col.size(), nadj = (int64_t)c->adj_tet.size();
  const int64_t ne = c->ne, nqt = c->nq * nt;
  d->tets = w.take<int32_t>(ne * nt);
  d->v2d = w.take<int32_t>(nv);
  d->xyz = w.take<double>(3 * nv);
  d->geo = w.take<double>(16 * nt);
  d->qpx = w.take<double>(3 * nqt);
  if (c->order == 2) d->qtab = w.take<double>(P2_TAB);
  d->vext = w.take<double>(nqt);
  d->vxc = w.take<double>(nqt);
  d->exc = w.take<double>(nqt);
  d->veff = w.take<double>(nqt);
  d->rho = w.take<double>(nqt);
  d->fld = w.take<double>(nqt);
  d->fld2 = w.take<double>(nqt);
  d->rhot = w.take<double>(nqt);
  d->rowptr = w.take<int32_t>(n + 1);
  d->col = w.take<int32_t>(nnz);
  d->adj_ptr = w.take<int32_t>(n + 1);
  d->adj_tet = w.take<int32_t>(nadj);
  d->adj_loc = w.take<int8_t>(nadj);
  d->bverts = w.take<int32_t>((int64_t)c->bverts.size());
  d->valA = w.take<double>(nnz);
  d->valF = w.take<double>(nnz);
  d->valW = w.take<double>(nnz);
  d->valM = w.take<double>(nnz);
  d->valK = w.take<double>(nnz);
  d->elem = w.take<double>(std::max<int64_t>(2 * (int64_t)c->slot_ptr.back(), 2 * ne * nt));
  d->slot_ptr = w.take<int32_t>(nnz + 1);
  d->slot_of = w.take<int32_t>(ne * ne * nt);
  d->diag_slot = w.take<int32_t>(n);
  d->dinvA = w.take<double>(n);
  d->dinvK = w.take<double>(n);
  d->Phi = w.take<double>(n * N);
  d->X = w.take<double>(n * N);
  d->R = w.take<double>(n * N);
  d->P = w.take<double>(n * N);
  d->Q = w.take<double>(n * N);
  d->B = w.take<double>(n * N);
  d->Y = w.take<double>(4 * n * N);
  d->Yh = w.take<double>(c->hartree ? 4 * n : 1);
  d->w = w.take<double>(nv);
  d->g = w.take<double>(nv);
  d->w0 = w.take<double>(n);
  d->lvec = w.take<double>(n);
  d->pb = w.take<double>(n);
  d->pr = w.take<double>(n);
  d->pp = w.take<double>(n);
  d->pq = w.take<double>(n);
  d->rho_nodal = w.take<double>(nv);
  d->Pk = w.take<int32_t>(4 * n);
  d->Pw = w.take<double>(4 * n);
  d->rch_seg = w.take<int32_t>((int64_t)c->rch_seg.size());
  d->rseg_ptr = w.take<int32_t>((int64_t)c->rseg_ptr.size());
  d->rent_row = w.take<int32_t>((int64_t)c->rent_row.size());
  d->rent_w = w.take<double>((int64_t)c->rent_w.size());
  d->kseg_ptr = w.take<int32_t>((int64_t)c->kseg_ptr.size());
  d->kseg = w.take<int32_t>((int64_t)c->kseg.size());
  d->rpart = w.take<double>((int64_t)c->kseg.size() * std::max<int64_t>(N, 1));
  d->rpartH = w.take<double>((int64_t)c->kseg.size());
  d->PTptr = w.take<int32_t>(nH + 1);
  d->PTidx = w.take<int32_t>((int64_t)c->PTidx.size());
  d->PTw = w.take<double>((int64_t)c->PTw.size());
  d->cgrp_ptr = w.take<int32_t>(cnt + 1);
  d->cgrp_tet = w.take<int32_t>(nt);
  d->cgrp_dof = w.take<int32_t>(ne * nt);
  d->cgeo = w.take<double>(12 * cnt);
  d->cel_ops = w.take<double>(40 * cnt);
  d->cel_orb = w.take<double>(14 * cnt * N);
  if (c->opt.variant == MLC_VARIANT_JOINT) {
    const int64_t npair = N * (N + 1) / 2;
    d->cel_pairs = w.take<double>(4 * cnt * npair);
    d->pair_jl = w.take<int32_t>(2 * npair);
  }
  d->cel_tri = w.take<double>(20 * cnt);
  d->chat = w.take<double>((4 * c->nq + 1) * nt);
  d->small = w.take<double>(small_len(nH, (int)N));
  d->coarse_in = w.take<double>(nH * N + nH + N + N * N);
  d->occ = w.take<double>(N);
  d->RZ = w.take<double>(4 * std::max<int64_t>(1, c->n_nuclei));
  d->colv = w.take<double>(2 * N);
  // 5 per-block column sums per orbital: the Galerkin dots of the learned start (the most of any user)
  int64_t nred = std::max<int64_t>(5 * (int64_t)elem_blocks(n, (int)N) * N, 3 * (int64_t)elem_blocks(n, 1));
  nred = std::max<int64_t>(nred, 2 * (int64_t)cg_max_blocks() * 3 * std::max<int64_t>(N, 1));
  nred = std::max<int64_t>(nred, (int64_t)qp_blocks(nt) * 16);
  nred = std::max<int64_t>(nred, (int64_t)gram_blocks(n) * N * N);
  c->nred = nred;
  d->red = w.take<double>(nred);
  d->red2 = w.take<double>((int64_t)gram_blocks(n) * N * N);
  d->scal = w.take<double>(10 * N);
  d->scalP = w.take<double>(10);
  d->flags = w.take<int32_t>(8);
  d->flagsP = w.take<int32_t>(8);
  if (c->opt.precision == MLC_PREC_FP32_IR) {
    d->valA32 = w.take<float>(nnz);
    d->dinvA32 = w.take<float>(n);
    d->X32 = w.take<float>(n * N);
    d->R32 = w.take<float>(n * N);
    d->P32 = w.take<float>(n * N);
    d->Q32 = w.take<float>(n * N);
    d->B32 = w.take<float>(n * N);
  }
  d->scal32 = w.take<double>(10 * N);
  d->flags32 = w.take<int32_t>(8);
  // learned initial guess: features, network outputs, column scales, choices
  d->F = w.take<float>(6 * n * N);
  d->Ynn = w.take<float>(n * N);
  d->gscale = w.take<double>(N);
  d->gsel = w.take<double>(4 * N);
  d->gdots = w.take<double>(5 * N);
  d->d2v = w.take<int32_t>(n);
  d->dof_user = w.take<int32_t>(n);
  d->chk = w.take<int32_t>(4);
  d->lmax = w.take<double>(2);
  d->lanc = w.take<double>(2 * 64 + 4);
  if (c->hartree && hartree_pc(c->opt) == MLC_PC_CHEBYSHEV) d->valK32 = w.take<float>(nnz);
  if (c->opt.hartree_coarse && c->hartree) {
    d->KHinv = w.take<double>(nH * nH);
    d->rH = w.take<double>(nH);
    d->eH = w.take<double>(nH);
  }
  if (c->opt.estimator) {
    d->nbr = w.take<int32_t>(4 * nt);
    d->tord = w.take<int32_t>(nt);
  }
  return w.off + 256;
}

#define HIPCHK(x)                                     \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return hip_fail(c, e_, #x); \
  } while (0)

template <class T>
static hipError_t up(hipStream_t s, T* dst, const std::vector<T>& src) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s);
}

mlc_status upload_and_init(mlc_ctx* c) {
  auto& d = c->d;
  hipStream_t s = c->stream;
  // quadrature points: barycentric combinations of each tet's vertices (its first 4 nodes)
  const int nq = c->nq, ne = c->ne;
  std::vector<double> qpx(3 * nq * c->nt);
  for (int64_t t = 0; t < c->nt; ++t)
    for (int q = 0; q < nq; ++q)
      for (int k = 0; k < 3; ++k) {
        double v = 0.0;
        for (int j = 0; j < 4; ++j) {
          const double lq = c->order == 2 ? c->qtab[P2_T_L + 4 * q + j] : (q == j ? QA : QB);
          v += lq * c->xyz[3 * (int64_t)c->tets[ne * t + j] + k];
        }
        qpx[3 * (nq * t + q) + k] = v;
      }
  std::vector<double> RZ(4 * std::max(1, c->n_nuclei), 0.0);
  for (int k = 0; k < c->n_nuclei; ++k) {
    for (int x = 0; x < 3; ++x) RZ[4 * k + x] = c->R[3 * k + x];
    RZ[4 * k + 3] = c->Z[k];
  }
  HIPCHK(up(s, d.tets, c->tets));
  HIPCHK(up(s, d.v2d, c->v2d));
  HIPCHK(up(s, d.xyz, c->xyz));
  HIPCHK(up(s, d.geo, c->geo));
  HIPCHK(up(s, d.qpx, qpx));
  if (d.qtab) HIPCHK(up(s, d.qtab, c->qtab));
  HIPCHK(up(s, d.rowptr, c->rowptr));
  HIPCHK(up(s, d.col, c->col));
  HIPCHK(up(s, d.adj_ptr, c->adj_ptr));
  HIPCHK(up(s, d.adj_tet, c->adj_tet));
  HIPCHK(up(s, d.adj_loc, c->adj_loc));
  HIPCHK(up(s, d.bverts, c->bverts));
  HIPCHK(up(s, d.slot_ptr, c->slot_ptr));
  HIPCHK(up(s, d.slot_of, c->slot_of));
  HIPCHK(up(s, d.diag_slot, c->diag_slot));
  HIPCHK(up(s, d.Pk, c->Pk));
  HIPCHK(up(s, d.Pw, c->Pw));
  HIPCHK(up(s, d.rch_seg, c->rch_seg));
  HIPCHK(up(s, d.rseg_ptr, c->rseg_ptr));
  HIPCHK(up(s, d.rent_row, c->rent_row));
  HIPCHK(up(s, d.rent_w, c->rent_w));
  HIPCHK(up(s, d.kseg_ptr, c->kseg_ptr));
  HIPCHK(up(s, d.kseg, c->kseg));
  HIPCHK(up(s, d.PTptr, c->PTptr));
  HIPCHK(up(s, d.PTidx, c->PTidx));
  HIPCHK(up(s, d.PTw, c->PTw));
  HIPCHK(up(s, d.cgrp_ptr, c->cgrp_ptr));
  HIPCHK(up(s, d.cgrp_tet, c->cgrp_tet));
  HIPCHK(up(s, d.cgrp_dof, c->cgrp_dof));
  HIPCHK(up(s, d.cgeo, c->cgeo));
  HIPCHK(up(s, d.occ, c->occ));
  HIPCHK(up(s, d.RZ, RZ));
  HIPCHK(up(s, d.d2v, c->d2v));
  HIPCHK(up(s, d.dof_user, c->dof_user));
  if (d.nbr) {
    HIPCHK(up(s, d.nbr, c->nbr));
    HIPCHK(up(s, d.tord, c->tord));
  }
  if (d.pair_jl) {
    std::vector<int32_t> jl;
    for (int j = 0; j < c->N; ++j)
      for (int l = j; l < c->N; ++l) {
        jl.push_back(j);
        jl.push_back(l);
      }
    HIPCHK(up(s, d.pair_jl, jl));
  }
  HIPCHK(hipMemsetAsync(d.w, 0, sizeof(double) * c->nv, s));
  HIPCHK(hipMemsetAsync(d.g, 0, sizeof(double) * c->nv, s));
  HIPCHK(hipMemsetAsync(d.small, 0, sizeof(double) * small_len(c->nH, c->N), s));
  HIPCHK(hipMemsetAsync(d.w0, 0, sizeof(double) * c->n, s));
  // fixed quantities: V_ext at the quadrature points, K, M, coarse trilinear tensor
  launch_vext(s, nq * c->nt, d.qpx, d.RZ, c->n_nuclei, c->potential, c->rc, c->omega, d.vext);
  const int64_t nnz = (int64_t)c->col.size();
  const int64_t ns = c->slot_ptr.back();
  if (c->order == 2) {
    launch_assemble2_p2(s, c->nt, c->n, nnz, d.geo, d.slot_ptr, d.slot_of, d.diag_slot, d.elem, 1.0, nullptr, 0.0,
                        d.valK, d.dinvK, 0.0, nullptr, d.valM, d.qtab);
    launch_assemble2_p2(s, c->nt, c->n, nnz, d.geo, d.slot_ptr, d.slot_of, d.diag_slot, d.elem, 0.0, nullptr, 1.0,
                        d.valM, nullptr, 0.0, nullptr, nullptr, d.qtab);
  } else {
    launch_assemble2(s, c->nt, c->n, nnz, d.geo, d.slot_ptr, d.slot_of, ns, d.diag_slot, d.elem, 1.0, nullptr, 0.0,
                     d.valK, d.dinvK, 0.0, nullptr, d.valM);
    launch_assemble2(s, c->nt, c->n, nnz, d.geo, d.slot_ptr, d.slot_of, ns, d.diag_slot, d.elem, 0.0, nullptr, 1.0,
                     d.valM, nullptr, 0.0, nullptr, nullptr);
  }
  launch_gershgorin(s, c->n, d.rowptr, d.valK, d.dinvK, d.red, d.lmax + 1);
  if (c->opt.cheb_lanczos)
    launch_lanczos_lmax(s, c->n, d.rowptr, d.col, d.valK, d.dinvK, c->opt.cheb_lanczos, 1.1, d.Y, d.red, d.lanc,
                        d.lmax + 1);
  if (d.valK32) launch_to_f32(s, nnz, d.valK, d.valK32);
  if (c->order == 2) {
    launch_coarse_tri_p2(s, c->cnt, d.cgrp_ptr, d.cgrp_tet, d.tets, d.geo, d.xyz, d.cgeo, d.qtab, d.cel_tri);
    launch_coarse_hats_p2(s, c->cnt, c->nt, d.cgrp_ptr, d.cgrp_tet, d.tets, d.geo, d.xyz, d.cgeo, d.qtab, d.chat);
  } else {
    launch_coarse_tri(s, c->cnt, d.cgrp_ptr, d.cgrp_tet, d.tets, d.geo, d.xyz, d.cgeo, d.cel_tri);
    launch_coarse_hats(s, c->cnt, c->nt, d.cgrp_ptr, d.cgrp_tet, d.tets, d.geo, d.xyz, d.cgeo, d.chat);
  }
  if (d.KHinv) {
    // coarse stiffness K_H = P^T K P of the nested P1 spaces (element by element: the coarse hat
    // gradients are constant on a coarse tet), its Cholesky factor and explicit inverse
    const int64_t nH = c->nH;
    c->h_KHinv.assign(nH * nH, 0.0);
    std::vector<double> L(nH * nH, 0.0);
    for (int64_t C = 0; C < c->cnt; ++C) {
      const double* g = &c->cgeo[12 * C];
      double gr[4][3];
      for (int x = 0; x < 3; ++x) {
        gr[1][x] = g[3 + x];
        gr[2][x] = g[6 + x];
        gr[3][x] = g[9 + x];
        gr[0][x] = -(gr[1][x] + gr[2][x] + gr[3][x]);
      }
      int k[4];
      for (int a = 0; a < 4; ++a) k[a] = c->cv2d[c->ctets[4 * C + a]];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          if (k[a] >= 0 && k[b] >= 0)
            L[(int64_t)k[a] * nH + k[b]] +=
                c->cvol[C] * (gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2]);
    }
    if (!dense::cholesky(L, nH)) return fail(c, MLC_ERR_NONFINITE, "coarse stiffness not SPD");
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nH; ++j) {
      std::vector<double> e(nH, 0.0);
      e[j] = 1.0;
      dense::forward(L, nH, e.data());
      dense::backward(L, nH, e.data());
      for (int64_t i = 0; i < nH; ++i) c->h_KHinv[i * nH + j] = e[i];
    }
    HIPCHK(up(s, d.KHinv, c->h_KHinv));
  }
  c->h_tri.resize(20 * c->cnt);
  HIPCHK(hipMemcpyAsync(c->h_tri.data(), d.cel_tri, sizeof(double) * c->h_tri.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  c->h_Mh_chol.clear();
  c->h_Kh_chol.clear();
  return MLC_OK;
}

mlc_status probe(mlc_ctx* c, int which, double* out, int64_t count) {
  const int64_t n = c->n, nH = c->nH, nv = c->nv, nt = c->nt;
  const int N = c->N;
  auto need = [&](int64_t k) { return count == k ? MLC_OK : fail(c, MLC_ERR_ARG, "probe size mismatch"); };
  hipStream_t s = c->stream;
  auto& d = c->d;
  auto dev_perm = [&](const double* src, int64_t cols) -> mlc_status {
    std::vector<double> h(n * cols);
    HIPCHK(hipMemcpyAsync(h.data(), src, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t a = 0; a < n; ++a)
      for (int64_t j = 0; j < cols; ++j) out[(int64_t)c->dof_user[a] * cols + j] = h[a * cols + j];
    return MLC_OK;
  };
  std::vector<double> tmp;
  const double* h = c->last_small.data();
  int64_t hn = nH * N, nn = (int64_t)N * N;
  mlc_status st;
  switch (which) {
    case MLC_PROBE_U:
      if ((st = need(n * N))) return st;
      return dev_perm(d.X, N);
    case MLC_PROBE_W0:
      if ((st = need(n))) return st;
      return dev_perm(d.w0, 1);
    case MLC_PROBE_G:
      if ((st = need(nv))) return st;
      HIPCHK(hipMemcpyAsync(out, d.g, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      return MLC_OK;
    case MLC_PROBE_VXC_QP: {
      if ((st = need(c->nq * nt))) return st;
      // library tet order -> caller tet order is not tracked; return per library tet
      HIPCHK(hipMemcpyAsync(out, d.vxc, sizeof(double) * c->nq * nt, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      return MLC_OK;
    }
    case MLC_PROBE_PT_AFIX_U:
    case MLC_PROBE_PT_MW0_U:
    case MLC_PROBE_PT_M_U:
    case MLC_PROBE_PT_K_U:
      if ((st = need(hn))) return st;
      std::memcpy(out, h + (which - MLC_PROBE_PT_AFIX_U) * hn, sizeof(double) * hn);
      return MLC_OK;
    case MLC_PROBE_UT_AFIX_U:
    case MLC_PROBE_UT_MW0_U:
    case MLC_PROBE_UT_M_U:
    case MLC_PROBE_UT_K_U:
      if ((st = need(nn))) return st;
      std::memcpy(out, h + 4 * hn + (which - MLC_PROBE_UT_AFIX_U) * nn, sizeof(double) * nn);
      return MLC_OK;
    case MLC_PROBE_HARTREE_D:
      if ((st = need(nH + 2))) return st;
      std::memcpy(out, h + 4 * hn + 4 * nn, sizeof(double) * nH);
      out[nH] = h[4 * hn + 4 * nn + 2 * nH + 0];
      out[nH + 1] = h[4 * hn + 4 * nn + 2 * nH + 1];
      return MLC_OK;
    case MLC_PROBE_AFIX_H:
    case MLC_PROBE_MW0_H:
    case MLC_PROBE_M_H:
    case MLC_PROBE_K_H: {
      if ((st = need(nH * nH))) return st;
      int off = 10 * (which - MLC_PROBE_AFIX_H);
      std::fill(out, out + nH * nH, 0.0);
      static const int base[4] = {0, 4, 7, 9};
      for (int64_t C = 0; C < c->cnt; ++C)
        for (int a = 0; a < 4; ++a) {
          int ka = c->cv2d[c->ctets[4 * C + a]];
          if (ka < 0) continue;
          for (int b = 0; b < 4; ++b) {
            int kb = c->cv2d[c->ctets[4 * C + b]];
            if (kb < 0) continue;
            int j = std::min(a, b), k = std::max(a, b);
            out[(int64_t)ka * nH + kb] += c->last_cel_ops[40 * C + off + base[j] + (k - j)];
          }
        }
      return MLC_OK;
    }
    case MLC_PROBE_AH4: {
      if ((st = need(N * nH * nH))) return st;
      std::fill(out, out + N * nH * nH, 0.0);
      static const int base[4] = {0, 4, 7, 9};
      for (int64_t C = 0; C < c->cnt; ++C)
        for (int i = 0; i < N; ++i)
          for (int a = 0; a < 4; ++a) {
            int ka = c->cv2d[c->ctets[4 * C + a]];
            if (ka < 0) continue;
            for (int b = 0; b < 4; ++b) {
              int kb = c->cv2d[c->ctets[4 * C + b]];
              if (kb < 0) continue;
              int j = std::min(a, b), k = std::max(a, b);
              out[(int64_t)i * nH * nH + (int64_t)ka * nH + kb] += c->last_cel_orb[(C * N + i) * 14 + base[j] + (k - j)];
            }
          }
      return MLC_OK;
    }
    case MLC_PROBE_RHS: {
      if ((st = need(N * nH))) return st;
      std::fill(out, out + N * nH, 0.0);
      for (int64_t C = 0; C < c->cnt; ++C)
        for (int i = 0; i < N; ++i)
          for (int a = 0; a < 4; ++a) {
            int ka = c->cv2d[c->ctets[4 * C + a]];
            if (ka >= 0) out[(int64_t)i * nH + ka] += c->last_cel_orb[(C * N + i) * 14 + 10 + a];
          }
      return MLC_OK;
    }
    case MLC_PROBE_THETA2:
      if ((st = need(N))) return st;
      std::copy(c->last_theta2.begin(), c->last_theta2.end(), out);
      return MLC_OK;
    case MLC_PROBE_PHI_H:
      if ((st = need(nH * N))) return st;
      std::copy(c->last_phiH.begin(), c->last_phiH.end(), out);
      return MLC_OK;
    case MLC_PROBE_WH:
      if ((st = need(nH + 1))) return st;
      std::copy(c->last_wH.begin(), c->last_wH.end(), out);
      out[nH] = c->last_theta1;
      return MLC_OK;
    case MLC_PROBE_SIGMA:
      if ((st = need(1))) return st;
      out[0] = c->last_sigma;
      return MLC_OK;
    case MLC_PROBE_FEATURES:
    case MLC_PROBE_NN_OUT: {
      const int per = which == MLC_PROBE_FEATURES ? 6 : 1;
      if ((st = need(n * N * per))) return st;
      std::vector<float> h(n * N * per);
      HIPCHK(hipMemcpyAsync(h.data(), which == MLC_PROBE_FEATURES ? d.F : d.Ynn, sizeof(float) * h.size(),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int64_t a = 0; a < n; ++a)
        for (int64_t j = 0; j < (int64_t)N * per; ++j)
          out[(int64_t)c->dof_user[a] * N * per + j] = h[a * N * per + j];
      return MLC_OK;
    }
    case MLC_PROBE_GUESS_SCALE:
      if ((st = need(N))) return st;
      HIPCHK(hipMemcpyAsync(out, d.gscale, sizeof(double) * N, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      return MLC_OK;
    case MLC_PROBE_LMAX:
      if ((st = need(2))) return st;
      HIPCHK(hipMemcpyAsync(out, d.lmax, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      return MLC_OK;
    case MLC_PROBE_PATTERN:
      if ((st = need(3))) return st;
      out[0] = (double)c->col.size();
      out[1] = c->ne;
      out[2] = c->nq;
      return MLC_OK;
    default:
      return fail(c, MLC_ERR_ARG, "unknown probe");
  }
}

}  // namespace mlc

using namespace mlc;

extern "C" {

void mlc_options_default(mlc_options* o) {
  if (!o) return;
  o->cg_rtol = 1e-10;
  o->cg_maxit = 20000;
  o->check_every = 25;
  o->shift = 1;
  o->sigma0 = 1.0;
  o->poisson_rtol = 1e-12;
  o->inner_maxit = 500;
  o->inner_tol = 1e-10;
  o->n_extra = 8;
  o->reorder = 1;
  o->time_kernels = 0;
  o->use_graphs = 1;
  o->precision = MLC_PREC_FP64;
  o->ir_inner_rtol = 1e-4;
  o->ir_max_outer = 30;
  o->precond = MLC_PC_JACOBI;
  o->cheb_degree = 4;
  o->cheb_ratio = 30.0;
  o->hartree_coarse = 0;
  o->hartree_precond = -1;
  o->inner_mix_history = 6;
  o->inner_mix_beta = 0.5;
  o->variant = MLC_VARIANT_EIGENPAIRWISE;
  o->estimator = 0;
  o->cheb_lanczos = 0;
  o->hartree_cheb_degree = 0;
  o->hartree_cheb_ratio = 0.0;
}

mlc_status mlc_create(const mlc_mesh* fine, const mlc_mesh* coarse, const mlc_system* sys, const mlc_options* opt,
                      mlc_ctx** out) {
  if (!out) return MLC_ERR_ARG;
  *out = nullptr;
  if (!fine || !coarse || !sys || !fine->xyz || !fine->tets || !coarse->xyz || !coarse->tets) return MLC_ERR_ARG;
  if (sys->n_orbitals < 1 || sys->n_orbitals > MLC_MAX_ORBITALS || !sys->occupations) return MLC_ERR_ARG;
  if (sys->potential < 0 || sys->potential > 2 || sys->xc < 0 || sys->xc > 2) return MLC_ERR_ARG;
  if (sys->n_nuclei < 0 || (sys->n_nuclei > 0 && (!sys->R || !sys->Z))) return MLC_ERR_ARG;
  if (sys->potential != MLC_POT_HARMONIC && sys->n_nuclei == 0) return MLC_ERR_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(sys->box_hi[k] > sys->box_lo[k]) || !std::isfinite(sys->box_lo[k]) || !std::isfinite(sys->box_hi[k]))
      return MLC_ERR_ARG;
  if ((fine->order != 1 && fine->order != 2) || coarse->order != 1) return MLC_ERR_ARG;
  if (sys->potential == MLC_POT_ERF && !(sys->rc > 0)) return MLC_ERR_ARG;
  for (int i = 0; i < sys->n_orbitals; ++i)
    if (!(sys->occupations[i] >= 0.0) || !std::isfinite(sys->occupations[i])) return MLC_ERR_ARG;
  mlc_ctx* c = new (std::nothrow) mlc_ctx();
  if (!c) return MLC_ERR_ARG;
  if (opt)
    c->opt = *opt;
  else
    mlc_options_default(&c->opt);
  if (!(c->opt.cg_rtol > 0) || c->opt.cg_maxit < 1 || c->opt.check_every < 1 || c->opt.inner_maxit < 1 ||
      c->opt.n_extra < 0 || !(c->opt.poisson_rtol > 0) ||
      (c->opt.precision != MLC_PREC_FP64 && c->opt.precision != MLC_PREC_FP32_IR) ||
      (c->opt.precision == MLC_PREC_FP32_IR && (!(c->opt.ir_inner_rtol > 0) || c->opt.ir_max_outer < 1)) ||
      (c->opt.precond != MLC_PC_JACOBI && c->opt.precond != MLC_PC_CHEBYSHEV) ||
      (c->opt.hartree_precond != -1 && c->opt.hartree_precond != MLC_PC_JACOBI &&
       c->opt.hartree_precond != MLC_PC_CHEBYSHEV) ||
      ((c->opt.precond == MLC_PC_CHEBYSHEV || hartree_pc(c->opt) == MLC_PC_CHEBYSHEV) &&
       (c->opt.cheb_degree < 2 || c->opt.cheb_degree > 16 || !(c->opt.cheb_ratio > 1.0))) ||
      c->opt.inner_mix_history < 0 || c->opt.inner_mix_history > 16 ||
      (c->opt.variant != MLC_VARIANT_EIGENPAIRWISE && c->opt.variant != MLC_VARIANT_JOINT) ||
      (c->opt.variant == MLC_VARIANT_JOINT && sys->n_orbitals > 64) ||
      (c->opt.estimator != 0 && c->opt.estimator != 1) ||
      (c->opt.cheb_lanczos != 0 && (c->opt.cheb_lanczos < 2 || c->opt.cheb_lanczos > 64)) ||
      (c->opt.hartree_cheb_degree != 0 && (c->opt.hartree_cheb_degree < 2 || c->opt.hartree_cheb_degree > 16)) ||
      !(c->opt.hartree_cheb_ratio == 0.0 || c->opt.hartree_cheb_ratio > 1.0) ||
      (fine->order == 2 && (c->opt.estimator != 0 || c->opt.variant == MLC_VARIANT_JOINT)) ||
      !(c->opt.inner_mix_beta > 0.0 && c->opt.inner_mix_beta <= 1.0)) {
    delete c;
    return MLC_ERR_ARG;
  }
  c->n_nuclei = sys->n_nuclei;
  c->R.assign(sys->R ? sys->R : nullptr, sys->R ? sys->R + 3 * sys->n_nuclei : nullptr);
  c->Z.assign(sys->Z ? sys->Z : nullptr, sys->Z ? sys->Z + sys->n_nuclei : nullptr);
  c->N = sys->n_orbitals;
  c->occ.assign(sys->occupations, sys->occupations + c->N);
  c->potential = sys->potential;
  c->rc = sys->rc;
  c->omega = sys->omega;
  c->xc = sys->xc;
  c->xalpha = sys->xalpha;
  c->hartree = sys->hartree ? 1 : 0;
  for (int k = 0; k < 3; ++k) {
    c->lo[k] = sys->box_lo[k];
    c->hi[k] = sys->box_hi[k];
  }
  mlc_status st = build_mesh(c, fine, coarse);
  if (st != MLC_OK) {
    // keep the message reachable for the caller through a temporary context
    *out = c;
    return st;
  }
  *out = c;
  return MLC_OK;
}

mlc_status mlc_sizes(const mlc_ctx* c, int64_t* n_dof, int64_t* n_coarse_dof, int64_t* n_vertices,
                     int32_t* n_orbitals) {
  if (!c) return MLC_ERR_ARG;
  if (n_dof) *n_dof = c->n;
  if (n_coarse_dof) *n_coarse_dof = c->nH;
  if (n_vertices) *n_vertices = c->nv;
  if (n_orbitals) *n_orbitals = c->N;
  return MLC_OK;
}

mlc_status mlc_workspace_bytes(const mlc_ctx* c, size_t* bytes) {
  if (!c || !bytes) return MLC_ERR_ARG;
  Dev tmp;
  *bytes = workspace_layout(const_cast<mlc_ctx*>(c), nullptr, &tmp);
  return MLC_OK;
}

mlc_status mlc_bind(mlc_ctx* c, void* dev_workspace, size_t bytes, void* hip_stream) {
  if (!c) return MLC_ERR_ARG;
  if (c->n == 0) return fail(c, MLC_ERR_STATE, "context was not built");
  Dev tmp;
  size_t need = workspace_layout(c, nullptr, &tmp);
  if (!dev_workspace || bytes < need) return fail(c, MLC_ERR_WORKSPACE, "workspace missing or too small");
  c->ws = static_cast<char*>(dev_workspace);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(hip_stream);
  workspace_layout(c, c->ws, &c->d);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  c->ev_used = 0;
  for (int k = 0; k < 3; ++k) {
    for (auto& g : c->cg_graph[k]) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
    c->cg_pred[k] = 0;
  }
  if (!c->side) {
    hipError_t he = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (he != hipSuccess) return hip_fail(c, he, "side stream");
  }
  if (c->opt.use_graphs && !c->cap_stream) {
    hipError_t he = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_fail(c, he, "hipStreamCreateWithFlags");
  }
  if (c->opt.time_kernels) {
    c->ev_pool.resize(2 * std::max(1, c->opt.check_every));
    for (auto& e : c->ev_pool) {
      hipError_t he = hipEventCreate(&e);
      if (he != hipSuccess) return hip_fail(c, he, "hipEventCreate");
    }
  }
  mlc_status st = upload_and_init(c);
  if (st != MLC_OK) return st;
  c->bound = true;
  c->has_state = false;
  c->has_step = false;
  return MLC_OK;
}

mlc_status mlc_initial_state(mlc_ctx* c, double tol, int32_t maxit, int32_t* iters) {
  if (!c) return MLC_ERR_ARG;
  if (!c->bound) return fail(c, MLC_ERR_STATE, "mlc_bind first");
  if (!(tol > 0) || maxit < 1) return fail(c, MLC_ERR_ARG, "bad tolerance or iteration cap");
  int it = 0;
  mlc_status st = coarse_scf(c, tol, maxit, &it);
  if (iters) *iters = it;
  return st;
}

mlc_status mlc_set_state(mlc_ctx* c, const double* lambda, const double* phi_dev, const double* w_dev) {
  if (!c || !lambda || !phi_dev || !w_dev) return MLC_ERR_ARG;
  if (!c->bound) return fail(c, MLC_ERR_STATE, "mlc_bind first");
  const int N = c->N;
  for (int i = 0; i < N; ++i)
    if (!std::isfinite(lambda[i])) return fail(c, MLC_ERR_NONFINITE, "non-finite eigenvalue");
  hipStream_t s = c->stream;
  auto& d = c->d;
  // the caller's arrays are checked before anything of the state is overwritten
  int32_t bad = 0;
  launch_count_nonfinite(s, c->n * N, phi_dev, c->nv, w_dev, d.chk);
  HIPCHK(hipMemcpyAsync(&bad, d.chk, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (bad) return fail(c, MLC_ERR_NONFINITE, "non-finite value in phi or w");
  launch_permute_rows(s, c->n, N, d.dof_user, phi_dev, d.Phi, /*gather=*/1);
  HIPCHK(hipMemcpyAsync(d.w, w_dev, sizeof(double) * c->nv, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  c->lam.assign(lambda, lambda + N);
  c->has_state = true;
  c->has_step = false;
  return MLC_OK;
}

mlc_status mlc_correction_step(mlc_ctx* c, mlc_step_report* rep) {
  if (!c) return MLC_ERR_ARG;
  if (!c->bound || !c->has_state) return fail(c, MLC_ERR_STATE, "bind and set a state first");
  return fine_stage_and_step(c, rep);
}

mlc_status mlc_get_results(mlc_ctx* c, double* lambda, double* phi_dev, double* rho_dev, double* w_dev) {
  if (!c) return MLC_ERR_ARG;
  if (!c->bound || !c->has_state) return fail(c, MLC_ERR_STATE, "no state");
  const int N = c->N;
  hipStream_t s = c->stream;
  auto& d = c->d;
  if (lambda) std::copy(c->lam.begin(), c->lam.end(), lambda);
  if (phi_dev) launch_permute_rows(s, c->n, N, d.dof_user, d.Phi, phi_dev, /*gather=*/0);
  if (rho_dev) launch_rho_nodal(s, c->nv, d.v2d, d.Phi, N, d.occ, rho_dev);
  if (w_dev) HIPCHK(hipMemcpyAsync(w_dev, d.w, sizeof(double) * c->nv, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return MLC_OK;
}

mlc_status mlc_probe(mlc_ctx* c, int32_t which, double* out, int64_t count) {
  if (!c || !out) return MLC_ERR_ARG;
  if (!c->has_step) return fail(c, MLC_ERR_STATE, "no correction step has run");
  return probe(c, which, out, count);
}

mlc_status mlc_estimate(mlc_ctx* c, double* eta2) {
  if (!c || !eta2) return MLC_ERR_ARG;
  if (!c->bound || !c->has_state) return fail(c, MLC_ERR_STATE, "bind and set a state first");
  if (!c->opt.estimator) return fail(c, MLC_ERR_STATE, "created without options.estimator");
  auto& d = c->d;
  hipStream_t s = c->stream;
  // V_eff of the current state at the quadrature points, then eta^2 per tet
  launch_qp_fields(s, c->nt, d.tets, d.v2d, d.Phi, c->N, d.occ, d.w, d.vext, d.geo, d.qpx, c->xc, c->xalpha, d.vxc,
                   d.exc, d.veff, d.rho, d.red);
  HIPCHK(hipMemcpyAsync(d.colv, c->lam.data(), sizeof(double) * c->N, hipMemcpyHostToDevice, s));
  launch_estimate(s, c->nt, c->N, d.tets, d.v2d, d.Phi, d.colv, d.veff, d.geo, d.xyz, d.nbr, d.tord, eta2);
  HIPCHK(hipGetLastError());
  return MLC_OK;
}

mlc_status mlc_transfer_vertices(int64_t nv_old, int64_t nv_new, const int64_t* parents, int32_t nbatch,
                                 const int64_t* batch_ptr, int32_t ncols, double* values, void* stream) {
  if (nv_old < 1 || nv_new < nv_old || nbatch < 0 || ncols < 1 || !values || (nv_new > nv_old && !parents) ||
      (nbatch > 0 && !batch_ptr))
    return MLC_ERR_ARG;
  if (nbatch > 0 && (batch_ptr[0] != 0 || batch_ptr[nbatch] != nv_new - nv_old)) return MLC_ERR_ARG;
  for (int32_t b = 0; b < nbatch; ++b)
    if (batch_ptr[b + 1] < batch_ptr[b]) return MLC_ERR_ARG;
  if (nbatch == 0 && nv_new != nv_old) return MLC_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  for (int32_t b = 0; b < nbatch; ++b)
    launch_transfer(s, batch_ptr[b + 1] - batch_ptr[b], batch_ptr[b], nv_old, parents, ncols, values);
  return hipGetLastError() == hipSuccess ? MLC_OK : MLC_ERR_HIP;
}

mlc_status mlc_time_kernel(mlc_ctx* c, int32_t which, int32_t reps, double* avg_us) {
  if (!c || !avg_us || reps < 1 || reps > 100000 || which < MLC_KERNEL_CG_SPMM ||
      which > MLC_KERNEL_HARTREE_CHEB_STEP)
    return MLC_ERR_ARG;
  if (!c->has_step) return fail(c, MLC_ERR_STATE, "no correction step has run");
  const bool cheb = which == MLC_KERNEL_CHEB_STEP || which == MLC_KERNEL_HARTREE_CHEB_STEP;
  const bool hart = which >= MLC_KERNEL_HARTREE_SPMM;
  if (cheb && (hart ? hartree_pc(c->opt) : c->opt.precond) != MLC_PC_CHEBYSHEV)
    return fail(c, MLC_ERR_ARG, "no polynomial preconditioner");
  if (hart && !c->hartree) return fail(c, MLC_ERR_ARG, "no Hartree problem");
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const int N = hart ? 1 : c->N;
  const bool f32 = !hart && c->opt.precision == MLC_PREC_FP32_IR;
  float* Yf = reinterpret_cast<float*>(d.Y);
  // one interior Chebyshev step (j = 2: both iterate blocks read, the older
  // one overwritten, no r.z partials): the launch of every step but the first
  // and the last
  double* Yd = hart ? d.Yh : d.Y;
  PolyPC<double> pd{hart ? d.lmax + 1 : d.lmax, hart ? hartree_ratio(c->opt) : c->opt.cheb_ratio, 3, {Yd, Yd + n * N}, nullptr,
                    hart ? d.valK32 : nullptr};
  PolyPC<float> pf{d.lmax, c->opt.cheb_ratio, 3, {Yf, Yf + n * N}, nullptr};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, MLC_ERR_HIP, "hipEventCreate");
  }
  auto one = [&]() {
    if (hart) {
      if (cheb)
        launch_cheb_step_t<double>(s, n, 1, d.rowptr, d.col, d.valK, d.dinvK, d.pr, pd, 2, pd.Z[1], pd.Z[0], pd.Z[0],
                                   nullptr, nullptr);
      else
        launch_spmm2(s, n, 1, d.rowptr, d.col, d.valK, d.pp, d.pq, d.red, nullptr);
    } else if (f32) {
      if (cheb)
        launch_cheb_step_t<float>(s, n, N, d.rowptr, d.col, d.valA32, d.dinvA32, d.R32, pf, 2, pf.Z[1], pf.Z[0],
                                  pf.Z[0], nullptr, nullptr);
      else
        launch_spmm2_f32(s, n, N, d.rowptr, d.col, d.valA32, d.P32, d.Q32, d.red, nullptr);
    } else {
      if (cheb)
        launch_cheb_step_t<double>(s, n, N, d.rowptr, d.col, d.valA, d.dinvA, d.R, pd, 2, pd.Z[1], pd.Z[0], pd.Z[0],
                                   nullptr, nullptr);
      else
        launch_spmm2(s, n, N, d.rowptr, d.col, d.valA, d.P, d.Q, d.red, nullptr);
    }
  };
  hipError_t err = hipSuccess;
  if (c->opt.use_graphs && c->cap_stream && reps <= 4096) {
    // the launches back to back in one graph, as the solver replays its chunks
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipStream_t keep = s;
    err = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
      s = c->cap_stream;
      for (int k = 0; k < reps; ++k) one();
      s = keep;
      err = hipStreamEndCapture(c->cap_stream, &g);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (err == hipSuccess) err = hipGraphLaunch(ge, s);  // warm-up replay
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = hipGraphLaunch(ge, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (ge) (void)hipGraphExecDestroy(ge);
  } else {
    err = hipEventRecord(e0, s);
    for (int k = 0; k < reps && err == hipSuccess; ++k) {
      one();
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
  }
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_fail(c, err, "mlc_time_kernel");
  *avg_us = 1e3 * (double)ms / reps;
  return MLC_OK;
}

mlc_status mlc_set_guess(mlc_ctx* c, const mlc_nn* nn) {
  if (!c) return MLC_ERR_ARG;
  if (nn && !nn_device(nn)) return fail(c, MLC_ERR_STATE, "network not bound or without parameters");
  c->nn = nn;
  return MLC_OK;
}

mlc_status mlc_set_sample_sink(mlc_ctx* c, float* x, float* t, int64_t capacity, int32_t stride) {
  if (!c || capacity < 0) return MLC_ERR_ARG;
  if (capacity > 0 && (!x || !t || stride < 1)) return fail(c, MLC_ERR_ARG, "sink needs x, t and stride >= 1");
  c->sink_x = capacity > 0 ? x : nullptr;
  c->sink_t = capacity > 0 ? t : nullptr;
  c->sink_cap = capacity;
  c->sink_stride = capacity > 0 ? stride : 1;
  c->sink_count = 0;
  return MLC_OK;
}

mlc_status mlc_sample_count(const mlc_ctx* c, int64_t* rows) {
  if (!c || !rows) return MLC_ERR_ARG;
  *rows = c->sink_count;
  return MLC_OK;
}

const char* mlc_status_string(mlc_status s) {
  switch (s) {
    case MLC_OK: return "ok";
    case MLC_ERR_ARG: return "invalid argument";
    case MLC_ERR_MESH: return "invalid mesh";
    case MLC_ERR_NOT_NESTED: return "meshes are not nested";
    case MLC_ERR_WORKSPACE: return "workspace missing or too small";
    case MLC_ERR_HIP: return "HIP runtime error";
    case MLC_ERR_NOT_CONVERGED: return "CG not converged";
    case MLC_ERR_BREAKDOWN: return "CG breakdown";
    case MLC_ERR_NONFINITE: return "non-finite value";
    case MLC_ERR_STATE: return "call order";
    case MLC_WARN_INNER_MAXIT: return "inner iteration stopped at inner_maxit";
  }
  return "unknown status";
}

const char* mlc_last_error(const mlc_ctx* c) { return c ? c->err.c_str() : "null context"; }

void mlc_destroy(mlc_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& gk : c->cg_graph)
    for (hipGraphExec_t g : gk)
      if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  delete c;
}

}  // extern "C"
