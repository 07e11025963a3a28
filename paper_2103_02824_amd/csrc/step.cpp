// One outer step of Algorithm 1 (steps 5-7): the fine stage on the GPU, the
// inner Hartree iteration on the host, and the reconstruction on the GPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "nn.h"
#include "phases.h"

namespace mlc {

static double box_diagonal(const mlc_ctx* c) {
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) d2 += (c->hi[k] - c->lo[k]) * (c->hi[k] - c->lo[k]);
  return std::sqrt(d2);
}

// Offsets into the packed small-block buffer (doubles).
struct SmallLayout {
  int64_t ptF, ptW, ptM, ptK, utF, utW, utM, utK, d, liftH, sc, mom, ovl, colv, total;
  SmallLayout(int64_t nH, int N) {
    int64_t hn = nH * N, nn = (int64_t)N * N;
    ptF = 0;
    ptW = hn;
    ptM = 2 * hn;
    ptK = 3 * hn;
    utF = 4 * hn;
    utW = utF + nn;
    utM = utW + nn;
    utK = utM + nn;
    d = utK + nn;
    liftH = d + nH;
    sc = liftH + nH;   // [0] zeta [1] w0.l [2] int rho [3] energy piece
    mom = sc + 8;      // 11 moments (+ min V_eff)
    ovl = mom + 16;    // N x N overlaps
    colv = ovl + nn;   // 2N per-column values
    total = colv + 2 * N;
  }
};

int64_t small_len(int64_t nH, int N) { return SmallLayout(nH, N).total; }

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) return hip_fail(c, e_, #x); \
  } while (0)

namespace {

// Exact correction over the nested coarse space, added to the preconditioner:
// z += P K_H^-1 P^T r (additive two-level preconditioner).
struct CoarsePC {
  const double* KHinv;
  int64_t nH;
  const int32_t* PTptr;
  const int32_t* PTidx;
  const double* PTw;
  const int32_t* Pk;
  const double* Pw;
  double* rH;
  double* eH;
  double* Z;        // z without the polynomial preconditioner
  double* rz_part;  // per-block r.z partials
};

template <typename T>
struct CgArgs {
  const T* val;
  const T* dinv;
  const T* B;
  T *X, *R, *P, *Q;
  double* scal;
  int32_t* flags;
  const double* mask;  // optional: column c may be active only if mask[active c] != 0
  const PolyPC<T>* pc = nullptr;  // Chebyshev polynomial preconditioner (null: Jacobi)
  const CoarsePC* cc = nullptr;  // additive coarse-space correction (one FP64 column only)
};

// The preconditioned residual of the iteration (or of the start, into P).
template <typename T>
void enqueue_precond(mlc_ctx* c, hipStream_t s, int64_t n, int N, const CgArgs<T>& a, const int32_t* flags,
                     bool start, const double** rz_part, const T** Zl) {
  auto& d = c->d;
  *rz_part = nullptr;
  *Zl = nullptr;
  if (a.pc) {
    launch_cheb_steps_t<T>(s, n, N, d.rowptr, d.col, a.val, a.dinv, a.R, *a.pc, start ? a.P : nullptr, flags);
    *rz_part = a.pc->rz_part;
    *Zl = start ? a.P : a.pc->Z[(a.pc->degree - 1) & 1];
  }
  if constexpr (std::is_same<T, double>::value) {
    if (a.cc) {
      const CoarsePC& cc = *a.cc;
      launch_restrict_chunks(s, n, cc.nH, 1, d, a.R, cc.rH, d.rpartH);
      launch_dense_mv(s, cc.nH, cc.KHinv, cc.rH, cc.eH);
      double* zout = start ? a.P : (a.pc ? const_cast<double*>(*Zl) : cc.Z);
      launch_zcoarse(s, n, a.dinv, a.R, a.pc ? *Zl : nullptr, cc.Pk, cc.Pw, cc.eH, zout, cc.rz_part);
      *rz_part = cc.rz_part;
      *Zl = zout;
    }
  }
}

// type-dispatched launchers
inline void L_spmm(hipStream_t s, int64_t n, int N, const int32_t* rp, const int32_t* ci, const double* v,
                   const double* X, double* Y, double* part, const int32_t* fl) {
  launch_spmm2(s, n, N, rp, ci, v, X, Y, part, fl);
}
inline void L_spmm(hipStream_t s, int64_t n, int N, const int32_t* rp, const int32_t* ci, const float* v,
                   const float* X, float* Y, double* part, const int32_t* fl) {
  launch_spmm2_f32(s, n, N, rp, ci, v, X, Y, part, fl);
}
inline void L_init(hipStream_t s, int64_t n, int N, const double* B, const double* AX, const double* dinv, double* R,
                   double* P, double* part) {
  launch_cg_init2(s, n, N, B, AX, dinv, R, P, part);
}
inline void L_init(hipStream_t s, int64_t n, int N, const float* B, const float* AX, const float* dinv, float* R,
                   float* P, double* part) {
  launch_cg_init2_f32(s, n, N, B, AX, dinv, R, P, part);
}
template <typename T>
mlc_status enqueue_iteration(mlc_ctx* c, hipStream_t s, int64_t n, int N, const CgArgs<T>& a, double rt2, int p,
                             hipEvent_t* ev = nullptr) {
  auto& d = c->d;
  double* red_pq = d.red;
  double* red_upd = d.red + c->nred / 2;
  double* sc_in = a.scal + (p ? 5 * N : 0);
  double* sc_out = a.scal + (p ? 0 : 5 * N);
  int32_t* fl_in = a.flags + (p ? 2 : 0);
  int32_t* fl_out = a.flags + (p ? 0 : 2);
  if (ev) HIPCHK(hipEventRecord(ev[0], s));
  L_spmm(s, n, N, d.rowptr, d.col, a.val, a.P, a.Q, red_pq, fl_in);
  if (ev) HIPCHK(hipEventRecord(ev[1], s));
  launch_cg_update_t<T>(s, n, N, a.dinv, a.X, a.R, a.P, a.Q, red_pq, sc_in, fl_in, red_upd, a.flags + 4, a.pc);
  const double* rz_part;
  const T* Zl;
  enqueue_precond<T>(c, s, n, N, a, fl_in, false, &rz_part, &Zl);
  launch_cg_direction_z<T>(s, n, N, a.dinv, a.R, a.P, red_upd, sc_in, fl_in, sc_out, fl_out, rt2, rz_part, Zl);
  return MLC_OK;
}

// Start of a solve: R = B - A X, P = M^-1 R (Jacobi, or the polynomial with
// its last step written into P), scalars and active flags.
template <typename T>
void enqueue_start(mlc_ctx* c, hipStream_t s, int64_t n, int N, const CgArgs<T>& a, double rt2) {
  auto& d = c->d;
  double* red_upd = d.red + c->nred / 2;
  L_spmm(s, n, N, d.rowptr, d.col, a.val, a.X, a.Q, nullptr, nullptr);
  launch_cg_init_t<T>(s, n, N, a.B, a.Q, a.dinv, a.R, a.P, red_upd, a.pc);
  const double* rz_part;
  const T* Zl;
  enqueue_precond<T>(c, s, n, N, a, nullptr, true, &rz_part, &Zl);
  launch_cg_start2(s, n, N, red_upd, rt2, a.mask, a.scal, a.flags, rz_part);
}

// Multi-column preconditioned CG, one independent recurrence per column;
// per-column scalars stay on the device; the host checks the number of
// active columns after every chunk of iterations (chunk_length). Chunks are
// replayed from captured HIP graphs (per solve kind and size); with
// timed = true they are launched eagerly and every SpMM launch is bracketed
// by HIP events. On exit the true residual is evaluated in T.
template <typename T>
mlc_status cg(mlc_ctx* c, int kind, int64_t n, int N, const CgArgs<T>& a, double rtol, int maxit, bool timed,
              double* spmm_ms, int64_t* n_spmm, CgRes* out) {
  hipStream_t s = c->stream;
  auto& d = c->d;
  const double rt2 = rtol * rtol;
  double* red_upd = d.red + c->nred / 2;
  HIPCHK(hipMemsetAsync(a.flags, 0, 8 * sizeof(int32_t), s));
  enqueue_start<T>(c, s, n, N, a, rt2);
  int it = 0;
  int32_t hf[8];
  const int every = 2 * ((std::max(1, c->opt.check_every) + 1) / 2);
  const bool graph = c->opt.use_graphs && !timed && c->cap_stream;
  const int pcdeg = (a.pc ? a.pc->degree : 0) + (a.cc ? 100 : 0);
  auto* graphs = c->cg_graph[kind];
  if (graph && (c->cg_graph_rt2[kind] != rt2 || c->cg_graph_pc[kind] != pcdeg)) {
    for (int g = 0; g < CHUNK_GRAPHS; ++g) {
      if (graphs[g]) HIPCHK(hipGraphExecDestroy(graphs[g]));
      graphs[g] = nullptr;
    }
    c->cg_graph_rt2[kind] = rt2;
    c->cg_graph_pc[kind] = pcdeg;
  }
  // every chunk size is captured at the first solve of a kind (a one-time
  // cost), so that later predicted chunks never wait for an instantiation
  if (graph && !graphs[0]) {
    for (int g = 0; g < CHUNK_GRAPHS; ++g) {
      hipGraph_t gr;
      HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < (2 << g); ++k) (void)enqueue_iteration<T>(c, c->cap_stream, n, N, a, rt2, k & 1);
      HIPCHK(hipStreamEndCapture(c->cap_stream, &gr));
      hipError_t e = hipGraphInstantiate(&graphs[g], gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) {
        for (int h = 0; h <= g; ++h) {
          if (graphs[h]) (void)hipGraphExecDestroy(graphs[h]);
          graphs[h] = nullptr;
        }
        return hip_fail(c, e, "hipGraphInstantiate");
      }
    }
  }
  auto launch_graph = [&](int g) -> mlc_status {
    HIPCHK(hipGraphLaunch(graphs[g], s));
    return MLC_OK;
  };
  int len = 0;
  for (int chunk = 0;; ++chunk) {
    HIPCHK(hipMemcpyAsync(hf, a.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (timed && c->ev_used > 0) {
      for (int k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
        *spmm_ms += ms;
      }
      c->ev_used = 0;
    }
    if (hf[4]) {
      out->breakdown = true;
      break;
    }
    if (hf[0] == 0) {
      out->converged = true;
      break;
    }
    if (it >= maxit) break;
    len = chunk_length(chunk, len, c->cg_pred[kind], every);
    if (graph) {
      mlc_status st = MLC_OK;
      for_chunk_graphs(len, [&](int g) {
        if (st == MLC_OK) st = launch_graph(g);
      });
      if (st != MLC_OK) return st;
    } else {
      for (int k = 0; k < len; ++k) {
        bool rec = timed && c->ev_used + 2 <= (int)c->ev_pool.size();
        mlc_status st = enqueue_iteration<T>(c, s, n, N, a, rt2, k & 1, rec ? &c->ev_pool[c->ev_used] : nullptr);
        if (st != MLC_OK) return st;
        if (rec) {
          c->ev_used += 2;
          ++*n_spmm;
        }
      }
    }
    it += len;
  }
  // per-column iteration counts, then the true residual ||B - A X|| / ||B||
  std::vector<double> hs(5 * N);
  HIPCHK(hipMemcpyAsync(hs.data(), a.scal, sizeof(double) * 5 * N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int itmax = 0;
  int64_t itsum = 0;
  for (int j = 0; j < N; ++j) {
    int ij = (int)hs[4 * N + j];
    itmax = std::max(itmax, ij);
    itsum += ij;
  }
  out->iters = itmax;
  out->iters_sum = itsum;
  if (out->converged) c->cg_pred[kind] = itmax;
  L_spmm(s, n, N, d.rowptr, d.col, a.val, a.X, a.Q, nullptr, nullptr);
  L_init(s, n, N, a.B, a.Q, a.dinv, a.R, a.P, red_upd);
  launch_cg_start(s, n, N, red_upd, 0.0, nullptr, a.scal, a.flags);
  HIPCHK(hipMemcpyAsync(hs.data(), a.scal, sizeof(double) * 5 * N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double mx = 0.0;
  for (int j = 0; j < N; ++j) {
    double bb = hs[2 * N + j];
    double rr = hs[1 * N + j];
    mx = std::max(mx, bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr));
  }
  out->relres = mx;
  if (!std::isfinite(mx)) return fail(c, MLC_ERR_NONFINITE, "non-finite CG residual");
  return MLC_OK;
}

// Step 5 with FP32 CG inside FP64 iterative refinement: the residual
// R = B - A X is formed in FP64, the correction D solves A D = R in FP32 (CG
// to ir_inner_rtol relative to ||R|| for the columns not yet converged in
// FP64), and X += D in FP64; until ||B - A X||_2 <= cg_rtol ||B||_2 per column.
mlc_status solve_ir(mlc_ctx* c, int64_t n, int N, bool timed, double* spmm_ms, int64_t* n_spmm, CgRes* out,
                    int* outer_iters) {
  hipStream_t s = c->stream;
  auto& d = c->d;
  double* red_upd = d.red + c->nred / 2;
  const double rt2 = c->opt.cg_rtol * c->opt.cg_rtol;
  int total = 0;
  int64_t total_sum = 0;
  int outer = 0;
  int32_t hf[8];
  bool converged = false;
  for (; outer < c->opt.ir_max_outer; ++outer) {
    launch_spmm2(s, n, N, d.rowptr, d.col, d.valA, d.X, d.Q, nullptr, nullptr);
    launch_cg_init2(s, n, N, d.B, d.Q, d.dinvA, d.R, d.P, red_upd);
    launch_cg_start(s, n, N, red_upd, rt2, nullptr, d.scal, d.flags);
    HIPCHK(hipMemcpyAsync(hf, d.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hf[0] == 0) {
      converged = true;
      break;
    }
    launch_to_f32(s, n * N, d.R, d.B32);
    HIPCHK(hipMemsetAsync(d.X32, 0, sizeof(float) * n * N, s));
    float* Yf = reinterpret_cast<float*>(d.Y);
    PolyPC<float> pcF{d.lmax, c->opt.cheb_ratio, c->opt.cheb_degree, {Yf, Yf + n * N},
                      d.red + (int64_t)cg_max_blocks() * N};
    CgArgs<float> fa{d.valA32, d.dinvA32, d.B32, d.X32, d.R32, d.P32, d.Q32, d.scal32, d.flags32, d.scal,
                     c->opt.precond == MLC_PC_CHEBYSHEV ? &pcF : nullptr};
    CgRes ir;
    mlc_status st = cg<float>(c, 2, n, N, fa, c->opt.ir_inner_rtol, c->opt.cg_maxit, timed, spmm_ms, n_spmm, &ir);
    if (st != MLC_OK) return st;
    if (ir.breakdown) {
      out->breakdown = true;
      return MLC_OK;
    }
    launch_add_f32(s, n * N, d.X32, d.X);
    total += ir.iters;
    total_sum += ir.iters_sum;
  }
  out->converged = converged;
  out->iters = total;
  out->iters_sum = total_sum;
  // true FP64 residual
  launch_spmm2(s, n, N, d.rowptr, d.col, d.valA, d.X, d.Q, nullptr, nullptr);
  launch_cg_init2(s, n, N, d.B, d.Q, d.dinvA, d.R, d.P, red_upd);
  launch_cg_start(s, n, N, red_upd, 0.0, nullptr, d.scal, d.flags);
  std::vector<double> hs(5 * N);
  HIPCHK(hipMemcpyAsync(hs.data(), d.scal, sizeof(double) * 5 * N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double mx = 0.0;
  for (int j = 0; j < N; ++j) {
    double bb = hs[2 * N + j], rr = hs[N + j];
    mx = std::max(mx, bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr));
  }
  out->relres = mx;
  *outer_iters = outer;
  if (!std::isfinite(mx)) return fail(c, MLC_ERR_NONFINITE, "non-finite CG residual");
  return MLC_OK;
}

}  // namespace

// ---- phases of one correction step ---------------------------------------------
// The single-system step runs them in order with its own CG solves; a batch runs
// each phase for every system and replaces the two solves by batched launches.

StepRun::StepRun(mlc_ctx* ctx) : c(ctx) { std::memset(&r, 0, sizeof(r)); }
StepRun::~StepRun() {
  for (int k = 0; k < 8; ++k)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
}

// Density, XC and V_eff at the quadrature points; multipole moments and
// min V_eff copied to the host (the caller synchronises before phase_operators).
mlc_status phase_fields(StepRun& S) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  hipStream_t s = c->stream;
  SmallLayout L(c->nH, c->N);
  for (int k = 0; k < 8; ++k) HIPCHK(hipEventCreate(&S.ev[k]));
  HIPCHK(hipEventRecord(S.ev[0], s));
  if (c->order == 2)
    launch_qp_fields_p2(s, c->nt, d.tets, d.v2d, d.Phi, c->N, d.occ, d.w, d.vext, d.geo, d.qpx, c->xc, c->xalpha,
                        d.qtab, d.vxc, d.exc, d.veff, d.rho, d.red);
  else
    launch_qp_fields(s, c->nt, d.tets, d.v2d, d.Phi, c->N, d.occ, d.w, d.vext, d.geo, d.qpx, c->xc, c->xalpha, d.vxc,
                     d.exc, d.veff, d.rho, d.red);
  launch_reduce_rows(s, d.red, qp_blocks(c->nt), nmom(), 1, d.small + L.mom);
  return S.defer_copies ? MLC_OK : phase_fields_copy(S);
}

mlc_status phase_fields_copy(StepRun& S) {
  mlc_ctx* c = S.c;
  SmallLayout L(c->nH, c->N);
  HIPCHK(hipMemcpyAsync(S.mom, c->d.small + L.mom, sizeof(double) * nmom(), hipMemcpyDeviceToHost, c->stream));
  return MLC_OK;
}

// Boundary data g, the operators A + sigma M and A_fix, the right-hand sides
// B = (lambda_i + sigma) M phi_i and the initial iterate X = Phi (step 5).
mlc_status phase_operators(StepRun& S) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t n = c->n, nt = c->nt, nv = c->nv;
  const int N = c->N;
  SmallLayout L(c->nH, N);
  S.sigma = c->opt.shift ? c->opt.sigma0 - S.mom[nmom() - 1] : 0.0;
  c->last_sigma = S.sigma;
  for (int i = 0; i < N; ++i) S.colv[i] = c->lam[i] + S.sigma;
  HIPCHK(hipMemcpyAsync(d.colv, S.colv, sizeof(double) * N, hipMemcpyHostToDevice, s));
  // multipole Dirichlet data g (remark after Algorithm 3)
  HIPCHK(hipMemsetAsync(d.g, 0, sizeof(double) * nv, s));
  if (c->hartree && S.mom[0] > 0.0)
    launch_boundary_g(s, (int64_t)c->bverts.size(), d.bverts, d.xyz, d.small + L.mom, d.g);
  // V_ext + V_xc + g at the quadrature points (A_fix of the inner problems)
  const int64_t nnz = (int64_t)c->col.size();
  if (c->order == 2) {
    launch_field_p2(s, nt, d.tets, d.g, d.v2d, nullptr, d.vext, d.vxc, d.qtab, d.fld);
    launch_assemble2_p2(s, nt, n, nnz, d.geo, d.slot_ptr, d.slot_of, d.diag_slot, d.elem, 0.5, d.veff, S.sigma,
                        d.valA, d.dinvA, 0.5, d.fld, d.valF, d.qtab);
  } else {
    launch_field(s, nt, d.tets, d.g, d.v2d, nullptr, d.vext, d.vxc, d.fld);
    launch_assemble2(s, nt, n, nnz, d.geo, d.slot_ptr, d.slot_of, c->slot_ptr.back(), d.diag_slot, d.elem, 0.5,
                     d.veff, S.sigma, d.valA, d.dinvA, 0.5, d.fld, d.valF);
  }
  if (c->opt.precond == MLC_PC_CHEBYSHEV) {
    launch_gershgorin(s, n, d.rowptr, d.valA, d.dinvA, d.red, d.lmax);
    if (c->opt.cheb_lanczos)
      launch_lanczos_lmax(s, n, d.rowptr, d.col, d.valA, d.dinvA, c->opt.cheb_lanczos, 1.1, d.Y, d.red, d.lanc, d.lmax);
  }
  launch_spmm2(s, n, N, d.rowptr, d.col, d.valM, d.Phi, d.Q, nullptr, nullptr);
  launch_scale_cols_to(s, n, N, d.Q, d.colv, d.B);
  HIPCHK(hipMemcpyAsync(d.X, d.Phi, sizeof(double) * n * N, hipMemcpyDeviceToDevice, s));
  // learned start: direction delta = s NN(features), start = minimiser of the
  // energy 1/2 x.Ax - b.x over span{phi, delta} (phi where J does not drop)
  const NnDev* nd = c->nn ? nn_device(c->nn) : nullptr;
  if (c->nn && !nd) return fail(c, MLC_ERR_STATE, "the guess network lost its parameters or binding");
  const bool sink = c->sink_cap > 0 && c->sink_count < c->sink_cap;
  S.guess = nd != nullptr;
  if (nd || sink) {
    launch_spmm2(s, n, N, d.rowptr, d.col, d.valA, d.Phi, d.Q, nullptr, nullptr);
    launch_colmax_abs(s, n, N, d.Phi, d.red, d.gscale);
    launch_features(s, n, N, d.d2v, d.xyz, d.w, d.Phi, d.Q, d.B, d.dinvA, d.occ, d.RZ, c->n_nuclei, c->potential,
                    c->rc, c->omega, c->xc, c->xalpha, box_diagonal(c), d.gscale, d.F);
  }
  if (nd) {
    launch_nn_forward(s, *nd, d.F, n * N, 0, 1, n * N, d.Ynn);
    launch_guess_delta(s, n, N, d.gscale, d.Ynn, d.X);
    launch_spmm2(s, n, N, d.rowptr, d.col, d.valA, d.X, d.R, nullptr, nullptr);
    launch_guess_galerkin(s, n, N, d.Phi, d.Q, d.R, d.B, d.X, d.red, d.gdots, d.gsel);
  }
  if (c->opt.precision == MLC_PREC_FP32_IR) {
    launch_to_f32(s, nnz, d.valA, d.valA32);
    launch_to_f32(s, n, d.dinvA, d.dinvA32);
  }
  return MLC_OK;
}

// After step 5: M-normalise u_i; density of the u_i and the Hartree load
// vector (the caller then solves K w0 = b with zero boundary values).
mlc_status phase_after_solve(StepRun& S) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t n = c->n, nt = c->nt;
  const int N = c->N;
  S.r.cg_iters_max = S.cr.iters;
  S.r.cg_iters_sum = (int32_t)S.cr.iters_sum;
  S.r.cg_relres_max = S.cr.relres;
  S.r.spmm_rows = n;
  S.r.spmm_cols_sum = N;
  if (S.cr.breakdown) return fail(c, MLC_ERR_BREAKDOWN, "CG breakdown in the auxiliary problems");
  // training samples from this solve (before the M-normalisation)
  if (c->sink_cap > 0 && c->sink_count < c->sink_cap) {
    const int st = c->sink_stride;
    launch_collect(s, n, N, st, d.F, d.X, d.Phi, d.gscale, c->sink_count, c->sink_cap, c->sink_x, c->sink_t);
    c->sink_count = std::min<int64_t>(c->sink_cap, c->sink_count + ((n + st - 1) / st) * N);
  }
  launch_spmm2(s, n, N, d.rowptr, d.col, d.valM, d.X, d.Q, nullptr, nullptr);
  launch_coldot(s, n, N, d.X, d.Q, d.red);
  launch_reduce_cols(s, N, elem_blocks(n, N), d.red, d.colv + N);
  launch_normalize_cols(s, n, N, d.colv + N, d.X);
  if (c->hartree) {
    // start of the Hartree CG: the interior values of the current Hartree
    // potential w^l, the Hartree potential of rho^l (rho~ differs from it by
    // the step's change of the orbitals; the boundary data are zero inside)
    launch_gather_nodal(s, n, d.d2v, d.w, d.w0);
    if (c->order == 2) {
      launch_qp_density_p2(s, nt, d.tets, d.v2d, d.X, N, d.occ, d.qtab, d.rhot);
      launch_load_p2(s, n, nt, d.adj_ptr, d.adj_tet, d.adj_loc, d.tets, d.geo, d.rhot, 4.0 * 3.14159265358979323846,
                     d.g, d.v2d, d.qtab, d.elem, d.pb, d.lvec);
    } else {
      launch_qp_density(s, nt, d.tets, d.v2d, d.X, N, d.occ, d.rhot);
      launch_load(s, n, nt, d.adj_ptr, d.adj_tet, d.adj_loc, d.tets, d.geo, d.rhot, 4.0 * 3.14159265358979323846,
                  d.g, d.v2d, d.elem, d.pb, d.lvec);
    }
  }
  return MLC_OK;
}

// Algorithm 3 step 1, the part that does not involve w0: the Gram blocks
// P^T O U and U^T O U of O = A_fix, M, K (eqs. Adef, bdef, betadef) and the
// per-orbital coarse-pattern integrals (eqs. Ah4def, rhsdef), on stream s
// with partials in red. It may run beside the Hartree solve: it reads U and
// the fixed operators and writes only its own blocks.
mlc_status phase_gram_fixed(StepRun& S, hipStream_t s, double* red) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  const int64_t n = c->n, nH = c->nH, cnt = c->cnt;
  const int N = c->N;
  SmallLayout L(nH, N);
  const double* vals[4] = {d.valF, d.valW, d.valM, d.valK};
  for (int o : {0, 2, 3}) {
    double* Yo = d.Y + (int64_t)o * n * N;
    launch_spmm2(s, n, N, d.rowptr, d.col, vals[o], d.X, Yo, nullptr, nullptr);
    launch_restrict_chunks(s, n, nH, N, d, Yo, d.small + L.ptF + (int64_t)o * nH * N);
    launch_gram(s, n, N, d.X, Yo, red);
    launch_reduce_cols(s, N * N, gram_blocks(n), red, d.small + L.utF + (int64_t)o * N * N);
  }
  if (c->order == 2)
    launch_coarse_orb_p2(s, cnt, c->nt, d.cgrp_ptr, d.cgrp_dof, d.chat, d.X, N, d.qtab, d.cel_orb);
  else
    launch_coarse_orb(s, cnt, c->nt, d.cgrp_ptr, d.cgrp_dof, d.chat, d.X, N, d.cel_orb);
  if (d.cel_pairs) launch_coarse_pairs(s, cnt, c->nt, d.cgrp_ptr, d.cgrp_dof, d.chat, d.X, N, d.pair_jl, N * (N + 1) / 2,
                                       d.cel_pairs);
  HIPCHK(hipGetLastError());
  return MLC_OK;
}

// Step 6 continued and Algorithm 3 step 1 (after phase_gram_fixed): M_{w0},
// its Gram blocks, the Hartree pieces and the coarse-pattern integrals of the
// fixed operators and of M_{w0}, copied to the host (the caller synchronises
// before phase_inner).
mlc_status phase_gram(StepRun& S) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t n = c->n, nt = c->nt, nH = c->nH, cnt = c->cnt;
  const int N = c->N;
  SmallLayout L(nH, N);
  const int64_t nnz = (int64_t)c->col.size();
  if (c->hartree) {
    if (S.pr.breakdown) return fail(c, MLC_ERR_BREAKDOWN, "CG breakdown in the Hartree problem");
    if (c->order == 2) {
      launch_field_p2(s, nt, d.tets, nullptr, d.v2d, d.w0, nullptr, nullptr, d.qtab, d.fld2);
      launch_assemble2_p2(s, nt, n, nnz, d.geo, d.slot_ptr, d.slot_of, d.diag_slot, d.elem, 0.0, d.fld2, 0.0,
                          d.valW, nullptr, 0.0, nullptr, nullptr, d.qtab);
    } else {
      launch_field(s, nt, d.tets, nullptr, d.v2d, d.w0, nullptr, nullptr, d.fld2);
      launch_assemble2(s, nt, n, nnz, d.geo, d.slot_ptr, d.slot_of, c->slot_ptr.back(), d.diag_slot, d.elem, 0.0,
                       d.fld2, 0.0, d.valW, nullptr, 0.0, nullptr, nullptr);
    }
  } else {
    HIPCHK(hipMemsetAsync(d.w0, 0, sizeof(double) * n, s));
    HIPCHK(hipMemsetAsync(d.lvec, 0, sizeof(double) * n, s));
    HIPCHK(hipMemsetAsync(d.fld2, 0, sizeof(double) * c->nq * nt, s));
    HIPCHK(hipMemsetAsync(d.valW, 0, sizeof(double) * nnz, s));
  }
  S.r.poisson_iters = S.pr.iters;
  S.r.poisson_relres = S.pr.relres;
  {
    double* Yo = d.Y + (int64_t)n * N;
    launch_spmm2(s, n, N, d.rowptr, d.col, d.valW, d.X, Yo, nullptr, nullptr);
    launch_restrict_chunks(s, n, nH, N, d, Yo, d.small + L.ptF + (int64_t)nH * N);
    launch_gram(s, n, N, d.X, Yo, d.red);
    launch_reduce_cols(s, N * N, gram_blocks(n), d.red, d.small + L.utF + (int64_t)N * N);
  }
  HIPCHK(hipMemsetAsync(d.small + L.d, 0, sizeof(double) * (2 * nH + 8), s));
  if (c->hartree) {
    launch_spmm2(s, n, 1, d.rowptr, d.col, d.valK, d.w0, d.pq, nullptr, nullptr);
    launch_restrict_chunks(s, n, nH, 1, d, d.pq, d.small + L.d);
    launch_restrict_chunks(s, n, nH, 1, d, d.lvec, d.small + L.liftH);
    launch_coldot(s, n, 1, d.w0, d.pq, d.red);
    launch_reduce_cols(s, 1, elem_blocks(n, 1), d.red, d.small + L.sc + 0);
    launch_coldot(s, n, 1, d.w0, d.lvec, d.red);
    launch_reduce_cols(s, 1, elem_blocks(n, 1), d.red, d.small + L.sc + 1);
  }
  // coarse-pattern integrals (eqs. Adef, Ah4def, rhsdef, FG)
  if (c->order == 2)
    launch_coarse_ops_p2(s, cnt, nt, d.cgrp_ptr, d.cgrp_tet, d.chat, d.cgeo, d.fld, d.fld2, d.qtab, d.cel_ops);
  else
    launch_coarse_ops(s, cnt, nt, d.cgrp_ptr, d.cgrp_tet, d.chat, d.cgeo, d.fld, d.fld2, d.cel_ops);
  HIPCHK(hipEventRecord(S.ev[1], s));
  return S.defer_copies ? MLC_OK : phase_gram_copy(S);
}

mlc_status phase_gram_copy(StepRun& S) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t cnt = c->cnt;
  const int N = c->N;
  SmallLayout L(c->nH, N);
  c->last_small.resize(L.total);
  c->last_cel_ops.resize(40 * cnt);
  c->last_cel_orb.resize(14 * cnt * N);
  HIPCHK(hipMemcpyAsync(c->last_small.data(), d.small, sizeof(double) * L.total, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->last_cel_ops.data(), d.cel_ops, sizeof(double) * 40 * cnt, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->last_cel_orb.data(), d.cel_orb, sizeof(double) * 14 * cnt * N, hipMemcpyDeviceToHost, s));
  if (d.cel_pairs) {
    c->last_cel_pairs.resize(4 * cnt * (N * (N + 1) / 2));
    HIPCHK(hipMemcpyAsync(c->last_cel_pairs.data(), d.cel_pairs, sizeof(double) * c->last_cel_pairs.size(),
                          hipMemcpyDeviceToHost, s));
  }
  if (S.guess) HIPCHK(hipMemcpyAsync(S.gsel, d.gsel, sizeof(double) * 4 * N, hipMemcpyDeviceToHost, s));
  return MLC_OK;
}

// Algorithm 2 via Algorithm 3 step 2 on the host (FP64). Touches no device memory.
mlc_status phase_inner(StepRun& S) {
  mlc_ctx* c = S.c;
  const int64_t nH = c->nH;
  const int N = c->N;
  SmallLayout L(nH, N);
  FineBlocks fb;
  const double* h = c->last_small.data();
  fb.ptF.assign(h + L.ptF, h + L.ptF + nH * N);
  fb.ptW.assign(h + L.ptW, h + L.ptW + nH * N);
  fb.ptM.assign(h + L.ptM, h + L.ptM + nH * N);
  fb.ptK.assign(h + L.ptK, h + L.ptK + nH * N);
  fb.utF.assign(h + L.utF, h + L.utF + N * N);
  fb.utW.assign(h + L.utW, h + L.utW + N * N);
  fb.utM.assign(h + L.utM, h + L.utM + N * N);
  fb.utK.assign(h + L.utK, h + L.utK + N * N);
  fb.d.assign(h + L.d, h + L.d + nH);
  fb.liftH.assign(h + L.liftH, h + L.liftH + nH);
  fb.zeta = h[L.sc + 0];
  fb.liftT = h[L.sc + 1];
  fb.cel_ops = c->last_cel_ops;
  fb.cel_orb = c->last_cel_orb;
  if (c->opt.variant == MLC_VARIANT_JOINT) {
    fb.cel_pairs = c->last_cel_pairs;
    S.ist = inner_loop_joint(c, fb, S.io);
  } else {
    S.ist = inner_loop(c, fb, S.io);
  }
  if (S.ist < 0) return S.ist;
  // everything the reconstruction writes into the state is checked here, on
  // the host, before any device write: on failure the state stays as it was
  bool finite = std::isfinite(S.io.theta1);
  for (double v : S.io.lam) finite = finite && std::isfinite(v);
  for (double v : S.io.theta2) finite = finite && std::isfinite(v);
  for (double v : S.io.phiH) finite = finite && std::isfinite(v);
  for (double v : S.io.wH) finite = finite && std::isfinite(v);
  for (double v : S.io.D) finite = finite && std::isfinite(v);
  if (!finite) return fail(c, MLC_ERR_NONFINITE, "non-finite result of the augmented problems");
  S.r.inner_iters = S.io.iters;
  S.r.inner_last_diff = S.io.last_diff;
  S.r.t_inner_ms = S.io.ms;
  S.r.theta1 = S.io.theta1;
  S.r.sigma = S.sigma;
  return MLC_OK;
}

// Algorithm 3 step 3: phi_i = phi_{i,H} + theta2_i u_i, w = g + w_H + theta1 w0,
// the density, the energy pieces and the overlaps, copied to the host.
mlc_status phase_recon(StepRun& S) {
  mlc_ctx* c = S.c;
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t n = c->n, nt = c->nt, nH = c->nH, nv = c->nv;
  const int N = c->N;
  SmallLayout L(nH, N);
  const bool joint = c->opt.variant == MLC_VARIANT_JOINT;
  S.cin.assign(nH * N + nH + N + (joint ? N * N : 0), 0.0);
  std::copy(S.io.phiH.begin(), S.io.phiH.end(), S.cin.begin());
  std::copy(S.io.wH.begin(), S.io.wH.end(), S.cin.begin() + nH * N);
  std::copy(S.io.theta2.begin(), S.io.theta2.end(), S.cin.begin() + nH * N + nH);
  if (joint) std::copy(S.io.D.begin(), S.io.D.end(), S.cin.begin() + nH * N + nH + N);
  HIPCHK(hipMemcpyAsync(d.coarse_in, S.cin.data(), sizeof(double) * S.cin.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(S.ev[2], s));
  if (joint)
    launch_reconstruct_joint(s, n, N, d.Pk, d.Pw, d.coarse_in, d.coarse_in + nH * N + nH + N, d.X, d.Phi);
  else
    launch_reconstruct(s, n, N, d.Pk, d.Pw, d.coarse_in, d.coarse_in + nH * N + nH, d.X, d.Phi);
  launch_hartree_nodal(s, nv, d.v2d, d.Pk, d.Pw, d.coarse_in + nH * N, S.io.theta1, d.w0, d.g, d.w);
  launch_rho_nodal(s, nv, d.v2d, d.Phi, N, d.occ, d.rho_nodal);
  if (c->order == 2)
    launch_energy_p2(s, nt, d.tets, d.v2d, d.Phi, N, d.occ, d.w, d.vxc, d.geo, c->xc, c->xalpha, d.qtab, d.red);
  else
    launch_energy(s, nt, d.tets, d.v2d, d.Phi, N, d.occ, d.w, d.vxc, d.geo, c->xc, c->xalpha, d.red);
  launch_reduce_rows(s, d.red, qp_blocks(nt), 2, 0, d.small + L.sc + 2);
  launch_spmm2(s, n, N, d.rowptr, d.col, d.valM, d.Phi, d.Q, nullptr, nullptr);
  launch_gram(s, n, N, d.Phi, d.Q, d.red);
  launch_reduce_cols(s, N * N, gram_blocks(n), d.red, d.small + L.ovl);
  HIPCHK(hipEventRecord(S.ev[3], s));
  return S.defer_copies ? MLC_OK : phase_recon_copy(S);
}

mlc_status phase_recon_copy(StepRun& S) {
  mlc_ctx* c = S.c;
  SmallLayout L(c->nH, c->N);
  S.tail.assign(L.total - L.sc, 0.0);
  HIPCHK(hipMemcpyAsync(S.tail.data(), c->d.small + L.sc, sizeof(double) * S.tail.size(), hipMemcpyDeviceToHost,
                        c->stream));
  return MLC_OK;
}

// After the caller synchronised: timings, energy, overlaps, state update.
mlc_status phase_finish(StepRun& S, mlc_step_report* rep) {
  mlc_ctx* c = S.c;
  const int N = c->N;
  SmallLayout L(c->nH, N);
  std::copy(S.tail.begin(), S.tail.end(), c->last_small.begin() + L.sc);
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, S.ev[0], S.ev[1]));
  S.r.t_fine_ms = ms;
  HIPCHK(hipEventElapsedTime(&ms, S.ev[2], S.ev[3]));
  S.r.t_recon_ms = ms;
  if (S.solve_timed) {
    HIPCHK(hipEventElapsedTime(&ms, S.ev[4], S.ev[5]));
    S.r.t_solve_ms = ms;
    HIPCHK(hipEventElapsedTime(&ms, S.ev[6], S.ev[7]));
    S.r.t_poisson_ms = ms;
  }
  double E = S.tail[3];
  for (int i = 0; i < N; ++i) E += c->occ[i] * S.io.lam[i];
  S.r.energy = E;
  S.r.rho_integral = S.tail[2];
  double mo = 0.0;
  const double* ov = S.tail.data() + (L.ovl - L.sc);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      if (i != j) mo = std::max(mo, std::fabs(ov[i * N + j]));
  S.r.max_offdiag_overlap = mo;
  if (S.guess) {
    double worst = 0.0;
    int used = 0;
    for (int i = 0; i < N; ++i) {
      used += S.gsel[i] != 0.0;
      double l = S.gsel[3 * N + i], p = S.gsel[2 * N + i];
      worst = std::max(worst, p > 0.0 ? std::sqrt(l / p) : (l > 0.0 ? 1e300 : 1.0));
    }
    S.r.guess_learned_cols = used;
    S.r.guess_resid_ratio = worst;
  }
  for (int i = 0; i < N; ++i)
    if (!std::isfinite(S.io.lam[i])) return fail(c, MLC_ERR_NONFINITE, "non-finite eigenvalue");
  c->lam = S.io.lam;
  c->last_theta2 = S.io.theta2;
  c->last_phiH = S.io.phiH;
  c->last_wH = S.io.wH;
  c->last_theta1 = S.io.theta1;
  c->has_step = true;
  if (rep) *rep = S.r;
  if (!S.cr.converged) return fail(c, MLC_ERR_NOT_CONVERGED, "CG did not reach cg_rtol within cg_maxit");
  if (c->hartree && !S.pr.converged) return fail(c, MLC_ERR_NOT_CONVERGED, "Hartree CG did not converge");
  return S.ist;
}

#define PHASE(x)                      \
  do {                                \
    mlc_status st_ = (x);             \
    if (st_ != MLC_OK) return st_;    \
  } while (0)

mlc_status fine_stage_and_step(mlc_ctx* c, mlc_step_report* rep) {
  auto& d = c->d;
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const int N = c->N;
  const bool timed = c->opt.time_kernels != 0;
  StepRun S(c);
  PHASE(phase_fields(S));
  HIPCHK(hipStreamSynchronize(s));
  PHASE(phase_operators(S));
  // step 5: (A + sigma M) u_i = (lambda_i + sigma) M phi_i
  int outer_iters = 0;
  const bool cheb = c->opt.precond == MLC_PC_CHEBYSHEV;
  double* rz_part = d.red + (int64_t)cg_max_blocks() * N;
  PolyPC<double> pcA{d.lmax, c->opt.cheb_ratio, c->opt.cheb_degree, {d.Y, d.Y + n * N}, rz_part};
  HIPCHK(hipEventRecord(S.ev[4], s));
  if (c->opt.precision == MLC_PREC_FP32_IR) {
    PHASE(solve_ir(c, n, N, timed, &S.r.t_spmm_ms, &S.r.n_spmm, &S.cr, &outer_iters));
  } else {
    CgArgs<double> ca{d.valA, d.dinvA, d.B, d.X, d.R, d.P, d.Q, d.scal, d.flags, nullptr, cheb ? &pcA : nullptr};
    PHASE(cg<double>(c, 0, n, N, ca, c->opt.cg_rtol, c->opt.cg_maxit, timed, &S.r.t_spmm_ms, &S.r.n_spmm, &S.cr));
  }
  HIPCHK(hipEventRecord(S.ev[5], s));
  S.r.ir_outer = outer_iters;
  PHASE(phase_after_solve(S));
  // the w0-independent Gram blocks beside the Hartree solve (which is
  // latency-bound), on the side stream
  const bool side = c->hartree && c->side;
  if (side) {
    HIPCHK(hipEventRecord(c->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    PHASE(phase_gram_fixed(S, c->side, d.red2));
    HIPCHK(hipEventRecord(c->ev_join, c->side));
  } else {
    PHASE(phase_gram_fixed(S, s, d.red));
  }
  // step 6: Hartree direction w0, started from the interior values of w^l (phase_after_solve)
  HIPCHK(hipEventRecord(S.ev[6], s));
  if (c->hartree) {
    double dummy = 0.0;
    int64_t dn = 0;
    PolyPC<double> pcK{d.lmax + 1, hartree_ratio(c->opt), hartree_deg(c->opt), {d.Yh, d.Yh + n},
                       d.red + cg_max_blocks(), d.valK32};
    CoarsePC ccK{d.KHinv, c->nH, d.PTptr, d.PTidx, d.PTw, d.Pk, d.Pw, d.rH, d.eH, d.Yh + 3 * n,
                 d.red + cg_max_blocks()};
    CgArgs<double> pa{d.valK, d.dinvK, d.pb, d.w0, d.pr, d.pp, d.pq, d.scalP, d.flagsP, nullptr,
                      hartree_pc(c->opt) == MLC_PC_CHEBYSHEV ? &pcK : nullptr,
                      c->opt.hartree_coarse && d.KHinv ? &ccK : nullptr};
    PHASE(cg<double>(c, 1, n, 1, pa, c->opt.poisson_rtol, c->opt.cg_maxit, false, &dummy, &dn, &S.pr));
  }
  HIPCHK(hipEventRecord(S.ev[7], s));
  S.solve_timed = true;
  if (side) HIPCHK(hipStreamWaitEvent(s, c->ev_join, 0));
  PHASE(phase_gram(S));
  HIPCHK(hipStreamSynchronize(s));
  PHASE(phase_inner(S));
  PHASE(phase_recon(S));
  HIPCHK(hipStreamSynchronize(s));
  return phase_finish(S, rep);
}

}  // namespace mlc
