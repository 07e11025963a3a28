// Batches of independent systems: one correction step of every system, with
// the step-5 solves of all systems (and their Hartree solves) run as batched
// CG launches over a tile table, replayed from captured HIP graphs; the other
// phases run per system on the batch stream and the host inner iterations run
// in parallel over the systems.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "batch.h"
#include "phases.h"

using mlc::BCoarse;
using mlc::BProb;

struct mlc_batch {
  std::vector<mlc_ctx*> ctx;
  int K = 0;       // systems
  int KP = 0;      // systems with a Hartree problem
  int NB = 1;      // max orbitals over systems
  int prec = MLC_PREC_FP64;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<hipStream_t> sys_stream;  // per-system streams of the non-solver phases
  std::vector<hipEvent_t> sys_event;    // their join events (+ one fork event at the end)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  // shape (autotuned on the first step unless fixed)
  int TR = 0, G = 0, ntiles = 0, ntilesP = 0;
  bool tuned = false;
  int fixed_TR = 0, fixed_G = 0;
  double tune_ms = 0.0;
  int64_t max_tiles = 0;
  // device
  BProb<double>* dA = nullptr;   // step-5 problems, FP64
  BProb<float>* dA32 = nullptr;  // step-5 problems, FP32 (refinement)
  BProb<double>* dP = nullptr;   // Hartree problems
  int32_t* tile_prob = nullptr;  // step-5 tile table
  int32_t* tile_probP = nullptr; // Hartree tile table
  double* part = nullptr;
  double* part_rz = nullptr;     // r.z partials of the polynomial preconditioner
  BCoarse* dC = nullptr;         // Hartree coarse corrections (null: none)
  int32_t* crow_prob = nullptr;  // global coarse row -> Hartree problem
  int64_t ncrows = 0;
  double *bsA = nullptr, *bsA32 = nullptr, *bsP = nullptr;
  int32_t *flA = nullptr, *flA32 = nullptr, *flP = nullptr;
  // graphs: 0 step-5 FP64, 1 Hartree, 2 step-5 FP32
  // per kind and chunk size (2 << g iterations), with the tolerance they were
  // captured with and the last solve's iterations
  hipGraphExec_t graph[3][mlc::CHUNK_GRAPHS] = {};
  double graph_rt2[3] = {0, 0, 0};
  int pred[3] = {0, 0, 0};
  std::string err;
};

namespace mlc {
namespace {

constexpr int TR_MIN = 128;

mlc_status bfail(mlc_batch* b, mlc_status s, const std::string& m) {
  b->err = m;
  return s;
}

#define BCHK(x)                                                                         \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return bfail(b, MLC_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

int64_t tiles_for(const mlc_batch* b, int TR, bool hartree_only) {
  int64_t t = 0;
  for (mlc_ctx* c : b->ctx)
    if (!hartree_only || c->hartree) t += (c->n + TR - 1) / TR;
  return t;
}

struct Carve {
  char* p;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* r = p ? reinterpret_cast<T*>(p + off) : nullptr;
    off += count * sizeof(T);
    return r;
  }
};

size_t layout(mlc_batch* b, char* base) {
  Carve cv{base};
  const int K = b->K, KP = std::max(b->KP, 1), NB = b->NB;
  b->dA = cv.take<BProb<double>>(K);
  b->dA32 = cv.take<BProb<float>>(K);
  b->dP = cv.take<BProb<double>>(KP);
  b->tile_prob = cv.take<int32_t>(b->max_tiles);
  b->tile_probP = cv.take<int32_t>(b->max_tiles);
  b->part = cv.take<double>(b->max_tiles * 3 * NB);
  b->part_rz = cv.take<double>(b->max_tiles * NB);
  b->bsA = cv.take<double>((size_t)K * 8 * NB);
  b->bsA32 = cv.take<double>((size_t)K * 8 * NB);
  b->bsP = cv.take<double>((size_t)KP * 8 * NB);
  b->flA = cv.take<int32_t>(K + 1);
  b->flA32 = cv.take<int32_t>(K + 1);
  b->flP = cv.take<int32_t>(KP + 1);
  if (b->ncrows > 0) {
    b->dC = cv.take<BCoarse>(KP);
    b->crow_prob = cv.take<int32_t>(b->ncrows);
  }
  return cv.off + 256;
}

// Tile tables and descriptors for rows-per-tile TR.
mlc_status upload_shape(mlc_batch* b, int TR) {
  std::vector<int32_t> tp, tpP;
  std::vector<BProb<double>> hA, hP;
  std::vector<BProb<float>> hA32;
  int kp = 0;
  for (int s = 0; s < b->K; ++s) {
    mlc_ctx* c = b->ctx[s];
    auto& d = c->d;
    int nt = (int)((c->n + TR - 1) / TR);
    // polynomial preconditioner scratch: the context's Gram blocks, free during the solves
    const bool pc = c->opt.precond == MLC_PC_CHEBYSHEV;
    const int64_t nN = c->n * c->N;
    float* Yf = reinterpret_cast<float*>(d.Y);
    BProb<double> a{d.rowptr, d.col, d.valA, d.dinvA, d.B, d.X, d.R, d.P, d.Q,
                    d.Y, d.Y + nN, d.Y + 2 * nN, pc ? d.lmax : nullptr, c->n, c->N, (int32_t)tp.size(), nt, 0};
    BProb<float> f{d.rowptr, d.col, d.valA32, d.dinvA32, d.B32, d.X32, d.R32, d.P32, d.Q32,
                   Yf, Yf + nN, Yf + 2 * nN, pc ? d.lmax : nullptr, c->n, c->N, (int32_t)tp.size(), nt, 0};
    hA.push_back(a);
    hA32.push_back(f);
    for (int k = 0; k < nt; ++k) tp.push_back(s);
    if (c->hartree) {
      BProb<double> pp{d.rowptr, d.col, d.valK, d.dinvK, d.pb, d.w0, d.pr, d.pp, d.pq,
                       d.Yh, d.Yh + c->n, d.Yh + 2 * c->n,
                       hartree_pc(c->opt) == MLC_PC_CHEBYSHEV ? d.lmax + 1 : nullptr, c->n, 1, (int32_t)tpP.size(),
                       nt, 0};
      hP.push_back(pp);
      for (int k = 0; k < nt; ++k) tpP.push_back(kp);
      ++kp;
    }
  }
  if ((int64_t)tp.size() > b->max_tiles) return bfail(b, MLC_ERR_ARG, "tile table larger than reserved");
  hipStream_t s = b->stream;
  BCHK(hipMemcpyAsync(b->tile_prob, tp.data(), sizeof(int32_t) * tp.size(), hipMemcpyHostToDevice, s));
  BCHK(hipMemcpyAsync(b->dA, hA.data(), sizeof(BProb<double>) * hA.size(), hipMemcpyHostToDevice, s));
  BCHK(hipMemcpyAsync(b->dA32, hA32.data(), sizeof(BProb<float>) * hA32.size(), hipMemcpyHostToDevice, s));
  if (!hP.empty()) {
    BCHK(hipMemcpyAsync(b->tile_probP, tpP.data(), sizeof(int32_t) * tpP.size(), hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(b->dP, hP.data(), sizeof(BProb<double>) * hP.size(), hipMemcpyHostToDevice, s));
  }
  if (b->ncrows > 0) {
    std::vector<BCoarse> hC;
    std::vector<int32_t> crow;
    int kq = 0;
    for (mlc_ctx* c : b->ctx) {
      if (!c->hartree) continue;
      auto& d = c->d;
      hC.push_back(BCoarse{d.PTptr, d.PTidx, d.PTw, d.Pk, d.Pw, d.KHinv, d.rH, d.eH, d.Yh + 3 * c->n, c->nH,
                           (int32_t)crow.size(), 0});
      for (int64_t k = 0; k < c->nH; ++k) crow.push_back(kq);
      ++kq;
    }
    BCHK(hipMemcpyAsync(b->dC, hC.data(), sizeof(BCoarse) * hC.size(), hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(b->crow_prob, crow.data(), sizeof(int32_t) * crow.size(), hipMemcpyHostToDevice, s));
  }
  BCHK(hipStreamSynchronize(s));
  b->TR = TR;
  b->ntiles = (int)tp.size();
  b->ntilesP = (int)tpP.size();
  for (auto& gk : b->graph)
    for (auto& g : gk)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  return MLC_OK;
}

// Autotuner: time the step-5 SpMM (Q = A X over every system, the dominant
// launch) for each rows-per-tile x lanes-per-row candidate on the assembled
// operators of this batch and keep the fastest.
mlc_status autotune(mlc_batch* b) {
  auto t0 = std::chrono::steady_clock::now();
  static const int TRs[] = {128, 256, 512, 1024};
  static const int Gs[] = {2, 4, 8};
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  float best = 1e30f;
  int bTR = 256, bG = 4;
  mlc_status st = MLC_OK;
  for (int TR : TRs) {
    if (b->fixed_TR && TR != b->fixed_TR) continue;
    if ((st = upload_shape(b, TR)) != MLC_OK) break;
    for (int G : Gs) {
      if (b->fixed_G && G != b->fixed_G) continue;
      for (int w = 0; w < 2; ++w) {
        if (b->prec == MLC_PREC_FP32_IR)
          launch_b_spmm<float>(b->stream, b->dA32, b->tile_prob, b->ntiles, TR, G, b->NB, 1, b->part, b->flA32);
        else
          launch_b_spmm<double>(b->stream, b->dA, b->tile_prob, b->ntiles, TR, G, b->NB, 1, b->part, b->flA);
      }
      (void)hipEventRecord(e0, b->stream);
      const int reps = 5;
      for (int w = 0; w < reps; ++w) {
        if (b->prec == MLC_PREC_FP32_IR)
          launch_b_spmm<float>(b->stream, b->dA32, b->tile_prob, b->ntiles, TR, G, b->NB, 1, b->part, b->flA32);
        else
          launch_b_spmm<double>(b->stream, b->dA, b->tile_prob, b->ntiles, TR, G, b->NB, 1, b->part, b->flA);
      }
      (void)hipEventRecord(e1, b->stream);
      hipError_t e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = bfail(b, MLC_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
        break;
      }
      if (ms < best) {
        best = ms;
        bTR = TR;
        bG = G;
      }
    }
    if (st != MLC_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MLC_OK) return st;
  if ((st = upload_shape(b, bTR)) != MLC_OK) return st;
  b->G = bG;
  b->tuned = true;
  b->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return MLC_OK;
}

struct BRes {
  std::vector<int> iters;          // per problem: max over columns
  std::vector<int64_t> iters_sum;  // per problem: sum over columns
  std::vector<double> relres;      // per problem: max over columns of ||b - Ax|| / ||b||
  std::vector<char> done;          // per problem: every column converged
  bool breakdown = false;
};

// Batched CG from the current X of every problem; scalars in bs, counts in fl.
// Ns[p] = columns of problem p. Accumulates iteration counts into out.
BPoly batch_poly(const mlc_batch* b, int kind) {
  const mlc_options& o = b->ctx[0]->opt;
  if ((kind == 1 ? hartree_pc(o) : o.precond) != MLC_PC_CHEBYSHEV) return BPoly{0, 1.0, nullptr};
  if (kind == 1) return BPoly{hartree_deg(o), hartree_ratio(o), b->part_rz};
  return BPoly{o.cheb_degree, o.cheb_ratio, b->part_rz};
}

template <typename T>
mlc_status bcg(mlc_batch* b, int kind, const BProb<T>* probs, const int32_t* tile_prob, int ntiles,
               const std::vector<int>& Ns, double* bs, int32_t* fl, const double* mask_bs, double rtol, int maxit,
               BRes* out, const BCoarseSet* cs = nullptr) {
  BPoly poly = batch_poly(b, kind);
  if (cs && cs->coarse && !poly.rz_part) poly.rz_part = b->part_rz;  // the coarse term's r.z partials
  hipStream_t s = b->stream;
  const int K = (int)Ns.size();
  const double rt2 = rtol * rtol;
  const int NB = b->NB;
  BCHK(hipMemsetAsync(fl + K, 0, sizeof(int32_t), s));
  launch_b_start<T>(s, probs, tile_prob, ntiles, K, b->TR, b->G, NB, b->part, bs, mask_bs, fl, rt2, poly, cs);
  const int every = 2 * ((std::max(1, b->ctx[0]->opt.check_every) + 1) / 2);
  const bool graph = b->ctx[0]->opt.use_graphs != 0;
  auto* graphs = b->graph[kind];
  if (graph && b->graph_rt2[kind] != rt2) {
    for (int g = 0; g < mlc::CHUNK_GRAPHS; ++g) {
      if (graphs[g]) BCHK(hipGraphExecDestroy(graphs[g]));
      graphs[g] = nullptr;
    }
    b->graph_rt2[kind] = rt2;
  }
  // every chunk size is captured at the first solve of a kind and shape
  if (graph && !graphs[0]) {
    for (int g = 0; g < mlc::CHUNK_GRAPHS; ++g) {
      hipGraph_t gr;
      BCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < (2 << g); ++k)
        launch_b_iteration<T>(b->cap_stream, probs, tile_prob, ntiles, K, b->TR, b->G, NB, b->part, bs, fl, rt2,
                              poly, cs);
      BCHK(hipStreamEndCapture(b->cap_stream, &gr));
      hipError_t e = hipGraphInstantiate(&graphs[g], gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) {
        for (int h = 0; h <= g; ++h) {
          if (graphs[h]) (void)hipGraphExecDestroy(graphs[h]);
          graphs[h] = nullptr;
        }
        return bfail(b, MLC_ERR_HIP, "hipGraphInstantiate (batch)");
      }
    }
  }
  auto launch_graph = [&](int g) -> mlc_status {
    BCHK(hipGraphLaunch(graphs[g], s));
    return MLC_OK;
  };
  std::vector<int32_t> hf(K + 1);
  int it = 0, len = 0;
  for (int chunk = 0;; ++chunk) {
    BCHK(hipMemcpyAsync(hf.data(), fl, sizeof(int32_t) * (K + 1), hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    if (hf[K]) {
      out->breakdown = true;
      break;
    }
    bool any = false;
    for (int p = 0; p < K; ++p) any = any || hf[p] != 0;
    if (!any || it >= maxit) break;
    len = mlc::chunk_length(chunk, len, b->pred[kind], every);
    if (graph) {
      mlc_status st = MLC_OK;
      mlc::for_chunk_graphs(len, [&](int g) {
        if (st == MLC_OK) st = launch_graph(g);
      });
      if (st != MLC_OK) return st;
    } else {
      for (int k = 0; k < len; ++k)
        launch_b_iteration<T>(s, probs, tile_prob, ntiles, K, b->TR, b->G, NB, b->part, bs, fl, rt2, poly, cs);
    }
    it += len;
  }
  std::vector<double> hs((size_t)K * 8 * NB);
  BCHK(hipMemcpyAsync(hs.data(), bs, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, s));
  BCHK(hipStreamSynchronize(s));
  if (out->iters.empty()) {
    out->iters.assign(K, 0);
    out->iters_sum.assign(K, 0);
  }
  out->done.assign(K, 0);
  for (int p = 0; p < K; ++p) out->done[p] = hf[p] == 0 && !hf[K];
  int itmax = 0;
  for (int p = 0; p < K; ++p) {
    int mx = 0;
    for (int c = 0; c < Ns[p]; ++c) {
      int ic = (int)hs[((size_t)p * 8 + B_IT) * NB + c];
      mx = std::max(mx, ic);
      out->iters_sum[p] += ic;
    }
    out->iters[p] += mx;
    itmax = std::max(itmax, mx);
  }
  bool all = !hf[K];
  for (int p = 0; p < K; ++p) all = all && hf[p] == 0;
  if (all) b->pred[kind] = itmax;
  return MLC_OK;
}

// True FP64 residuals ||B - A X|| / ||B|| per problem (max over columns) and
// the per-column activity for tolerance rtol (into bs, fl).
mlc_status residuals(mlc_batch* b, const BProb<double>* probs, const int32_t* tile_prob, int ntiles,
                     const std::vector<int>& Ns, double* bs, int32_t* fl, double rtol, std::vector<double>* rel,
                     std::vector<int>* active) {
  hipStream_t s = b->stream;
  const int K = (int)Ns.size(), NB = b->NB;
  launch_b_start<double>(s, probs, tile_prob, ntiles, K, b->TR, b->G, NB, b->part, bs, nullptr, fl, rtol * rtol,
                         BPoly{0, 1.0, nullptr});
  std::vector<double> hs((size_t)K * 8 * NB);
  std::vector<int32_t> hf(K);
  BCHK(hipMemcpyAsync(hs.data(), bs, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, s));
  BCHK(hipMemcpyAsync(hf.data(), fl, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s));
  BCHK(hipStreamSynchronize(s));
  rel->assign(K, 0.0);
  active->assign(K, 0);
  for (int p = 0; p < K; ++p) {
    for (int c = 0; c < Ns[p]; ++c) {
      double rr = hs[((size_t)p * 8 + B_RR) * NB + c], bb = hs[((size_t)p * 8 + B_BB) * NB + c];
      (*rel)[p] = std::max((*rel)[p], bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr));
    }
    (*active)[p] = hf[p];
  }
  return MLC_OK;
}

// Step 5 of every system: FP64 CG, or FP32 CG inside FP64 refinement. A
// system counts as converged as in the single-system path: by the CG
// recurrence (FP64), or by its true FP64 residual (refinement).
mlc_status solve_step5(mlc_batch* b, BRes* res, int* outer) {
  std::vector<int> Ns(b->K);
  for (int p = 0; p < b->K; ++p) Ns[p] = b->ctx[p]->N;
  const mlc_options& o = b->ctx[0]->opt;
  mlc_status st;
  std::vector<int> act;
  *outer = 0;
  if (b->prec == MLC_PREC_FP32_IR) {
    for (;;) {
      if ((st = residuals(b, b->dA, b->tile_prob, b->ntiles, Ns, b->bsA, b->flA, o.cg_rtol, &res->relres, &act)) !=
          MLC_OK)
        return st;
      int nact = 0;
      for (int v : act) nact += v;
      if (nact == 0 || *outer >= o.ir_max_outer) break;
      launch_b_ir(b->stream, b->dA, b->dA32, b->tile_prob, b->ntiles, b->TR, 0);
      if ((st = bcg<float>(b, 2, b->dA32, b->tile_prob, b->ntiles, Ns, b->bsA32, b->flA32, b->bsA, o.ir_inner_rtol,
                           o.cg_maxit, res)) != MLC_OK)
        return st;
      if (res->breakdown) break;
      launch_b_ir(b->stream, b->dA, b->dA32, b->tile_prob, b->ntiles, b->TR, 1);
      ++*outer;
    }
    if (res->iters.empty()) {
      res->iters.assign(b->K, 0);
      res->iters_sum.assign(b->K, 0);
    }
    res->done.assign(b->K, 0);
    for (int p = 0; p < b->K; ++p) res->done[p] = act[p] == 0 && !res->breakdown;
    return MLC_OK;
  }
  if ((st = bcg<double>(b, 0, b->dA, b->tile_prob, b->ntiles, Ns, b->bsA, b->flA, nullptr, o.cg_rtol, o.cg_maxit,
                        res)) != MLC_OK)
    return st;
  std::vector<char> done = res->done;
  if ((st = residuals(b, b->dA, b->tile_prob, b->ntiles, Ns, b->bsA, b->flA, 0.0, &res->relres, &act)) != MLC_OK)
    return st;
  res->done = done;
  return MLC_OK;
}

mlc_status solve_hartree(mlc_batch* b, BRes* res) {
  std::vector<int> Ns(b->KP, 1);
  const mlc_options& o = b->ctx[0]->opt;
  mlc_status st;
  BCoarseSet cs{b->dC, b->crow_prob, b->ncrows};
  if ((st = bcg<double>(b, 1, b->dP, b->tile_probP, b->ntilesP, Ns, b->bsP, b->flP, nullptr, o.poisson_rtol,
                        o.cg_maxit, res, b->dC ? &cs : nullptr)) != MLC_OK)
    return st;
  std::vector<char> done = res->done;
  std::vector<int> act;
  if ((st = residuals(b, b->dP, b->tile_probP, b->ntilesP, Ns, b->bsP, b->flP, 0.0, &res->relres, &act)) != MLC_OK)
    return st;
  res->done = done;
  return MLC_OK;
}

struct StreamRestore {
  mlc_batch* b;
  std::vector<hipStream_t> saved;
  explicit StreamRestore(mlc_batch* bb) : b(bb) {
    for (mlc_ctx* c : b->ctx) saved.push_back(c->stream);
  }
  ~StreamRestore() {
    for (size_t i = 0; i < saved.size(); ++i) b->ctx[i]->stream = saved[i];
  }
};

// The systems' phases run concurrently on their own streams, which start
// after the work already on the batch stream (fork) and which the batch
// stream waits for before it goes on (join).
mlc_status fork(mlc_batch* b) {
  hipEvent_t ev = b->sys_event.back();
  BCHK(hipEventRecord(ev, b->stream));
  for (int i = 0; i < b->K; ++i) {
    BCHK(hipStreamWaitEvent(b->sys_stream[i], ev, 0));
    b->ctx[i]->stream = b->sys_stream[i];
  }
  return MLC_OK;
}
mlc_status join(mlc_batch* b) {
  for (int i = 0; i < b->K; ++i) {
    BCHK(hipEventRecord(b->sys_event[i], b->sys_stream[i]));
    BCHK(hipStreamWaitEvent(b->stream, b->sys_event[i], 0));
    b->ctx[i]->stream = b->stream;
  }
  return MLC_OK;
}

mlc_status sys_fail(mlc_batch* b, int s, mlc_status st) {
  return bfail(b, st, "system " + std::to_string(s) + ": " + b->ctx[s]->err);
}

}  // namespace
}  // namespace mlc

using namespace mlc;

extern "C" {

mlc_status mlc_batch_create(mlc_ctx* const* ctxs, int32_t count, mlc_batch** out) {
  if (!out) return MLC_ERR_ARG;
  *out = nullptr;
  if (!ctxs || count < 1) return MLC_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return MLC_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return MLC_ERR_ARG;
  }
  std::unique_ptr<mlc_batch> b(new mlc_batch());
  b->ctx.assign(ctxs, ctxs + count);
  b->K = count;
  b->prec = ctxs[0]->opt.precision;
  for (mlc_ctx* c : b->ctx) {
    if (!c->bound) return MLC_ERR_STATE;
    if (c->opt.precision != b->prec) return MLC_ERR_ARG;
    if (c->opt.precond != ctxs[0]->opt.precond || hartree_pc(c->opt) != hartree_pc(ctxs[0]->opt) ||
        ((c->opt.precond == MLC_PC_CHEBYSHEV || hartree_pc(c->opt) == MLC_PC_CHEBYSHEV) &&
         (c->opt.cheb_degree != ctxs[0]->opt.cheb_degree || c->opt.cheb_ratio != ctxs[0]->opt.cheb_ratio ||
          hartree_deg(c->opt) != hartree_deg(ctxs[0]->opt) ||
          hartree_ratio(c->opt) != hartree_ratio(ctxs[0]->opt))))
      return MLC_ERR_ARG;
    if (c->opt.hartree_coarse != ctxs[0]->opt.hartree_coarse) return MLC_ERR_ARG;
    b->NB = std::max(b->NB, (int)c->N);
    b->KP += c->hartree ? 1 : 0;
    if (c->hartree && c->opt.hartree_coarse) b->ncrows += c->nH;
  }
  b->max_tiles = std::max<int64_t>(tiles_for(b.get(), TR_MIN, false), 1);
  b->ws_bytes = layout(b.get(), nullptr);
  *out = b.release();
  return MLC_OK;
}

mlc_status mlc_batch_workspace_bytes(const mlc_batch* b, size_t* bytes) {
  if (!b || !bytes) return MLC_ERR_ARG;
  *bytes = b->ws_bytes;
  return MLC_OK;
}

mlc_status mlc_batch_bind(mlc_batch* b, void* workspace, size_t bytes, void* stream) {
  if (!b || !workspace) return MLC_ERR_ARG;
  if (bytes < b->ws_bytes) return bfail(b, MLC_ERR_WORKSPACE, "batch workspace too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return bfail(b, MLC_ERR_WORKSPACE, "batch workspace must be 256-byte aligned");
  for (auto& gk : b->graph)
    for (auto& g : gk)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  if (!b->cap_stream) BCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  while ((int)b->sys_stream.size() < b->K) {
    hipStream_t st;
    BCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    b->sys_stream.push_back(st);
  }
  while ((int)b->sys_event.size() < b->K + 1) {
    hipEvent_t ev;
    BCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->sys_event.push_back(ev);
  }
  b->ws = static_cast<char*>(workspace);
  b->stream = static_cast<hipStream_t>(stream);
  layout(b, b->ws);
  b->bound = true;
  b->tuned = false;
  return MLC_OK;
}

mlc_status mlc_batch_set_shape(mlc_batch* b, int32_t tile_rows, int32_t lanes) {
  if (!b) return MLC_ERR_ARG;
  if (tile_rows != 0 && tile_rows != 128 && tile_rows != 256 && tile_rows != 512 && tile_rows != 1024)
    return bfail(b, MLC_ERR_ARG, "tile_rows must be 0 (autotune), 128, 256, 512 or 1024");
  if (lanes != 0 && lanes != 2 && lanes != 4 && lanes != 8)
    return bfail(b, MLC_ERR_ARG, "lanes must be 0 (autotune), 2, 4 or 8");
  b->fixed_TR = tile_rows;
  b->fixed_G = lanes;
  b->tuned = false;
  return MLC_OK;
}

mlc_status mlc_batch_step(mlc_batch* b, mlc_step_report* reports, mlc_batch_report* br) {
  if (!b) return MLC_ERR_ARG;
  if (!b->bound) return bfail(b, MLC_ERR_STATE, "batch not bound");
  for (int s = 0; s < b->K; ++s) {
    mlc_ctx* c = b->ctx[s];
    if (!c->bound || !c->has_state) return bfail(b, MLC_ERR_STATE, "system " + std::to_string(s) + " has no state");
    if (c->opt.precision != b->prec) return bfail(b, MLC_ERR_ARG, "precision changed since mlc_batch_create");
  }
  StreamRestore restore(b);
  for (mlc_ctx* c : b->ctx) c->stream = b->stream;
  hipStream_t s = b->stream;
  const int K = b->K;
  std::vector<std::unique_ptr<StepRun>> runs;
  for (int i = 0; i < K; ++i) {
    runs.emplace_back(new StepRun(b->ctx[i]));
    runs.back()->defer_copies = true;
  }
  hipEvent_t ev[8];
  for (auto& e : ev) e = nullptr;
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int k = 0; k < 8; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    }
  } guard{ev};
  for (auto& e : ev) BCHK(hipEventCreate(&e));
  mlc_status st;
  BCHK(hipEventRecord(ev[0], s));
  if ((st = fork(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_fields(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  if ((st = join(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_fields_copy(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  BCHK(hipStreamSynchronize(s));
  if ((st = fork(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_operators(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  if ((st = join(b)) != MLC_OK) return st;
  if (!b->tuned) {
    BCHK(hipStreamSynchronize(s));
    BCHK(hipEventRecord(ev[0], s));  // the tuning is reported on its own
    if ((st = autotune(b)) != MLC_OK) return st;
  }
  BCHK(hipEventRecord(ev[1], s));
  BRes r5;
  int outer = 0;
  if ((st = solve_step5(b, &r5, &outer)) != MLC_OK) return st;
  BCHK(hipEventRecord(ev[2], s));
  for (int i = 0; i < K; ++i) {
    CgRes& cr = runs[i]->cr;
    cr.iters = r5.iters.empty() ? 0 : r5.iters[i];
    cr.iters_sum = r5.iters_sum.empty() ? 0 : r5.iters_sum[i];
    cr.relres = r5.relres[i];
    cr.breakdown = r5.breakdown;
    cr.converged = r5.done[i] != 0;
    runs[i]->r.ir_outer = outer;
  }
  if ((st = fork(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_after_solve(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  if ((st = join(b)) != MLC_OK) return st;
  BCHK(hipEventRecord(ev[3], s));
  // the w0-independent Gram blocks on the systems' streams, beside the
  // batched Hartree solve on the batch stream
  if ((st = fork(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_gram_fixed(*runs[i], b->sys_stream[i], b->ctx[i]->d.red)) != MLC_OK) return sys_fail(b, i, st);
  BRes rp;
  if (b->KP > 0) {
    if ((st = solve_hartree(b, &rp)) != MLC_OK) return st;
  }
  BCHK(hipEventRecord(ev[4], s));
  if ((st = join(b)) != MLC_OK) return st;
  int kp = 0;
  for (int i = 0; i < K; ++i) {
    if (b->ctx[i]->hartree) {
      CgRes& pr = runs[i]->pr;
      pr.iters = rp.iters[kp];
      pr.iters_sum = rp.iters_sum[kp];
      pr.relres = rp.relres[kp];
      pr.breakdown = rp.breakdown;
      pr.converged = rp.done[kp] != 0;
      ++kp;
    }
  }
  if ((st = fork(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_gram(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  if ((st = join(b)) != MLC_OK) return st;
  BCHK(hipEventRecord(ev[5], s));
  for (int i = 0; i < K; ++i)
    if ((st = phase_gram_copy(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  BCHK(hipStreamSynchronize(s));
  auto ti0 = std::chrono::steady_clock::now();
  std::vector<mlc_status> ist(K, MLC_OK);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < K; ++i) ist[i] = phase_inner(*runs[i]);
  double t_inner = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ti0).count();
  for (int i = 0; i < K; ++i)
    if (ist[i] < 0) return sys_fail(b, i, ist[i]);
  BCHK(hipEventRecord(ev[6], s));
  if ((st = fork(b)) != MLC_OK) return st;
  for (int i = 0; i < K; ++i)
    if ((st = phase_recon(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  if ((st = join(b)) != MLC_OK) return st;
  BCHK(hipEventRecord(ev[7], s));
  for (int i = 0; i < K; ++i)
    if ((st = phase_recon_copy(*runs[i])) != MLC_OK) return sys_fail(b, i, st);
  BCHK(hipStreamSynchronize(s));
  // every system's device state was rewritten by its reconstruction, so every
  // system's host state (eigenvalues, coarse coefficients) is brought up to
  // date before an error is returned; the first failing system is reported
  mlc_status worst = MLC_OK, first_err = MLC_OK;
  int first_bad = -1;
  for (int i = 0; i < K; ++i) {
    st = phase_finish(*runs[i], reports ? &reports[i] : nullptr);
    if (st < 0 && first_bad < 0) {
      first_bad = i;
      first_err = st;
    }
    if (st > 0) worst = st;
  }
  if (first_bad >= 0) return sys_fail(b, first_bad, first_err);
  if (br) {
    std::memset(br, 0, sizeof(*br));
    br->n_systems = K;
    br->tile_rows = b->TR;
    br->spmm_lanes = b->G;
    br->n_tiles = b->ntiles;
    int mx = 0, mp = 0;
    for (int v : r5.iters) mx = std::max(mx, v);
    for (int v : rp.iters) mp = std::max(mp, v);
    br->cg_iters = mx;
    br->poisson_iters = mp;
    br->ir_outer = outer;
    for (mlc_ctx* c : b->ctx) br->dof_orbitals += c->n * c->N;
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, ev[0], ev[5]));
    br->t_gpu_ms = ms;
    BCHK(hipEventElapsedTime(&ms, ev[1], ev[2]));
    br->t_solve_ms = ms;
    BCHK(hipEventElapsedTime(&ms, ev[3], ev[4]));
    br->t_poisson_ms = ms;
    BCHK(hipEventElapsedTime(&ms, ev[6], ev[7]));
    br->t_recon_ms = ms;
    br->t_inner_ms = t_inner;
    br->t_tune_ms = b->tune_ms;
  }
  b->tune_ms = 0.0;
  return worst;
}

const char* mlc_batch_last_error(const mlc_batch* b) { return b ? b->err.c_str() : "null batch"; }

void mlc_batch_destroy(mlc_batch* b) {
  if (!b) return;
  for (auto& gk : b->graph)
    for (hipGraphExec_t g : gk)
      if (g) (void)hipGraphExecDestroy(g);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (hipStream_t st : b->sys_stream) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->sys_event) (void)hipEventDestroy(ev);
  delete b;
}

}  // extern "C"
