// The phases of one correction step (Algorithm 1 steps 5-7), shared by the
// single-system step and the batched step. Not part of the ABI.
#pragma once

#include "inner.h"
#include "mlc_internal.h"

namespace mlc {

struct CgRes {
  int iters = 0;
  int64_t iters_sum = 0;
  double relres = 0.0;
  bool converged = false;
  bool breakdown = false;
};

struct StepRun {
  mlc_ctx* c;
  mlc_step_report r;
  // 0-1 fine stage, 2-3 reconstruction, 4-5 step-5 solve, 6-7 Hartree solve
  // (4-7 recorded by the single-system step only: solve_timed)
  hipEvent_t ev[8] = {};
  bool solve_timed = false;
  double mom[16] = {};
  double colv[2 * MLC_MAX_ORBITALS] = {};
  double sigma = 0.0;
  CgRes cr, pr;  // step-5 and Hartree solves
  InnerOut io;
  mlc_status ist = MLC_OK;
  std::vector<double> cin, tail;
  bool guess = false;                     // learned start evaluated this step
  bool defer_copies = false;              // the caller enqueues the *_copy phases itself
  double gsel[4 * MLC_MAX_ORBITALS] = {};  // its per-column choices and residuals
  explicit StepRun(mlc_ctx* ctx);
  ~StepRun();
  StepRun(const StepRun&) = delete;
  StepRun& operator=(const StepRun&) = delete;
};

// Enqueue on c->stream; phase_fields and phase_gram end with device-to-host
// copies that the caller must synchronise before phase_operators and
// phase_inner; phase_recon likewise before phase_finish. Host-to-device
// copies come first in their phases (phase_operators, phase_recon).
mlc_status phase_fields(StepRun& S);
mlc_status phase_operators(StepRun& S);
mlc_status phase_after_solve(StepRun& S);
mlc_status phase_gram_fixed(StepRun& S, hipStream_t s, double* red);
mlc_status phase_gram(StepRun& S);
mlc_status phase_inner(StepRun& S);
mlc_status phase_recon(StepRun& S);
mlc_status phase_finish(StepRun& S, mlc_step_report* rep);
// The device-to-host copies that end phase_fields, phase_gram and phase_recon;
// called by those phases unless defer_copies is set (a batch runs the phases
// of its systems on separate streams and copies after joining them).
mlc_status phase_fields_copy(StepRun& S);
mlc_status phase_gram_copy(StepRun& S);
mlc_status phase_recon_copy(StepRun& S);

}  // namespace mlc
