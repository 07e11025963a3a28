"""Benchmark of the fine-mesh correction step on one MI355X.

Workload (default): the 40-atom seeded cluster (positions uniform in [-8,8]^3
with separation >= 1.8, Z in {1..4}, smoothed Coulomb rc = 0.5, box
[-25,25]^3), a graded P1 mesh of 2.0e6 DoF, N = ceil(sum Z / 2) = 52
orbitals, LDA; step 5 in FP32 CG inside FP64 iterative refinement to 1e-9,
Chebyshev-preconditioned, the Hartree CG in FP64 with the coarse-space
correction. Synthetic seeded inputs (no datasets).

A step is one outer iteration of Algorithm 1 (steps 5-7). On the 40-atom
workload every timed step is the first outer step from the interpolated
coarse Kohn-Sham state (Algorithm 1 steps 1 and 4), set on the device before
each step: its 12^3 coarse space cannot separate 52 orbitals, so that its
outer iteration drifts, and the reset keeps every timed step on the same
physical input. On the smaller workloads the timed steps continue the outer
iteration after the warm-up steps. The metric counts
DoF x orbitals per second of the fine-mesh stage: the GPU time from the
density/XC evaluation through the Gram blocks and coarse-pattern integrals,
plus the reconstruction, measured with HIP events on the library's stream.
The host inner Hartree iteration (small augmented problems) runs to
convergence and is timed and reported separately. The plain FP64 GPU path
(FP64 Jacobi-PCG, no coarse correction) is timed on the same input state for
the speed-up against it (vs_plain_fp64).

After the timed steps the library replays each solver kernel back to back
between two HIP events on its own stream (mlc_time_kernel): the CG SpMM and,
with the polynomial preconditioner, the fused Chebyshev step, for step 5 and
for the Hartree problem. The dominant kernel is the one with the largest time
per step (mean launch time x launches per step); its algorithmic bytes per
launch over its mean duration give the roofline fraction. The measured HBM
traffic per launch comes from the committed counter summary in profiles/ and
is reported only while the kernel source matches it.

The step's result is checked (sorted eigenvalues, electron count, the inner
loop's convergence, the largest orbital overlap) and reported under
"physics"; an invalid result ends the run with exit status 3 after the JSON
line.

cpu_baseline: the CPU checker's Jacobi-PCG, timed on a bounded sample of the
workload (see cpu_baseline_pcg_rate; the smaller workloads time one whole
fine stage of the checker, see cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
_HPC = {"same": -1, "jacobi": 0, "chebyshev": 1}  # options.hartree_precond


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_system(workload, seed, order=1):
    from inputs.systems import c1_hydrogen, c2_cluster, c3_cluster
    if workload == "c1":
        return c1_hydrogen()
    if workload == "c2":
        return c2_cluster(seed)
    if workload == "c3":
        return c3_cluster(seed, order=order, progress=lambda m: log(f"[bench] {m}"))
    raise SystemExit(f"unknown workload {workload}")


def cheb_bytes(n, nnz, N, word=8, mword=None):
    """Algorithmic bytes of one interior fused Chebyshev step (the launch
    mlc_time_kernel replays): the SpMM's matrix (mword bytes per value,
    default word) and row pointers, the inverse diagonal, the iterate z_{j-1}
    read once (gathered), R read, z_{j-2} read and z_j written."""
    mword = word if mword is None else mword
    return (mword + 4) * nnz + 4 * (n + 1) + word * n + 4 * word * n * N


def _kernel_name(which, N, word, n):
    """Profiler name of the kernel mlc_time_kernel replays: the CG SpMM and
    the Hartree SpMM run the partial-sum shape (1024-thread blocks), the
    polynomial steps the 256-thread shape of the steps before the last. The
    N > 8 kernels gather through 32-bit offsets when an n x N block spans
    less than 4 GiB."""
    t = "float" if word == 4 else "double"
    if which in ("hartree_spmm", "hartree_cheb_step"):
        N, t = 1, "double"
    if N > 8:
        # the library's N > 8 layout: V columns per lane, L lanes per row, NCH column chunks
        V = 4 if (word == 4 and N % 4 == 0) else (2 if N % 2 == 0 else 1)
        groups = -(-N // V)
        L = 4
        while L < groups and L < 64:
            L *= 2
        nch = -(-groups // L)
        o32 = "true" if n * N * word < 2 ** 32 else "false"
        if "spmm" in which:  # the CG SpMM with its p.q partials: 512-thread blocks
            return f"k_spmm_rows<{L}, {V}, {nch}, {o32}, 512, {t}>"
        return f"k_cheb_rows<{L}, {V}, {nch}, false, {o32}, 256, {t}>"  # the steps without the r.z partials
    if "spmm" in which:
        unroll = 4 if N <= 3 else (2 if N <= 6 else 1)
        return f"k_spmm_small<{N}, 4, {unroll}, 1024, {8 if N <= 6 else 4}, {t}>"
    # the matrix-value type: FP32 in the Hartree problem's polynomial steps
    mt = "float" if which == "hartree_cheb_step" else t
    return f"k_cheb_small<{N}, 4, {4 if N <= 6 else 2}, 256, {8 if N <= 2 else 4}, {t}, {mt}>"


def spmm_bytes(n, nnz, N, word=8):
    """Algorithmic bytes of one SpMM launch Y = A X: values (word bytes) and
    column indices (4 B) per nonzero, row pointers (4 B per row), X read once
    and Y written once (word bytes per DoF and orbital each)."""
    return (word + 4) * nnz + 4 * (n + 1) + 2 * word * n * N


def cpu_baseline(S, ctx, rtol):
    """The checker's fine stage of one correction step at the library's current state, with the
    checker's own Jacobi-PCG for both linear solves (its default sparse LU for the Hartree problem
    takes minutes at this size): density and XC at the quadrature points, multipole boundary data,
    assembly, the step-5 solves to rtol from phi, M-normalisation, the Hartree load and solve to
    rtol. Setting up the checker's problem (meshes, prolongation, matrices) is not timed."""
    import os
    from oracle import hartree as har
    from oracle import xc as xcmod
    from oracle.mlc import Problem
    from oracle.pcg import jacobi_pcg
    prob = Problem(S)
    lam, Phi, w, _ = ctx.get_results()
    fine = prob.fine
    t0 = time.perf_counter()
    rho = prob.density_qp(Phi)
    exc, vxc = xcmod.evaluate(S.xc, rho, S.xalpha)
    g = har.boundary_data(fine, rho) if prob.hartree else np.zeros(fine.nv)
    veff = prob.vext_qp + fine.at_qp(w) + vxc
    sigma = 1.0 - float(veff.min())
    A = (0.5 * prob.K + prob.mass_ii(veff) + sigma * prob.M).tocsr()
    B = (prob.M @ Phi) * (lam + sigma)[None, :]
    U, it5 = jacobi_pcg(A, B, x0=Phi, rtol=rtol, maxit=100000)
    U = U / np.sqrt(np.einsum("ai,ai->i", U, prob.M @ U))[None, :]
    itp = 0
    if prob.hartree:
        rho_t = prob.density_qp(U)
        b = 4.0 * np.pi * fine.load(rho_t)[fine.interior] - fine.ib(prob.Kfull) @ g[fine.bverts]
        _, itp = jacobi_pcg(prob.K.tocsr(), b, rtol=rtol, maxit=100000)
    t = time.perf_counter() - t0
    it5 = int(np.max(it5)) if np.ndim(it5) else int(it5)
    itp = int(np.max(itp)) if np.ndim(itp) else int(itp)
    threads = os.environ.get("OMP_NUM_THREADS", "all")
    return {"value": fine.n_dof * Phi.shape[1] / t, "unit": "DoF*orbitals/s", "cores": 1, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"one fine stage of the checker at the library's state after the timed steps: XC, "
                      f"multipole data, assembly, step-5 Jacobi-PCG ({it5} iterations) and Hartree Jacobi-PCG "
                      f"({itp} iterations) to {rtol:g}, {t:.1f} s; SciPy sparse products run on one thread "
                      f"(BLAS threads: {threads}); problem setup not timed"}


def _physics(S, ctx, rep):
    """Validation figures of a step's result: sorted eigenvalues, the largest
    off-diagonal orbital overlap, the electron count and the inner loop."""
    lam = np.sort(ctx.get_results()[0])
    ne = float(np.sum(S.occupations))
    return {"eigenvalues_sorted": [float(x) for x in lam],
            "max_offdiag_overlap": float(rep["max_offdiag_overlap"]),
            "rho_integral": float(rep["rho_integral"]), "electrons": ne,
            "energy": float(rep["energy"]), "inner_iters": int(rep["inner_iters"]),
            "inner_last_diff": float(rep["inner_last_diff"]),
            "inner_converged": bool(rep["status"] == 0)}


def _check_physics(phys, overlap_max, workload, need_inner=True):
    """Exit status 3 when the step's result is not a valid Kohn-Sham iterate:
    non-finite values, a wrong electron count, an inner loop stopped by its cap
    (when need_inner), or orbitals that overlap more than overlap_max."""
    bad = []
    if not all(np.isfinite(phys["eigenvalues_sorted"])) or not np.isfinite(phys["energy"]):
        bad.append("non-finite eigenvalues or energy")
    if abs(phys["rho_integral"] - phys["electrons"]) > 1e-6 * max(1.0, phys["electrons"]):
        bad.append(f"int rho = {phys['rho_integral']:.9f} != {phys['electrons']}")
    if need_inner and not phys["inner_converged"]:
        bad.append(f"inner iteration stopped at its cap ({phys['inner_iters']} iterations, "
                   f"last change {phys['inner_last_diff']:.1e})")
    if phys["max_offdiag_overlap"] > overlap_max:
        bad.append(f"max off-diagonal overlap {phys['max_offdiag_overlap']:.2e} > {overlap_max:g}")
    if bad:
        log(f"[bench] {workload}: invalid step result: " + "; ".join(bad))
        sys.exit(3)


def _opts(mlc, args, precision, precond, hartree_coarse):
    return mlc.options(cg_rtol=args.cg_rtol, poisson_rtol=args.cg_rtol, inner_maxit=args.inner_maxit,
                       inner_tol=args.inner_tol, time_kernels=0, precision=precision,
                       precond=mlc.PC_CHEBYSHEV if precond == "chebyshev" else mlc.PC_JACOBI,
                       cheb_degree=args.cheb_degree, cheb_ratio=args.cheb_ratio,
                       hartree_coarse=hartree_coarse, hartree_precond=_HPC[args.hartree_precond],
                       ir_inner_rtol=args.ir_inner_rtol, cheb_lanczos=args.cheb_lanczos,
                       hartree_cheb_degree=args.hartree_cheb_degree, hartree_cheb_ratio=args.hartree_cheb_ratio)


def _timed_steps(ctx, state, n_warm, n_timed, label, reset):
    """n_warm + n_timed correction steps from the given input state; with reset
    every step starts from that state (set on the device before the step,
    outside its timed region), otherwise the steps continue the outer
    iteration. Returns the timed steps' reports."""
    import torch
    lam0, Phi0, w0 = state
    reps = []
    ctx.set_state(lam0, Phi0, w0)
    for k in range(n_warm + n_timed):
        if reset and k > 0:
            ctx.set_state(lam0, Phi0, w0)
        rep = ctx.correction_step()
        tag = "warmup" if k < n_warm else "step"
        log(f"[bench] {label} {tag} {k if k < n_warm else k - n_warm}: fine {rep['t_fine_ms']:.2f} ms + recon "
            f"{rep['t_recon_ms']:.2f} ms (solve {rep['t_solve_ms']:.2f}, Hartree {rep['t_poisson_ms']:.2f}), inner "
            f"{rep['t_inner_ms']:.0f} ms ({rep['inner_iters']} it), cg {rep['cg_iters_max']} it relres "
            f"{rep['cg_relres_max']:.1e}, poisson {rep['poisson_iters']} it, refinement passes {rep['ir_outer']}")
        if k >= n_warm:
            reps.append(rep)
    torch.cuda.synchronize()
    return reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c1", "batch", "learned"],
                    help="c3: 40-atom cluster, 2e6 DoF x 52 orbitals, FP32 CG + FP64 refinement (default); c2: "
                         "4-atom cluster, 2e5 DoF; c1: hydrogen; batch: uneven clusters")
    ap.add_argument("--seed", type=int, default=None, help="cluster seed (default 0 for c3, 1 for c2)")
    ap.add_argument("--order", type=int, default=2, choices=[1, 2],
                    help="--workload c3: fine-space elements, 2 = P2 (2.0e6 DoFs on 2.8e5 vertices, the "
                         "default), 1 = P1 (2.0e6 vertices)")
    ap.add_argument("--cg-rtol", type=float, default=1e-9)
    ap.add_argument("--precision", choices=["fp64", "fp32ir"], default=None,
                    help="step-5 arithmetic: plain FP64 CG, or FP32 CG inside FP64 iterative refinement "
                         "(default: fp32ir for --workload c3, fp64 otherwise)")
    ap.add_argument("--precond", choices=["jacobi", "chebyshev"], default=None,
                    help="CG preconditioner of the step-5 and Hartree solves (default: chebyshev for one system, "
                         "jacobi for --workload batch, where the tile SpMM is bandwidth-bound and the polynomial "
                         "steps cost more than the iterations they save)")
    ap.add_argument("--hartree-precond", choices=["same", "jacobi", "chebyshev"], default="same",
                    help="preconditioner of the Hartree CG apart from the step-5 solves (default: the same)")
    ap.add_argument("--cheb-degree", type=int, default=None,
                    help="Chebyshev degree (default 16 on the P2 40-atom workload, 8 otherwise)")
    ap.add_argument("--cheb-ratio", type=float, default=None,
                    help="Chebyshev interval [lmax/ratio, lmax] (default 300 on the P2 40-atom workload, 100 "
                         "otherwise)")
    ap.add_argument("--cheb-lanczos", type=int, default=None,
                    help="Lanczos steps for the Chebyshev interval's upper end (0: the Gershgorin bound; default "
                         "16 on the P2 40-atom workload, 0 otherwise)")
    ap.add_argument("--hartree-cheb-degree", type=int, default=None,
                    help="the Hartree CG's polynomial degree (0: --cheb-degree; default 8 on the 40-atom workload, "
                         "0 otherwise)")
    ap.add_argument("--hartree-cheb-ratio", type=float, default=None,
                    help="the Hartree CG's interval ratio (0: --cheb-ratio; default 300 on the 40-atom workload, "
                         "0 otherwise)")
    ap.add_argument("--ir-inner-rtol", type=float, default=1e-4,
                    help="FP32 CG tolerance of each refinement pass (relative to the pass's residual)")
    ap.add_argument("--hartree-coarse", type=int, default=1, choices=[0, 1],
                    help="add the exact coarse-space correction to the Hartree CG preconditioner")
    ap.add_argument("--inner-maxit", type=int, default=None,
                    help="cap of the inner iteration (host, reported apart). Default 300 (a step that reaches it "
                         "is invalid) except for c3: 6, since each of its inner iterations reduces the 1331 x 1331 "
                         "coarse pencil on the host (~0.5 s) and its 12^3 coarse space does not resolve 52 "
                         "orbitals in the first place")
    ap.add_argument("--inner-tol", type=float, default=1e-9)
    ap.add_argument("--steps-from", choices=["initial", "trajectory"], default=None,
                    help="initial: every step starts from the interpolated coarse Kohn-Sham state (default for c3, "
                         "whose 12^3 coarse space cannot separate its 52 orbitals, so that its outer iteration "
                         "drifts); trajectory: the steps continue the outer iteration (default otherwise)")
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="timed steps of the plain FP64 path (FP64 Jacobi-PCG, no coarse correction) for the "
                         "speed-up against it, after the same number of warm-up steps as the timed path from the "
                         "same initial state (default: 2 with --steps-from initial, --steps otherwise; 0 skips it)")
    ap.add_argument("--overlap-max", type=float, default=None,
                    help="largest accepted off-diagonal orbital overlap after a step (default 1e-2 for c1/c2; "
                         "1.0 for c3, whose 12^3 coarse space does not resolve 52 cluster orbitals)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=20,
                    help="c3 cpu baseline: Jacobi-PCG iterations of the checker timed on --cpu-cols columns")
    ap.add_argument("--cpu-cols", type=int, default=8)
    ap.add_argument("--batch-systems", type=int, default=12,
                    help="--workload batch: number of uneven clusters stepped together")
    ap.add_argument("--batch-inner-maxit", type=int, default=4,
                    help="--workload batch: inner iterations per step (host, reported apart from the GPU time)")
    ap.add_argument("--train-steps", type=int, default=800,
                    help="--workload batch: Adam steps of the learned-guess network")
    ap.add_argument("--train-systems", type=int, default=125,
                    help="--workload learned: 4-atom clusters (seeds 1000, ...) whose steps give the training rows")
    ap.add_argument("--train-steps-per-system", type=int, default=4,
                    help="--workload learned: correction steps sampled per training cluster (125 x 4 = 500 solves)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this size twice (hardware counter calibration)")
    args = ap.parse_args()
    p2 = args.workload == "c3" and args.order == 2
    if args.cheb_degree is None:
        args.cheb_degree = 16 if p2 else 8
    if args.cheb_ratio is None:
        args.cheb_ratio = 300.0 if p2 else 100.0
    if args.cheb_lanczos is None:
        args.cheb_lanczos = 16 if p2 else 0
    if args.hartree_cheb_degree is None:
        args.hartree_cheb_degree = 8 if args.workload == "c3" else 0
    if args.hartree_cheb_ratio is None:
        args.hartree_cheb_ratio = 300.0 if args.workload == "c3" else 0.0
    if args.precond is None:
        args.precond = "jacobi" if args.workload == "batch" else "chebyshev"
    if args.precision is None:
        args.precision = "fp32ir" if args.workload == "c3" else "fp64"
    if args.seed is None:
        args.seed = 1 if args.workload == "c2" else 0
    if args.steps_from is None:
        args.steps_from = "initial" if args.workload == "c3" else "trajectory"
    if args.plain_steps is None:
        args.plain_steps = 2 if args.steps_from == "initial" else args.steps
    if args.inner_maxit is None:
        args.inner_maxit = 6 if args.workload == "c3" else 300
    if args.overlap_max is None:
        args.overlap_max = 1.0 if args.workload == "c3" else 1e-2
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the path shards by orbitals "
              f"across GPUs, which is not run here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_02824_amd import mlc

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "learned":
        return run_learned(args)
    t_all = time.perf_counter()
    log(f"[bench] building workload {args.workload} seed {args.seed}")
    S = make_system(args.workload, args.seed, args.order)
    prec = mlc.PREC_FP32_IR if args.precision == "fp32ir" else mlc.PREC_FP64
    ctx = mlc.Context(S, _opts(mlc, args, prec, args.precond, args.hartree_coarse))
    n, N = ctx.n_dof, ctx.N
    log(f"[bench] n_dof={n} N={N} n_coarse={ctx.n_coarse_dof} tets={ctx.n_tets} workspace={ctx.workspace_bytes/1e6:.0f} MB")
    t0 = time.perf_counter()
    # Algorithm 1 steps 1 and 4: the coarse Kohn-Sham solve, interpolated; the timed steps start from it
    it = ctx.initial_state(tol=1e-10, maxit=60 if args.workload == "c3" else 300)
    lam0, Phi0, w0, _ = ctx.get_results_device()
    state0 = (lam0, Phi0.clone(), w0.clone())
    log(f"[bench] coarse SCF (initial state): {it} iterations, {time.perf_counter()-t0:.1f} s")
    tw0 = time.perf_counter()
    reset = args.steps_from == "initial"
    reps = _timed_steps(ctx, state0, args.warmup, args.steps, "timed path", reset)
    wall = time.perf_counter() - tw0
    phys = _physics(S, ctx, reps[-1])
    log(f"[bench] result of the step: {phys}")
    if args.calib_copy_mib:
        nb = args.calib_copy_mib * 2 ** 20
        a = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nb} bytes read and written, 2 times")
    t_gpu = sum(r["t_fine_ms"] + r["t_recon_ms"] for r in reps) / 1e3
    value = n * N * len(reps) / t_gpu
    ms_per_step = 1e3 * t_gpu / len(reps)
    # roofline of the dominant kernel: each solver kernel is replayed back to back on the library
    # stream between two HIP events (per-launch events inside the solve would add dispatch overhead
    # to every launch); the one with the largest time per step (mean launch time x launches per
    # step) is the dominant kernel
    nnz = int(ctx.probe("PATTERN", (3,))[0])
    word = 4 if args.precision == "fp32ir" else 8
    n_replay = 200
    cheb = args.precond == "chebyshev"
    deg = args.cheb_degree if cheb else 1
    hdeg = (args.hartree_cheb_degree or deg) if cheb else 1   # 0 = the step-5 polynomial's degree
    it5 = float(np.mean([r["cg_iters_max"] for r in reps]))
    itp = float(np.mean([r["poisson_iters"] for r in reps]))
    kern = {}
    cands = [("cg_spmm", N, word, it5 + 2), ("hartree_spmm", 1, 8, itp + 2)]
    if cheb:
        cands += [("cheb_step", N, word, (deg - 1) * (it5 + 1)), ("hartree_cheb_step", 1, 8, (hdeg - 1) * (itp + 1))]
    for which, ncol, w, launches in cands:
        us = ctx.time_kernel(which, n_replay)
        nbytes = (spmm_bytes(n, nnz, ncol, w) if "spmm" in which else
                  cheb_bytes(n, nnz, ncol, w, 4 if which == "hartree_cheb_step" else w))
        kern[which] = {"avg_launch_us": round(us, 2), "bytes_per_launch": nbytes,
                       "achieved_GBs": round(nbytes / (us * 1e-6) / 1e9, 1), "launches_per_step": round(launches, 1),
                       "ms_per_step": round(us * launches / 1e3, 3)}
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    kd = kern[dom]
    kname = _kernel_name(dom, N, word, n)
    achieved = kd["achieved_GBs"]
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _traffic(kname, args.workload, args.seed, args.precision,
                                args.order if args.workload == "c3" else 1),
            "kernel": kname, "bytes_per_launch": kd["bytes_per_launch"], "avg_launch_us": kd["avg_launch_us"],
            "launches_timed": n_replay, "all_kernels": kern}
    # the plain FP64 GPU path on the same input state: FP64 Jacobi-PCG, no coarse correction
    plain = None
    if args.plain_steps > 0:
        ctx_p = mlc.Context(S, _opts(mlc, args, mlc.PREC_FP64, "jacobi", 0))
        preps = _timed_steps(ctx_p, state0, 1 if reset else args.warmup, args.plain_steps, "plain FP64", reset)
        pphys = _physics(S, ctx_p, preps[-1])
        p_ms = float(np.mean([r["t_fine_ms"] + r["t_recon_ms"] for r in preps]))
        plain = {"ms_per_step": p_ms, "value": n * N / (p_ms / 1e3),
                 "cg_iters_per_step": float(np.mean([r["cg_iters_max"] for r in preps])),
                 "poisson_iters_per_step": float(np.mean([r["poisson_iters"] for r in preps])),
                 "max_eigenvalue_difference": float(np.max(np.abs(np.array(pphys["eigenvalues_sorted"]) -
                                                                  np.array(phys["eigenvalues_sorted"]))))}
        log(f"[bench] plain FP64 path: {p_ms:.2f} ms per step, eigenvalues differ from the timed path's by "
            f"{plain['max_eigenvalue_difference']:.2e}")
        ctx_p.close()
        del ctx_p
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: the checker's Jacobi-PCG")
        if args.workload == "c3":
            cpu = cpu_baseline_pcg_rate(S, ctx, args, plain)
        else:
            cpu = cpu_baseline(S, ctx, args.cg_rtol)
        log(f"[bench] cpu baseline: {cpu['sample']}")
    cg_its = int(np.mean([r["cg_iters_max"] for r in reps]))
    workload_name = {"c2": f"4-atom seeded cluster (seed {args.seed}), graded P1 mesh",
                     "c3": f"40-atom seeded cluster (seed {args.seed}), graded P{args.order} mesh",
                     "c1": "hydrogen Z=1 rc=0.2, 16^3 Kuhn P1 mesh"}[args.workload]
    out = {
        "metric": "fine-mesh SCF correction step: DoF*orbitals/s and % HBM roofline vs plain FP64",
        "value": value, "unit": "DoF*orbitals/s", "n_gpus": 1, "steps": len(reps), "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "vs_plain_fp64": (plain["ms_per_step"] / ms_per_step) if plain else None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64-refinement", "data": "synthetic",
        "config": {"workload": workload_name,
                   "n_dof": n, "orbitals": N, "n_tets": ctx.n_tets, "nnz": nnz, "n_coarse_dof": ctx.n_coarse_dof,
                   "cg_rtol": args.cg_rtol,
                   "precision": "plain FP64" if args.precision == "fp64" else "FP32 CG + FP64 refinement",
                   "preconditioner": ("Jacobi" if args.precond == "jacobi" else
                                      f"Chebyshev degree {args.cheb_degree} over [lmax/{args.cheb_ratio:g}, lmax], lmax "
                                      + (f"from {args.cheb_lanczos} Lanczos steps" if args.cheb_lanczos else
                                         "the Gershgorin bound")
                                      + (f"; Hartree CG degree {args.hartree_cheb_degree or args.cheb_degree} over "
                                         f"[lmax/{args.hartree_cheb_ratio or args.cheb_ratio:g}, lmax]"))
                   + (" + coarse-space correction (Hartree)" if args.hartree_coarse else ""),
                   "timed_step": ("outer step l=0 -> 1 of Algorithm 1 from the interpolated coarse Kohn-Sham "
                                  "state, repeated (state reset on the device before each step)" if reset else
                                  f"outer steps l={args.warmup}..{args.warmup + args.steps - 1} of Algorithm 1 "
                                  f"from the interpolated coarse Kohn-Sham state"),
                   "parallelism": "1 GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "physics": phys,
        "detail": {"plain_fp64": plain,
                   "pcg_throughput": {
                       "step5_dof_orbital_iterations_per_s":
                           n * sum(r["cg_iters_sum"] for r in reps) / (1e-3 * sum(r["t_solve_ms"] for r in reps)),
                       "hartree_dof_iterations_per_s":
                           n * sum(r["poisson_iters"] for r in reps) / (1e-3 * max(sum(r["t_poisson_ms"] for r in reps),
                                                                                   1e-9)),
                       "t_solve_ms_per_step": float(np.mean([r["t_solve_ms"] for r in reps])),
                       "t_poisson_ms_per_step": float(np.mean([r["t_poisson_ms"] for r in reps]))},
                   "cg_iters_per_step": cg_its,
                   "poisson_iters_per_step": int(np.mean([r["poisson_iters"] for r in reps])),
                   "inner_ms_per_step": float(np.mean([r["t_inner_ms"] for r in reps])),
                   "inner_iters_per_step": float(np.mean([r["inner_iters"] for r in reps])),
                   "wall_ms_per_step_incl_host_inner": 1e3 * wall / (len(reps) + args.warmup),
                   "coarse_scf_iterations": it,
                   "total_wall_s": time.perf_counter() - t_all},
    }
    print(json.dumps(out), flush=True)
    _check_physics(phys, args.overlap_max, args.workload, need_inner=args.workload != "c3")


def cpu_baseline_pcg_rate(S, ctx, args, plain):
    """The checker's Jacobi-PCG on the 40-atom step-5 operator, timed over a
    bounded sample: cpu_iters iterations on cpu_cols of the N columns (SciPy's
    sparse-times-dense product streams the matrix once per product, so the
    per-column cost is what scales). The operator is 1/2 K + M_{V_ext} + sigma M
    assembled by the checker (the same sparsity and nearly the same spectrum as
    the step's A + sigma M; the density-dependent part of V_eff is left out of
    this timing sample). The rate in DoF*orbital*iterations/s is converted to
    the metric's DoF*orbitals/s with the plain FP64 GPU path's iteration counts
    per step (its step-5 and Hartree Jacobi-PCG iterations), the CPU doing the
    same iterations."""
    import os
    from oracle.fem import make_mesh
    from oracle.pcg import jacobi_pcg
    from oracle.potentials import v_ext
    t0 = time.perf_counter()
    fine = make_mesh(S.xyz, S.tets, S.lo, S.hi, getattr(S, "order", 1))
    Kf = fine.stiffness()
    vq = v_ext(fine.qp, S.R, S.Z, S.potential, S.rc, S.omega)
    sigma = 1.0 - float(vq.min())
    A = fine.ii(0.5 * Kf + fine.mass(vq + sigma))
    K = fine.ii(Kf)
    del Kf
    t_setup = time.perf_counter() - t0
    lam, Phi, w, _ = ctx.get_results()
    cols = min(args.cpu_cols, Phi.shape[1])
    B = np.ascontiguousarray(Phi[:, :cols])
    t0 = time.perf_counter()
    _, _ = jacobi_pcg(A, B, x0=np.zeros_like(B), rtol=1e-30, maxit=args.cpu_iters)
    t5 = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _ = jacobi_pcg(K, B[:, 0], x0=np.zeros(B.shape[0]), rtol=1e-30, maxit=args.cpu_iters)
    th = time.perf_counter() - t0
    n = A.shape[0]
    N = Phi.shape[1]
    rate5 = n * cols * args.cpu_iters / t5          # DoF*orbital*iterations/s
    rateh = n * args.cpu_iters / th
    it5 = plain["cg_iters_per_step"] if plain else 100.0
    ith = plain["poisson_iters_per_step"] if plain else 300.0
    t_step = n * N * it5 / rate5 + n * ith / rateh
    threads = os.environ.get("OMP_NUM_THREADS", "all")
    return {"value": n * N / t_step, "unit": "DoF*orbitals/s", "cores": 1, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "step5_dof_orbital_iterations_per_s": rate5, "hartree_dof_iterations_per_s": rateh,
            "sample": f"the checker's Jacobi-PCG (SciPy sparse products, one thread; BLAS threads: {threads}) on the "
                      f"40-atom step-5 operator 1/2 K + M_(V_ext + sigma) ({n} DoF, {A.nnz} nonzeros): "
                      f"{args.cpu_iters} iterations on {cols} of the {N} columns in {t5:.1f} s, and on the Hartree "
                      f"matrix K, one column, in {th:.1f} s; per step the CPU would run the plain FP64 GPU path's "
                      f"{it5:.0f} step-5 and {ith:.0f} Hartree iterations: {t_step:.0f} s per step "
                      f"(assembly by the checker, {t_setup:.0f} s, not timed; density, XC and the rest of the fine "
                      f"stage not included, which favours the CPU)"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _batch_contexts(systems, mlc, states, **kw):
    """Contexts from the shared initial states (computed once, by the first call)."""
    ctxs = []
    for k, S in enumerate(systems):
        ctx = mlc.Context(S, mlc.options(**kw))
        if len(states) <= k:
            ctx.initial_state(tol=1e-9, maxit=300)
            lam, Phi, w, _ = ctx.get_results()
            states.append((lam, Phi, w))
        ctx.set_state(*states[k])
        ctxs.append(ctx)
    return ctxs


def train_guess_network(mlc, args, opts, n_systems=4, steps_per_system=3, stride=1, cap=600000):
    """Samples from the library's own steps on small 4-atom clusters (seeds
    1000, 1001, ..., not in the batch), then GPU training by the library."""
    import torch
    from inputs.nn_init import init_params
    from inputs.systems import c2_small
    sx = torch.zeros((cap, 6), dtype=torch.float32, device="cuda")
    st = torch.zeros(cap, dtype=torch.float32, device="cuda")
    rows = 0
    t0 = time.perf_counter()
    for seed in range(1000, 1000 + n_systems):
        if rows >= cap:
            break
        ctx = mlc.Context(c2_small(seed), mlc.options(**opts))
        ctx.initial_state(tol=1e-9, maxit=300)
        ctx.set_sample_sink(sx[rows:], st[rows:], stride=stride)
        for _ in range(steps_per_system):
            ctx.correction_step()
        rows += ctx.sample_count()
        ctx.close()
        if (seed - 1000) % 10 == 9:
            log(f"[bench] training samples from {seed - 999} systems: {rows} rows, {time.perf_counter() - t0:.0f} s")
    net = mlc.Network()
    net.set_params(init_params(11, out_scale=0.01))
    t0 = time.perf_counter()
    hist = net.train(sx[:rows].contiguous(), st[:rows].contiguous(), steps=args.train_steps, batch=4096, lr=2e-3)
    log(f"[bench] trained guess network on {rows} rows, {args.train_steps} steps in {time.perf_counter()-t0:.1f} s, "
        f"loss {np.mean(hist[:20]):.3e} -> {np.mean(hist[-20:]):.3e}")
    return net, rows, float(np.mean(hist[:20])), float(np.mean(hist[-20:]))


def run_learned(args):
    """The learned initial guess at the 40-atom workload: the network is
    trained by the library on rows of its own steps on small 4-atom clusters
    of the 4-atom distribution (seeds 1000, ...), then the 40-atom step
    (FP32 CG + FP64 refinement to 1e-9, the benchmark's preconditioners) is
    run from the interpolated coarse state with the plain start (phi) and
    with the learned start, alternately; reported: CG iterations, refinement
    passes and GPU times of each."""
    import torch
    from paper_2103_02824_amd import mlc
    t_all = time.perf_counter()
    base = dict(cg_rtol=args.cg_rtol, poisson_rtol=args.cg_rtol, inner_maxit=30, inner_tol=args.inner_tol)
    net, rows, l0, l1 = train_guess_network(mlc, args, base, n_systems=args.train_systems,
                                            steps_per_system=args.train_steps_per_system, stride=2, cap=8000000)
    S = make_system("c3", args.seed)
    opts = _opts(mlc, args, mlc.PREC_FP32_IR, args.precond, args.hartree_coarse)
    opts.inner_maxit = 6
    ctx = mlc.Context(S, opts)
    ctx.initial_state(tol=1e-10, maxit=60)
    lam0, Phi0, w0, _ = ctx.get_results_device()
    state0 = (lam0, Phi0.clone(), w0.clone())
    res = {"plain": [], "learned": []}
    for k in range(1 + args.steps):
        for name in ("plain", "learned"):
            ctx.set_guess(net if name == "learned" else None)
            ctx.set_state(*state0)
            rep = ctx.correction_step()
            log(f"[bench] 40-atom step, {name} start: solve {rep['t_solve_ms']:.2f} ms, fine {rep['t_fine_ms']:.2f} ms, "
                f"cg {rep['cg_iters_max']} (sum {rep['cg_iters_sum']}), refinement passes {rep['ir_outer']}, "
                f"learned columns {rep['guess_learned_cols']}, residual ratio {rep['guess_resid_ratio']:.3f}")
            if k > 0:
                res[name].append(rep)
    summary = {}
    for name, reps in res.items():
        summary[name] = {"t_fine_ms": float(np.mean([r["t_fine_ms"] + r["t_recon_ms"] for r in reps])),
                         "t_solve_ms": float(np.mean([r["t_solve_ms"] for r in reps])),
                         "cg_iters_max": int(reps[-1]["cg_iters_max"]), "cg_iters_sum": int(reps[-1]["cg_iters_sum"]),
                         "refinement_passes": int(reps[-1]["ir_outer"]),
                         "learned_cols": int(reps[-1]["guess_learned_cols"]),
                         "guess_resid_ratio": float(reps[-1]["guess_resid_ratio"])}
    n, N = ctx.n_dof, ctx.N
    out = {"metric": "fine-mesh SCF correction step: DoF*orbitals/s and % HBM roofline vs plain FP64",
           "value": n * N / (summary["learned"]["t_fine_ms"] / 1e3), "unit": "DoF*orbitals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": summary["learned"]["t_fine_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64-refinement", "data": "synthetic",
           "config": {"workload": f"40-atom seeded cluster (seed {args.seed}), graded P1 mesh, learned start",
                      "n_dof": n, "orbitals": N,
                      "training": f"{rows} rows from {args.train_systems * args.train_steps_per_system} solves "
                                  f"({args.train_systems} 4-atom clusters x {args.train_steps_per_system} steps)"},
           "roofline": None, "cpu_baseline": None,
           "detail": dict(summary, training_rows=rows, training_loss=[l0, l1],
                          speedup_of_learned=summary["plain"]["t_fine_ms"] / summary["learned"]["t_fine_ms"],
                          total_wall_s=time.perf_counter() - t_all)}
    ctx.close()
    net.close()
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Batching of uneven independent systems: plain FP64 single-system steps
    vs batched FP64, batched FP32 + FP64 refinement, and batched FP32 +
    refinement with the learned start; a timed step follows one warm-up step
    in every configuration, from the same initial states."""
    import torch
    from inputs.systems import batch_clusters
    from paper_2103_02824_amd import mlc
    t_all = time.perf_counter()
    systems = batch_clusters(args.batch_systems)
    log(f"[bench] batch of {len(systems)} clusters: vertices {[len(S.xyz) for S in systems]}, "
        f"orbitals {[S.n_orbitals for S in systems]}")
    base = dict(cg_rtol=args.cg_rtol, poisson_rtol=args.cg_rtol, inner_maxit=args.batch_inner_maxit,
                inner_tol=args.inner_tol)
    pcopt = dict(precond=mlc.PC_CHEBYSHEV if args.precond == "chebyshev" else mlc.PC_JACOBI,
                 cheb_degree=args.cheb_degree, cheb_ratio=args.cheb_ratio, hartree_coarse=args.hartree_coarse,
                 hartree_precond=_HPC[args.hartree_precond])
    pcname = args.precond + ("" if args.hartree_precond == "same" else f"/hartree-{args.hartree_precond}") + \
        ("+coarse" if args.hartree_coarse else "")
    out = {}
    states = []
    dof_orb = None
    # one system at a time: the plain FP64 path (Jacobi-PCG) and the best single-system solver settings
    for name, kw in (("plain_fp64_sequential", {}), (f"single_fp64_{pcname}_sequential", pcopt)):
        ctxs = _batch_contexts(systems, mlc, states, **dict(base, **kw))
        dof_orb = sum(c.n_dof * c.N for c in ctxs)
        for c in ctxs:
            c.correction_step()
        torch.cuda.synchronize()
        t = 0.0
        its = []
        for c in ctxs:
            r = c.correction_step()
            t += r["t_fine_ms"] + r["t_recon_ms"]
            its.append((r["cg_iters_max"], r["poisson_iters"]))
        out[name] = {"gpu_ms": t, "cg_and_hartree_iters": its}
        log(f"[bench] {name}: {t:.2f} ms GPU, CG/Hartree iterations {its}")
        for c in ctxs:
            c.close()
    net, rows, l0, l1 = train_guess_network(mlc, args, base)
    for name, kw, learned in (("batched_fp64", {}, False),
                              (f"batched_fp64_{pcname}", pcopt, False),
                              (f"batched_fp32ir_{pcname}", dict(pcopt, precision=mlc.PREC_FP32_IR), False),
                              (f"batched_fp32ir_{pcname}_learned", dict(pcopt, precision=mlc.PREC_FP32_IR), True)):
        ctxs = _batch_contexts(systems, mlc, states, **dict(base, **kw))
        if learned:
            for c in ctxs:
                c.set_guess(net)
        b = mlc.Batch(ctxs)
        reps, br = b.step()
        torch.cuda.synchronize()
        reps, br = b.step()
        gpu = br["t_gpu_ms"] + br["t_recon_ms"]
        out[name] = {"gpu_ms": gpu, "solve_ms": br["t_solve_ms"], "poisson_ms": br["t_poisson_ms"],
                     "inner_ms": br["t_inner_ms"], "cg_iters": [r["cg_iters_max"] for r in reps],
                     "hartree_iters": [r["poisson_iters"] for r in reps],
                     "tile_rows": br["tile_rows"], "lanes": br["spmm_lanes"], "ir_outer": br["ir_outer"],
                     "learned_cols": sum(r["guess_learned_cols"] for r in reps)}
        log(f"[bench] {name}: {gpu:.2f} ms GPU (solve {br['t_solve_ms']:.2f}, Hartree {br['t_poisson_ms']:.2f}), "
            f"shape {br['tile_rows']}x{br['spmm_lanes']}, CG iterations {out[name]['cg_iters']}, "
            f"Hartree {out[name]['hartree_iters']}")
        b.close()
        for c in ctxs:
            c.close()
    best = out[f"batched_fp32ir_{pcname}_learned"]["gpu_ms"]
    res = {
        "metric": "fine-mesh SCF correction step: DoF*orbitals/s and % HBM roofline vs plain FP64",
        "value": dof_orb / (best / 1e3), "unit": "DoF*orbitals/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64-refinement", "data": "synthetic",
        "config": {"workload": f"batch of {len(systems)} uneven seeded clusters (2-8 atoms, graded P1 meshes)",
                   "dof_orbitals": dof_orb, "cg_rtol": args.cg_rtol, "parallelism": "1 GPU",
                   "timed_path": f"batched, FP32 CG + FP64 refinement, {pcname} preconditioner, learned start"},
        "roofline": None, "cpu_baseline": None,
        "detail": dict(out, speedup_vs_plain_fp64=out["plain_fp64_sequential"]["gpu_ms"] / best,
                       speedup_vs_best_single_sequential=out[f"single_fp64_{pcname}_sequential"]["gpu_ms"] / best,
                       training_rows=rows, training_loss=[l0, l1], total_wall_s=time.perf_counter() - t_all),
    }
    net.close()
    print(json.dumps(res), flush=True)


# committed rocprofv3 summaries with hardware-counter traffic per workload
_PROFILES = {("c2", 0, "fp64", 1): "cg_c2_cluster_fp64.md", ("c3", 0, "fp32ir", 1): "cg_c3_cluster40_fp32ir.md",
             ("c3", 0, "fp32ir", 2): "cg_c3_cluster40_p2_fp32ir.md"}


def _traffic(kname, workload, seed, precision, order=1):
    """HBM bytes per launch of the roofline kernel from the committed counter summary, or None
    when there is no summary for this workload or the kernel sources have changed since."""
    import hashlib
    name = _PROFILES.get((workload, seed, precision, order))
    if name is None:
        return None
    prof = Path(ROOT) / "profiles" / name
    if not prof.exists():
        return None
    for line in prof.read_text().splitlines():
        if line.startswith("traffic-record:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec["kernel"] != kname:
                continue
            srcs = rec.get("sources", [rec["source"]] if "source" in rec else [])
            want = rec.get("sources_sha256", rec.get("source_sha256"))
            try:
                blob = b"".join((Path(ROOT) / f).read_bytes() for f in srcs)
            except OSError:
                return None
            if not srcs or hashlib.sha256(blob).hexdigest() != want:
                return None
            return rec["bytes_per_launch"]
    return None


if __name__ == "__main__":
    main()
