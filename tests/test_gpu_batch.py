"""Batched stepping of uneven independent systems (mlc_batch_*) vs the FP64
CPU checker, through the C ABI.

The batch mixes one hydrogen system (N = 1, LDA + Hartree), a two-orbital
nonlinear system and a twelve-orbital linear system without a Hartree problem
(the wide SpMM path), on meshes of different sizes. Tolerances as for single
contexts: eigenvalues 1e-8 Ha, density 1e-6 relative L2, step-5 solutions
1e-8 relative.
"""
import numpy as np
import pytest

from inputs.systems import c1_hydrogen, tiny_system
from oracle.mlc import Options, Problem, correction_step, fine_stage
from oracle.scf import initial_state

pytestmark = pytest.mark.gpu

LIB_OPTS = dict(cg_rtol=1e-12, poisson_rtol=1e-13, inner_tol=1e-11, inner_maxit=500, n_extra=8, shift=1,
                sigma0=1.0)
ORA_OPTS = Options(shift=True, sigma0=1.0, inner_tol=1e-11, inner_maxit=500, n_extra=8)


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _systems():
    tiny12 = tiny_system(n_fine=10, n_coarse=5, box=6.0, nonlinear=False, n_orbitals=12, seed=3)
    tiny12.occupations = np.ones(12)
    return [("c1", c1_hydrogen(), True),
            ("tiny2", tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=7), True),
            ("tiny12", tiny12, False)]


@pytest.fixture(scope="module")
def cases(gpu):
    out = []
    for name, S, full in _systems():
        prob = Problem(S)
        st0, _ = initial_state(prob)
        ref = correction_step(prob, st0, ORA_OPTS) if full else None
        fs = ref.inter["fine"] if full else fine_stage(prob, st0, ORA_OPTS)
        out.append((name, S, st0, ref, fs, full))
    return out


def _contexts(cases, **kw):
    from paper_2103_02824_amd import mlc
    ctxs = []
    for name, S, st0, ref, fs, full in cases:
        ctx = mlc.Context(S, mlc.options(**dict(LIB_OPTS, **kw)))
        ctx.set_state(st0.lam, st0.Phi, st0.w)
        ctxs.append(ctx)
    return ctxs


@pytest.mark.parametrize("prec,pc", [("fp64", "jacobi"), ("fp32ir", "jacobi"), ("fp64", "chebyshev"),
                                     ("fp32ir", "chebyshev"), ("fp64", "jacobi+coarse"),
                                     ("fp64", "chebyshev+coarse"), ("fp32ir", "chebyshev+coarse"),
                                     ("fp32ir", "jacobi/hartree-chebyshev+coarse")])
def test_batch_step_matches_checker(cases, prec, pc):
    from paper_2103_02824_amd import mlc
    kw = {} if prec == "fp64" else dict(precision=mlc.PREC_FP32_IR, ir_inner_rtol=1e-4)
    if pc.startswith("chebyshev"):
        kw.update(precond=mlc.PC_CHEBYSHEV, cheb_degree=6, cheb_ratio=100.0)
    if pc.endswith("coarse"):
        kw.update(hartree_coarse=1)
    if "/hartree-chebyshev" in pc:  # Jacobi for step 5, the polynomial only in the Hartree CG
        kw.update(hartree_precond=mlc.PC_CHEBYSHEV, cheb_degree=6, cheb_ratio=100.0)
    print(f"case batch of {[c[0] for c in cases]} precision {prec} preconditioner {pc}", flush=True)
    ctxs = _contexts(cases, **kw)
    batch = mlc.Batch(ctxs)
    reps, br = batch.step()
    print(br, flush=True)
    assert br["n_systems"] == 3
    assert br["tile_rows"] in (128, 256, 512, 1024) and br["spmm_lanes"] in (2, 4, 8)
    assert br["dof_orbitals"] == sum(c.n_dof * c.N for c in ctxs)
    for (name, S, st0, ref, fs, full), ctx, rep in zip(cases, ctxs, reps):
        assert rep["cg_relres_max"] <= 1e-12 * (1 + 1e-6), (name, rep)
        U = ctx.probe("U", (ctx.n_dof, ctx.N))
        assert relerr(U, fs["U"]) < 1e-8, (name, relerr(U, fs["U"]))
        if S.hartree:
            assert relerr(ctx.probe("W0", (ctx.n_dof,)), fs["w0"]) < 1e-8, name
        if full:
            lam, Phi, w, rho = ctx.get_results()
            assert np.max(np.abs(lam - ref.state.lam)) < 1e-8, (name, lam, ref.state.lam)
            assert relerr(rho, ref.rho_nodal) < 1e-6, name
            assert abs(rep["energy"] - ref.energy) < 1e-8, name
    batch.close()
    for c in ctxs:
        c.close()


def test_batch_equals_single_steps_over_two_steps(cases):
    """Two batch steps with a fixed tile shape give the same results as two
    single-context steps of each system (to rounding order)."""
    from paper_2103_02824_amd import mlc
    print("case batch vs single contexts, two steps, shape 128 x 2", flush=True)
    single = _contexts(cases)
    for c in single:
        c.correction_step()
        c.correction_step()
    ctxs = _contexts(cases)
    batch = mlc.Batch(ctxs, tile_rows=128, lanes=2)
    for _ in range(2):
        reps, br = batch.step()
        assert br["tile_rows"] == 128 and br["spmm_lanes"] == 2
    for (name, S, st0, ref, fs, full), a, b in zip(cases, single, ctxs):
        ua, ub = a.probe("U", (a.n_dof, a.N)), b.probe("U", (b.n_dof, b.N))
        assert relerr(ub, ua) < 1e-9, (name, relerr(ub, ua))
        if full:
            la, lb = a.get_results()[0], b.get_results()[0]
            assert np.max(np.abs(la - lb)) < 1e-9, (name, la, lb)
    batch.close()
    for c in single + ctxs:
        c.close()


def test_batch_coarse_correction_matches_single_context_iterations(cases):
    """The batched Hartree CG with the coarse-space correction takes the
    iterations of the single-context two-level solve (Jacobi and polynomial
    smoothers, within one) and reaches its potential; the hydrogen system's
    count against plain Jacobi is reported."""
    from paper_2103_02824_amd import mlc
    for pc in ("jacobi", "chebyshev"):
        print(f"case batch vs single contexts, two-level Hartree, {pc}", flush=True)
        kw = dict(hartree_coarse=1)
        if pc == "chebyshev":
            kw.update(precond=mlc.PC_CHEBYSHEV, cheb_degree=6, cheb_ratio=100.0)
        single = _contexts(cases, **kw)
        srep = [c.correction_step() for c in single]
        ctxs = _contexts(cases, **kw)
        batch = mlc.Batch(ctxs)
        reps, br = batch.step()
        for (name, S, *_), a, b, ra, rb in zip(cases, single, ctxs, srep, reps):
            if not S.hartree:
                continue
            assert abs(ra["poisson_iters"] - rb["poisson_iters"]) <= 1, (name, pc, ra["poisson_iters"],
                                                                        rb["poisson_iters"])
            wa, wb = a.probe("W0", (a.n_dof,)), b.probe("W0", (b.n_dof,))
            assert relerr(wb, wa) < 1e-9, (name, pc, relerr(wb, wa))
        batch.close()
        for c in single + ctxs:
            c.close()
    plain = _contexts(cases[:1])
    rp = plain[0].correction_step()
    plain[0].close()
    print(f"c1 Hartree iterations: Jacobi {rp['poisson_iters']}, two-level (batched) {reps[0]['poisson_iters']}",
          flush=True)
