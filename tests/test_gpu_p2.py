"""P2 (quadratic) fine spaces on the GPU against the checker's P2 space
(oracle/fem2.py), through the C ABI: every fine-stage block of a correction
step (step-5 solutions per column, Hartree direction, boundary data, Gram
blocks, coarse-pattern integrals), then eigenvalues, density and energy, on
a P2 space over the coarse mesh itself and over a refinement of it; the
initial state; whole steps in a row; the FP32 + Chebyshev configuration of
the large workloads; and P2 systems in a batch beside a P1 one. Tolerances
as for P1: eigenvalues 1e-8 Ha, density 1e-6 relative L2, blocks 1e-8 at CG
tolerance 1e-12."""
import numpy as np
import pytest

from inputs.systems import tiny_system
from oracle.mlc import Options, Problem, correction_step
from oracle.scf import initial_state
from test_gpu_parity import LIB_OPTS, ORA_OPTS, _compare_fine_stage, relerr

pytestmark = pytest.mark.gpu

CASES = {
    # P1 coarse space on the same mesh (p-nested), 343 DoFs
    "same_mesh": lambda: tiny_system(n_fine=4, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=7, order=2),
    # P1 coarse space on a mesh refined once (h-nested as well), 1331 DoFs
    "nested": lambda: tiny_system(n_fine=6, n_coarse=3, box=5.0, nonlinear=True, n_orbitals=2, seed=7, order=2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_p2_fine_stage_and_step(gpu, case):
    from paper_2103_02824_amd import mlc
    S = CASES[case]()
    prob = Problem(S)
    assert prob.fine.order == 2
    st0, _ = initial_state(prob)
    ctx = mlc.Context(S, mlc.options(**LIB_OPTS))
    print(f"case P2 {case}: n_dof={ctx.n_dof} nodes={ctx.n_vertices} nH={ctx.n_coarse_dof}", flush=True)
    assert ctx.n_dof == prob.fine.n_dof and ctx.n_vertices == prob.fine.nv
    ctx.set_state(st0.lam, st0.Phi, st0.w)
    rep = ctx.correction_step()
    ref = correction_step(prob, st0, ORA_OPTS)
    _compare_fine_stage(ctx, prob, ref.inter["fine"])
    lam, Phi, w, rho = ctx.get_results()
    print(f"lambda {lam} / {ref.state.lam}, energy {rep['energy']:.10f} / {ref.energy:.10f}", flush=True)
    assert np.max(np.abs(lam - ref.state.lam)) < 1e-8, (lam, ref.state.lam)
    assert relerr(rho, ref.rho_nodal) < 1e-6
    assert relerr(w, ref.state.w) < 1e-6
    assert abs(rep["energy"] - ref.energy) < 1e-8
    assert abs(rep["rho_integral"] - float(np.sum(S.occupations))) < 1e-9
    ctx.close()


def test_p2_initial_state(gpu):
    """Algorithm 1 step 1 on the coarse mesh and the transfer Phi = P Phi_H,
    w = P w_H to every P2 node (edge midpoints included)."""
    from paper_2103_02824_amd import mlc
    S = CASES["nested"]()
    prob = Problem(S)
    st0, _ = initial_state(prob, tol=1e-11, maxit=400)
    ctx = mlc.Context(S, mlc.options(**LIB_OPTS))
    ctx.initial_state(tol=1e-11, maxit=400)
    lam, Phi, w, rho = ctx.get_results()
    assert np.max(np.abs(lam - st0.lam)) < 1e-8, (lam, st0.lam)
    s = np.sign(np.sum(Phi * st0.Phi, axis=0))
    assert relerr(Phi * s, st0.Phi) < 1e-6
    assert relerr(w, st0.w) < 1e-6
    ctx.close()


def test_p2_three_steps_in_a_row(gpu):
    """Three outer steps, each side continuing from its own state."""
    from paper_2103_02824_amd import mlc
    S = CASES["nested"]()
    prob = Problem(S)
    st, _ = initial_state(prob)
    ctx = mlc.Context(S, mlc.options(**LIB_OPTS))
    ctx.set_state(st.lam, st.Phi, st.w)
    for k in range(3):
        rep = ctx.correction_step()
        ref = correction_step(prob, st, ORA_OPTS)
        st = ref.state
        lam, Phi, w, rho = ctx.get_results()
        print(f"P2 step {k}: lambda {lam} / {ref.state.lam}, inner {rep['inner_iters']}/{ref.inner_iters}",
              flush=True)
        assert np.max(np.abs(lam - ref.state.lam)) < 1e-8, (lam, ref.state.lam)
        assert relerr(rho, ref.rho_nodal) < 1e-6
    ctx.close()


def test_p2_fp32_refinement_with_chebyshev(gpu):
    """The large workloads' solver configuration on P2: FP32 CG inside FP64
    refinement, Chebyshev preconditioner (degree 8, ratio 100), coarse
    correction of the Hartree CG."""
    from paper_2103_02824_amd import mlc
    S = CASES["nested"]()
    prob = Problem(S)
    st0, _ = initial_state(prob)
    ctx = mlc.Context(S, mlc.options(**dict(LIB_OPTS, precision=mlc.PREC_FP32_IR, precond=mlc.PC_CHEBYSHEV,
                                            cheb_degree=8, cheb_ratio=100.0, hartree_coarse=1)))
    ctx.set_state(st0.lam, st0.Phi, st0.w)
    rep = ctx.correction_step()
    assert rep["cg_relres_max"] <= 1e-12
    ref = correction_step(prob, st0, ORA_OPTS)
    assert relerr(ctx.probe("U", (ctx.n_dof, ctx.N)), ref.inter["fine"]["U"]) < 1e-8
    lam, Phi, w, rho = ctx.get_results()
    assert np.max(np.abs(lam - ref.state.lam)) < 1e-8, (lam, ref.state.lam)
    assert relerr(rho, ref.rho_nodal) < 1e-6
    ctx.close()


def test_p2_systems_in_a_batch(gpu):
    """A batch mixing two P2 systems and a P1 one (mlc_batch_*: the batched
    CG over every system's rows, the other phases per system with their own
    element kernels) reaches each system's checker results."""
    from paper_2103_02824_amd import mlc
    systems = [CASES["same_mesh"](), CASES["nested"](),
               tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=7)]
    kw = dict(LIB_OPTS, precision=mlc.PREC_FP32_IR, ir_inner_rtol=1e-4, precond=mlc.PC_CHEBYSHEV, cheb_degree=6,
              cheb_ratio=100.0, hartree_coarse=1)
    refs, ctxs = [], []
    for S in systems:
        prob = Problem(S)
        st0, _ = initial_state(prob)
        refs.append(correction_step(prob, st0, ORA_OPTS))
        ctx = mlc.Context(S, mlc.options(**kw))
        ctx.set_state(st0.lam, st0.Phi, st0.w)
        ctxs.append(ctx)
    print("case batch of two P2 systems and one P1 system", flush=True)
    batch = mlc.Batch(ctxs)
    reps, br = batch.step()
    for S, ctx, rep, ref in zip(systems, ctxs, reps, refs):
        assert rep["cg_relres_max"] <= 1e-12 * (1 + 1e-6)
        assert relerr(ctx.probe("U", (ctx.n_dof, ctx.N)), ref.inter["fine"]["U"]) < 1e-8
        lam, Phi, w, rho = ctx.get_results()
        assert np.max(np.abs(lam - ref.state.lam)) < 1e-8, (S.order, lam, ref.state.lam)
        assert relerr(rho, ref.rho_nodal) < 1e-6
    batch.close()
    for c in ctxs:
        c.close()
