"""The adaptive loop on the GPU against the checker: the residual estimator
per tet on the checker's states, the transfer of nodal values to a bisected
mesh, and whole adaptive runs (estimate, mark, refine, transfer, correction
steps) level by level."""
import numpy as np
import pytest

from inputs.meshgen import AdaptiveMesh
from inputs.systems import lih_small, tiny_system
from oracle import afem
from oracle.mlc import Options, Problem
from oracle.scf import initial_state

pytestmark = pytest.mark.gpu

LIB_OPTS = dict(cg_rtol=1e-12, poisson_rtol=1e-13, inner_tol=1e-11)
CASES = {
    "tiny2": lambda: tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=7),
    "lih_small": lih_small,
}


@pytest.mark.parametrize("case", list(CASES))
def test_estimator_matches_the_checker(gpu, case):
    """eta^2 per tet of the checker's coarse-interpolated state, set into the
    library; per-tet relative difference below 1e-10 of the largest."""
    from paper_2103_02824_amd import mlc
    S = CASES[case]()
    prob = Problem(S)
    st0, _ = initial_state(prob)
    ref = afem.estimator(prob.fine, st0.lam, prob.fine.full(st0.Phi), afem.veff_qp(prob, st0))
    print(f"case {case}: estimator on {len(S.tets)} tets", flush=True)
    ctx = mlc.Context(S, mlc.options(**LIB_OPTS, estimator=1))
    ctx.set_state(st0.lam, st0.Phi, st0.w)
    got = ctx.estimate().cpu().numpy()
    ctx.close()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"eta^2: max relative difference {err:.2e}, total {np.sqrt(ref.sum()):.4e}", flush=True)
    assert err < 1e-10


def test_estimate_needs_the_option_and_a_state(gpu):
    from paper_2103_02824_amd import mlc
    S = CASES["tiny2"]()
    ctx = mlc.Context(S, mlc.options(**LIB_OPTS))
    with pytest.raises(mlc.MlcError):
        ctx.estimate()                           # no state
    st0, _ = initial_state(Problem(S))
    ctx.set_state(st0.lam, st0.Phi, st0.w)
    with pytest.raises(mlc.MlcError):
        ctx.estimate()                           # created without the estimator option
    ctx.close()


def test_transfer_matches_the_checker(gpu):
    """Seeded nodal values (3 columns) on a Kuhn mesh refined twice at random
    marks: the library's batch-by-batch transfer equals the checker's
    sequential one bit for bit (both are the mean of the two parents)."""
    import torch
    from paper_2103_02824_amd import mlc
    from inputs.meshgen import kuhn_mesh
    xyz, tets = kuhn_mesh(3, -1.0, 1.0)
    X, T, G = xyz, tets.astype(np.int32), np.full(len(tets), 3, dtype=np.int8)
    rng = np.random.default_rng(21)
    vals = rng.normal(size=(len(X), 3))
    for step in range(2):
        r = mlc.refine(X, T, G, rng.random(len(T)) < 0.2)
        ref = afem.transfer(vals, len(r["xyz"]), r["parents"])
        V = torch.zeros((len(r["xyz"]), 3), dtype=torch.float64, device="cuda")
        V[:len(X)] = torch.as_tensor(vals, device="cuda")
        mlc.transfer_vertices(V, len(X), r["parents"], r["batch_ptr"])
        assert np.array_equal(V.cpu().numpy(), ref)
        X, T, G, vals = r["xyz"], r["tets"], r["tags"], ref


@pytest.mark.parametrize("case", ["tiny2", "tiny3"])
def test_adaptive_loop_matches_the_checker(gpu, case):
    """Three meshes of the adaptive loop (theta 0.4, one correction step
    each) from the checker's initial state: on every mesh the library and
    the checker have the same number of tets and DoFs (the same marks, so
    the same refined meshes), eigenvalues within 1e-8 and estimates within
    1e-8 relative, and the mesh grows. Random two-atom clusters on Kuhn
    meshes (tags 3 to start): no symmetry, so no two tets tie in eta^2 at the
    marking threshold."""
    from paper_2103_02824_amd import afem as lafem
    from paper_2103_02824_amd import mlc
    S = (CASES["tiny2"]() if case == "tiny2" else
         tiny_system(n_fine=10, n_coarse=5, box=5.0, nonlinear=True, n_orbitals=3, seed=11))
    prob = Problem(S)
    st0, _ = initial_state(prob)
    am = AdaptiveMesh(S.xyz, S.tets)

    def refine(mark):
        am.refine(mark)
        return am.xyz.copy(), am.tets.copy(), am.new_parents.copy()

    ref = afem.adapt(S, Options(), 0.4, 3, 1, st0, refine)
    print(f"case {case}: adaptive loop, 3 meshes", flush=True)
    got, ctx = lafem.adapt(S, mlc.options(**LIB_OPTS), theta=0.4, levels=3, steps=1,
                           state=(st0.lam, st0.Phi, st0.w))
    ctx.close()
    for g, r in zip(got, ref):
        print(f"level {g['level']}: tets {g['n_tets']} / {r['n_tets']}, lam {g['lam']} / {r['lam']}, "
              f"eta {g['eta']:.6e} / {r['eta']:.6e}", flush=True)
        assert g["n_tets"] == r["n_tets"] and g["n_dof"] == r["n_dof"]
        assert np.max(np.abs(g["lam"] - r["lam"])) < 1e-8
        assert abs(g["eta"] - r["eta"]) < 1e-8 * r["eta"]
        if r["mark"] is not None:
            assert g["marked"] == int(r["mark"].sum())
    assert got[-1]["n_tets"] > got[0]["n_tets"]
