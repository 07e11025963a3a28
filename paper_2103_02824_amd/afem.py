"""The adaptive loop of Algorithm 1 on the library (the outer loop around the
correction step): on each fine mesh, correction steps, then the residual
estimator (mlc_estimate), Doerfler marking (mlc_mark_dorfler), refinement of
the marked tets by tagged bisection (mlc_refine) and the transfer of the
state (Lambda, Phi, w) to the refined mesh (mlc_transfer_vertices). The
coarse mesh, and with it V_H, stays the same. This module only orders the
calls and moves arrays between them."""
from __future__ import annotations

import dataclasses

import numpy as np

from . import mlc


def interior_vertices(xyz, lo, hi):
    """Vertices off the box faces, ascending: the library's DoFs in the
    caller's order (the same face test as the library, per axis)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    lo3, hi3 = mlc.box3(lo), mlc.box3(hi)
    on = np.zeros(len(xyz), dtype=bool)
    for k in range(3):
        tol = 1e-12 * max(1.0, abs(lo3[k]), abs(hi3[k]))
        on |= (np.abs(xyz[:, k] - lo3[k]) <= tol) | (np.abs(xyz[:, k] - hi3[k]) <= tol)
    return np.nonzero(~on)[0]


def adapt(system, opts=None, theta=0.4, levels=3, steps=1, state=None, tags=None, init=(1e-10, 200),
          progress=None, tol=None):
    """Run `levels` meshes of the adaptive loop from system's fine mesh.

    opts: library options (estimator is switched on); theta: Doerfler
    parameter (0.4 in Section 4); steps: correction steps per mesh, or with
    tol the most steps per mesh, stopping once the eigenvalues change by less
    than tol between two steps (the outer iteration of Algorithm 1 run to
    convergence on each mesh, as the iteration counts of Section 4 are); state:
    optional (lam, Phi, w) on the first mesh (host arrays or device tensors;
    else mlc_initial_state with init = (tol, maxit)); tags: bisection tags of
    the first mesh's tets (default 3, right for a Kuhn-ordered mesh).
    Returns (levels: list of dicts with the mesh sizes, eigenvalues, the
    estimate sqrt(sum eta^2), the marked count and the step reports; the last
    context, still open)."""
    import torch

    o = opts if opts is not None else mlc.options()
    o.estimator = 1
    S = system
    tg = np.full(len(S.tets), 3, dtype=np.int8) if tags is None else np.asarray(tags, dtype=np.int8)
    ctx = mlc.Context(S, o)
    if state is None:
        ctx.initial_state(*init)
    else:
        ctx.set_state(*state)
    out = []
    for lev in range(levels):
        reps = []
        lam_prev = ctx.get_results()[0] if tol is not None else None
        for _ in range(steps):
            reps.append(ctx.correction_step())
            if tol is not None:
                lam_now = ctx.get_results()[0]
                done = float(np.max(np.abs(lam_now - lam_prev))) < tol
                lam_prev = lam_now
                if done:
                    break
        eta2 = ctx.estimate().cpu().numpy()
        lam, Phi, w, _ = ctx.get_results_device()
        rec = {"level": lev, "n_dof": ctx.n_dof, "n_tets": ctx.n_tets, "lam": lam.copy(),
               "eta": float(np.sqrt(eta2.sum())), "reports": reps, "marked": 0, "outer": len(reps),
               "inner": [int(r["inner_iters"]) for r in reps]}
        out.append(rec)
        if progress:
            progress(rec)
        if lev == levels - 1:
            break
        mark, k = mlc.mark_dorfler(eta2, theta)
        rec["marked"] = k
        r = mlc.refine(S.xyz, S.tets, tg, mark)
        nv_old, N = len(S.xyz), ctx.N
        V = torch.zeros((len(r["xyz"]), N + 1), dtype=torch.float64, device=ctx.device)
        old_int = torch.as_tensor(interior_vertices(S.xyz, S.lo, S.hi), device=ctx.device)
        V[old_int, :N] = Phi
        V[:nv_old, N] = w
        mlc.transfer_vertices(V, nv_old, r["parents"], r["batch_ptr"], stream=ctx.stream)
        S = dataclasses.replace(S, xyz=r["xyz"], tets=r["tets"])
        tg = r["tags"]
        ctx.close()
        ctx = mlc.Context(S, o)
        new_int = torch.as_tensor(interior_vertices(S.xyz, S.lo, S.hi), device=ctx.device)
        ctx.set_state(lam, V[new_int, :N].contiguous(), V[:, N].contiguous())
    return out, ctx
