"""The host parts of the library's adaptive loop (no GPU): Doerfler marking
against the checker's, and the library's bisection refinement against the
mesh generator's (the same tagged bisection and closure written twice: the
meshes must agree vertex for vertex and tet for tet)."""
import numpy as np
import pytest

from inputs.meshgen import AdaptiveMesh, kuhn_mesh
from oracle import afem
from paper_2103_02824_amd import mlc


def test_dorfler_marking_matches_the_checker_including_ties():
    rng = np.random.default_rng(4)
    for trial in range(60):
        n = int(rng.integers(1, 400))
        eta2 = rng.exponential(size=n)
        if trial % 3 == 0:
            eta2 = np.round(eta2, 1)            # many ties: broken by index on both sides
        theta = float(rng.uniform(0.05, 1.0))
        m, k = mlc.mark_dorfler(eta2, theta)
        ref = afem.dorfler_mark(eta2, theta)
        assert np.array_equal(m, ref) and k == int(ref.sum())


def test_dorfler_marking_rejects_bad_input():
    with pytest.raises(mlc.MlcError):
        mlc.mark_dorfler(np.array([1.0, -1.0]), 0.4)
    with pytest.raises(mlc.MlcError):
        mlc.mark_dorfler(np.array([1.0, np.nan]), 0.4)
    with pytest.raises(mlc.MlcError):
        mlc.mark_dorfler(np.array([1.0, 2.0]), 0.0)


def test_refinement_matches_the_mesh_generator():
    """Random marks on a Kuhn mesh over four refinements: the library's
    vertices, tets, tags and new-vertex parents equal the generator's; every
    refined mesh is conforming (each interior face in exactly two tets) and
    keeps the volume."""
    xyz, tets = kuhn_mesh(3, -1.0, 1.0)
    am = AdaptiveMesh(xyz, tets)
    X, T, G = xyz.copy(), tets.astype(np.int32), np.full(len(tets), 3, dtype=np.int8)
    rng = np.random.default_rng(9)
    for step in range(4):
        mark = rng.random(len(T)) < 0.15
        am.refine(mark)
        r = mlc.refine(X, T, G, mark)
        assert np.array_equal(r["xyz"], am.xyz)
        assert np.array_equal(r["tets"], am.tets.astype(np.int32))
        assert np.array_equal(r["parents"], am.new_parents)
        assert r["batch_ptr"][0] == 0 and r["batch_ptr"][-1] == len(r["parents"])
        # each batch's parents were created before the batch
        nv0 = len(X)
        for b in range(len(r["batch_ptr"]) - 1):
            lo, hi = r["batch_ptr"][b], r["batch_ptr"][b + 1]
            assert np.all(r["parents"][lo:hi] < nv0 + lo)
        X, T, G = r["xyz"], r["tets"], r["tags"]
        P = X[T]
        vol = np.abs(np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6
        assert abs(vol.sum() - 8.0) < 1e-12
        faces = np.sort(np.concatenate([np.delete(T, a, axis=1) for a in range(4)]), axis=1)
        _, cnt = np.unique(faces, axis=0, return_counts=True)
        assert cnt.max() == 2


def test_refinement_rejects_bad_input():
    xyz, tets = kuhn_mesh(1, 0.0, 1.0)
    T = tets.astype(np.int32)
    G = np.full(len(T), 3, dtype=np.int8)
    with pytest.raises(mlc.MlcError):
        mlc.refine(xyz, T, np.zeros(len(T), dtype=np.int8), np.ones(len(T), bool))   # tag 0
    bad = T.copy()
    bad[0, 0] = len(xyz)
    with pytest.raises(mlc.MlcError):
        mlc.refine(xyz, bad, G, np.ones(len(T), bool))
