"""The seeded mesh generator: after each bisection it searches for hanging
edges only around the edges that bisection split. That must give exactly the
mesh that searching every tet gives, and the result must be a conforming
nested mesh: every interior face in exactly two tets, every boundary face in
one box plane, and every fine tet inside one coarse tet."""
import math

import numpy as np
import pytest

from inputs.meshgen import graded_mesh
from inputs.systems import random_cluster


@pytest.mark.parametrize("atoms,hw,box,n_base,h,coarse", [
    (4, 3.0, 15.0, 8, 0.5, (1.4, 0.6, 1.4)),
    (40, 8.0, 25.0, 12, 0.6, None),
])
def test_restricted_hanging_search_gives_the_full_scan_mesh(atoms, hw, box, n_base, h, coarse):
    R, _ = random_cluster(0, atoms, hw, 1.5 if atoms == 4 else 1.8)
    hm = 2 * box / n_base * math.sqrt(3.0)
    cg = None if coarse is None else (*coarse, hm)
    kw = dict(h0=h, kappa=h, h_min=h, h_max=hm, coarse=cg)
    fast = graded_mesh(n_base, -box, box, R, **kw)
    ref = graded_mesh(n_base, -box, box, R, full_scan=True, **kw)
    for a, b in zip(fast, ref):
        assert a.shape == b.shape and np.array_equal(a, b)
    xyz, tets = fast[0], fast[1]
    # conforming: every edge's midpoint (if a vertex) would make it hanging; each
    # interior face is shared by exactly two tets
    faces = np.sort(np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 3]],
                                    tets[:, [1, 2, 3]]]), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert counts.max() <= 2
    on = np.zeros(len(xyz), bool)
    for ax in range(3):
        on |= np.isclose(xyz[:, ax], -box) | np.isclose(xyz[:, ax], box)
    uf, cnt = np.unique(faces, axis=0, return_counts=True)
    single = uf[cnt == 1]
    assert np.all(on[single].all(axis=1)), "a face seen once must lie on the box boundary"
    # ... and on one box face: its three vertices share one coordinate at -box or +box
    P = xyz[single]
    one_plane = np.zeros(len(single), bool)
    for ax in range(3):
        for side in (-box, box):
            one_plane |= np.all(np.isclose(P[:, :, ax], side), axis=1)
    assert one_plane.all(), "a boundary face must lie in one box plane"
    # nested: every fine tet lies in one coarse tet (its centroid's), all four vertices inside it
    cxyz, ctets = fast[2], fast[3]
    cP = cxyz[ctets]
    Jinv = np.linalg.inv(np.stack([cP[:, 1] - cP[:, 0], cP[:, 2] - cP[:, 0], cP[:, 3] - cP[:, 0]], axis=2))
    from scipy.spatial import cKDTree
    fP = xyz[tets]
    cen = fP.mean(axis=1)
    _, cand = cKDTree(cP.mean(axis=1)).query(cen, k=min(32, len(ctets)))
    host = np.full(len(tets), -1)
    best = np.full(len(tets), -np.inf)
    for c in range(cand.shape[1]):
        t = cand[:, c]
        l123 = np.einsum("nij,nj->ni", Jinv[t], cen - cP[t, 0])
        m = np.minimum(l123.min(axis=1), 1.0 - l123.sum(axis=1))
        better = m > best
        best, host = np.where(better, m, best), np.where(better, t, host)
    assert np.all(best > 0), "every fine centroid strictly inside a coarse tet"
    for a in range(4):
        l123 = np.einsum("nij,nj->ni", Jinv[host], fP[:, a] - cP[host, 0])
        m = np.minimum(l123.min(axis=1), 1.0 - l123.sum(axis=1))
        assert m.min() > -1e-10, "a fine tet crosses a coarse face"
