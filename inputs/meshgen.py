"""Seeded tetrahedral meshes: a structured Kuhn base mesh and its graded
refinement by tagged (Maubach) newest-vertex bisection.

This module produces inputs only (vertex coordinates and tetrahedra). It
holds no finite-element arithmetic: no basis functions, quadrature,
assembly or prolongation. Both the CPU checker and the GPU library derive
those from the arrays returned here.

The paper discretises on shape-regular, conforming tetrahedral meshes whose
coarsest level is a uniform mesh of 24576 tetrahedra (= 16^3 cubes x 6,
Section 4) refined locally toward the nuclei (Section 2, AFEM). The graded
meshes here follow that shape: a Kuhn cube mesh, then conforming bisection
wherever the longest edge of a tetrahedron exceeds a target size that grows
with the distance to the nearest nucleus. Every fine tetrahedron lies inside
exactly one base tetrahedron, so the base mesh is a nested coarse mesh.
"""
from __future__ import annotations

import hashlib
import itertools
import os

import numpy as np
from scipy.spatial import cKDTree

# Kuhn subdivision of the unit cube: one tetrahedron per permutation of the
# axes, x0 = corner (0,0,0), x_{k} = x_{k-1} + e_{perm[k-1]}, x3 = (1,1,1).
_PERMS = list(itertools.permutations(range(3)))


def kuhn_mesh(n, lo, hi):
    """Structured Kuhn mesh of the box [lo,hi]^3 with n^3 cubes.

    Returns (xyz float64 (V,3), tets int64 (6 n^3, 4)). Vertices are numbered
    lexicographically, x fastest: id = i + (n+1) j + (n+1)^2 k. Every tet is
    stored in Kuhn order (x0, x1, x2, x3) with x0-x3 the cube diagonal, which
    is the tag-3 vertex order that tagged bisection starts from.
    """
    n = int(n)
    g = np.linspace(lo, hi, n + 1)
    k, j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    xyz = np.stack([g[i.ravel()], g[j.ravel()], g[k.ravel()]], axis=1)

    def vid(ii, jj, kk):
        return ii + (n + 1) * (jj + (n + 1) * kk)

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = []
    for perm in _PERMS:
        off = np.zeros((4, 3), dtype=np.int64)
        for s in range(1, 4):
            off[s] = off[s - 1]
            off[s, perm[s - 1]] += 1
        tets.append(np.stack([vid(ci + off[s, 0], cj + off[s, 1], ck + off[s, 2]) for s in range(4)], axis=1))
    # order: cube-major, then permutation
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int64)
    return xyz, tets


class _Bisector:
    """Conforming tagged bisection (Maubach) of a Kuhn mesh, vectorised.

    A tagged tet (x0,x1,x2,x3; k) is cut at the midpoint z of edge x0-xk into
      (x0..x_{k-1}, z, x_{k+1}..x3) and (x1..x_k, z, x_{k+1}..x3),
    both tagged k-1 (or 3 after tag 1). Starting from Kuhn order with tag 3
    the refinement of neighbouring tets is compatible, and closing every
    hanging edge by further bisection yields a conforming mesh.
    """

    def __init__(self, xyz, tets, full_scan=False):
        self.full_scan = full_scan  # search every tet for hanging edges (reference behaviour)
        self.xyz = [np.asarray(xyz, dtype=np.float64)]
        self.nv = len(xyz)
        self.tets = np.asarray(tets, dtype=np.int64).copy()
        self.tags = np.full(len(tets), 3, dtype=np.int8)
        self.mid_keys = np.zeros(0, dtype=np.int64)  # sorted edge keys
        self.mid_ids = np.zeros(0, dtype=np.int64)
        self.key_base = np.int64(1) << np.int64(31)
        # after a bisection: endpoints of the edges it split and the number of
        # children it appended (the only places a new hanging edge can be)
        self.split_ends = None
        self.n_children = 0
        self.parents = []  # (lo, hi) edge of each created vertex, in creation (id) order

    def _key(self, a, b):
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        return lo * self.key_base + hi

    def coords(self):
        if len(self.xyz) > 1:
            self.xyz = [np.concatenate(self.xyz, axis=0)]
        return self.xyz[0]

    def bisect(self, mask):
        idx = np.nonzero(mask)[0]
        if len(idx) == 0:
            return 0
        T = self.tets[idx]
        k = self.tags[idx].astype(np.int64)
        a = T[:, 0]
        b = T[np.arange(len(idx)), k]
        keys = self._key(a, b)
        # look up existing midpoints, create the missing ones
        pos = np.searchsorted(self.mid_keys, keys)
        pos_c = np.minimum(pos, max(len(self.mid_keys) - 1, 0))
        found = (len(self.mid_keys) > 0) & (self.mid_keys[pos_c] == keys) if len(self.mid_keys) else np.zeros(len(keys), bool)
        new_keys, inv = np.unique(keys[~found], return_inverse=True)
        mids = np.empty(len(keys), dtype=np.int64)
        if len(self.mid_keys):
            mids[found] = self.mid_ids[pos_c[found]]
        if len(new_keys):
            lo = new_keys // self.key_base
            hi = new_keys % self.key_base
            X = self.coords()
            newxyz = 0.5 * (X[lo] + X[hi])
            new_ids = self.nv + np.arange(len(new_keys), dtype=np.int64)
            self.nv += len(new_keys)
            self.parents.append(np.stack([lo, hi], axis=1))
            self.xyz.append(newxyz)
            mids[~found] = new_ids[inv]
            allk = np.concatenate([self.mid_keys, new_keys])
            alli = np.concatenate([self.mid_ids, new_ids])
            order = np.argsort(allk, kind="stable")
            self.mid_keys = allk[order]
            self.mid_ids = alli[order]
        z = mids
        c1 = np.empty_like(T)
        c2 = np.empty_like(T)
        for kk in (1, 2, 3):
            s = k == kk
            if not np.any(s):
                continue
            Ts = T[s]
            zs = z[s]
            # child 1: (x0..x_{k-1}, z, x_{k+1}..x3)
            ch1 = Ts.copy()
            ch1[:, kk] = zs
            # child 2: (x1..x_k, z, x_{k+1}..x3)
            ch2 = np.empty_like(Ts)
            ch2[:, :kk] = Ts[:, 1:kk + 1]
            ch2[:, kk] = zs
            ch2[:, kk + 1:] = Ts[:, kk + 1:]
            c1[s] = ch1
            c2[s] = ch2
        ends = np.zeros(self.nv, dtype=bool)
        ends[a] = True
        ends[b] = True
        self.split_ends = ends
        self.n_children = 2 * len(idx)
        newtag = np.where(k > 1, k - 1, 3).astype(np.int8)
        keep = np.ones(len(self.tets), dtype=bool)
        keep[idx] = False
        self.tets = np.concatenate([self.tets[keep], c1, c2], axis=0)
        self.tags = np.concatenate([self.tags[keep], newtag, newtag])
        return len(idx)

    def hanging(self):
        """Mask of tets that own an edge whose midpoint already exists.

        Called on a mesh that had no hanging edge before the last bisection:
        a tet that bisection did not create can then only hang on an edge it
        split, so only the new children and the tets with a vertex at an end
        of a split edge are searched."""
        if len(self.mid_keys) == 0:
            return np.zeros(len(self.tets), dtype=bool)
        cand = None
        if self.split_ends is not None and not self.full_scan:
            cand = self.split_ends[self.tets].any(axis=1)
            cand[len(self.tets) - self.n_children:] = True
            cand = np.nonzero(cand)[0]
        T = self.tets if cand is None else self.tets[cand]
        hang_c = np.zeros(len(T), dtype=bool)
        for (p, q) in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
            keys = self._key(T[:, p], T[:, q])
            pos = np.searchsorted(self.mid_keys, keys)
            pos = np.minimum(pos, len(self.mid_keys) - 1)
            hang_c |= self.mid_keys[pos] == keys
        if cand is None:
            return hang_c
        hang = np.zeros(len(self.tets), dtype=bool)
        hang[cand] = hang_c
        return hang

    def close(self, max_rounds=1000):
        for _ in range(max_rounds):
            h = self.hanging()
            if not np.any(h):
                return
            self.bisect(h)
        raise RuntimeError("bisection closure did not terminate")


class AdaptiveMesh:
    """A conforming tetrahedral mesh refined step by step by tagged bisection
    of marked tets plus the closure that removes hanging edges (the refinement
    of an adaptive loop). Mesh data only: after each refine(), xyz and tets
    describe the new mesh and new_parents holds, for each vertex created by
    that refine() in id order, the two ends of the edge it bisects."""

    def __init__(self, xyz, tets):
        self._b = _Bisector(xyz, tets)
        self.new_parents = np.zeros((0, 2), dtype=np.int64)

    @classmethod
    def kuhn(cls, n, lo, hi):
        return cls(*kuhn_mesh(n, lo, hi))

    @property
    def xyz(self):
        return self._b.coords()

    @property
    def tets(self):
        return self._b.tets

    def refine(self, marked):
        """Bisect the marked tets once (marked: boolean mask over the current
        tets), then close the mesh."""
        marked = np.asarray(marked, dtype=bool)
        if marked.shape != (len(self._b.tets),):
            raise ValueError("marked must be a mask over the current tets")
        nv0 = self._b.nv
        start = len(self._b.parents)
        self._b.bisect(marked)
        self._b.close()
        par = self._b.parents[start:]
        self.new_parents = np.concatenate(par, axis=0) if par else np.zeros((0, 2), dtype=np.int64)
        assert len(self.new_parents) == self._b.nv - nv0
        return self


def _longest_edge(xyz, tets):
    P = xyz[tets]
    h2 = np.zeros(len(tets))
    for (p, q) in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        d = P[:, p] - P[:, q]
        h2 = np.maximum(h2, np.einsum("ij,ij->i", d, d))
    return np.sqrt(h2)


def _refine_to(B, C, h0, kappa, h_min, h_max, max_levels=200, progress=None):
    tree = cKDTree(np.asarray(C, dtype=np.float64).reshape(-1, 3))
    for level in range(max_levels):
        X = B.coords()
        cen = X[B.tets].mean(axis=1)
        d, _ = tree.query(cen)  # distance to the nearest centre
        target = np.clip(h0 + kappa * d, h_min, h_max)
        mark = _longest_edge(X, B.tets) > target * (1.0 + 1e-12)
        if not np.any(mark):
            return
        B.bisect(mark)
        B.close()
        if progress:
            progress(f"mesh refinement level {level}: {B.nv} vertices, {len(B.tets)} tets")


def graded_mesh(n_base, lo, hi, centres, h0, kappa, h_min, h_max=np.inf, coarse=None, progress=None,
                full_scan=False):
    """Kuhn base mesh refined until every tet satisfies
    longest_edge <= clip(h0 + kappa * d(centroid), h_min, h_max), d = distance
    of the centroid to the nearest centre.

    coarse: None (the coarse mesh is the Kuhn base) or a tuple
    (h0, kappa, h_min, h_max) of a first, milder grading; the fine mesh then
    refines that graded mesh further, so the two meshes stay nested.
    Returns (xyz, tets, coarse_xyz, coarse_tets). Coarse vertices keep their
    ids in the fine mesh. progress: optional callable given one line per
    refinement level (long generations stay visibly alive). full_scan: search
    every tet for hanging edges after each bisection (the reference for the
    restricted search, which must give the same mesh).
    """
    C = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    cache = _cache_path(n_base, lo, hi, C, h0, kappa, h_min, h_max, coarse)
    if cache is not None and os.path.exists(cache):
        with np.load(cache, allow_pickle=False) as z:
            return z["xyz"], z["tets"], z["cxyz"], z["ctets"]
    bxyz, btets = kuhn_mesh(n_base, lo, hi)
    B = _Bisector(bxyz, btets, full_scan=full_scan)
    if coarse is not None:
        _refine_to(B, C, *coarse, progress=progress)
    cxyz = B.coords().copy()
    ctets = B.tets.copy()
    _refine_to(B, C, h0, kappa, h_min, h_max, progress=progress)
    X = B.coords()
    out = (X.copy(), B.tets.copy(), cxyz, ctets)
    if cache is not None and not full_scan:
        tmp = cache + ".tmp.npz"
        np.savez(tmp, xyz=out[0], tets=out[1], cxyz=out[2], ctets=out[3])
        os.replace(tmp, cache)
    return out


def _cache_path(*params):
    """File of a generated mesh in the directory named by the environment
    variable MLC_MESH_CACHE (None when it is unset): generating the largest
    meshes takes minutes, and a second process on the same machine can load
    them instead. The name is a hash of every generation parameter."""
    d = os.environ.get("MLC_MESH_CACHE")
    if not d:
        return None
    os.makedirs(d, exist_ok=True)
    h = hashlib.sha256(repr([np.asarray(p).tolist() if isinstance(p, np.ndarray) else p
                             for p in params]).encode()).hexdigest()[:24]
    return os.path.join(d, f"graded_{h}.npz")


def boundary_mask(xyz, lo, hi, tol=1e-12):
    """Vertices on the box boundary (where the homogeneous Dirichlet condition
    applies). Pure geometry of the input box."""
    on = np.zeros(len(xyz), dtype=bool)
    for ax in range(3):
        on |= np.abs(xyz[:, ax] - lo) <= tol * max(1.0, abs(lo))
        on |= np.abs(xyz[:, ax] - hi) <= tol * max(1.0, abs(hi))
    return on
