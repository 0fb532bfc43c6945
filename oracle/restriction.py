"""Element restriction matrices R_e by point location (oracle; test infrastructure only).

Sec. 3.2.1 (and the caption of figure "hanging"): the values at the nodes of
element K_e are obtained from the global nodal vector by R_e.  A node of
K_e that is a global node gives a unit row.  A dependent (hanging) node lies
on a face or edge of a coarser neighbour; its value is the neighbour's
polynomial evaluated there, so its row holds the neighbour's Lagrange basis
at that point (tensor-product interpolation, dense along the interface).

This module finds every element node in the mesh's logical coordinates:
first as a global node (nearest-neighbour search), otherwise by locating it
in an unrefined element whose logical box contains it, mapping it to that
element's reference coordinates and evaluating all of its basis functions.
It does not use the mesh's ``elem_nodes`` or ``cmask`` arrays.

Periodic lateral axes (the slab problem of Sec. 4.3): a logical position and
its translates by the number of columns along that axis are the same point.
Nodes are matched modulo that translation, and a point is located in a
coarse element through its translate nearest to the element.  The element
geometry then takes, for every node that a slot depends on, the node's
periodic image nearest to the slot.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .reference import ReferenceElement

_TOL = 1e-9


def _periods(mesh):
    """Logical period per axis (number of columns), 0 where the axis is not periodic."""
    per = getattr(mesh, "periodic", (False, False))
    return np.array([mesh.nx if per[0] else 0, mesh.ny if per[1] else 0, 0], dtype=np.float64)


class _Locator:
    def __init__(self, mesh, ref: ReferenceElement):
        self.mesh, self.ref = mesh, ref
        self.per = _periods(mesh)
        self.tree = cKDTree(mesh.node_logical)
        self.lo, self.size = mesh.elem_box()
        lvl0 = np.nonzero(mesh.elem_level == 0)[0]
        self.coarse = {tuple(mesh.elem_cell[e]): e for e in lvl0}

    def canonical(self, pts):
        """Translate positions into [0, n) along periodic axes (n - tol counts as 0)."""
        out = np.array(pts, dtype=np.float64, copy=True)
        for d in range(3):
            n = self.per[d]
            if n > 0:
                v = np.mod(out[..., d], n)
                out[..., d] = np.where(v > n - _TOL, v - n, v)
        return out

    def slot_points(self, elems):
        i0, i1, i2 = self.ref.lex
        s = (self.ref.xi + 1.0) / 2.0
        frac = np.stack([s[i0], s[i1], s[i2]], 1)                 # [P^3, 3]
        return self.lo[elems][:, None, :] + self.size[elems][:, None, None] * frac[None]

    def match(self, pts):
        d, i = self.tree.query(self.canonical(pts), distance_upper_bound=_TOL)
        return np.where(np.isfinite(d), i, -1)

    def coarse_row(self, p):
        """(node ids, weights) of the unrefined element containing logical point p."""
        cand = [sorted({int(np.floor(p[d] - _TOL)), int(np.floor(p[d] + _TOL))}) for d in range(3)]
        for cell in itertools.product(*cand):
            cell = tuple(int(np.mod(c, self.per[d])) if self.per[d] > 0 else c for d, c in enumerate(cell))
            e = self.coarse.get(cell)
            if e is None:
                continue
            lo = self.lo[e]
            # the translate of p nearest to the element's centre
            q = p + self.per * np.round((lo + 0.5 - p) / np.where(self.per > 0, self.per, 1.0))
            if np.all(q >= lo - _TOL) and np.all(q <= lo + 1.0 + _TOL):
                xi = 2.0 * (q - lo) - 1.0
                w = self.ref.eval_basis(xi[None, :])[0]
                nodes = self.match(self.slot_points(np.array([e]))[0])
                if np.any(nodes < 0):
                    raise RuntimeError("coarse element with a node that is not a global node")
                keep = w != 0.0
                return nodes[keep], w[keep]
        raise RuntimeError(f"node at logical point {p} is neither global nor on an unrefined element")


def element_coordinates(mesh, ref: ReferenceElement, R: sp.csr_matrix, elems=None) -> np.ndarray:
    """Physical slot coordinates X_e = R_e X [len(elems), P^3, 3], each node entering through its
    periodic image nearest to the slot (plain R X without periodic axes)."""
    if elems is None:
        elems = np.arange(mesh.n_el)
    elems = np.asarray(elems, dtype=np.int64)
    loc = _Locator(mesh, ref)
    pts = loc.slot_points(elems).reshape(-1, 3)
    C = R.tocoo()
    X = np.zeros((pts.shape[0], 3))
    period = np.asarray(getattr(mesh, "period", (0.0, 0.0, 0.0)), dtype=np.float64)
    img = np.zeros((C.row.shape[0], 3))
    for d in range(3):
        if loc.per[d] > 0:
            img[:, d] = np.round((pts[C.row, d] - mesh.node_logical[C.col, d]) / loc.per[d])
    contrib = C.data[:, None] * (mesh.coords[:, C.col].T + img * period[None, :])
    np.add.at(X, C.row, contrib)
    return X.reshape(elems.shape[0], ref.P ** 3, 3)


def build_restriction(mesh, ref: ReferenceElement, elems=None) -> sp.csr_matrix:
    """Stacked restriction R = [R_e0; R_e1; ...] of shape [len(elems)*P^3, n_nodes]."""
    if elems is None:
        elems = np.arange(mesh.n_el)
    elems = np.asarray(elems, dtype=np.int64)
    loc = _Locator(mesh, ref)
    n_s = ref.P ** 3
    pts = loc.slot_points(elems).reshape(-1, 3)
    ids = loc.match(pts)
    rows = [np.nonzero(ids >= 0)[0]]
    cols = [ids[ids >= 0]]
    vals = [np.ones(rows[0].shape[0])]
    for r in np.nonzero(ids < 0)[0]:
        c, w = loc.coarse_row(pts[r])
        rows.append(np.full(c.shape[0], r))
        cols.append(c)
        vals.append(w)
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(elems.shape[0] * n_s, mesh.n_nodes))
    return R
