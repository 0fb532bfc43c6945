"""Column meshes of hexahedra with one level of 2:1 refinement (Sec. 3.1 "Meshing").

The mesh is a structured grid of ``nx x ny`` columns, each ``nz`` elements high
(the column organisation of Sec. 3.1, where every column spans the full
height).  A *refined* column is split isotropically 2x2x2 in every element,
so it becomes 2x2 fine columns of ``2*nz`` elements; neighbouring columns
differ by at most one level (the 2:1 condition of Sec. 3.1).  Fine elements
next to unrefined columns have nonconforming (hanging) faces or edges
(Sec. 3.2.1, figure "hanging").  With ``refine_from = z0 > 0`` only layers
z0 and above of a refined column are split (an octree-like mesh whose
columns no longer span the full height in one level); the fine elements of
the lowest refined layer then also hang on the coarse element below them
through their -z face.  With ``periodic = (px, py)`` the lateral boundaries
of a periodic axis are identified (the slab problem of Sec. 4.3): nodes at
logical x = nx are the nodes at x = 0, and columns on opposite boundaries are
neighbours, with hanging faces across the boundary where their levels
differ; ``period`` holds the physical translation between the boundaries.
With ``base_frames=True`` every basal node gets a local frame whose third
axis is the unit normal of the bed surface there (tangents: the x-direction
tangent of the bed and normal x tangent), and the normal component is
flagged in ``dmask``: u . n = 0 on a curved base (eq. (robin)) by rotation.

Everything here is topology and node placement:

* element list (level, integer cell at that level), in column order;
* the global (independent) nodes, i.e. all element Gauss-Lobatto positions
  except the dependent ones: every fine-element node lying on a face or edge
  of a coarse neighbour is dependent, also where it coincides with a coarse
  node (Sec. 3.2.1);
* ``elem_nodes``: for each element slot the global node id; a dependent slot
  holds the id of the coarse neighbour's node at the *same local index*
  along the face/edge tangent directions ("parent value in the child slot"),
  which the GPU engine then interpolates in place;
* ``cmask``: per element the child position inside its refined parent and
  flags for hanging faces / edges (bit layout below);
* logical node positions (in coarse-cell units) and physical coordinates
  from a caller-supplied geometry map.

``cmask`` bit layout (shared contract with the engine's C header):

* bits 0..2  : child position (hx, hy, hz) in {0,1}^3 of a refined element;
* bits 3..8  : hanging face  -x, +x, -y, +y, -z, +z;
* bits 9..20 : hanging edge  4*dir + s0 + 2*s1, dir 0/1/2 = parallel to x/y/z,
  (s0, s1) = side (0 low, 1 high) along the two other axes in increasing
  axis order.  An edge bit is set only when no hanging face already covers it.

No quadrature, basis functions or interpolation weights appear here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import sqrt
from typing import Callable, Optional

import numpy as np

# Gauss-Lobatto points on [-1, 1]: the endpoints and the roots of P_k'
# (closed forms; the node set of Sec. 3.2.1).
GLL_CLOSED_FORM = {
    1: (-1.0, 1.0),
    2: (-1.0, 0.0, 1.0),
    3: (-1.0, -1.0 / sqrt(5.0), 1.0 / sqrt(5.0), 1.0),
    4: (-1.0, -sqrt(3.0 / 7.0), 0.0, sqrt(3.0 / 7.0), 1.0),
}

FACE_BIT0 = 3
EDGE_BIT0 = 9


@dataclass
class ColumnMesh:
    k: int
    nx: int
    ny: int
    nz: int
    refined: np.ndarray          # (nx, ny) bool
    elem_level: np.ndarray       # int8  [n_el]
    elem_cell: np.ndarray        # int32 [n_el, 3] cell index at the element's level
    elem_nodes: np.ndarray       # int32 [n_el, (k+1)^3], slot a = a0 + P*(a1 + P*a2)
    cmask: np.ndarray            # uint32 [n_el]
    node_logical: np.ndarray     # float64 [n_nodes, 3] in coarse-cell units
    coords: np.ndarray           # float64 [3, n_nodes]
    bface_elem: np.ndarray       # int32 [n_bface], elements whose zeta=-1 face is basal
    dmask: np.ndarray            # uint8 [3, n_nodes]
    extent: tuple = (1.0, 1.0, 1.0)
    meta: dict = field(default_factory=dict)
    pspace: str = "P"            # pressure space: "P" = P_{k-1}, "Q" = Q_{k-2} (a label only)
    periodic: tuple = (False, False)
    period: tuple = (0.0, 0.0, 0.0)  # physical translation between identified boundaries, 0 = none
    frame_nodes: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))   # [n_frames]
    frames: np.ndarray = field(default_factory=lambda: np.zeros((0, 3, 3)))         # [n_frames, 3, 3]

    @property
    def P(self) -> int:
        return self.k + 1

    @property
    def n_el(self) -> int:
        return int(self.elem_level.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.node_logical.shape[0])

    @property
    def n_bface(self) -> int:
        return int(self.bface_elem.shape[0])

    @property
    def n_p(self) -> int:
        """Pressure unknowns per element: dim P_{k-1} or dim Q_{k-2} on the reference cube."""
        k = self.k
        return (k - 1) ** 3 if self.pspace == "Q" else k * (k + 1) * (k + 2) // 6

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes + self.n_el * self.n_p

    def elem_box(self):
        """Logical box of each element: (lo[n_el,3], size[n_el]) in coarse-cell units."""
        size = np.where(self.elem_level == 0, 1.0, 0.5)
        lo = self.elem_cell.astype(np.float64) * size[:, None]
        return lo, size

    def submesh_elements(self, elems: np.ndarray) -> np.ndarray:
        return np.asarray(elems, dtype=np.int64)


def _axis_tables(k: int):
    """Per-axis position codes.

    Every node position along one axis is ``cell + frac`` with ``cell`` a
    coarse cell and ``frac`` one of the finitely many Gauss-Lobatto fractions
    of a coarse cell or of its two halves.  ``U`` lists those fractions in
    [0, 1); a position is encoded as ``cell*len(U) + index``.  Returns
    (U, off, idx) with off/idx of shape [2 levels][2 halves][k+1].
    """
    xi = np.asarray(GLL_CLOSED_FORM[k], dtype=np.float64)
    fr = np.empty((2, 2, k + 1))
    fr[0, 0] = (xi + 1.0) / 2.0
    fr[0, 1] = fr[0, 0]
    fr[1, 0] = (xi + 1.0) / 4.0
    fr[1, 1] = 0.5 + (xi + 1.0) / 4.0
    off = (fr >= 1.0 - 1e-14).astype(np.int64)
    frac = np.where(off == 1, 0.0, fr)
    # merge equal fractions through a rounded key, but keep the unrounded values
    keys, first = np.unique(np.round(frac.ravel(), 13), return_index=True)
    U = frac.ravel()[first]
    idx = np.searchsorted(keys, np.round(frac, 13))
    assert np.allclose(U[idx], frac, rtol=0, atol=1e-15)
    return U, off, idx


def _codes(level, cell, k, U, off, idx):
    """Codes [n, k+1] of the k+1 node positions of cells along one axis."""
    level = np.asarray(level)
    cell = np.asarray(cell, dtype=np.int64)
    coarse = np.where(level == 0, cell, cell // 2)
    half = np.where(level == 0, 0, cell % 2)
    o = off[level, half]            # [n, k+1]
    ix = idx[level, half]
    return (coarse[:, None] + o) * len(U) + ix


def column_mesh(k: int, nx: int, ny: int, nz: int,
                refined: Optional[np.ndarray] = None,
                geometry: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                extent=(1.0, 1.0, 1.0),
                base_normal_dirichlet: bool = False, pspace: str = "P", refine_from: int = 0,
                periodic=(False, False), base_frames: bool = False) -> ColumnMesh:
    """Build a column mesh.

    ``geometry`` maps logical positions [n, 3] (coarse-cell units, x in
    [0, nx], ...) to physical coordinates [n, 3].  Default: the axis-aligned
    box ``extent`` (affine slab).  ``base_normal_dirichlet`` flags the
    z-component of every base node (logical z = 0) in ``dmask``.  ``pspace``
    labels the pressure space the mesh is used with ("P" or "Q").  ``refine_from``
    = z0 > 0 refines the marked columns only from coarse layer z0 upwards (an
    octree-like mesh, T_xyz of the slab tests): the fine elements of layer 2 z0
    then hang on the coarse elements below through their -z face.
    """
    if pspace not in ("P", "Q"):
        raise ValueError("pspace must be 'P' or 'Q'")
    if k not in (2, 3, 4):
        raise ValueError("k must be 2, 3 or 4")
    P = k + 1
    if refined is None:
        refined = np.zeros((nx, ny), dtype=bool)
    refined = np.asarray(refined, dtype=bool)
    assert refined.shape == (nx, ny)
    z0 = int(refine_from)
    assert 0 <= z0 < nz
    per = (bool(periodic[0]), bool(periodic[1]))
    ncell = (nx, ny)
    # an element must be shorter than half a period along a periodic axis
    assert all(ncell[d] >= 3 for d in range(2) if per[d]), "periodic axes need at least 3 columns"

    def wrap(c, d):
        return np.mod(c, ncell[d]) if per[d] else c

    # ---- element list, column by column (y-major, then x), layers innermost
    lev, cx, cy, cz = [], [], [], []
    for j in range(ny):
        for i in range(nx):
            if not refined[i, j]:
                lev.append(np.zeros(nz, np.int8))
                cx.append(np.full(nz, i)); cy.append(np.full(nz, j)); cz.append(np.arange(nz))
            else:
                if z0 > 0:                      # coarse layers below the refined part
                    lev.append(np.zeros(z0, np.int8))
                    cx.append(np.full(z0, i)); cy.append(np.full(z0, j)); cz.append(np.arange(z0))
                nf = 2 * (nz - z0)
                for hy in (0, 1):
                    for hx in (0, 1):
                        lev.append(np.ones(nf, np.int8))
                        cx.append(np.full(nf, 2 * i + hx))
                        cy.append(np.full(nf, 2 * j + hy))
                        cz.append(np.arange(2 * z0, 2 * nz))
    elem_level = np.concatenate(lev)
    elem_cell = np.stack([np.concatenate(cx), np.concatenate(cy), np.concatenate(cz)], 1).astype(np.int32)
    n_el = elem_level.shape[0]

    # ---- hanging faces / edges of fine elements
    fine = elem_level == 1
    cmask = np.zeros(n_el, dtype=np.uint32)
    I, J, L = (elem_cell[:, d].astype(np.int64) for d in range(3))
    ci, cj = np.where(fine, I // 2, I), np.where(fine, J // 2, J)
    hx, hy, hz = I % 2, J % 2, L % 2

    def coarse_col(ii, jj):
        ii, jj = wrap(ii, 0), wrap(jj, 1)
        inside = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        iic, jjc = np.clip(ii, 0, nx - 1), np.clip(jj, 0, ny - 1)
        return inside & ~refined[iic, jjc]

    face = np.zeros((n_el, 6), dtype=bool)
    face[:, 0] = fine & (hx == 0) & coarse_col(ci - 1, cj)
    face[:, 1] = fine & (hx == 1) & coarse_col(ci + 1, cj)
    face[:, 2] = fine & (hy == 0) & coarse_col(ci, cj - 1)
    face[:, 3] = fine & (hy == 1) & coarse_col(ci, cj + 1)
    face[:, 4] = fine & (L == 2 * z0) & (z0 > 0)          # fine on top of the coarse part of the column
    # z-parallel edges at the column corners (sx, sy)
    zedge = np.zeros((n_el, 4), dtype=bool)
    for sy in (0, 1):
        for sx in (0, 1):
            zedge[:, sx + 2 * sy] = (fine & (hx == sx) & (hy == sy)
                                     & coarse_col(ci + 2 * sx - 1, cj + 2 * sy - 1)
                                     & ~face[:, sx] & ~face[:, 2 + sy])
    cmask |= np.where(fine, (hx | (hy << 1) | (hz << 2)), 0).astype(np.uint32)
    for f in range(6):
        cmask |= (face[:, f].astype(np.uint32) << np.uint32(FACE_BIT0 + f))
    for e in range(4):
        cmask |= (zedge[:, e].astype(np.uint32) << np.uint32(EDGE_BIT0 + 8 + e))

    # ---- position codes and slot keys
    U, off, idx = _axis_tables(k)
    nU = len(U)
    Cx, Cz = (nx + 1) * nU, (nz + 1) * nU
    codes = [_codes(elem_level, elem_cell[:, d], k, U, off, idx) for d in range(3)]  # [n_el, P]
    for d in range(2):
        if per[d]:
            codes[d] = np.mod(codes[d], ncell[d] * nU)       # logical position n_d is position 0
    a = np.arange(P)
    a0 = np.tile(a, P * P)
    a1 = np.tile(np.repeat(a, P), P)
    a2 = np.repeat(a, P * P)
    slot_key = ((codes[1][:, a1] * Cx + codes[0][:, a0]) * Cz + codes[2][:, a2])  # [n_el, P^3]

    # dependent slots
    dep = np.zeros((n_el, P ** 3), dtype=bool)
    on = [a0 == 0, a0 == k, a1 == 0, a1 == k]
    for f in range(4):
        dep |= face[:, f][:, None] & on[f][None, :]
    dep |= face[:, 4][:, None] & (a2 == 0)[None, :]
    for sy in (0, 1):
        for sx in (0, 1):
            dep |= zedge[:, sx + 2 * sy][:, None] & (on[sx] & on[2 + sy])[None, :]

    keys = np.unique(slot_key[~dep])
    elem_nodes = np.full((n_el, P ** 3), -1, dtype=np.int64)
    elem_nodes[~dep] = np.searchsorted(keys, slot_key[~dep])

    # parent slot of each dependent slot: neighbour coarse element, opposite
    # index along the face/edge normal(s), same index along the tangent(s)
    if dep.any():
        e_idx, s_idx = np.nonzero(dep)
        pa = [a0[s_idx].copy(), a1[s_idx].copy(), a2[s_idx].copy()]
        pc = [ci[e_idx].copy(), cj[e_idx].copy(), L[e_idx] // 2]
        done = np.zeros(e_idx.shape[0], dtype=bool)
        for f in range(4):
            d, side = f // 2, f % 2
            sel = ~done & face[e_idx, f] & (pa[d] == side * k)
            pc[d][sel] += (2 * side - 1)
            pa[d][sel] = (1 - side) * k
            done |= sel
        sel = ~done & face[e_idx, 4] & (pa[2] == 0)          # -z face: the coarse element below
        pc[2][sel] -= 1
        pa[2][sel] = k
        done |= sel
        for sy in (0, 1):
            for sx in (0, 1):
                sel = (~done & zedge[e_idx, sx + 2 * sy]
                       & (pa[0] == sx * k) & (pa[1] == sy * k))
                pc[0][sel] += 2 * sx - 1
                pc[1][sel] += 2 * sy - 1
                pa[0][sel] = (1 - sx) * k
                pa[1][sel] = (1 - sy) * k
                done |= sel
        assert done.all()
        lev0 = np.zeros(e_idx.shape[0], dtype=np.int64)
        pcode = []
        for d in range(3):
            c = _codes(lev0, wrap(pc[d], d) if d < 2 else pc[d], k, U, off, idx)          # [m, P]
            c = np.mod(c, ncell[d] * nU) if d < 2 and per[d] else c
            pcode.append(c[np.arange(c.shape[0]), pa[d]])
        pkey = (pcode[1] * Cx + pcode[0]) * Cz + pcode[2]
        pos = np.searchsorted(keys, pkey)
        assert np.all(pos < keys.shape[0]) and np.all(keys[np.minimum(pos, keys.shape[0] - 1)] == pkey), \
            "parent node of a hanging slot is not an independent node"
        elem_nodes[e_idx, s_idx] = pos
    assert (elem_nodes >= 0).all()

    # ---- logical and physical node positions
    kz = keys % Cz
    kyx = keys // Cz
    kx, ky = kyx % Cx, kyx // Cx
    node_logical = np.stack([kc // nU + U[kc % nU] for kc in (kx, ky, kz)], 1)
    if geometry is None:
        Lx, Ly, Lz = extent
        geometry = lambda lg: lg * np.array([Lx / nx, Ly / ny, Lz / nz])
    phys = np.asarray(geometry(node_logical), dtype=np.float64)
    coords = np.ascontiguousarray(phys.T)
    period = [0.0, 0.0, 0.0]
    for d in range(2):
        if per[d]:
            shift = np.zeros(3)
            shift[d] = ncell[d]
            dx = np.asarray(geometry(node_logical + shift), dtype=np.float64) - phys
            period[d] = float(dx[0, d])
            assert period[d] > 0 and np.allclose(dx, np.eye(3)[d] * period[d], rtol=0, atol=1e-12 * period[d]), \
                "geometry is not periodic along a periodic axis"


    bface_elem = np.nonzero(elem_cell[:, 2] == 0)[0].astype(np.int32)
    dmask = np.zeros((3, keys.shape[0]), dtype=np.uint8)
    if base_normal_dirichlet:
        dmask[2, node_logical[:, 2] == 0.0] = 1
    frame_nodes = np.zeros(0, np.int32)
    frames = np.zeros((0, 3, 3))
    if base_frames:
        assert not base_normal_dirichlet
        frame_nodes = np.nonzero(node_logical[:, 2] == 0.0)[0].astype(np.int32)
        lg = node_logical[frame_nodes]
        h = 1e-5                                     # central differences of the geometry map
        ex, ey = np.array([h, 0.0, 0.0]), np.array([0.0, h, 0.0])
        tx = (np.asarray(geometry(lg + ex)) - np.asarray(geometry(lg - ex))) / (2 * h)
        ty = (np.asarray(geometry(lg + ey)) - np.asarray(geometry(lg - ey))) / (2 * h)
        nrm = np.cross(tx, ty)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        t1 = tx - np.sum(tx * nrm, axis=1, keepdims=True) * nrm
        t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
        t2 = np.cross(nrm, t1)
        frames = np.stack([t1, t2, nrm], axis=2)     # columns: local axes
        dmask[2, frame_nodes] = 1

    return ColumnMesh(k=k, nx=nx, ny=ny, nz=nz, refined=refined,
                      elem_level=elem_level, elem_cell=elem_cell,
                      elem_nodes=elem_nodes.astype(np.int32), cmask=cmask,
                      node_logical=node_logical, coords=coords,
                      bface_elem=bface_elem, dmask=dmask, extent=tuple(extent), pspace=pspace,
                      periodic=per, period=tuple(period), frame_nodes=frame_nodes, frames=frames)


def random_refined_columns(nx: int, ny: int, fraction: float, rng: np.random.Generator) -> np.ndarray:
    """A seeded random set of round(fraction*nx*ny) refined columns."""
    n = int(round(fraction * nx * ny))
    flat = np.zeros(nx * ny, dtype=bool)
    flat[rng.choice(nx * ny, size=n, replace=False)] = True
    return flat.reshape(nx, ny)
