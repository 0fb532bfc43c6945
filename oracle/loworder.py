"""Low-order approximation F~ of the velocity block on the Gauss-Lobatto sub-grid (oracle; test
infrastructure only).

Sec. 5, "Construction of low-order approximation F~": the (k+1)^3 Gauss-Lobatto nodes of element K_e
are taken as the corners of a k x k x k grid of trilinear (Q1) sub-cells, and F~_e is the matrix of the
bilinear form of F on that grid.  Read here as follows (the paper gives the construction in words):

* sub-cell geometry: the trilinear map of the sub-cell's 8 corners, the physical positions of the
  element's nodes X_e = R_e X (watertight, as the high-order map);
* quadrature: the 2-point Gauss-Lobatto rule per direction on each sub-cell (the paper's F~_GL, whose
  points are the sub-cell corners, i.e. the element's nodes), weight 1/8 per corner of the unit cube
  times |det J| of the sub-cell map at the corner;
* integrand: the Newton tensor of eq. (rank4), C(u) = mu (I - (n-1)/(2n) D0 (x) D0 / (II + eps)), with
  mu, D0, II evaluated at each node from the high-order state u_h differentiated inside K_e (the
  Picard operator drops the D0 (x) D0 part), tested with the sym-gradients of the Q1 basis;
* basal Robin term of eq. (robin) on the element's base: the k x k bilinear sub-faces with the 2 x 2
  Gauss-Lobatto rule, giving per base node the lumped block sum (1/4) |x_s x x_t| beta (I - n n^T)
  over the sub-faces at that node, n the sub-face's unit normal at the node;
* assembly with the high-order restriction, F~ = sum_e R_e^T F~_e R_e (the "R_i" construction of
  figure "interp" (a) at nonconforming faces), the nodal frames and the Dirichlet rows as for F:
  J~_c = P Q^T F~ Q P + (I - P).

Element matrices are formed from the dense sub-cell matrices of this definition, one sub-cell and
one quadrature corner at a time.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .reference import gll_nodes, lagrange
from .restriction import element_coordinates
from .stokes import glen_viscosity

_CORNERS = list(itertools.product((0, 1), repeat=3))      # (dx, dy, dz), x fastest below


def _q1_ref_gradients():
    """grad_s psi_c(q) for the 8 trilinear basis functions c at the 8 corners q of [0, 1]^3: [q, c, 3]."""
    G = np.zeros((8, 8, 3))
    for qi, q in enumerate(_CORNERS):
        for ci, c in enumerate(_CORNERS):
            for d in range(3):
                # psi_c(s) = prod_e (s_e if c_e else 1 - s_e); d/ds_d at s = q
                val = 1.0 if c[d] else -1.0
                for e in range(3):
                    if e != d:
                        val *= (q[e] if c[e] else 1.0 - q[e])
                G[qi, ci, d] = val
    return G


def nodal_coefficients(oracle):
    """mu, kappa' = mu (n-1)/(2n)/(II+eps) (0 for Picard) and D0 at every node of every element of the
    oracle's subset, from the high-order state differentiated inside the element: [E, P^3], [E, P^3],
    [E, P^3, 3, 3]."""
    ref, mesh = oracle.ref, oracle.mesh
    P = ref.P
    xi = gll_nodes(ref.k)
    _, dV = lagrange(xi, xi)                         # dV[g, a] = l_a'(xi_g)
    V = np.eye(P)
    i0, i1, i2 = ref.lex
    dPhiN = np.empty((P ** 3, P ** 3, 3))            # d phi_a / d xi_r at node g
    dPhiN[:, :, 0] = dV[i0][:, i0] * V[i1][:, i1] * V[i2][:, i2]
    dPhiN[:, :, 1] = V[i0][:, i0] * dV[i1][:, i1] * V[i2][:, i2]
    dPhiN[:, :, 2] = V[i0][:, i0] * V[i1][:, i1] * dV[i2][:, i2]
    X = element_coordinates(mesh, ref, oracle.R, oracle.elems)
    X = X - X[:, :1, :]
    J = np.einsum("esi,gsr->egir", X, dPhiN)
    Jinv = np.linalg.inv(J)                          # [e, g, r, i]
    ue = oracle.gather(oracle.u)
    G = np.einsum("esc,gsr,egri->egci", ue, dPhiN, Jinv)
    D0 = 0.5 * (G + np.swapaxes(G, 2, 3))
    II = 0.5 * np.einsum("egij,egij->eg", D0, D0)
    mu = glen_viscosity(II, oracle.Be[:, None], oracle.n, oracle.eps)
    kap = np.zeros_like(mu) if oracle.picard else mu * (oracle.n - 1.0) / (2.0 * oracle.n) / (II + oracle.eps)
    return mu, kap, D0, X


def element_matrices(oracle):
    """Dense F~_e [E, 3 P^3, 3 P^3] (rows/cols (c, a): component-major, node index a) of the oracle's
    subset, including the lumped basal term."""
    ref = oracle.ref
    P, k = ref.P, ref.k
    S = P ** 3
    mu, kap, D0, X = nodal_coefficients(oracle)
    Gs = _q1_ref_gradients()
    E = X.shape[0]
    A = np.zeros((E, 3, S, 3, S))
    node = lambda i, j, l: i + P * (j + P * l)
    eye = np.eye(3)
    for (i, j, l) in itertools.product(range(k), repeat=3):
        nodes = np.array([node(i + c[0], j + c[1], l + c[2]) for c in _CORNERS])
        Xc = X[:, nodes, :]                                          # [E, 8, 3]
        for qi in range(8):
            g = nodes[qi]
            Jq = np.einsum("eci,cr->eir", Xc, Gs[qi])                  # dx_i / ds_r at the corner
            det = np.linalg.det(Jq)
            if np.any(det == 0):
                raise ValueError("degenerate sub-cell")
            grad = np.einsum("cr,eri->eci", Gs[qi], np.linalg.inv(Jq))  # physical grad psi_c: [E, 8, 3]
            w = np.abs(det) / 8.0
            # E(c, comp) = sym(grad psi_c (x) e_comp): [E, 8, comp, 3, 3]
            Ecm = 0.5 * (np.einsum("eci,mj->ecmij", grad, eye) + np.einsum("ecj,mi->ecmij", grad, eye))
            s = np.einsum("ecmij,eij->ecm", Ecm, D0[:, g])             # D0 : E(c, comp)
            blk = (np.einsum("e,ecmij,ednij->ecmdn", w * mu[:, g], Ecm, Ecm)
                   - np.einsum("e,ecm,edn->ecmdn", w * kap[:, g], s, s))
            for a_i, a in enumerate(nodes):
                for b_i, b in enumerate(nodes):
                    A[:, :, a, :, b] += blk[:, a_i, :, b_i, :]
    # lumped basal sub-faces
    for j_f, el in enumerate(oracle.fl):
        beta = oracle.beta[oracle.fid[j_f]]
        Xe = X[el]
        for (i, j) in itertools.product(range(k), repeat=2):
            for (qx, qy) in itertools.product((0, 1), repeat=2):
                a = node(i + qx, j + qy, 0)
                xs = Xe[node(i + 1, j + qy, 0)] - Xe[node(i, j + qy, 0)]
                xt = Xe[node(i + qx, j + 1, 0)] - Xe[node(i + qx, j, 0)]
                cr = np.cross(xs, xt)
                area = np.linalg.norm(cr)
                nrm = cr / area
                A[el, :, a, :, a] += 0.25 * area * beta * (eye - np.outer(nrm, nrm))
    return A.reshape(E, 3 * S, 3 * S)


def low_order_matrix(oracle):
    """Assembled J~_c [3 n_nodes, 3 n_nodes] (CSR): sum_e R_e^T F~_e R_e with frames and Dirichlet rows,
    velocity block only.  With a subset of elements the rows are exact where every incident element is
    in the subset."""
    mesh = oracle.mesh
    N = mesh.n_nodes
    A = element_matrices(oracle)
    R3 = oracle._R3()
    K = R3.T @ (sp.block_diag(list(A), format="csr") @ R3)
    pm = oracle.pmask.reshape(-1)
    Pd = sp.diags(pm)
    return (Pd @ K @ Pd + sp.diags(1.0 - pm)).tocsr()
