"""Dense-quadrature FP64 Newton-Stokes residual, Jacobian and VJP (oracle; test infrastructure only).

Definitions followed (Sec. 2 and 3 of the paper):

* strain rate D(u) = (grad u + grad u^T)/2, second invariant II = D:D/2;
* Glen law, eq. (glen): viscosity mu = B (II + eps)^((1-n)/(2n)); here
  B = B0 exp(-logA_e / n) per element;
* weak residual, eq. (weak):
  r(v, q) = int mu D(v):D(u) - p div v - q div u + int_base beta Tv.Tu - f(v),
  T = I - n n^T the tangential projector of eq. (robin);
* Newton linearisation, eq. (newton) with the 4th-order tensor of eq. (rank4):
  C(u) = mu (I - (n-1)/(2n) D (x) D / (II + eps));
  with picard=True the Picard operator of Sec. 2.3 instead: C(u) = mu I (the
  D (x) D part dropped, the viscosity kept);
* the saddle-point Jacobian A(u) = [[F, B^T], [B, 0]] (Sec. 4.1) assembled as
  sum_e R_e^T A_e R_e (Sec. 3.2.1);
* normal Dirichlet condition u.n = 0 on flat bases (eq. (robin)) as a
  component mask P: state and residual use P u, residual rows of masked
  components are u itself, Jacobian J_c = P K P + (I - P);
* on a curved base the same condition by nodal frames: a node with frame Q
  holds u_hat, u = Q u_hat, so with Q the block-diagonal change of variables
  the operator is J_c = P Q^T K Q P + (I - P) and the residual
  P Q^T r(Q P u_hat) + (I - P) u_hat, the mask acting on local components;
* energy of the appendix (with the friction coefficient beta written into the
  boundary term): Pi(u) = int 2n/(n+1) B (II+eps)^((n+1)/(2n)) + 1/2 int beta |Tu|^2 - f(u).

Element matrices are formed by full tensor quadrature over dense basis
tables; nothing is sum-factorised.  All arithmetic is analytic in u (no
absolute values or conjugates), so complex-step differentiation works.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .reference import ReferenceElement
from .restriction import build_restriction, element_coordinates


def glen_viscosity(II, Be, n, eps):
    """mu = B (II + eps)^((1-n)/(2n)) -- eq. (glen)."""
    return Be * (II + eps) ** ((1.0 - n) / (2.0 * n))


def newton_tensor(D0, mu, II, n, eps):
    """C(u) of eq. (rank4) as a 9x9 matrix acting on row-major 3x3 tensors."""
    I9 = np.eye(9)
    d = D0.reshape(9)
    return mu * (I9 - (n - 1.0) / (2.0 * n) * np.outer(d, d) / (II + eps))


class StokesOracle:
    """FP64 oracle on a column mesh (or on a subset of its elements).

    With ``elems`` given, only those elements (and the basal faces they own)
    are assembled; rows of the global result are then exact only where every
    incident element is in the subset (row-sampled checks).
    """

    def __init__(self, mesh, n=3.0, eps=1e-10, B0=0.5, logA=None, beta=None, body=(0.0, 0.0, 0.0),
                 elems=None, picard=False):
        self.mesh = mesh
        self.picard = bool(picard)
        self.n, self.eps, self.B0 = float(n), float(eps), float(B0)
        self.ref = ReferenceElement(mesh.k, getattr(mesh, "pspace", "P"))
        ref = self.ref
        self.S = ref.P ** 3
        self.elems = np.arange(mesh.n_el) if elems is None else np.asarray(elems, dtype=np.int64)
        self.logA = np.zeros(mesh.n_el) if logA is None else np.asarray(logA, dtype=np.float64)
        self.beta = np.zeros(mesh.n_bface) if beta is None else np.asarray(beta, dtype=np.float64)
        self.body = np.asarray(body, dtype=np.float64)
        self.pmask = 1.0 - mesh.dmask.astype(np.float64)          # [3, n_nodes]
        # nodal frames: Qn[n] with the local axes as columns (identity for nodes without one)
        fnodes = getattr(mesh, "frame_nodes", None)
        self.Qn = None
        if fnodes is not None and len(fnodes):
            self.Qn = np.tile(np.eye(3), (mesh.n_nodes, 1, 1))
            self.Qn[np.asarray(fnodes)] = np.asarray(mesh.frames, dtype=np.float64).reshape(-1, 3, 3)
        E = self.elems.shape[0]

        self.R = build_restriction(mesh, ref, self.elems)          # [E*S, n_nodes]
        # geometry: X_e = R_e X (watertight), J = dX/dxi at quadrature points
        Xs = element_coordinates(mesh, ref, self.R, self.elems)
        # the map's derivative is translation invariant: differentiate coordinates relative
        # to each element's first node so that rounding stays relative to the element size
        Xs = Xs - Xs[:, :1, :]
        J = np.einsum("esi,qsr->eqir", Xs, ref.dPhi)
        self.detJ = np.linalg.det(J)
        if np.any(self.detJ <= 0):
            raise ValueError("inverted element (detJ <= 0 at a quadrature point)")
        Jinv = np.linalg.inv(J)                                     # [e, q, r, i] = d xi_r / d x_i
        self.Gp = np.einsum("qsr,eqri->eqsi", ref.dPhi, Jinv)       # physical basis gradients
        self.W = ref.wq[None, :] * self.detJ                        # w_q detJ_q

        # basal faces owned by the subset
        where = {int(e): f for f, e in enumerate(mesh.bface_elem)}
        self.fl = np.array([i for i, e in enumerate(self.elems) if int(e) in where], dtype=np.int64)
        self.fid = np.array([where[int(self.elems[i])] for i in self.fl], dtype=np.int64)
        if self.fl.size:
            Xf = Xs[self.fl]
            xa = np.einsum("fsi,gs->fgi", Xf, ref.dPhif[:, :, 0])
            xb = np.einsum("fsi,gs->fgi", Xf, ref.dPhif[:, :, 1])
            cr = np.cross(xa, xb)
            area = np.sqrt(np.einsum("fgi,fgi->fg", cr, cr))
            self.fn = cr / area[..., None]
            self.Wf = ref.wf[None, :] * area
        else:
            self.fn = np.zeros((0, ref.P ** 2, 3))
            self.Wf = np.zeros((0, ref.P ** 2))
        self.Be = self.B0 * np.exp(-self.logA[self.elems] / self.n)
        self._K = None

    # ------------------------------------------------------------------ helpers
    def to_cartesian(self, v):
        """Q v: node vectors [3, n_nodes] from local to Cartesian components."""
        return v if self.Qn is None else np.einsum("nij,jn->in", self.Qn, v)

    def to_local(self, v):
        """Q^T v: node vectors [3, n_nodes] from Cartesian to local components."""
        return v if self.Qn is None else np.einsum("nji,jn->in", self.Qn, v)

    def gather(self, v_u):
        """R_e Q (P v) for every element of the subset: [E, S, 3]."""
        return (self.R @ self.to_cartesian(self.pmask * v_u).T).reshape(self.elems.shape[0], self.S, 3)

    def _tangential(self, v):
        """T v = v - n (n.v) at face quadrature points."""
        return v - self.fn * np.einsum("fgc,fgc->fg", self.fn, v)[..., None]

    def scatter(self, r_e):
        """Q^T sum_e R_e^T r_e for r_e [E, 3, S] -> [3, n_nodes] (local components)."""
        out = np.stack([self.R.T @ r_e[:, c, :].reshape(-1) for c in range(3)])
        return self.to_local(out)

    # ------------------------------------------------------------------ state
    def set_state(self, u, p):
        self.u = np.asarray(u)
        self.p = np.asarray(p)
        ue = self.gather(self.u)
        G = np.einsum("esc,eqsi->eqci", ue, self.Gp)
        self.D0 = 0.5 * (G + np.swapaxes(G, 2, 3))
        self.II = 0.5 * np.einsum("eqij,eqij->eq", self.D0, self.D0)
        self.mu = glen_viscosity(self.II, self.Be[:, None], self.n, self.eps)
        self.cpr = self.mu * (self.n - 1.0) / (2.0 * self.n) / (self.II + self.eps)
        if self.picard:
            self.cpr = np.zeros_like(self.cpr)
        self.pq = np.einsum("em,qm->eq", self.p[self.elems], self.ref.Psi)
        self.divu = np.einsum("eqcc->eq", G)
        if self.fl.size:
            self.uf = np.einsum("gs,fsc->fgc", self.ref.Phif, ue[self.fl])
        self._K = None

    # ------------------------------------------------------------------ residual
    def residual(self, f_u=None):
        """Residual of eq. (weak) with Dirichlet rows: (r_u [3, n_nodes], r_p [n_el, n_p])."""
        W = self.W
        r_e = (np.einsum("eq,eqci,eqsi->ecs", W * self.mu, self.D0, self.Gp)
               - np.einsum("eq,eqsc->ecs", W * self.pq, self.Gp))
        if self.fl.size:
            tb = self.Wf * self.beta[self.fid][:, None]
            rb = np.einsum("fg,gs,fgc->fcs", tb, self.ref.Phif, self._tangential(self.uf))
            r_e = r_e.astype(np.result_type(r_e, rb))
            np.add.at(r_e, self.fl, rb)
        if np.any(self.body != 0.0):
            r_e = r_e - np.einsum("eq,c,qs->ecs", W, self.body, self.ref.Phi)
        r_u = self.scatter(r_e)
        if f_u is not None:
            r_u = r_u - f_u
        r_u = self.pmask * r_u + (1.0 - self.pmask) * self.u
        r_p = np.zeros((self.mesh.n_el, self.ref.n_p), dtype=r_u.dtype)
        r_p[self.elems] = -np.einsum("eq,qm,eq->em", W, self.ref.Psi, self.divu)
        return r_u, r_p

    def load_vector(self):
        """f(v) = int b . v for the constant body force b: [3, n_nodes] (without Dirichlet masking)."""
        f_e = np.einsum("eq,c,qs->ecs", self.W, self.body, self.ref.Phi)
        return self.scatter(f_e)

    # ------------------------------------------------------------------ element matrices
    def element_matrices(self, sl=slice(None)):
        """Dense A_e [E, 3S, 3S] (velocity block incl. basal term) and B_e [E, n_p, 3S]."""
        S = self.S
        Gp, W = self.Gp[sl], self.W[sl]
        E = Gp.shape[0]
        Wmu = W * self.mu[sl]
        Wc = W * self.cpr[sl]
        Z = np.ascontiguousarray(np.transpose(Gp, (0, 3, 2, 1)))        # [e, i, s, q] = d_i phi_s at q
        V = np.einsum("eqci,eqsi->ecsq", self.D0[sl], Gp)               # [e, c, s, q] = (D0 . grad phi_s)_c
        # K_st = sum_q W mu grad phi_s . grad phi_t
        K = sum(np.matmul(Z[:, i] * Wmu[:, None, :], np.swapaxes(Z[:, i], 1, 2)) for i in range(3))
        A = np.empty((E, 3, S, 3, S))
        for c in range(3):
            for d in range(3):
                # 1/2 sum_q W mu d_d phi_s d_c phi_t  -  sum_q W c' (D0 grad phi_s)_c (D0 grad phi_t)_d
                A[:, c, :, d, :] = (0.5 * np.matmul(Z[:, d] * Wmu[:, None, :], np.swapaxes(Z[:, c], 1, 2))
                                    - np.matmul(V[:, c] * Wc[:, None, :], np.swapaxes(V[:, d], 1, 2)))
            A[:, c, :, c, :] += 0.5 * K
        # B_e[m, (d, t)] = - sum_q W psi_m d_d phi_t
        Bm = -np.einsum("eq,qm,edtq->emdt", W, self.ref.Psi, Z, optimize=True)
        E = A.shape[0]
        A = A.reshape(E, 3 * S, 3 * S)
        # basal Robin term  sum_fq w|S| beta phi_s phi_t (I - n n^T)_cd
        idx = np.arange(self.elems.shape[0])[sl]
        pos = {int(v): i for i, v in enumerate(idx)}
        for j, el in enumerate(self.fl):
            if int(el) in pos:
                tb = self.Wf[j] * self.beta[self.fid[j]]
                T = np.eye(3)[None] - np.einsum("gc,gd->gcd", self.fn[j], self.fn[j])
                M = np.einsum("g,gs,gt,gcd->csdt", tb, self.ref.Phif, self.ref.Phif, T)
                A[pos[int(el)]] += M.reshape(3 * S, 3 * S)
        return A, Bm.reshape(E, self.ref.n_p, 3 * S)

    def _R3(self):
        """Restriction on velocity dofs, R_e Q: rows (e, c, s) -> global c*n_nodes + node (local components)."""
        R = self.R.tocoo()
        E, S, N = self.elems.shape[0], self.S, self.mesh.n_nodes
        e, s = R.row // S, R.row % S
        rows = np.concatenate([e * 3 * S + c * S + s for c in range(3)])
        cols = np.concatenate([c * N + R.col for c in range(3)])
        vals = np.concatenate([R.data] * 3)
        R3 = sp.csr_matrix((vals, (rows, cols)), shape=(E * 3 * S, 3 * N))
        if self.Qn is None:
            return R3
        # block-diagonal change of variables: Cartesian (c, n) <- local (d, n), weight Q_n[c, d]
        n = np.arange(N)
        qr = np.concatenate([c * N + n for c in range(3) for d in range(3)])
        qc = np.concatenate([d * N + n for c in range(3) for d in range(3)])
        qv = np.concatenate([self.Qn[:, c, d] for c in range(3) for d in range(3)])
        return R3 @ sp.csr_matrix((qv, (qr, qc)), shape=(3 * N, 3 * N))

    def jacobian(self, chunk=128):
        """Assembled J_c = P K P + (I - P) of shape [n_dof, n_dof] (CSR), velocity dofs first."""
        if self._K is not None:
            return self._K
        mesh, S = self.mesh, self.S
        N, npp = mesh.n_nodes, self.ref.n_p
        R3 = self._R3()
        E = self.elems.shape[0]
        Kuu = sp.csr_matrix((3 * N, 3 * N))
        Bg = sp.csr_matrix((mesh.n_el * npp, 3 * N))
        for c0 in range(0, E, chunk):
            sl = slice(c0, min(E, c0 + chunk))
            A, Bm = self.element_matrices(sl)
            m = A.shape[0]
            R3c = R3[c0 * 3 * S:(c0 + m) * 3 * S]
            Abd = sp.block_diag(list(A), format="csr")
            Kuu = Kuu + (R3c.T @ (Abd @ R3c))
            rows = (self.elems[sl][:, None] * npp + np.arange(npp)[None, :]).ravel()
            Bbd = sp.block_diag(list(Bm), format="csr")
            Pm = sp.csr_matrix((np.ones(rows.shape[0]), (rows, np.arange(rows.shape[0]))),
                               shape=(mesh.n_el * npp, rows.shape[0]))
            Bg = Bg + Pm @ (Bbd @ R3c)
        K = sp.bmat([[Kuu, Bg.T], [Bg, None]], format="csr")
        pm = np.concatenate([self.pmask.reshape(-1), np.ones(mesh.n_el * npp)])
        Pd = sp.diags(pm)
        self._K = (Pd @ K @ Pd + sp.diags(1.0 - pm)).tocsr()
        return self._K

    def jacobian_apply(self, x_u, x_p):
        K = self.jacobian()
        y = K @ np.concatenate([np.asarray(x_u).reshape(-1), np.asarray(x_p).reshape(-1)])
        N = self.mesh.n_nodes
        return y[:3 * N].reshape(3, N), y[3 * N:].reshape(self.mesh.n_el, self.ref.n_p)

    # ------------------------------------------------------------------ VJP
    def vjp(self, w_u, w_p):
        """Cotangent w -> (J_c^T w, d<w,r>/dlogA [n_el], d<w,r>/dbeta [n_bface])."""
        K = self.jacobian()
        N = self.mesh.n_nodes
        g = K.T @ np.concatenate([np.asarray(w_u).reshape(-1), np.asarray(w_p).reshape(-1)])
        g_u, g_p = g[:3 * N].reshape(3, N), g[3 * N:].reshape(self.mesh.n_el, self.ref.n_p)
        we = self.gather(w_u)
        Gw = np.einsum("esc,eqsi->eqci", we, self.Gp)
        Dw = 0.5 * (Gw + np.swapaxes(Gw, 2, 3))
        g_logA = np.zeros(self.mesh.n_el)
        g_logA[self.elems] = -(1.0 / self.n) * np.einsum("eq,eqij,eqij->e", self.W * self.mu, self.D0, Dw)
        g_beta = np.zeros(self.mesh.n_bface)
        if self.fl.size:
            wf = np.einsum("gs,fsc->fgc", self.ref.Phif, we[self.fl])
            g_beta[self.fid] = np.einsum("fg,fgc,fgc->f", self.Wf, self._tangential(self.uf),
                                         self._tangential(wf))
        return g_u, g_p, g_logA, g_beta

    # ------------------------------------------------------------------ energy
    def energy(self, u):
        """Pi(Pu) of the appendix (beta inside the boundary term)."""
        n, eps = self.n, self.eps
        ue = self.gather(u)
        G = np.einsum("esc,eqsi->eqci", ue, self.Gp)
        D = 0.5 * (G + np.swapaxes(G, 2, 3))
        II = 0.5 * np.einsum("eqij,eqij->eq", D, D)
        val = np.sum(self.W * (2 * n / (n + 1)) * self.Be[:, None] * (II + eps) ** ((n + 1) / (2 * n)))
        if self.fl.size:
            uf = self._tangential(np.einsum("gs,fsc->fgc", self.ref.Phif, ue[self.fl]))
            val = val + 0.5 * np.sum(self.Wf * self.beta[self.fid][:, None] * np.einsum("fgc,fgc->fg", uf, uf))
        if np.any(self.body != 0.0):
            uq = np.einsum("qs,esc->eqc", self.ref.Phi, ue)
            val = val - np.sum(self.W[..., None] * uq * self.body)
        return val
