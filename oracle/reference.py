"""Reference-element tables, built directly from their definitions (oracle; test infrastructure only).

* Velocity: isoparametric Q_k Lagrange basis on the tensor Gauss-Lobatto
  nodes of [-1, 1]^3 (Sec. 3.2.1).  Gauss-Lobatto nodes are +-1 and the roots
  of P_k' (numpy's Legendre module).
* Quadrature: tensor Gauss-Legendre rule with k+1 points per direction (the
  paper says "Gauss nodes of order k"; read as k+1 points, exact for
  polynomials of degree 2k+1 per direction).
* Pressure, two spaces (Sec. 3.2.2):
  - "P": P_{k-1} on the reference cube, basis of products of normalised
    Legendre polynomials Lhat_i(x) Lhat_j(y) Lhat_l(z) with i+j+l <= k-1 and
    Lhat_i = sqrt((2i+1)/2) P_i, ordered by (i+j+l, l, j, i).  The paper does
    not fix the basis for this pair; this one is orthonormal on the reference
    cube, so the pressure mass is near-diagonal on near-affine elements, which
    is the property the paper asks of its pressure basis (Sec. 6);
  - "Q": Q_{k-2}, the Lagrange basis on the tensor product of the k-1 Gauss
    points per direction (the basis Sec. 6 gives for this pair), ordered with
    the x index fastest.

The 3D tables are formed as dense products over all (quadrature point, node)
pairs -- deliberately no sum factorisation.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k: int) -> np.ndarray:
    """Gauss-Lobatto nodes of degree k on [-1, 1]: -1, roots of P_k', +1."""
    c = np.zeros(k + 1)
    c[k] = 1.0
    d1 = npleg.legder(c)
    d2 = npleg.legder(d1)
    inner = np.sort(np.real(npleg.legroots(d1))) if k >= 2 else np.array([])
    # companion-matrix roots are accurate to a few ulp; polish them as roots of P_k'
    for _ in range(3):
        inner = inner - npleg.legval(inner, d1) / npleg.legval(inner, d2)
    inner = 0.5 * (inner - inner[::-1])          # the roots are symmetric about 0
    return np.concatenate([[-1.0], inner, [1.0]])


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Lagrange basis l_a(x) on ``nodes`` and its derivative, by the product formula.

    Returns (V, dV) of shape [len(x), len(nodes)].
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x)
    n = nodes.shape[0]
    V = np.ones((x.shape[0], n), dtype=np.result_type(x, np.float64))
    dV = np.zeros_like(V)
    for a in range(n):
        others = [b for b in range(n) if b != a]
        denom = np.prod([nodes[a] - nodes[b] for b in others])
        fac = [(x - nodes[b]) for b in others]
        V[:, a] = np.prod(fac, axis=0) / denom if others else 1.0
        tot = np.zeros(x.shape[0], dtype=V.dtype)
        for skip in range(len(others)):
            term = np.ones(x.shape[0], dtype=V.dtype)
            for t, f in enumerate(fac):
                if t != skip:
                    term = term * f
            tot = tot + term
        dV[:, a] = tot / denom
    return V, dV


def legendre_normalised(i: int, x: np.ndarray) -> np.ndarray:
    c = np.zeros(i + 1)
    c[i] = np.sqrt((2 * i + 1) / 2.0)
    return npleg.legval(x, c)


def pressure_q_indices(k: int):
    """(i, j, l) of the Q_{k-2} Gauss-point Lagrange basis, x index fastest."""
    m = k - 1
    return [(i, j, l) for l in range(m) for j in range(m) for i in range(m)]


def pressure_exponents(k: int):
    """(i, j, l) with i+j+l <= k-1, ordered by (i+j+l, l, j, i)."""
    out = []
    for d in range(k):
        for l in range(d + 1):
            for j in range(d - l + 1):
                out.append((d - l - j, j, l))
    return out


class ReferenceElement:
    """Dense tables on the reference cube for polynomial degree k."""

    def __init__(self, k: int, pspace: str = "P"):
        self.k = k
        self.pspace = pspace
        self.P = k + 1
        P = self.P
        self.xi = gll_nodes(k)
        self.g, self.w1 = npleg.leggauss(k + 1)
        B1, D1 = lagrange(self.xi, self.g)                  # [q, a]
        self.B1, self.D1 = B1, D1
        # lexicographic index: a = a0 + P*(a1 + P*a2); same for quadrature points
        idx = np.arange(P)
        i0 = np.tile(idx, P * P)
        i1 = np.tile(np.repeat(idx, P), P)
        i2 = np.repeat(idx, P * P)
        self.lex = (i0, i1, i2)
        # Phi[q, a] and dPhi[q, a, r] (r = xi, eta, zeta)
        self.Phi = B1[i0][:, i0] * B1[i1][:, i1] * B1[i2][:, i2]
        dPhi = np.empty((P ** 3, P ** 3, 3))
        dPhi[:, :, 0] = D1[i0][:, i0] * B1[i1][:, i1] * B1[i2][:, i2]
        dPhi[:, :, 1] = B1[i0][:, i0] * D1[i1][:, i1] * B1[i2][:, i2]
        dPhi[:, :, 2] = B1[i0][:, i0] * B1[i1][:, i1] * D1[i2][:, i2]
        self.dPhi = dPhi
        self.wq = self.w1[i0] * self.w1[i1] * self.w1[i2]
        self.qpts = np.stack([self.g[i0], self.g[i1], self.g[i2]], 1)
        # pressure basis psi_m at volume quadrature points
        if pspace == "P":
            self.pexp = pressure_exponents(k)
            self.Psi = np.stack([legendre_normalised(i, self.qpts[:, 0]) * legendre_normalised(j, self.qpts[:, 1])
                                 * legendre_normalised(l, self.qpts[:, 2]) for (i, j, l) in self.pexp], 1)
        elif pspace == "Q":
            self.pexp = pressure_q_indices(k)
            self.gp, _ = npleg.leggauss(k - 1)
            Lx, _ = lagrange(self.gp, self.qpts[:, 0])
            Ly, _ = lagrange(self.gp, self.qpts[:, 1])
            Lz, _ = lagrange(self.gp, self.qpts[:, 2])
            self.Psi = np.stack([Lx[:, i] * Ly[:, j] * Lz[:, l] for (i, j, l) in self.pexp], 1)
        else:
            raise ValueError("pspace must be 'P' or 'Q'")
        self.n_p = len(self.pexp)
        # bottom face zeta = -1: face Gauss points (g_i, g_j, -1), face weights w_i w_j
        f0 = np.tile(idx, P)
        f1 = np.repeat(idx, P)
        Bm1, Dm1 = lagrange(self.xi, np.array([-1.0]))
        self.Phif = B1[f0][:, i0] * B1[f1][:, i1] * Bm1[0][i2][None, :]
        dPhif = np.empty((P * P, P ** 3, 2))
        dPhif[:, :, 0] = D1[f0][:, i0] * B1[f1][:, i1] * Bm1[0][i2][None, :]
        dPhif[:, :, 1] = B1[f0][:, i0] * D1[f1][:, i1] * Bm1[0][i2][None, :]
        self.dPhif = dPhif
        self.wf = self.w1[f0] * self.w1[f1]

    def eval_pressure_basis(self, xi3: np.ndarray) -> np.ndarray:
        """Values of the n_p pressure basis functions at reference points xi3 [m, 3] -> [m, n_p]."""
        if self.pspace == "P":
            return np.stack([legendre_normalised(i, xi3[:, 0]) * legendre_normalised(j, xi3[:, 1])
                             * legendre_normalised(l, xi3[:, 2]) for (i, j, l) in self.pexp], 1)
        Lx, _ = lagrange(self.gp, xi3[:, 0])
        Ly, _ = lagrange(self.gp, xi3[:, 1])
        Lz, _ = lagrange(self.gp, xi3[:, 2])
        return np.stack([Lx[:, i] * Ly[:, j] * Lz[:, l] for (i, j, l) in self.pexp], 1)

    def eval_basis(self, xi3: np.ndarray) -> np.ndarray:
        """Values of all P^3 nodal basis functions at reference points xi3 [m, 3] -> [m, P^3]."""
        i0, i1, i2 = self.lex
        V0, _ = lagrange(self.xi, xi3[:, 0])
        V1, _ = lagrange(self.xi, xi3[:, 1])
        V2, _ = lagrange(self.xi, xi3[:, 2])
        return V0[:, i0] * V1[:, i1] * V2[:, i2]
