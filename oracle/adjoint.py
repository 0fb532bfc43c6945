"""Solved state and adjoint gradient by direct sparse solves (oracle; test infrastructure only).

Sec. 2.3: the adjoint of the Newton linearisation uses the same fourth-order tensor, so for
a functional Phi(u(theta), p(theta)) of the state that solves r(u, p; theta) = 0, with
theta = (logA, beta),

    J_c^T lambda = dPhi/d(u, p),        dPhi/dtheta = -(dr/dtheta)^T lambda,

J_c the assembled Jacobian with the Dirichlet rows of the oracle.  Here the linear systems are
solved directly (scipy.sparse.linalg.spsolve) and (dr/dtheta)^T lambda is the oracle's own VJP.
Pinned by central differences of Phi at re-solved states (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def newton_solve(oracle, u, p, f_u=None, tol=1e-12, max_steps=60):
    """Newton's method with backtracking on ||r|| from (u, p), direct solves of J_c d = -r.
    Returns the solved (u, p) and the residual norms; sets the oracle's state to the solution."""
    N = oracle.mesh.n_nodes
    x = np.concatenate([np.asarray(u, dtype=np.float64).ravel(), np.asarray(p, dtype=np.float64).ravel()])

    def split(v):
        return v[:3 * N].reshape(3, N), v[3 * N:].reshape(oracle.mesh.n_el, -1)

    def res(v):
        oracle.set_state(*split(v))
        ru, rp = oracle.residual(f_u)
        return np.concatenate([ru.ravel(), rp.ravel()])

    r = res(x)
    hist = [float(np.linalg.norm(r))]
    for _ in range(max_steps):
        if hist[-1] <= tol * hist[0]:
            break
        d = spla.spsolve(oracle.jacobian().tocsc(), -r)
        alpha = 1.0
        while True:
            xt = x + alpha * d
            rt = res(xt)
            if np.linalg.norm(rt) <= (1.0 - 1e-4 * alpha) * hist[-1] or alpha < 1e-6:
                break
            alpha *= 0.5
        x, r = xt, rt
        hist.append(float(np.linalg.norm(r)))
    uu, pp = split(x)
    oracle.set_state(uu, pp)
    return uu.copy(), pp.copy(), hist


def adjoint_gradient(oracle, dphi_u, dphi_p=None):
    """dPhi/dlogA [n_el] and dPhi/dbeta [n_bface] at the oracle's current (solved) state for the
    cotangent dPhi/d(u, p): lambda = J_c^-T dPhi/d(u, p), then minus the parameter parts of the
    residual VJP at lambda.  Returns (g_logA, g_beta, lambda_u, lambda_p)."""
    N = oracle.mesh.n_nodes
    n_p = oracle.ref.n_p
    if dphi_p is None:
        dphi_p = np.zeros((oracle.mesh.n_el, n_p))
    rhs = np.concatenate([np.asarray(dphi_u).ravel(), np.asarray(dphi_p).ravel()])
    lam = spla.spsolve(oracle.jacobian().T.tocsc(), rhs)
    lu, lp = lam[:3 * N].reshape(3, N), lam[3 * N:].reshape(oracle.mesh.n_el, n_p)
    _, _, g_logA, g_beta = oracle.vjp(lu, lp)
    return -g_logA, -g_beta, lu, lp
