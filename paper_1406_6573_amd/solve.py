"""Newton-Krylov driver on the engine (Sec. 4.1-4.2 of the paper).

Each Newton step linearises at (u, p), evaluates the FP64 residual, builds the
block-diagonal preconditioner (an approximation of F, lumped -M(1/mu) for the
Schur block) and solves J_c d = -r with right-preconditioned FGMRES(m) using
classical Gram-Schmidt with a second pass.  The velocity block is approximated
either by its diagonal ("jacobi") or by its vertical-line blocks ("line"):
banded Cholesky factors of F restricted to each column of nodes, which resolve
the strong vertical coupling of thin columns.  With triangular=True the
preconditioner is the block upper-triangular [[F~, B^T], [0, S~]] of Sec. 4.2
instead of the block-diagonal one: z_p = S~^-1 v_p, z_u = F~^-1 (v_u - B^T z_p),
with B^T z_p from the engine's pressure-gradient apply (the velocity rows of the
Jacobian apply at zero velocity; one more, lighter, element pass per iteration,
fewer iterations).  A backtracking line search on ||r|| accepts
the step.  With linearization="picard" the steps solve with the Picard operator
instead (viscosity kept, the anisotropic part of the Newton tensor dropped;
Sec. 2.3), which converges linearly where Newton converges quadratically.
Every vector operation runs in the engine's kernels (multi-dots with FP64
accumulation, basis combinations, scaling); the host holds only the small
Hessenberg least-squares problem.

Precision modes:
* "fp64": FP64 Krylov basis and FP64 Jacobian applies;
* "mixed": FP32 Krylov basis and FP32 Jacobian applies, inner products
  accumulated in FP64, FP64 right-hand side and FP64 outer refinement of the
  correction (d += FGMRES_32(b - J_64 d) for ``refine`` cycles).

The preconditioners are plain fallbacks (the paper's AMG is not part of this
engine): neither is h-robust in the horizontal directions, so convergence per
Krylov iteration degrades with mesh size; point Jacobi also degrades with the
aspect ratio.
"""
from __future__ import annotations

import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np
import torch


def column_coarse_space(mesh, cells):
    """Host arrays of the horizontal coarse space on a column mesh: a lattice of cells[0] x cells[1]
    coarse cells over the bounding box of the nodes' (x, y), each node's coarse cell corners (lattice
    point i + (cells[0] + 1) j) with bilinear weights, and its relative height zeta (logical height over
    the number of layers).  Returns (n_cpts, node_cpt [N, 4], node_w [N, 4], zeta [N], lattice shape)."""
    ncx, ncy = int(cells[0]), int(cells[1])
    # coarse cells made of whole columns: then no element straddles a lattice line, a hat function
    # couples only with the hats of the neighbouring lattice points, and the probing colours stay exact
    if mesh.nx % ncx or mesh.ny % ncy:
        raise ValueError(f"coarse cells {cells} must divide the column counts ({mesh.nx}, {mesh.ny})")
    x, y = np.asarray(mesh.coords[0]), np.asarray(mesh.coords[1])
    zeta = np.clip(np.asarray(mesh.node_logical[:, 2], dtype=np.float64) / mesh.nz, 0.0, 1.0)
    cols = []
    for v, nc in ((x, ncx), (y, ncy)):
        lo, hi = float(v.min()), float(v.max())
        f = (v - lo) / max(hi - lo, 1e-300) * nc
        i = np.clip(np.floor(f).astype(np.int64), 0, nc - 1)
        cols.append((i, f - i))
    (i, s), (j, t) = cols
    npx = ncx + 1
    cpt = np.stack([i + npx * j, i + 1 + npx * j, i + npx * (j + 1), i + 1 + npx * (j + 1)], 1).astype(np.int32)
    w = np.stack([(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t], 1)
    return npx * (ncy + 1), cpt, w, zeta, (npx, ncy + 1)


class CoarseCorrection:
    """Two-level part of the velocity preconditioner: coarse functions = bilinear hats of a horizontal
    lattice times three vertical profiles (the engine's coarse space), Galerkin coarse matrix
    A_c = P_c^T J~_c P_c with the low-order approximation J~_c of Sec. 5 (probed with the engine's
    matrix-free F~ apply: lattice points whose indices agree modulo 3 have disjoint coupled supports, so
    9 colours x 3 components x 3 profiles = 81 applies give every entry), and its dense inverse by
    Cholesky.  apply(r) = P_c A_c^-1 P_c^T r."""

    def __init__(self, engine, mesh, cells, krylov_dtype):
        self.eng = engine
        n_cpts, cpt, w, zeta, (npx, npy) = column_coarse_space(mesh, cells)
        engine.coarse_setup(n_cpts, cpt, w, zeta)
        self.n_cpts, self.npx, self.npy = n_cpts, npx, npy
        self.nc = 9 * n_cpts
        dev = engine.dev
        self.kt = krylov_dtype
        N = engine.sizes["n_nodes"]
        self.xc = torch.zeros((3, n_cpts, 3), dtype=torch.float64, device=dev)
        self.rc = torch.empty((3, n_cpts, 3), dtype=torch.float64, device=dev)
        self.xu = torch.empty((3, N), dtype=torch.float64, device=dev)
        self.yu = torch.empty((3, N), dtype=torch.float64, device=dev)
        pi = torch.arange(n_cpts, device=dev) % npx
        pj = torch.arange(n_cpts, device=dev) // npx
        self.colours = []
        for a in range(3):
            for b in range(3):
                members = (pi % 3 == a) & (pj % 3 == b)
                # partner[J'] = the lattice point of colour (a, b) within distance 1 of J' (unique), or -1
                di = (a - pi) % 3
                di = torch.where(di == 2, -1, di)
                dj = (b - pj) % 3
                dj = torch.where(dj == 2, -1, dj)
                qi, qj = pi + di, pj + dj
                ok = (qi >= 0) & (qi < npx) & (qj >= 0) & (qj < npy)
                partner = torch.where(ok, qi + npx * qj, torch.full_like(qi, -1))
                self.colours.append((members, partner))
        self.Ainv = None

    def setup(self):
        """Probe A_c at the engine's current state and factor it."""
        eng, n, dev = self.eng, self.n_cpts, self.eng.dev
        A = torch.zeros((self.nc, self.nc), dtype=torch.float64, device=dev)
        rows_c = torch.arange(3, device=dev).view(3, 1, 1).expand(3, n, 3)
        rows_m = torch.arange(3, device=dev).view(1, 1, 3).expand(3, n, 3)
        for members, partner in self.colours:
            pj = partner.view(1, n, 1).expand(3, n, 3)
            valid = (pj >= 0).reshape(-1)
            rows = torch.arange(self.nc, device=dev)[valid]
            for c in range(3):
                for m in range(3):
                    self.xc.zero_()
                    self.xc[c, members, m] = 1.0
                    eng.coarse_prolong(self.xc, self.xu)
                    eng.lowo_apply(self.xu, out=self.yu)
                    eng.coarse_restrict(self.yu, self.rc)
                    cols = ((c * n + pj) * 3 + m).reshape(-1)[valid]
                    A[rows, cols] = self.rc.reshape(-1)[valid]
        A = 0.5 * (A + A.T)
        self.asym = None
        L, info = torch.linalg.cholesky_ex(A)
        if int(info) != 0:                      # singular coarse matrix (no basal friction nor mask)
            shift = 1e-10 * float(torch.diagonal(A).abs().max())
            L = torch.linalg.cholesky(A + shift * torch.eye(self.nc, dtype=A.dtype, device=dev))
        self.Ainv = torch.cholesky_inverse(L)
        self.Ainv32 = self.Ainv.float() if self.kt == torch.float32 else None
        self.A = A

    def apply(self, r_u, out):
        """out = P_c A_c^-1 P_c^T r_u (r_u, out [3, n_nodes] in the Krylov precision)."""
        eng = self.eng
        eng.coarse_restrict(r_u, self.rc)
        rc = self.rc.reshape(-1)
        if self.Ainv32 is not None:
            ec = (self.Ainv32 @ rc.float()).double()
        else:
            ec = self.Ainv @ rc
        self.xc.copy_(ec.view(3, self.n_cpts, 3))
        eng.coarse_prolong(self.xc, out)
        return out


@dataclass
class SolveStats:
    newton_residuals: list = field(default_factory=list)
    linear_reductions: list = field(default_factory=list)
    krylov_iterations: list = field(default_factory=list)
    step_lengths: list = field(default_factory=list)
    # per step: True when the accepted step met the sufficient-decrease test of the line search
    sufficient_decrease: list = field(default_factory=list)
    # set when no trial step lowered ||r||: the iterate was kept and the iteration stopped
    stalled: bool = False
    seconds: float = 0.0


class NewtonKrylov:
    def __init__(self, engine, restart: int = 50, precision: str = "fp64", refine: int = 1,
                 precond: str = "jacobi", triangular: bool = False, linearization: str = "newton",
                 coarse=None, coarse_mode: str = "mult"):
        """coarse = (mesh, (cells_x, cells_y)) adds the horizontal coarse correction built from the
        low-order F~ to the velocity preconditioner (two-level with the line blocks as smoother,
        multiplicative "coarse then smooth" or additive)."""
        if restart + 1 > 64:
            raise ValueError("restart must be at most 63")
        if precond not in ("jacobi", "line"):
            raise ValueError("precond must be 'jacobi' or 'line'")
        if coarse_mode not in ("mult", "add"):
            raise ValueError("coarse_mode must be 'mult' or 'add'")
        if engine.linearization != linearization:         # switching discards the engine's state
            engine.set_linearization(linearization)
        self.linearization = linearization
        self.eng, self.m, self.precision, self.refine, self.precond = engine, restart, precision, refine, precond
        self.triangular = triangular
        sz = engine.sizes
        self.N, self.n_el, self.n_p = sz["n_nodes"], sz["n_el"], sz["n_p"]
        self.n = 3 * self.N + self.n_el * self.n_p
        dev = engine.dev
        kt = torch.float64 if precision == "fp64" else torch.float32
        self.kt = kt
        # basis rows padded to a multiple of 64 entries: every row starts 256-byte aligned, which lets the
        # multi-dot and basis-combination kernels use 16-byte loads
        ld = (self.n + 63) // 64 * 64
        self.V = torch.empty((restart + 1, ld), dtype=kt, device=dev)[:, :self.n]
        self.Z = torch.empty((restart, ld), dtype=kt, device=dev)[:, :self.n]
        self.h = torch.empty(64, dtype=torch.float64, device=dev)
        # Hessenberg columns of one cycle: the two Gram-Schmidt passes (the second zero when not taken)
        # and the squared norm per step, on the device and their pinned host copies
        self.Hd = torch.zeros((restart, 3, 64), dtype=torch.float64, device=dev)
        self.Hh = torch.zeros((restart, 3, 64), dtype=torch.float64, pin_memory=True)
        self.reorth = torch.zeros(1, dtype=torch.int32, device=dev)   # second Gram-Schmidt pass taken
        # second Gram-Schmidt pass when the projection kept less than eta2 of |w|^2: 0.01 (a pass may
        # lose one digit of orthogonality) for cycles whose target is 1e-6 or looser, 1/2 (the
        # classical constant) for tighter targets, whose attainable residual the loss would limit
        self.reorth_eta2_loose, self.reorth_eta2_tight, self.reorth_tol = 0.01, 0.5, 1e-6
        self.events = [torch.cuda.Event() for _ in range(restart)]
        self.minv = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.w64 = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.r64 = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.d64 = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.tmp = torch.empty(self.n, dtype=kt, device=dev)
        if triangular:
            self.bt = torch.empty(self.n, dtype=kt, device=dev)
        self.coarse, self.coarse_mode = None, coarse_mode
        if coarse is not None:
            self.coarse = CoarseCorrection(engine, coarse[0], coarse[1], kt)
            self.zc = torch.empty((3, self.N), dtype=kt, device=dev)
            self.zero_p = torch.zeros((self.n_el, self.n_p), dtype=kt, device=dev)
            self.fz = torch.empty(self.n, dtype=kt, device=dev)

    # ------------------------------------------------------------ views
    def split(self, x):
        return x[:3 * self.N].view(3, self.N), x[3 * self.N:].view(self.n_el, self.n_p)

    def apply(self, x, y):
        """y = J_c x in the precision of x."""
        prec = "fp64" if x.dtype == torch.float64 else "fp32"
        self.eng.jacobian_apply(*self.split(x), prec, out=self.split(y))

    def precondition(self, v, z):
        """z = M^-1 v (vectors of the Krylov precision)."""
        eng = self.eng
        if self.precond == "jacobi" and not self.triangular and self.coarse is None:
            eng.vec_mul(self.minv, v, z)
            return
        vu, vp = self.split(v)
        zu, zp = self.split(z)
        eng.vec_mul(self.minv[3 * self.N:], vp.reshape(-1), zp.reshape(-1))      # z_p = S~^-1 v_p
        ru = vu
        if self.triangular:                                                       # v_u - B^T z_p
            bu, _ = self.split(self.bt)
            prec = "fp64" if v.dtype == torch.float64 else "fp32"
            eng.gradient_apply(zp, prec, out=bu)
            eng.vec_axpby(1.0, vu.reshape(-1), -1.0, bu.reshape(-1))
            ru = bu
        if self.coarse is not None:
            zc = self.coarse.apply(ru, self.zc)                                  # coarse correction
            if self.coarse_mode == "mult":                                      # smooth r - F z_c
                fu, fp = self.split(self.fz)
                prec = "fp64" if v.dtype == torch.float64 else "fp32"
                eng.jacobian_apply(zc, self.zero_p, prec, out=(fu, fp))
                eng.vec_axpby(1.0, ru.reshape(-1), -1.0, fu.reshape(-1))
                ru = fu
        if self.precond == "line":
            eng.line_apply(ru, out=zu)
        else:
            eng.vec_mul(self.minv[:3 * self.N], ru.reshape(-1), zu.reshape(-1))
        if self.coarse is not None:
            eng.vec_axpby(1.0, self.zc.reshape(-1), 1.0, zu.reshape(-1))

    def setup_preconditioner(self):
        mu, mp = self.split(self.minv)
        self.eng.jacobi_diag(invert=True, out=(mu, mp))
        if self.precond == "line":
            self.eng.line_setup()
        if self.coarse is not None:
            self.coarse.setup()

    def norm(self, x):
        self.eng.vec_dots(x.view(1, -1), 1, x, self.h)
        return math.sqrt(max(float(self.h[0]), 0.0))

    # ------------------------------------------------------------ FGMRES
    def fgmres(self, b, x, tol):
        """Approximately solve J x = b (vectors of the Krylov precision), x += correction.
        Returns (iterations, residual estimate / ||b||).

        An Arnoldi step runs entirely on the device: the Gram-Schmidt pass (multi-dots into a device
        Hessenberg column, basis combination), the norm, the test for a second pass and that pass when
        the test asks for it (both on the device), and the normalisation.  The column is
        copied to pinned host memory asynchronously, and the host applies the Givens rotations to
        column j - 1 while step j is queued, so no step waits for the host.  When column j - 1 meets
        the tolerance, the already computed column j is used as well (one step more than a
        synchronous loop would take)."""
        eng, V, Z, m = self.eng, self.V, self.Z, self.m
        eta2 = self.reorth_eta2_loose if tol >= self.reorth_tol else self.reorth_eta2_tight
        w = V[0]
        self.apply(x, w)
        eng.vec_axpby(1.0, b, -1.0, w)                   # r = b - J x, stored in V[0]
        beta = self.norm(w)
        bnorm = self.norm(b)
        if beta == 0.0 or bnorm == 0.0:
            return 0, 0.0
        eng.vec_axpby(0.0, w, 1.0 / beta, w)
        Hd, Hh = self.Hd, self.Hh
        Hn = Hh.numpy()
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        events = self.events

        def column(j):
            """Givens-reduce column j; returns (converged, breakdown)."""
            hcol = np.zeros(j + 2)
            hcol[:j + 1] = Hn[j, 0, :j + 1] + Hn[j, 1, :j + 1]
            hn = math.sqrt(max(Hn[j, 2, 0], 0.0))
            hcol[j + 1] = hn
            for i in range(j):                             # previous Givens rotations
                t = cs[i] * hcol[i] + sn[i] * hcol[i + 1]
                hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1]
                hcol[i] = t
            rho = math.hypot(hcol[j], hcol[j + 1])
            cs[j], sn[j] = (hcol[j] / rho, hcol[j + 1] / rho) if rho > 0 else (1.0, 0.0)
            hcol[j], hcol[j + 1] = rho, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[:j + 2, j] = hcol
            return abs(g[j + 1]) <= tol * bnorm, hn == 0.0

        k = m
        for j in range(m):
            self.precondition(V[j], Z[j])                  # z_j = M^-1 v_j
            wj = V[j + 1]
            self.apply(Z[j], wj)
            # classical Gram-Schmidt; the rows include w itself, so the last dot is |w|^2.  The squared
            # norm after the projection follows from the dots; a second pass runs, decided on the device,
            # only when it fell below eta2 |w|^2 (the Daniel-Gragg-Kaufman-Stewart test)
            h1, h2, hn = Hd[j, 0], Hd[j, 1], Hd[j, 2]
            eng.vec_dots(V, j + 2, wj, h1)
            eng.vec_gemv(V, j + 1, h1, -1.0, wj)
            eng.gs_norm(j + 1, h1, eta2, None, self.reorth, hn)
            eng.vec_dots_if(self.reorth, V, j + 2, wj, h2)
            eng.vec_gemv_if(self.reorth, V, j + 1, h2, -1.0, wj)
            eng.gs_norm(j + 1, h2, 0.0, self.reorth, None, hn)
            eng.vec_normalize(hn, wj)
            Hh[j].copy_(Hd[j], non_blocking=True)
            events[j].record()
            if j >= 1:
                events[j - 1].synchronize()
                conv, brk = column(j - 1)
                if brk:                                    # v_j = 0: the space is invariant
                    k = j
                    break
                if conv:
                    events[j].synchronize()
                    column(j)
                    k = j + 1
                    break
        else:
            events[m - 1].synchronize()
            column(m - 1)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k else np.zeros(0)
        if k:
            self.h[:k].copy_(torch.from_numpy(y))
            eng.vec_gemv(Z, k, self.h, 1.0, x)            # x += Z y
        return k, abs(g[k]) / bnorm

    def linear_solve(self, rhs64, tol):
        """d64 = approx J^-1 rhs64 (FP64 in and out) by ``refine`` cycles of FGMRES(m).  FP64: restarted
        FGMRES, stopping once the residual is below tol relative to rhs64.  Mixed: each cycle solves
        for the FP64 residual r = rhs - J_64 d in FP32 to tol relative to r (the outer iterative
        refinement), all ``refine`` cycles."""
        eng = self.eng
        self.d64.zero_()
        if self.precision == "fp64":
            its, red = 0, 1.0
            for _ in range(self.refine):
                k, red = self.fgmres(rhs64, self.d64, tol)
                its += k
                if red <= tol:
                    break
            return its, red
        its = 0
        for _ in range(self.refine):                       # FP64 outer refinement of the correction
            self.apply(self.d64, self.w64)
            eng.vec_axpby(1.0, rhs64, 0.0, self.r64)
            eng.vec_axpby(-1.0, self.w64, 1.0, self.r64)  # r = rhs - J_64 d
            b32 = self.V[0].new_empty(self.n)
            eng.vec_convert(self.r64, b32)
            x32 = self.tmp
            x32.zero_()
            k, _ = self.fgmres(b32, x32, tol)
            its += k
            eng.vec_convert(x32, self.w64)
            eng.vec_axpby(1.0, self.w64, 1.0, self.d64)
        self.apply(self.d64, self.w64)
        eng.vec_axpby(1.0, rhs64, 0.0, self.r64)
        eng.vec_axpby(-1.0, self.w64, 1.0, self.r64)
        return its, self.norm(self.r64) / max(self.norm(rhs64), 1e-300)

    # ------------------------------------------------------------ Newton
    def residual_vec(self, out):
        ru, rp = self.split(out)
        self.eng.residual(out=(ru, rp))
        return out

    def solve(self, u, p, n_newton=5, lin_tol=1e-8, max_backtrack=6, verbose=False):
        """Newton iterations from (u, p) (FP64 tensors, updated in place)."""
        eng, st = self.eng, SolveStats()
        t0 = time.perf_counter()
        x = torch.cat([u.reshape(-1), p.reshape(-1)])
        r = torch.empty_like(x)
        trial = torch.empty_like(x)
        xu, xp = self.split(x)
        eng.set_state(xu, xp)
        self.residual_vec(r)
        rn = self.norm(r)
        st.newton_residuals.append(rn)
        for it in range(n_newton):
            self.setup_preconditioner()
            eng.vec_axpby(0.0, r, -1.0, r)                  # rhs = -r
            its, red = self.linear_solve(r, lin_tol)
            st.krylov_iterations.append(its)
            st.linear_reductions.append(red)
            alpha, ok = 1.0, False
            for b in range(max_backtrack + 1):               # backtracking on ||r||
                if b:
                    alpha *= 0.5
                eng.vec_axpby(1.0, x, 0.0, trial)
                eng.vec_axpby(alpha, self.d64, 1.0, trial)
                tu, tp = self.split(trial)
                eng.set_state(tu, tp)
                self.residual_vec(r)
                rt = self.norm(r)
                if rt <= (1.0 - 1e-4 * alpha) * rn:
                    ok = True
                    break
            if not ok and not rt < rn:                        # no trial lowered ||r||: keep x and stop
                xu, xp = self.split(x)
                eng.set_state(xu, xp)
                self.residual_vec(r)
                st.stalled = True
                if verbose:
                    print(f"[newton {self.precision}] step {it + 1}: no step length down to {alpha} lowers "
                          f"|r| = {rn:.6e}; stopping", file=sys.stderr, flush=True)
                break
            eng.vec_axpby(1.0, trial, 0.0, x)
            rn = rt
            st.newton_residuals.append(rn)
            st.step_lengths.append(alpha)
            st.sufficient_decrease.append(ok)
            if verbose:
                print(f"[newton {self.precision}] step {it + 1}: |r| = {rn:.6e}, krylov {its}, "
                      f"linear reduction {red:.2e}, alpha {alpha}", file=sys.stderr, flush=True)
        u.copy_(self.split(x)[0])
        p.copy_(self.split(x)[1])
        torch.cuda.synchronize()
        st.seconds = time.perf_counter() - t0
        return st


def adjoint_gradient(nk: NewtonKrylov, u, p, dphi_u, dphi_p=None, tol: float = 1e-12):
    """Gradient of a functional Phi(u(theta), p(theta)) of the solved state with respect to the
    per-element log rate factors and the per-face basal friction, theta = (logA, beta)
    (the inverse-problem use of the adjoint, Sec. 2.3):

        J_c^T lambda = (dPhi/du, dPhi/dp),   dPhi/dtheta = -(dr/dtheta)^T lambda,

    with J_c symmetric (the same FGMRES solve as a Newton step) and (dr/dtheta)^T lambda from the
    residual VJP.  (u, p) must solve r(u, p) = 0; dphi_u [3, n_nodes] and dphi_p [n_el, n_p] are
    FP64 device tensors.  Returns (dPhi/dlogA [n_el], dPhi/dbeta [n_bface], Krylov iterations,
    relative residual of the adjoint solve)."""
    if nk.linearization != "newton":
        raise ValueError("the adjoint needs the Newton linearization")
    eng = nk.eng
    eng.set_state(u.contiguous(), p.contiguous())
    nk.setup_preconditioner()
    if dphi_p is None:
        dphi_p = torch.zeros((nk.n_el, nk.n_p), dtype=torch.float64, device=u.device)
    rhs = torch.cat([dphi_u.reshape(-1), dphi_p.reshape(-1)]).contiguous()
    its, red = nk.linear_solve(rhs, tol)
    lu, lp = nk.split(nk.d64)
    _, _, g_logA, g_beta = eng.residual_vjp(lu.contiguous(), lp.contiguous(), "fp64")
    return -g_logA, -g_beta, its, red
