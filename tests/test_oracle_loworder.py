"""Pins of the oracle's low-order matrix F~ (Gauss-Lobatto sub-grid, Sec. 5) against closed forms.

Each targets a plausible slip: a wrong quadrature weight or sym-gradient factor, a transposed
direction in the Kronecker structure, a missing |det J|, coefficients evaluated at the wrong point,
an unlumped or wrongly normalised basal term, or R_e dropped at hanging faces.
"""
import numpy as np
import pytest
import sympy

from meshgen.columns import column_mesh, random_refined_columns
from oracle import StokesOracle
from oracle.loworder import element_matrices, low_order_matrix, nodal_coefficients
from oracle.reference import gll_nodes


def mesh_for(k, nx=3, ny=2, nz=2, frac=0.35, seed=4, extent=(9.0, 6.0, 1.2), geometry=None, mask=False):
    rng = np.random.default_rng(seed)
    ref = random_refined_columns(nx, ny, frac, rng) if frac > 0 else None
    return column_mesh(k, nx, ny, nz, refined=ref, extent=extent, geometry=geometry, base_normal_dirichlet=mask)


def terrain(nx, ny, nz, L):
    def geo(lg):
        x, y = lg[:, 0] * L / nx, lg[:, 1] * L / ny
        return np.stack([x, y, 0.2 * np.sin(2 * np.pi * x / L) + lg[:, 2] / nz * (1.0 + 0.2 * np.cos(2 * np.pi * y / L))], 1)
    return geo


@pytest.mark.parametrize("k,mapped", [(2, False), (3, True), (4, True)])
def test_rigid_modes_in_kernel(k, mapped):
    """Translations and infinitesimal rotations are trilinear on every sub-cell (the sub-cell map is
    trilinear), so F~ annihilates them (beta = 0, no mask), on hanging and mapped meshes, n = 3."""
    nx, ny, nz, L = 3, 2, 2, 9.0
    m = mesh_for(k, nx, ny, nz, geometry=terrain(nx, ny, nz, L) if mapped else None)
    rng = np.random.default_rng(k)
    o = StokesOracle(m, 3.0, 1e-10, 0.5, rng.normal(0, 0.5, m.n_el), np.zeros(m.n_bface))
    o.set_state(rng.uniform(-1, 1, (3, m.n_nodes)), np.zeros((m.n_el, m.n_p)))
    K = low_order_matrix(o)
    x, y, z = m.coords
    for a, w in ((np.array([1.0, -2.0, 0.5]), np.zeros(3)), (np.zeros(3), np.array([0.3, -0.7, 1.1]))):
        u = a[:, None] + np.cross(w, np.stack([x, y, z]).T).T
        r = K @ u.ravel()
        assert np.max(np.abs(r)) < 1e-13 * np.max(abs(K) @ np.abs(u.ravel()))


def q1_1d(nodes):
    """1D Q1 matrices on the sub-grid `nodes` (length P), 2-point trapezoid rule per sub-interval:
    stiffness K (exact), lumped mass M (diagonal), C[a][b] = rule of psi_a' psi_b."""
    P = len(nodes)
    K, M, C = (sympy.zeros(P, P) for _ in range(3))
    for i in range(P - 1):
        h = nodes[i + 1] - nodes[i]
        loc = [i, i + 1]
        dpsi = [-1 / h, 1 / h]
        for a in range(2):
            M[loc[a], loc[a]] += h / 2
            for b in range(2):
                K[loc[a], loc[b]] += dpsi[a] * dpsi[b] * h
                C[loc[a], loc[b]] += dpsi[a] * h / 2          # psi_b is 1 at one of the two points
    return K, M, C


@pytest.mark.parametrize("k", [2, 3])
def test_affine_box_n1_kronecker_closed_form(k):
    """One axis-aligned box element at n = 1 (C = mu I, mu = B0 constant): F~_e equals the Kronecker
    closed form mu (1/2 delta_cd sum_i K_i (x) M_j (x) M_l + 1/2 C_d (x) C_c^T ...) built from 1D Q1
    matrices on the Gauss-Lobatto sub-grid in exact arithmetic (k = 2: nodes -1, 0, 1; k = 3: +-1/sqrt 5)."""
    hx, hy, hz = sympy.Rational(3), sympy.Rational(2), sympy.Rational(1, 2)
    xi = [-1, 0, 1] if k == 2 else [-1, -1 / sympy.sqrt(5), 1 / sympy.sqrt(5), 1]
    mats = []
    for h in (hx, hy, hz):
        mats.append(q1_1d([(sympy.nsimplify(s) + 1) * h / 2 for s in xi]))
    P = k + 1
    m = column_mesh(k, 1, 1, 1, extent=(float(hx), float(hy), float(hz)))
    B0 = 0.7
    o = StokesOracle(m, 1.0, 1e-10, B0, np.zeros(1), np.zeros(m.n_bface))
    o.set_state(np.random.default_rng(0).uniform(-1, 1, (3, m.n_nodes)), np.zeros((1, m.n_p)))
    A = element_matrices(o)[0].reshape(3, P ** 3, 3, P ** 3)

    def kron3(ax, ay, az):      # node index a = ax + P (ay + P az)
        return np.kron(np.array(az, dtype=float), np.kron(np.array(ay, dtype=float), np.array(ax, dtype=float)))

    (Kx, Mx, Cx), (Ky, My, Cy), (Kz, Mz, Cz) = mats
    lap = kron3(Kx, My, Mz) + kron3(Mx, Ky, Mz) + kron3(Mx, My, Kz)
    # d_i psi_a d_j psi_b integrated: i == j -> stiffness in i; i != j -> C in i (row), C^T in j
    def mixed(i, j):
        f = [[Mx, My, Mz][d] for d in range(3)]
        if i == j:
            f[i] = [Kx, Ky, Kz][i]
        else:
            f[i] = [Cx, Cy, Cz][i]
            f[j] = [Cx, Cy, Cz][j].T
        return kron3(*f)
    for c in range(3):
        for d in range(3):
            # a(psi_a e_c, psi_b e_d) = mu/2 (delta_cd grad psi_a . grad psi_b + d_d psi_a d_c psi_b)
            expect = 0.5 * B0 * ((lap if c == d else 0.0) + mixed(d, c))
            assert np.max(np.abs(A[c, :, d, :] - expect)) < 1e-13 * np.max(np.abs(expect))


@pytest.mark.parametrize("k", [2, 3, 4])
def test_linear_fields_match_high_order_energy(k):
    """For linear u, v on an affine hanging mesh at n = 1 both F and F~ give v^T F u = mu vol D(u):D(v)
    (the Q1 interpolant and R_e reproduce linear fields, the trapezoid rule integrates constants):
    a closed form independent of both discretisations."""
    m = mesh_for(k, extent=(9.0, 6.0, 1.2))
    B0 = 0.6
    o = StokesOracle(m, 1.0, 1e-10, B0, np.zeros(m.n_el), np.zeros(m.n_bface))
    o.set_state(np.zeros((3, m.n_nodes)), np.zeros((m.n_el, m.n_p)))
    Kt = low_order_matrix(o)
    X = m.coords
    Gu = np.array([[0.3, -1.0, 0.2], [0.5, 0.1, -0.4], [0.0, 0.7, 0.25]])
    Gv = np.array([[-0.2, 0.4, 1.0], [0.9, 0.3, 0.0], [0.1, -0.6, 0.5]])
    u, v = (G @ X for G in (Gu, Gv))
    Du, Dv = 0.5 * (Gu + Gu.T), 0.5 * (Gv + Gv.T)
    vol = 9.0 * 6.0 * 1.2
    expect = B0 * vol * np.sum(Du * Dv)
    got = v.ravel() @ (Kt @ u.ravel())
    assert abs(got - expect) < 1e-12 * abs(expect)


def test_nodal_coefficients_closed_form():
    """A quadratic velocity is represented exactly for k >= 2, so D0 at each node is the closed-form
    strain rate at the node's position, and mu follows eq. (glen) there."""
    k = 3
    m = mesh_for(k, frac=0.0)
    x, y, z = m.coords
    u = np.stack([x * y, 0.5 * z * z, x * z])
    rng = np.random.default_rng(1)
    logA = rng.normal(0, 0.5, m.n_el)
    n, eps, B0 = 3.0, 1e-10, 0.5
    o = StokesOracle(m, n, eps, B0, logA, np.zeros(m.n_bface))
    o.set_state(u, np.zeros((m.n_el, m.n_p)))
    mu, kap, D0, X = nodal_coefficients(o)
    Xabs = o.R @ m.coords.T                                       # node positions per slot
    Xabs = Xabs.reshape(m.n_el, (k + 1) ** 3, 3)
    xs, ys, zs = Xabs[..., 0], Xabs[..., 1], Xabs[..., 2]
    G = np.zeros(Xabs.shape[:2] + (3, 3))
    G[..., 0, 0], G[..., 0, 1] = ys, xs
    G[..., 1, 2] = zs
    G[..., 2, 0], G[..., 2, 2] = zs, xs
    D = 0.5 * (G + np.swapaxes(G, 2, 3))
    assert np.max(np.abs(D0 - D)) < 1e-11 * np.max(np.abs(D))
    II = 0.5 * np.einsum("egij,egij->eg", D, D)
    Be = B0 * np.exp(-logA / n)[:, None]
    assert np.max(np.abs(mu - Be * (II + eps) ** ((1 - n) / (2 * n))) / mu) < 1e-10
    assert np.max(np.abs(kap - mu * (n - 1) / (2 * n) / (II + eps)) / kap) < 1e-10


def test_basal_term_inclined_plane():
    """beta = 1 on a planar inclined base (hanging columns): the lumped basal blocks of F~ sum to
    area (delta_cd - n_c n_d) (constant fields see only the basal term), and each base node's block is
    diagonal in the nodes (lumping of the Gauss-Lobatto rule)."""
    a, b, Lx, Ly, nx, ny, nz = 0.3, -0.2, 12.0, 9.0, 4, 3, 2

    def geo(lg):
        x, y = lg[:, 0] * Lx / nx, lg[:, 1] * Ly / ny
        return np.stack([x, y, a * x + b * y + lg[:, 2] / nz * (1.0 + 0.02 * x)], 1)

    m = mesh_for(3, nx, ny, nz, frac=0.35, seed=3, geometry=geo)
    o = StokesOracle(m, 3.0, 1e-10, 0.5, np.zeros(m.n_el), np.ones(m.n_bface))
    o.set_state(np.zeros((3, m.n_nodes)), np.zeros((m.n_el, m.n_p)))
    K = low_order_matrix(o)
    N = m.n_nodes
    s = np.sqrt(1 + a * a + b * b)
    nrm = np.array([-a, -b, 1.0]) / s
    area = Lx * Ly * s
    tot = np.zeros((3, 3))
    for c in range(3):
        ec = np.zeros(3 * N)
        ec[c * N:(c + 1) * N] = 1.0
        Kc = K @ ec
        for d in range(3):
            tot[d, c] = Kc[d * N:(d + 1) * N].sum()
    mag = np.max(np.abs(K).sum(axis=1))
    assert np.max(np.abs(tot - area * (np.eye(3) - np.outer(nrm, nrm)))) < 1e-12 * mag * N


def test_nodal_coefficient_placement_linear_fields():
    """n = 3 with a varying state: for linear u, v (constant strain rates Du, Dv) the sub-cell rule gives
    v^T F~ u = sum_e sum_g V_g [mu_g Du:Dv - kappa_g (D0_g:Du)(D0_g:Dv)] with V_g = prod_d m_d(g) the
    lumped (trapezoid) volume of node g inside its box element and (mu, kappa, D0)_g the element's
    nodal coefficients: a coefficient used at the wrong corner or a dropped Newton term fails it."""
    k = 3
    m = mesh_for(k, frac=0.35, extent=(9.0, 6.0, 1.2))
    rng = np.random.default_rng(5)
    o = StokesOracle(m, 3.0, 1e-10, 0.5, rng.normal(0, 0.5, m.n_el), np.zeros(m.n_bface))
    x, y, z = m.coords
    o.set_state(np.stack([np.sin(x) * z, np.cos(y) * z * z, 0.3 * x * y]), np.zeros((m.n_el, m.n_p)))
    mu, kap, D0, _ = nodal_coefficients(o)
    Kt = low_order_matrix(o)
    Gu = np.array([[0.3, -1.0, 0.2], [0.5, 0.1, -0.4], [0.0, 0.7, 0.25]])
    Gv = np.array([[-0.2, 0.4, 1.0], [0.9, 0.3, 0.0], [0.1, -0.6, 0.5]])
    Du, Dv = 0.5 * (Gu + Gu.T), 0.5 * (Gv + Gv.T)
    u, v = Gu @ m.coords, Gv @ m.coords
    xi = gll_nodes(k)
    m1 = np.zeros(k + 1)                                    # lumped 1D mass on [-1, 1]
    for i in range(k):
        h = xi[i + 1] - xi[i]
        m1[i] += h / 2
        m1[i + 1] += h / 2
    P = k + 1
    lo, size = m.elem_box()
    scale = np.array([9.0 / 3, 6.0 / 2, 1.2 / 2])            # physical size of a coarse cell
    idx = np.arange(P ** 3)
    mw = m1[idx % P] * m1[(idx // P) % P] * m1[idx // (P * P)] / 8.0     # reference cube volume 8
    expect = 0.0
    for e in range(m.n_el):
        vol = np.prod(size[e] * scale)
        Vg = mw * vol
        s_u = np.einsum("gij,ij->g", D0[e], Du)
        s_v = np.einsum("gij,ij->g", D0[e], Dv)
        expect += np.sum(Vg * (mu[e] * np.sum(Du * Dv) - kap[e] * s_u * s_v))
    got = v.ravel() @ (Kt @ u.ravel())
    assert abs(got - expect) < 1e-11 * np.sum(np.abs(Kt) @ np.abs(u.ravel()) * np.abs(v.ravel()))
