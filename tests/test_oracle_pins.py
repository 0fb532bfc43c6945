"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

Each test targets a plausible mistake in the oracle (dropped term, wrong sign
or factor, transposed index, wrong hanging weight) and fails if it is made.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import sympy

from meshgen.columns import column_mesh, random_refined_columns
from oracle import StokesOracle
from oracle.reference import ReferenceElement, gll_nodes, lagrange
from oracle.stokes import newton_tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def hanging_mesh(k, seed=1, nx=4, ny=4, nz=2, frac=0.3, extent=(40.0, 40.0, 1.0), mask=False, geometry=None,
                 pspace="P", refine_from=0):
    rng = np.random.default_rng(seed)
    ref = random_refined_columns(nx, ny, frac, rng)
    return column_mesh(k, nx, ny, nz, refined=ref, extent=extent, base_normal_dirichlet=mask, geometry=geometry,
                       pspace=pspace, refine_from=refine_from)


def exact_gauss(m):
    """m-point Gauss-Legendre nodes and weights from the exact roots of P_m (sympy), w = 2/((1-x^2) P_m'(x)^2)."""
    x = sympy.Symbol("x")
    if m == 1:
        return np.array([0.0]), np.array([2.0])
    roots = sorted(sympy.solve(sympy.legendre(m, x), x), key=lambda r: float(r))
    dP = sympy.diff(sympy.legendre(m, x), x)
    w = [2 / ((1 - r ** 2) * dP.subs(x, r) ** 2) for r in roots]
    return np.array([float(r) for r in roots]), np.array([float(sympy.nsimplify(v)) for v in w])


def terrain(nx, ny, nz, L):
    def geo(lg):
        x, y = lg[:, 0] * L / nx, lg[:, 1] * L / ny
        b = 0.05 * np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L)
        H = 1.0 + 0.3 * np.cos(2 * np.pi * x / L + 0.4) * np.sin(2 * np.pi * y / L + 0.2)
        return np.stack([x, y, b + lg[:, 2] / nz * H], 1)
    return geo


def rigid(mesh, a=(0.3, -0.2, 0.5), om=(0.7, 0.1, -0.4)):
    return np.asarray(a)[:, None] + np.cross(np.asarray(om), mesh.coords.T).T


def scale_of(K, x):
    return np.abs(K) @ np.abs(x)


# ---------------------------------------------------------------- reference tables
@pytest.mark.parametrize("k", [2, 3, 4])
def test_gll_gauss_tables(k):
    """GLL nodes are +-1 and the roots of P_k'; Gauss rule integrates degree 2k+1 exactly."""
    ref = ReferenceElement(k)
    xs = sympy.Symbol("x")
    exact = sorted(float(r) for r in sympy.solve(sympy.diff(sympy.legendre(k, xs), xs), xs))
    assert np.max(np.abs(ref.xi - np.array([-1.0] + exact + [1.0]))) <= 6e-17
    for deg in range(2 * k + 2):
        assert abs(np.sum(ref.w1 * ref.g ** deg) - (0.0 if deg % 2 else 2.0 / (deg + 1))) < 1e-14


@pytest.mark.parametrize("k", [2, 3, 4])
def test_pressure_basis_orthonormal(k):
    """Pressure mass on the reference cube is the identity (orthonormal P_{k-1} basis), dim = k(k+1)(k+2)/6."""
    ref = ReferenceElement(k)
    M = ref.Psi.T @ (ref.wq[:, None] * ref.Psi)
    assert ref.n_p == k * (k + 1) * (k + 2) // 6
    assert np.allclose(M, np.eye(ref.n_p), atol=1e-13)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_pressure_q_basis(k):
    """Q_{k-2} pressure basis (Sec. 6: Lagrange basis on the tensor Gauss points): dimension (k-1)^3, the
    interpolation property at the exact Gauss points, partition of unity, and a diagonal reference mass equal
    to the products of the exact Gauss weights (the (k+1)-point rule integrates psi_m psi_n exactly)."""
    ref = ReferenceElement(k, "Q")
    m = k - 1
    assert ref.n_p == m ** 3
    gx, gw = exact_gauss(m)
    pts = np.array([(gx[i], gx[j], gx[l]) for l in range(m) for j in range(m) for i in range(m)])
    assert np.allclose(ref.eval_pressure_basis(pts), np.eye(ref.n_p), atol=1e-13)
    rng = np.random.default_rng(5)
    r = rng.uniform(-1, 1, (50, 3))
    assert np.allclose(ref.eval_pressure_basis(r).sum(axis=1), 1.0, atol=1e-13)
    M = ref.Psi.T @ (ref.wq[:, None] * ref.Psi)
    W = np.array([gw[i] * gw[j] * gw[l] for l in range(m) for j in range(m) for i in range(m)])
    assert np.allclose(M, np.diag(W), atol=1e-13)


# ---------------------------------------------------------------- P8 worked example (figure "interp")
def test_hanging_interpolation_worked_example():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "interp_k3_right_half.txt")) if l[0] != "#"]
    parent = np.array([[float(a), float(b)] for kind, a, b in rows if kind == "parent"])
    child = np.array([[float(a), float(b)] for kind, a, b in rows if kind == "child"])
    # mesh: column 0 refined, column 1 coarse; the coarse column's -x face carries a cubic in y
    mesh = column_mesh(3, 2, 1, 1, refined=np.array([[True], [False]]), extent=(2.0, 1.0, 1.0))
    ref = ReferenceElement(3)
    V, _ = lagrange(ref.xi, 2.0 * mesh.node_logical[:, 1] - 1.0)
    u = np.zeros((3, mesh.n_nodes))
    u[0] = V @ parent[:, 1]
    o = StokesOracle(mesh)
    ue = o.gather(u)
    # fine element in column 0 with child position hy = 1 (upper half in y), bottom layer
    e = [i for i in range(mesh.n_el) if mesh.elem_level[i] == 1 and tuple(mesh.elem_cell[i]) == (1, 1, 0)][0]
    P = 4
    vals = np.array([ue[e, 3 + P * a1, 0] for a1 in range(P)])      # slots (a0 = 3, a1, a2 = 0)
    assert np.allclose(vals, child[:, 1], atol=2e-4)
    # and the positions printed are the half-interval GLL nodes
    assert np.allclose((ref.xi + 1) / 2, child[:, 0], atol=1e-4)


# ---------------------------------------------------------------- P9 continuity across hanging faces
@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("refine_from", [0, 1])
def test_hanging_continuity(k, refine_from):
    """The gathered field is continuous across every face between a fine and a coarse element:
    lateral faces, and with partially refined columns the -z face on top of a coarse element."""
    mesh = hanging_mesh(k, seed=3, nx=3, ny=3, frac=0.35, refine_from=refine_from)
    o = StokesOracle(mesh)
    ref = o.ref
    rng = np.random.default_rng(0)
    u = rng.uniform(-1, 1, (3, mesh.n_nodes))
    ue = o.gather(u)
    lo, size = mesh.elem_box()
    coarse = {tuple(mesh.elem_cell[e]): e for e in range(mesh.n_el) if mesh.elem_level[e] == 0}
    checked, checked_z = 0, 0
    for e in np.nonzero(mesh.elem_level == 1)[0]:
        for d in range(3):
            for side in range(2):
                # point on the fine element's face (d, side), random in the tangential directions
                xi = rng.uniform(-1, 1, 3)
                xi[d] = 2 * side - 1
                p = lo[e] + size[e] * (xi + 1) / 2
                nb = np.floor(p).astype(int)
                nb[d] = int(np.floor(p[d] + (1e-9 if side else -1e-9)))
                ce = coarse.get(tuple(nb))
                if ce is None:
                    continue
                xc = 2.0 * (p - lo[ce]) - 1.0
                vf = ref.eval_basis(xi[None])[0] @ ue[e]
                vc = ref.eval_basis(xc[None])[0] @ ue[ce]
                assert np.allclose(vf, vc, atol=1e-13), (e, d, side)
                checked += 1
                checked_z += d == 2
    assert checked > 10
    assert (checked_z > 4) == (refine_from > 0)


def _element_at(mesh, q):
    """An element whose logical box contains q (brute force), with q's reference coordinates."""
    lo, size = mesh.elem_box()
    inside = np.all((q >= lo - 1e-12) & (q <= lo + size[:, None] + 1e-12), axis=1)
    e = int(np.nonzero(inside)[0][0])
    return e, 2.0 * (q - lo[e]) / size[e] - 1.0


@pytest.mark.parametrize("k", [2, 3, 4])
def test_periodic_continuity(k):
    """Periodic x and y with refined columns on the boundary: the gathered field of every element
    agrees, at random points of its lateral faces, with the element on the other side -- across the
    identified boundaries through the translate of the point by the number of columns."""
    refined = np.zeros((4, 3), dtype=bool)
    refined[0, 1] = refined[3, 0] = refined[1, 2] = True
    mesh = column_mesh(k, 4, 3, 2, refined=refined, extent=(8.0, 6.0, 1.0), periodic=(True, True))
    o = StokesOracle(mesh)
    rng = np.random.default_rng(1)
    ue = o.gather(rng.uniform(-1, 1, (3, mesh.n_nodes)))
    lo, size = mesh.elem_box()
    n = np.array([mesh.nx, mesh.ny, 1e9])
    across = 0
    for e in range(mesh.n_el):
        for d in range(2):
            for side in range(2):
                xi = rng.uniform(-1, 1, 3)
                xi[d] = 2 * side - 1
                p = lo[e] + size[e] * (xi + 1) / 2
                q = p.copy()
                q[d] += (2 * side - 1) * 1e-9
                wrapped = q[d] < 0 or q[d] > n[d]
                q[d] = np.mod(q[d], n[d])
                f, _ = _element_at(mesh, q)
                q[d] -= (2 * side - 1) * 1e-9
                xf = 2.0 * (q - lo[f]) / size[f] - 1.0
                xf[d] = np.clip(xf[d], -1, 1)
                vf = o.ref.eval_basis(xi[None])[0] @ ue[e]
                vg = o.ref.eval_basis(xf[None])[0] @ ue[f]
                assert np.allclose(vf, vg, atol=1e-12), (e, d, side)
                across += wrapped
    assert across > 20


@pytest.mark.parametrize("k", [2, 3])
def test_periodic_equals_identified_assembly(k):
    """Refined columns away from the boundary: the periodic residual and Jacobian equal those of the
    non-periodic mesh with the boundary nodes identified, r_per = Pi^T r(Pi u), K_per = Pi^T K Pi, with
    Pi the map from the non-periodic nodes to their periodic nodes (logical position modulo the
    number of columns); the element geometry is the same."""
    refined = np.zeros((4, 4), dtype=bool)
    refined[1, 2] = refined[2, 1] = True
    kw = dict(refined=refined, geometry=terrain(4, 4, 2, 40.0))
    mp = column_mesh(k, 4, 4, 2, periodic=(True, True), **kw)
    mn = column_mesh(k, 4, 4, 2, **kw)
    key = lambda lg: np.round(np.mod(lg, [4, 4, 1e9]) * 64).astype(np.int64) @ np.array([1, 10 ** 5, 10 ** 10])
    kp = {int(v): i for i, v in enumerate(key(mp.node_logical))}
    pi = np.array([kp[int(v)] for v in key(mn.node_logical)])
    Pi = sp.csr_matrix((np.ones(mn.n_nodes), (np.arange(mn.n_nodes), pi)), shape=(mn.n_nodes, mp.n_nodes))
    rng = np.random.default_rng(4)
    logA, beta = rng.normal(0, 0.5, mp.n_el), np.exp(rng.normal(0, 1, mp.n_bface))
    u = rng.uniform(-1, 1, (3, mp.n_nodes))
    p = rng.uniform(-1, 1, (mp.n_el, mp.n_p))
    op = StokesOracle(mp, 3.0, 1e-10, 0.5, logA, beta, body=(0.0, 0.1, -1.0))
    on = StokesOracle(mn, 3.0, 1e-10, 0.5, logA, beta, body=(0.0, 0.1, -1.0))
    assert np.allclose(op.detJ, on.detJ, rtol=1e-13)
    op.set_state(u, p)
    on.set_state(np.stack([Pi @ u[c] for c in range(3)]), p)
    ru_p, rp_p = op.residual()
    ru_n, rp_n = on.residual()
    assert np.allclose(ru_p, np.stack([Pi.T @ ru_n[c] for c in range(3)]), rtol=0, atol=1e-12 * np.abs(ru_n).max())
    assert np.allclose(rp_p, rp_n, rtol=0, atol=1e-14)
    P3 = sp.block_diag([Pi] * 3 + [sp.eye(mp.n_el * mp.n_p)], format="csr")
    Kp, Kn = op.jacobian(), on.jacobian()
    D = (Kp - P3.T @ Kn @ P3).tocoo()
    assert np.max(np.abs(D.data), initial=0.0) < 1e-12 * np.abs(Kn.data).max()


def _random_frames(rng, n):
    q, _ = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    return q


def _frames_block(mesh, Qn):
    """Block-diagonal Q on velocity dofs (c*N + node) extended by the identity on pressures."""
    N = mesh.n_nodes
    Qb = sp.lil_matrix((3 * N, 3 * N))
    for c in range(3):
        for d in range(3):
            Qb[c * N + np.arange(N), d * N + np.arange(N)] = Qn[:, c, d]
    return sp.block_diag([Qb.tocsr(), sp.eye(mesh.n_el * mesh.n_p)], format="csr")


@pytest.mark.parametrize("k", [2, 3])
def test_frames_change_variables(k):
    """Random orthonormal frames on the basal nodes, no mask: the framed operator is Q^T K Q and the
    framed residual Q^T r(Q u_hat) for the unframed K and r (catches Q and Q^T swapped in the
    gather or in the scatter)."""
    mesh = hanging_mesh(k, nx=3, ny=3, frac=0.35, geometry=terrain(3, 3, 2, 40.0))
    rng = np.random.default_rng(9)
    base = np.nonzero(mesh.node_logical[:, 2] == 0.0)[0]
    Qn = np.tile(np.eye(3), (mesh.n_nodes, 1, 1))
    Qn[base] = _random_frames(rng, base.shape[0])
    logA, beta = rng.normal(0, 0.5, mesh.n_el), np.exp(rng.normal(0, 1, mesh.n_bface))
    uh = rng.uniform(-1, 1, (3, mesh.n_nodes))
    p = rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    o = StokesOracle(mesh, 3.0, 1e-10, 0.5, logA, beta, body=(0.0, 0.1, -1.0))
    o.set_state(np.einsum("nij,jn->in", Qn, uh), p)
    mesh.frame_nodes, mesh.frames = base.astype(np.int32), Qn[base]
    of = StokesOracle(mesh, 3.0, 1e-10, 0.5, logA, beta, body=(0.0, 0.1, -1.0))
    of.set_state(uh, p)
    Qb = _frames_block(mesh, Qn)
    K, Kf = o.jacobian(), of.jacobian()
    assert abs(Kf - Qb.T @ K @ Qb).max() < 1e-12 * abs(K).max()
    r = np.concatenate([a.ravel() for a in o.residual()])
    rf = np.concatenate([a.ravel() for a in of.residual()])
    assert np.allclose(rf, Qb.T @ r, rtol=0, atol=1e-12 * np.abs(r).max())


def test_frames_on_flat_base_match_component_mask():
    """Flat base, frames with the normal e_z and tangents turned in the plane by a per-node angle,
    normal component masked: the framed operator is Q~^T J_mask Q~, J_mask the operator with the
    z component of the basal nodes masked (u_z = 0)."""
    rng = np.random.default_rng(10)
    ref = random_refined_columns(3, 3, 0.35, rng)
    m0 = column_mesh(3, 3, 3, 2, refined=ref, extent=(30.0, 30.0, 1.0), base_normal_dirichlet=True)
    mf = column_mesh(3, 3, 3, 2, refined=ref, extent=(30.0, 30.0, 1.0), base_frames=True)
    assert np.array_equal(m0.dmask, mf.dmask)
    ang = rng.uniform(0, 2 * np.pi, mf.frame_nodes.shape[0])
    c, s = np.cos(ang), np.sin(ang)
    Qf = np.zeros((ang.shape[0], 3, 3))
    Qf[:, 0, 0], Qf[:, 0, 1], Qf[:, 1, 0], Qf[:, 1, 1], Qf[:, 2, 2] = c, -s, s, c, 1.0
    assert np.allclose(mf.frames[:, :, 2], [0, 0, 1])
    mf.frames = Qf
    Qn = np.tile(np.eye(3), (mf.n_nodes, 1, 1))
    Qn[mf.frame_nodes] = Qf
    logA, beta = rng.normal(0, 0.5, m0.n_el), np.exp(rng.normal(0, 1, m0.n_bface))
    u = rng.uniform(-1, 1, (3, m0.n_nodes))
    p = rng.uniform(-1, 1, (m0.n_el, m0.n_p))
    o0 = StokesOracle(m0, 3.0, 1e-10, 0.5, logA, beta)
    o0.set_state(u, p)
    of = StokesOracle(mf, 3.0, 1e-10, 0.5, logA, beta)
    of.set_state(np.einsum("nji,jn->in", Qn, u), p)
    Qb = _frames_block(mf, Qn)
    K0, Kf = o0.jacobian(), of.jacobian()
    assert abs(Kf - Qb.T @ K0 @ Qb).max() < 1e-12 * abs(K0).max()


# ---------------------------------------------------------------- P1 rigid modes, P2 kernel of B
@pytest.mark.parametrize("k,pspace", [(2, "P"), (3, "P"), (4, "P"), (3, "Q"), (4, "Q")])
@pytest.mark.parametrize("mapped", [False, True])
def test_rigid_modes_in_kernel(k, pspace, mapped):
    geo = terrain(4, 4, 2, 40.0) if mapped else None
    mesh = hanging_mesh(k, geometry=geo, pspace=pspace)
    rng = np.random.default_rng(2)
    o = StokesOracle(mesh, 3.0, 1e-10, 0.5, rng.normal(0, 0.5, mesh.n_el), np.zeros(mesh.n_bface))
    o.set_state(rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p)))
    K = o.jacobian()
    x = np.concatenate([rigid(mesh).ravel(), np.zeros(mesh.n_el * mesh.n_p)])
    y = K @ x
    assert np.max(np.abs(y) / (scale_of(K, x) + 1e-300)) < 1e-11
    # residual of a rigid motion with zero pressure vanishes (D(u) = 0, div u = 0)
    o.set_state(rigid(mesh), np.zeros((mesh.n_el, mesh.n_p)))
    r_u, r_p = o.residual()
    mu_max = np.max(o.mu)
    assert np.max(np.abs(r_u)) < 1e-11 * mu_max * np.max(np.abs(rigid(mesh)))
    assert np.max(np.abs(r_p)) < 1e-12


@pytest.mark.parametrize("k,pspace", [(2, "P"), (3, "Q"), (4, "P")])
def test_rigid_modes_zface_hanging(k, pspace):
    """Rigid motions stay in the kernel of the Jacobian on a mapped mesh whose refined columns start
    one layer up (fine elements hanging on a coarse element through their -z face)."""
    mesh = hanging_mesh(k, nx=3, ny=3, frac=0.35, geometry=terrain(3, 3, 2, 40.0), pspace=pspace, refine_from=1)
    assert ((mesh.cmask >> 7) & 1).sum() > 0
    rng = np.random.default_rng(5)
    o = StokesOracle(mesh, 3.0, 1e-10, 0.5, rng.normal(0, 0.5, mesh.n_el), np.zeros(mesh.n_bface))
    o.set_state(rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p)))
    K = o.jacobian()
    x = np.concatenate([rigid(mesh).ravel(), np.zeros(mesh.n_el * mesh.n_p)])
    assert np.max(np.abs(K @ x) / (scale_of(K, x) + 1e-300)) < 1e-11


@pytest.mark.parametrize("k,pspace", [(2, "P"), (3, "Q"), (4, "P")])
def test_picard_operator_reproduces_residual(k, pspace):
    """The Picard operator is the Stokes operator with the viscosity frozen at u, so applied to the
    state itself it returns the residual: J_picard(u) (u, p) = r(u, p) + P f (P the Dirichlet mask,
    f the load).  The Newton operator does not (its anisotropic term adds -c'(D:D) D), which the
    second check confirms."""
    mesh = hanging_mesh(k, nx=3, ny=3, frac=0.35, geometry=terrain(3, 3, 2, 40.0), mask=True, pspace=pspace)
    rng = np.random.default_rng(8)
    logA, beta = rng.normal(0, 0.5, mesh.n_el), np.exp(rng.normal(0, 1, mesh.n_bface))
    u = rng.uniform(-1, 1, (3, mesh.n_nodes))
    p = rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    x = np.concatenate([u.ravel(), p.ravel()])
    gaps = {}
    for picard in (True, False):
        o = StokesOracle(mesh, 3.0, 1e-10, 0.5, logA, beta, body=(0.0, 0.1, -1.0), picard=picard)
        o.set_state(u, p)
        K = o.jacobian()
        r = np.concatenate([a.ravel() for a in o.residual()])
        f = np.concatenate([(o.pmask * o.load_vector()).ravel(), np.zeros(mesh.n_el * mesh.n_p)])
        gaps[picard] = np.max(np.abs(K @ x - r - f) / (scale_of(K, x) + np.abs(f) + 1e-300))
    assert gaps[True] < 1e-12
    assert gaps[False] > 1e-3


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("pspace", ["P", "Q"])
def test_divergence_free_in_kernel_of_B(k, pspace):
    mesh = hanging_mesh(k, extent=(4.0, 4.0, 1.0), pspace=pspace)
    o = StokesOracle(mesh)
    o.set_state(np.zeros((3, mesh.n_nodes)), np.zeros((mesh.n_el, mesh.n_p)))
    x, y, z = mesh.coords
    K = o.jacobian()
    N = 3 * mesh.n_nodes
    Bg = K[N:, :N]
    u = np.stack([y ** 2, z ** 2, x ** 2]).ravel()                    # div u = 0, degree 2 <= k
    assert np.max(np.abs(Bg @ u)) < 1e-12 * np.max(np.abs(Bg)) * np.max(np.abs(u)) * 10
    # u = (x, 0, 0): div u = 1, so (B u)_m = -int psi_m: P_{k-1} (orthonormal) -2 sqrt(2) |K|/8 delta_m0;
    # Q_{k-2} (Gauss-point Lagrange) -|K|/8 times the product of the exact Gauss weights of mode m
    u1 = np.concatenate([x, 0 * x, 0 * x])
    Bu = (Bg @ u1).reshape(mesh.n_el, mesh.n_p)
    vol = np.where(mesh.elem_level == 0, 1.0, 0.125) * (4.0 / 4) * (4.0 / 4) * (1.0 / 2)
    expect = np.zeros_like(Bu)
    if pspace == "P":
        expect[:, 0] = -2.0 * np.sqrt(2.0) * vol / 8.0
    else:
        m = k - 1
        _, gw = exact_gauss(m)
        W = np.array([gw[i] * gw[j] * gw[l] for l in range(m) for j in range(m) for i in range(m)])
        expect[:] = -vol[:, None] / 8.0 * W[None, :]
    assert np.allclose(Bu, expect, atol=1e-13)


# ---------------------------------------------------------------- P3 linear Stokes (n = 1)
def _exact_1d(k):
    """1D mass M_ab = int l_a l_b, stiffness S_ab = int l_a' l_b', mixed G_ab = int l_a' l_b on [-1, 1],
    by exact symbolic integration of the Lagrange polynomials on the exact GLL nodes."""
    x = sympy.Symbol("x")
    roots = sorted(sympy.solve(sympy.diff(sympy.legendre(k, x), x), x), key=lambda r: float(r))
    nodes = [sympy.Integer(-1)] + roots + [sympy.Integer(1)]
    ell = []
    for a in range(k + 1):
        e = sympy.Integer(1)
        for b in range(k + 1):
            if b != a:
                e *= (x - nodes[b]) / (nodes[a] - nodes[b])
        ell.append(sympy.expand(e))
    M = np.array([[float(sympy.integrate(ell[a] * ell[b], (x, -1, 1))) for b in range(k + 1)] for a in range(k + 1)])
    S = np.array([[float(sympy.integrate(sympy.diff(ell[a], x) * sympy.diff(ell[b], x), (x, -1, 1)))
                   for b in range(k + 1)] for a in range(k + 1)])
    G = np.array([[float(sympy.integrate(sympy.diff(ell[a], x) * ell[b], (x, -1, 1))) for b in range(k + 1)]
                  for a in range(k + 1)])
    return M, S, G


@pytest.mark.parametrize("k", [2, 3])
def test_linear_stokes_kronecker_closed_form(k):
    """At n = 1, A_e = mu/2 (delta_cd int grad phi_s . grad phi_t + int d_d phi_s d_c phi_t) on a box,
    with each integral a Kronecker product of exact 1D matrices."""
    h = np.array([3.0, 2.0, 0.5])
    mesh = column_mesh(k, 1, 1, 1, extent=tuple(h))
    o = StokesOracle(mesh, n=1.0, eps=1e-10, B0=0.7)
    rng = np.random.default_rng(0)
    o.set_state(rng.uniform(-1, 1, (3, mesh.n_nodes)), np.zeros((1, mesh.n_p)))
    A, _ = o.element_matrices()
    M, S, G = _exact_1d(k)
    sc = 2.0 / h
    vol8 = np.prod(h) / 8.0
    one = [M, M, M]

    def integral(i, j):
        """int d_i phi_s d_j phi_t (s rows, t columns) as a Kronecker product (lexicographic a0 fastest)."""
        mats = []
        for ax in range(3):
            if ax == i and ax == j:
                mats.append(S * sc[ax] ** 2)
            elif ax == i:
                mats.append(G * sc[ax])
            elif ax == j:
                mats.append(G.T * sc[ax])
            else:
                mats.append(one[ax])
        return vol8 * np.kron(mats[2], np.kron(mats[1], mats[0]))

    P3 = (k + 1) ** 3
    mu = 0.7
    Kst = sum(integral(i, i) for i in range(3))
    ref = np.zeros((3, P3, 3, P3))
    for c in range(3):
        for d in range(3):
            ref[c, :, d, :] = 0.5 * mu * ((c == d) * Kst + integral(d, c))
    assert np.allclose(A.reshape(3, P3, 3, P3), ref, atol=1e-12 * np.abs(ref).max())


def test_linear_stokes_residual_is_linear():
    """n = 1: J is independent of u and r(u + v) - r(u) = J v (Sec. 2.1: linear rheology)."""
    mesh = hanging_mesh(3, mask=True)
    rng = np.random.default_rng(5)
    beta = rng.uniform(0.5, 2, mesh.n_bface)
    o = StokesOracle(mesh, n=1.0, eps=1e-10, B0=0.5, beta=beta)
    u, p = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    v, q = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    o.set_state(u, p)
    K1 = o.jacobian().copy()
    r0u, r0p = o.residual()
    o.set_state(u + v, p + q)
    K2 = o.jacobian()
    r1u, r1p = o.residual()
    assert abs(K1 - K2).max() < 1e-13 * abs(K1).max()
    ju, jp = o.jacobian_apply(v, q)
    assert np.allclose(r1u - r0u, ju, atol=1e-12 * np.abs(ju).max())
    assert np.allclose(r1p - r0p, jp, atol=1e-12 * np.abs(jp).max())


# ---------------------------------------------------------------- P4 symmetry, P5 Newton consistency
@pytest.mark.parametrize("k,pspace", [(2, "P"), (3, "P"), (3, "Q")])
def test_jacobian_symmetric_and_complex_step(k, pspace):
    geo = terrain(3, 3, 2, 30.0)
    mesh = hanging_mesh(k, seed=7, nx=3, ny=3, frac=0.35, mask=True, geometry=geo, pspace=pspace)
    rng = np.random.default_rng(11)
    o = StokesOracle(mesh, 3.0, 1e-10, 0.5, rng.normal(0, 0.5, mesh.n_el), np.exp(rng.normal(0, 1, mesh.n_bface)),
                     body=(0.0, 0.1, -1.0))
    u, p = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    o.set_state(u, p)
    K = o.jacobian()
    assert abs(K - K.T).max() < 1e-13 * abs(K).max()
    v, q = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    ju, jp = o.jacobian_apply(v, q)
    h = 1e-30
    o.set_state(u + 1j * h * v, p + 1j * h * q)
    ru, rp = o.residual()
    assert np.max(np.abs(ru.imag / h - ju)) < 1e-12 * np.max(np.abs(ju))
    assert np.max(np.abs(rp.imag / h - jp)) < 1e-12 * np.max(np.abs(jp))
    # central finite differences (h = 1e-6), the check named for the VJP workload
    hh = 1e-6
    o.set_state(u + hh * v, p + hh * q)
    ru1, _ = o.residual()
    o.set_state(u - hh * v, p - hh * q)
    ru0, _ = o.residual()
    assert np.max(np.abs((ru1 - ru0) / (2 * hh) - ju)) < 1e-6 * np.max(np.abs(ju))


# ---------------------------------------------------------------- P6 energy functional
def test_residual_is_energy_gradient():
    mesh = hanging_mesh(2, seed=4, mask=True, geometry=terrain(4, 4, 2, 40.0))
    rng = np.random.default_rng(3)
    o = StokesOracle(mesh, 3.0, 1e-10, 0.5, rng.normal(0, 0.5, mesh.n_el), rng.uniform(0.5, 2, mesh.n_bface),
                     body=(0.0, 0.0, -1.0))
    u = rng.uniform(-1, 1, (3, mesh.n_nodes))
    v = rng.uniform(-1, 1, (3, mesh.n_nodes)) * o.pmask
    o.set_state(u, np.zeros((mesh.n_el, mesh.n_p)))
    r_u, _ = o.residual()
    h = 1e-30
    dE = o.energy(u + 1j * h * v).imag / h
    assert abs(np.sum(r_u * v) - dE) < 1e-12 * np.sum(np.abs(r_u * v))


# ---------------------------------------------------------------- P7 positivity of the Newton tensor
def test_newton_tensor_eigenvalues():
    rng = np.random.default_rng(0)
    for n in (1.0, 2.0, 3.0, 4.0):
        for _ in range(50):
            A = rng.normal(size=(3, 3)) * 10 ** rng.uniform(-6, 3)
            D = 0.5 * (A + A.T)
            II = 0.5 * np.sum(D * D)
            C = newton_tensor(D, 1.0, II, n, 1e-10)
            # restrict to symmetric tensors: orthonormal basis of Sym(3)
            Bs = []
            for i in range(3):
                for j in range(i, 3):
                    E = np.zeros((3, 3))
                    E[i, j] = E[j, i] = 1.0
                    Bs.append(E.ravel() / np.linalg.norm(E))
            Bs = np.array(Bs)
            ev = np.linalg.eigvalsh(Bs @ C @ Bs.T)
            assert ev.min() >= 1.0 / n - 1e-12 and ev.max() <= 1.0 + 1e-12
            # the smallest one is 1 - (n-1)/n * II/(II+eps), attained along D
            assert abs(ev.min() - (1.0 - (n - 1.0) / n * II / (II + 1e-10))) < 1e-9


# ---------------------------------------------------------------- boundary / geometry closed forms
def test_basal_term_and_load_closed_forms():
    """beta = 1 on a flat base: <e_x, M e_x> = base area; <e_z, M e_z> = 0 (T removes the normal);
    f(1) = int b = b * volume."""
    mesh = hanging_mesh(3, extent=(6.0, 5.0, 0.8))
    o = StokesOracle(mesh, beta=np.ones(mesh.n_bface), body=(0.0, 0.0, -2.0))
    o.set_state(np.zeros((3, mesh.n_nodes)), np.zeros((mesh.n_el, mesh.n_p)))
    A, _ = o.element_matrices()
    S = o.S
    tot_x = tot_z = mag = 0.0
    for j, el in enumerate(o.fl):
        Ae = A[el].reshape(3, S, 3, S)
        tot_x += Ae[0, :, 0, :].sum()
        tot_z += Ae[2, :, 2, :].sum()
        mag += np.abs(Ae).sum()
    # the stress part of A annihilates constants, so only the basal term remains (up to the
    # rounding of the stress entries, mu ~ 1e3 at zero strain rate)
    assert abs(tot_x - 30.0) < 1e-14 * mag and abs(tot_z) < 1e-14 * mag
    f = o.load_vector()
    assert abs(f[2].sum() + 2.0 * 6.0 * 5.0 * 0.8) < 1e-11 and abs(f[0].sum()) < 1e-13


def test_mapped_volume_closed_form():
    """Sum of w detJ = exact volume for a thickness linear in x (reproduced by Q_k)."""
    L, nx, nz = 10.0, 3, 2

    def geo(lg):
        x, y = lg[:, 0] * L / nx, lg[:, 1] * L / nx
        return np.stack([x, y, lg[:, 2] / nz * (1.0 + 0.05 * x)], 1)

    mesh = hanging_mesh(3, nx=nx, ny=nx, nz=nz, geometry=geo)
    o = StokesOracle(mesh)
    vol = L * L * (1.0 + 0.05 * L / 2)
    assert abs(o.W.sum() - vol) < 1e-11 * vol


def basal_blocks(o):
    """sum over the basal elements of e_d^T A_e e_c (3x3) and the magnitude of the summands: the stress
    part of A_e annihilates constant fields, so for beta = 1 only int_base (T e_c).(T e_d) remains."""
    A, _ = o.element_matrices()
    S = o.S
    tot, mag = np.zeros((3, 3)), 0.0
    for el in o.fl:
        Ae = A[el].reshape(3, S, 3, S)
        tot += Ae.sum(axis=(1, 3))
        mag += np.abs(Ae).sum()
    return tot, mag


@pytest.mark.parametrize("k", [2, 4])
def test_basal_term_inclined_plane_closed_form(k):
    """Column-mapped mesh over a planar inclined base z = a x + b y (with hanging columns), beta = 1:
    the face measure integrates to the tilted area Lx Ly sqrt(1 + a^2 + b^2), the face normal is
    (-a, -b, 1)/sqrt(1 + a^2 + b^2) at every face point, and sum over the basal blocks of
    <e_d, M e_c> = area (delta_cd - n_c n_d) (eq. (robin), eq. (weak)).  A projected measure |cr_z|
    or the reference normal e_z instead of the mapped one fails it."""
    a, b, Lx, Ly, nx, ny, nz = 0.3, -0.2, 12.0, 9.0, 4, 3, 2

    def geo(lg):
        x, y = lg[:, 0] * Lx / nx, lg[:, 1] * Ly / ny
        H = 1.0 + 0.02 * x - 0.01 * y
        return np.stack([x, y, a * x + b * y + lg[:, 2] / nz * H], 1)

    mesh = hanging_mesh(k, seed=3, nx=nx, ny=ny, nz=nz, frac=0.35, geometry=geo)
    assert (mesh.cmask >> 3).any()                     # hanging faces present
    o = StokesOracle(mesh, beta=np.ones(mesh.n_bface))
    o.set_state(np.zeros((3, mesh.n_nodes)), np.zeros((mesh.n_el, mesh.n_p)))
    s = np.sqrt(1.0 + a * a + b * b)
    area = Lx * Ly * s
    nrm = np.array([-a, -b, 1.0]) / s
    assert abs(o.Wf.sum() - area) < 1e-12 * area
    assert np.max(np.abs(o.fn - nrm)) < 1e-13
    tot, mag = basal_blocks(o)
    expect = area * (np.eye(3) - np.outer(nrm, nrm))
    assert np.max(np.abs(tot - expect)) < 1e-13 * mag


def test_basal_term_twisted_base_quadrature():
    """Curved (doubly ruled) base z = c (x - x0)(y - y0), exactly reproduced by the Q_k map: the
    basal blocks sum to int_base (I - n n^T) dS with the mapped normal n = (-z_x, -z_y, 1)/s and
    dS = s dx dy, s = sqrt(1 + z_x^2 + z_y^2), here evaluated by adaptive 2D quadrature of the
    closed-form integrand (scipy), independent of the oracle's face quadrature; agreement to the
    (k+1)^2-point Gauss error on the smooth integrand."""
    from scipy.integrate import dblquad
    c, Lx, Ly, nx, ny, nz, k = 0.004, 20.0, 16.0, 4, 4, 2, 4
    x0, y0 = 7.0, 5.0

    def geo(lg):
        x, y = lg[:, 0] * Lx / nx, lg[:, 1] * Ly / ny
        return np.stack([x, y, c * (x - x0) * (y - y0) + lg[:, 2] / nz * 1.5], 1)

    mesh = hanging_mesh(k, seed=5, nx=nx, ny=ny, nz=nz, frac=0.3, geometry=geo)
    o = StokesOracle(mesh, beta=np.ones(mesh.n_bface))
    o.set_state(np.zeros((3, mesh.n_nodes)), np.zeros((mesh.n_el, mesh.n_p)))

    def integrand(i, j):
        def f(y, x):
            g = np.array([-c * (y - y0), -c * (x - x0), 1.0])
            sc = np.linalg.norm(g)
            n = g / sc
            return ((1.0 if i == j else 0.0) - n[i] * n[j]) * sc
        return f

    expect = np.zeros((3, 3))
    for i in range(3):
        for j in range(i, 3):
            expect[i, j] = expect[j, i] = dblquad(integrand(i, j), 0.0, Lx, 0.0, Ly, epsabs=1e-13, epsrel=1e-13)[0]
    tot, mag = basal_blocks(o)
    assert np.max(np.abs(tot - expect)) < 1e-9 * abs(expect).max()
    # the normal varies over the base: a constant (reference) normal would miss the x-y coupling
    assert abs(expect[0, 1]) > 1e-4 * abs(expect).max()


# ---------------------------------------------------------------- P11 VJP closed forms / complex step
def test_vjp_parameter_gradients_complex_step():
    mesh = hanging_mesh(2, seed=9, nx=3, ny=3, mask=True)
    rng = np.random.default_rng(4)
    logA = rng.normal(0, 0.5, mesh.n_el)
    beta = np.exp(rng.normal(0, 1, mesh.n_bface))
    u, p = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    w_u, w_p = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    o = StokesOracle(mesh, 3.0, 1e-10, 0.5, logA, beta)
    o.set_state(u, p)
    g_u, g_p, g_logA, g_beta = o.vjp(w_u, w_p)
    ju, jp = o.jacobian_apply(w_u, w_p)
    assert np.allclose(g_u, ju, atol=1e-13 * np.abs(ju).max())          # J symmetric
    h = 1e-30
    for e in rng.choice(mesh.n_el, 6, replace=False):
        la = logA.astype(complex)
        la[e] += 1j * h
        oc = StokesOracle(mesh, 3.0, 1e-10, 0.5, la.real, beta)
        oc.Be = oc.B0 * np.exp(-la[oc.elems] / oc.n)
        oc.set_state(u, p)
        ru, rp = oc.residual()
        d = (np.sum(w_u * ru) + np.sum(w_p * rp)).imag / h
        assert abs(d - g_logA[e]) < 1e-12 * (abs(g_logA[e]) + 1e-300) + 1e-14
    for f in rng.choice(mesh.n_bface, 6, replace=False):
        bc = beta.astype(complex)
        bc[f] += 1j * h
        oc = StokesOracle(mesh, 3.0, 1e-10, 0.5, logA, beta)
        oc.beta = bc
        oc.set_state(u, p)
        ru, rp = oc.residual()
        d = (np.sum(w_u * ru) + np.sum(w_p * rp)).imag / h
        assert abs(d - g_beta[f]) < 1e-12 * (abs(g_beta[f]) + 1e-300) + 1e-14
    # closed form: at w = u (unmasked, p-part zero), sum_e g_logA = -(1/n) int mu D0:D0
    _, _, gA, _ = o.vjp(u, np.zeros_like(p))
    tot = -(1.0 / 3.0) * np.sum(o.W * o.mu * np.einsum("eqij,eqij->eq", o.D0, o.D0))
    assert abs(gA.sum() - tot) < 1e-12 * abs(tot)


def test_dirichlet_rows():
    mesh = hanging_mesh(2, mask=True)
    rng = np.random.default_rng(8)
    o = StokesOracle(mesh, beta=np.ones(mesh.n_bface))
    u, p = rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    o.set_state(u, p)
    r_u, _ = o.residual()
    m = mesh.dmask.astype(bool)
    assert m.sum() > 0 and np.array_equal(r_u[m], u[m])
    x = rng.uniform(-1, 1, (3, mesh.n_nodes))
    y, _ = o.jacobian_apply(x, np.zeros_like(p))
    assert np.array_equal(y[m], x[m])
    # changing masked components of x changes nothing else
    x2 = x.copy()
    x2[m] += 5.0
    y2, _ = o.jacobian_apply(x2, np.zeros_like(p))
    assert np.allclose(y2[~m], y[~m], atol=1e-13 * np.abs(y).max())


# ---------------------------------------------------------------- adjoint gradient (Sec. 2.3)
def test_adjoint_gradient_matches_resolved_finite_differences():
    """Phi(u) = 1/2 |u - u_obs|^2 at the solved state: the oracle's adjoint gradient (direct solve with
    J_c^T, then the parameter VJP) equals central differences (h = 1e-6) of Phi at states re-solved by
    Newton's method, for entries of logA and beta.  A wrong sign, a missing transpose of a
    nonsymmetric part or an unsolved state would break it."""
    from oracle import adjoint_gradient, newton_solve
    rng = np.random.default_rng(21)
    L, nx, nz = 20.0, 2, 1

    def geo(lg):
        x, y = lg[:, 0] * L / nx, lg[:, 1] * L / nx
        return np.stack([x, y, 0.05 * np.sin(2 * np.pi * x / L) + lg[:, 2] / nz * (1.0 + 0.1 * np.cos(2 * np.pi * y / L))], 1)

    mesh = hanging_mesh(2, seed=2, nx=nx, ny=nx, nz=nz, frac=0.5, mask=True, geometry=geo)
    logA = rng.normal(0, 0.5, mesh.n_el)
    beta = np.exp(rng.normal(0, 1, mesh.n_bface))
    body = (0.0, 0.0, -1.0)
    u0 = 0.1 * rng.uniform(-1, 1, (3, mesh.n_nodes))
    p0 = np.zeros((mesh.n_el, mesh.n_p))
    u_obs = rng.uniform(-1, 1, (3, mesh.n_nodes))

    def solve(la, be):
        o = StokesOracle(mesh, 3.0, 1e-10, 0.5, la, be, body=body)
        u, p, hist = newton_solve(o, u0, p0, tol=1e-14)
        assert hist[-1] <= 1e-12 * hist[0]
        return o, u, p

    o, u, p = solve(logA, beta)
    gA, gB, _, _ = adjoint_gradient(o, u - u_obs)
    phi = lambda v: 0.5 * np.sum((v - u_obs) ** 2)
    h = 1e-6
    for kind, idx in (("logA", 0), ("logA", mesh.n_el - 1), ("beta", 0), ("beta", mesh.n_bface - 1)):
        vals = []
        for sgn in (1.0, -1.0):
            la, be = logA.copy(), beta.copy()
            (la if kind == "logA" else be)[idx] += sgn * h
            vals.append(phi(solve(la, be)[1]))
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = (gA if kind == "logA" else gB)[idx]
        assert abs(fd - ad) < 1e-6 * abs(ad) + 1e-10 * phi(u), (kind, idx, fd, ad)
