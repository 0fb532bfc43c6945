"""Parity at the workloads' full sizes, on sampled outputs.

The oracle assembles only the elements of a few windows of whole columns (all layers) at the
full mesh sizes; the rows of the nodes whose incident elements all lie in a window are then exact
(every element whose restriction touches a node names it in its connectivity, hanging slots
included), and so are the pressure rows of every window element.  The windows are chosen so that
at least 2,000 velocity rows and 500 pressure rows are compared per workload, one of them placed on
refined columns (hanging faces) where the workload has any.  The engine runs in the production
launch configuration; FP64 rows must match to 1e-12 relative to (|K||x|)_i, FP32 rows to
64 * 2^-24 and the BF16-operator rows to 16 * 2^-9 (the per-entry bounds of the small parity tests).
Properties that hold at any size (FP32 vs FP64 over all rows) cover the rest.  For the VJP workload,
parameter gradients are also checked by central finite differences (h = 1e-6) of the engine's own
residual.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
MIN_VEL_ROWS, MIN_PRES_ROWS = 2000, 500
# window side (coarse columns) per workload, and the number of windows
WINDOWS = {2: (3, 3), 3: (3, 2), 4: (3, 3), 5: (3, 4)}
# the workloads as stated (P_{k-1} pressure), and config 2 with the Q_{k-2} pair (Q3 x Q1, the pair of
# the paper's large runs)
CASES = [(2, "P"), (3, "P"), (4, "P"), (5, "P"), (2, "Q")]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def coarse_columns(mesh):
    """Coarse column (i, j) of every element (fine elements of refined columns map to their parent)."""
    fine = mesh.elem_level == 1
    ci = np.where(fine, mesh.elem_cell[:, 0] // 2, mesh.elem_cell[:, 0])
    cj = np.where(fine, mesh.elem_cell[:, 1] // 2, mesh.elem_cell[:, 1])
    return ci, cj


def window_sample(mesh, rng, side, count):
    """Elements of `count` windows of side x side coarse columns (one centred on a refined column when
    there are any), the exactly computable velocity rows (nodes named only by window elements) and the
    window elements (their pressure rows)."""
    ci, cj = coarse_columns(mesh)
    refined = np.argwhere(mesh.refined)
    corners = []
    if refined.shape[0]:
        i, j = refined[rng.integers(refined.shape[0])]
        corners.append((int(np.clip(i - side // 2, 0, mesh.nx - side)), int(np.clip(j - side // 2, 0, mesh.ny - side))))
    while len(corners) < count:
        corners.append((int(rng.integers(0, mesh.nx - side + 1)), int(rng.integers(0, mesh.ny - side + 1))))
    inw = np.zeros(mesh.n_el, dtype=bool)
    for (i0, j0) in corners:
        inw |= (ci >= i0) & (ci < i0 + side) & (cj >= j0) & (cj < j0 + side)
    elems = np.nonzero(inw)[0]
    named_in = np.unique(mesh.elem_nodes[inw])
    named_out = np.unique(mesh.elem_nodes[~inw])
    nodes = np.setdiff1d(named_in, named_out, assume_unique=True)
    return elems, nodes, corners


@pytest.mark.parametrize("cfg,pspace", CASES)
def test_fullsize_sampled_parity(torch_cuda, cfg, pspace):
    torch = torch_cuda
    from meshgen import make_config
    from oracle import StokesOracle
    from paper_1406_6573_amd import Engine
    w = make_config(cfg, n_dirs=1, pspace=pspace)
    m = w.mesh
    print(f"[gpu] full-size config{cfg} pressure {pspace}: n_el={m.n_el} n_dof={m.n_dof}", flush=True)
    eng = Engine()
    eng.upload_mesh(m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
    eng.set_state(t(w.u), t(w.p))
    xu, xp = w.directions[0]
    ru, rp = eng.residual()
    yu, yp = eng.jacobian_apply(t(xu), t(xp))
    y32u, y32p = eng.jacobian_apply(t(xu).float(), t(xp).float(), "fp32")
    wu, wp = (w.adjoint if w.adjoint is not None else w.directions[0])
    g_u, g_p, g_A, g_b = eng.residual_vjp(t(wu), t(wp))
    torch.cuda.synchronize()
    # FP32 vs FP64 over all rows
    full64 = torch.cat([yu.reshape(-1), yp.reshape(-1)])
    full32 = torch.cat([y32u.reshape(-1), y32p.reshape(-1)]).double()
    e32 = float((full32 - full64).norm() / full64.norm())
    print(f"  fp32 vs fp64 over all {full64.numel()} rows: rel {e32:.2e}", flush=True)
    assert e32 < 1e-5
    ybu, ybp = eng.jacobian_apply(t(xu).float(), t(xp).float(), "bf16ops")
    # window rows against the oracle
    rng = np.random.default_rng(100 + cfg)
    side, count = WINDOWS[cfg]
    elems, nodes, corners = window_sample(m, rng, side, count)
    pel = elems
    N = m.n_nodes
    vrows = np.concatenate([c * N + nodes for c in range(3)])
    prow = (pel[:, None] * m.n_p + np.arange(m.n_p)[None, :]).ravel()
    print(f"  windows at {corners}: {len(elems)} elements, {vrows.size} velocity rows, {prow.size} pressure rows",
          flush=True)
    assert vrows.size >= MIN_VEL_ROWS and prow.size >= MIN_PRES_ROWS
    if m.refined.any():
        assert (m.cmask[elems] >> 3).any()          # hanging faces among the sampled elements
    o = StokesOracle(m, w.n, w.eps, w.B0, w.logA, w.beta, body=w.body, elems=elems)
    o.set_state(w.u, w.p)
    oru, orp = o.residual()
    K = o.jacobian()
    x = np.concatenate([xu.ravel(), xp.ravel()])
    oy = K @ x
    sc = abs(K) @ np.abs(x)
    gy = np.concatenate([yu.cpu().numpy().ravel(), yp.cpu().numpy().ravel()])
    rows = np.concatenate([vrows, 3 * N + prow])
    e_j = np.max(np.abs(gy[rows] - oy[rows]) / sc[rows])
    # mixed paths on the same rows, per entry against the FP64 oracle
    g32 = np.concatenate([y32u.double().cpu().numpy().ravel(), y32p.double().cpu().numpy().ravel()])
    gbf = np.concatenate([ybu.double().cpu().numpy().ravel(), ybp.double().cpu().numpy().ravel()])
    e_32 = np.max(np.abs(g32[rows] - oy[rows]) / sc[rows])
    e_bf = np.max(np.abs(gbf[rows] - oy[rows]) / sc[rows])
    print(f"  window rows: FP32 scaled {e_32:.2e} (bound {64 * U32:.2e}), BF16 operators scaled {e_bf:.2e} "
          f"(bound {16 * 2.0 ** -9:.2e})", flush=True)
    assert e_32 < 64 * U32 and e_bf < 16 * 2.0 ** -9
    gr = np.concatenate([ru.cpu().numpy().ravel(), rp.cpu().numpy().ravel()])
    orr = np.concatenate([oru.ravel(), orp.ravel()])
    rmag = np.max(np.abs(orr[rows]))
    e_r = np.max(np.abs(gr[rows] - orr[rows])) / rmag
    og_u, og_p, og_A, og_b = o.vjp(wu, wp)
    gg = np.concatenate([g_u.cpu().numpy().ravel(), g_p.cpu().numpy().ravel()])
    ogg = np.concatenate([og_u.ravel(), og_p.ravel()])
    wv = np.concatenate([np.asarray(wu).ravel(), np.asarray(wp).ravel()])
    e_v = np.max(np.abs(gg[rows] - ogg[rows]) / (abs(K) @ np.abs(wv))[rows])
    # logA gradient per element: a sum with cancellation over quadrature points; scale the error by the
    # sum of the magnitudes of its terms, (1/n) sum_q |w detJ mu D0 : D(w)|
    pos = np.searchsorted(o.elems, pel)
    we = o.gather(wu)
    Gw = np.einsum("esc,eqsi->eqci", we[pos], o.Gp[pos])
    Dw = 0.5 * (Gw + np.swapaxes(Gw, 2, 3))
    scale_A = np.sum(np.abs(o.W[pos] * o.mu[pos] * np.einsum("eqij,eqij->eq", o.D0[pos], Dw)), axis=1) / w.n
    e_a = np.max(np.abs(g_A.cpu().numpy()[pel] - og_A[pel]) / np.maximum(scale_A, 1e-300))
    print(f"  window rows: J scaled {e_j:.2e}, residual {e_r:.2e}, VJP u,p scaled {e_v:.2e}, logA {e_a:.2e}",
          flush=True)
    assert e_j < 1e-12 and e_r < 1e-12 and e_v < 1e-12 and e_a < 1e-12
    if m.n_bface and len(o.fid):
        fids = o.fid
        gb = g_b.cpu().numpy()[fids]
        e_b = np.max(np.abs(gb - og_b[fids]) / np.maximum(np.abs(og_b[fids]), 1e-300))
        print(f"  beta gradient on {len(fids)} faces: rel {e_b:.2e}", flush=True)
        assert e_b < 1e-11
    if cfg == 4:
        # central differences of <w, r> in logA and beta with the engine's own residual
        def wr(logA, beta):
            eng.set_params(w.n, w.eps, w.B0, w.body, t(logA), t(beta))
            eng.set_state(t(w.u), t(w.p))
            a, b = eng.residual()
            return float((a * t(wu)).sum() + (b * t(wp)).sum())
        h = 1e-6
        for e in rng.choice(m.n_el, 3, replace=False):
            la1, la0 = w.logA.copy(), w.logA.copy()
            la1[e] += h
            la0[e] -= h
            fd = (wr(la1, w.beta) - wr(la0, w.beta)) / (2 * h)
            print(f"  FD logA[{e}]: {fd:.8e} vs VJP {float(g_A[e]):.8e}", flush=True)
            assert abs(fd - float(g_A[e])) < 1e-5 * abs(float(g_A[e])) + 1e-8 * abs(wr(w.logA, w.beta))
        for f in rng.choice(m.n_bface, 3, replace=False):
            b1, b0 = w.beta.copy(), w.beta.copy()
            b1[f] += h
            b0[f] -= h
            fd = (wr(w.logA, b1) - wr(w.logA, b0)) / (2 * h)
            print(f"  FD beta[{f}]: {fd:.8e} vs VJP {float(g_b[f]):.8e}", flush=True)
            assert abs(fd - float(g_b[f])) < 1e-5 * abs(float(g_b[f])) + 1e-8 * abs(wr(w.logA, w.beta))
    eng.close()
