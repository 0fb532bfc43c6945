"""Block-Jacobi data, Krylov vector kernels and the Newton/FGMRES driver on the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import rel_err, small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def setup(torch, case):
    from paper_1406_6573_amd import Engine
    eng = Engine()
    eng.upload_mesh(case["mesh"])
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    eng.set_params(case["n"], case["eps"], case["B0"], case.get("body", (0, 0, 0)), t(case["logA"]), t(case["beta"]))
    eng.set_state(t(case["u"]), t(case["p"]))
    return eng, t


VARIANTS = {"": {}, "zface": dict(refine_from=1), "periodic": dict(periodic=(True, True), frac=0.4),
            "frames": dict(frames=True, frac=0.4),
            "all": dict(frames=True, frac=0.4, periodic=(True, True), refine_from=1)}


def node_frames(m):
    """Per-node frame Q_n [n_nodes, 3, 3] (identity for nodes without one)."""
    Qn = np.tile(np.eye(3), (m.n_nodes, 1, 1))
    if len(m.frame_nodes):
        Qn[m.frame_nodes] = m.frames
    return Qn


@pytest.mark.parametrize("k,mapped,pspace,variant", [(2, False, "P", ""), (3, True, "P", ""), (4, False, "P", ""),
                                                     (3, True, "Q", ""), (4, False, "Q", ""), (2, True, "P", "zface"),
                                                     (4, False, "P", "zface"), (3, True, "P", "periodic"),
                                                     (2, True, "P", "frames"), (4, True, "Q", "frames"),
                                                     (3, True, "P", "all")])
def test_jacobi_diag_matches_oracle(torch_cuda, k, mapped, pspace, variant):
    """d_u = sum_e sum_a R_e[a, n]^2 F_e[aa] (exact diagonal of F on conforming parts), 1 on masked
    rows; d_p = -sum_q w detJ psi_m^2 / mu."""
    from oracle import StokesOracle
    torch = torch_cuda
    case = small_case(k, mapped=mapped, pspace=pspace, **VARIANTS[variant])
    m = case["mesh"]
    eng, t = setup(torch, case)
    d_u, d_p = eng.jacobi_diag()
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"])
    o.set_state(case["u"], case["p"])
    A, _ = o.element_matrices()
    S = o.S
    # 3x3 slot blocks A_e[(c, a), (d, a)], summed with squared restriction weights per node, then
    # seen in the node's frame: d_c(n) = q_c(n)^T (sum_a R[a, n]^2 A_aa) q_c(n)
    idx = np.arange(S)
    blk = np.stack([np.stack([A[:, c * S + idx, d * S + idx].reshape(-1) for d in range(3)], -1)
                    for c in range(3)], -2)                       # [E*S, 3, 3]
    R2 = o.R.multiply(o.R).T.tocsr()
    Bn = np.stack([np.stack([R2 @ blk[:, c, d] for d in range(3)], -1) for c in range(3)], -2)   # [N, 3, 3]
    Qn = node_frames(m)
    ref_u = np.einsum("nca,ncd,nda->an", Qn, Bn, Qn)
    msk = m.dmask.astype(bool)
    ref_u[msk] = 1.0
    ref_p = -np.einsum("eq,qm->em", o.W / o.mu, o.ref.Psi ** 2)
    eu = np.max(np.abs(d_u.cpu().numpy() - ref_u) / np.abs(ref_u))
    ep = np.max(np.abs(d_p.cpu().numpy() - ref_p) / np.abs(ref_p))
    print(f"[gpu] jacobi diag k={k} mapped={mapped} {variant}: rel err u {eu:.2e} p {ep:.2e}", flush=True)
    assert eu < 1e-12 and ep < 1e-12
    # conforming slots: equals the assembled diagonal of J_c
    if not (m.cmask >> 3).any():
        assert np.allclose(ref_u.ravel(), o.jacobian().diagonal()[:3 * m.n_nodes], rtol=1e-13)
    inv_u, inv_p = eng.jacobi_diag(invert=True)
    assert torch.allclose(inv_u * d_u, torch.ones_like(d_u), rtol=1e-15, atol=0)
    eng.close()


def test_vector_kernels(torch_cuda):
    torch = torch_cuda
    from paper_1406_6573_amd import Engine
    eng = Engine()
    eng.upload_mesh(small_case(2)["mesh"])
    g = torch.Generator(device="cuda").manual_seed(0)
    n, k = 100003, 7
    for dt in (torch.float64, torch.float32):
        V = torch.rand((k, n), dtype=dt, device="cuda", generator=g) - 0.5
        w = torch.rand(n, dtype=dt, device="cuda", generator=g) - 0.5
        h = torch.empty(64, dtype=torch.float64, device="cuda")
        eng.vec_dots(V, k, w, h)
        ref = (V.double() @ w.double())
        assert torch.allclose(h[:k], ref, rtol=1e-12, atol=1e-12)
        w2 = w.clone()
        eng.vec_gemv(V, k, h, -0.5, w2)
        ref2 = (w.double() - 0.5 * (V.double().T @ h[:k]))
        assert torch.allclose(w2.double(), ref2, rtol=1e-6 if dt == torch.float32 else 1e-13, atol=1e-6)
        y = w.clone()
        eng.vec_axpby(2.0, V[0], -1.0, y)
        assert torch.allclose(y, 2.0 * V[0] - w)
        d = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
        z = torch.empty_like(w)
        eng.vec_mul(d, w, z)
        assert torch.allclose(z.double(), d * w.double(), rtol=1e-6)
        # device-side normalisation by a squared norm held on the device (0 for a zero norm)
        nrm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        eng.vec_dots(w.view(1, -1), 1, w, nrm2)
        y = w.clone()
        eng.vec_normalize(nrm2, y)
        assert torch.allclose(y.double(), w.double() / w.double().norm(), rtol=1e-6 if dt == torch.float32 else 1e-14)
        nrm2.zero_()
        eng.vec_normalize(nrm2, y)
        assert torch.count_nonzero(y) == 0
        # b = 0: y is written without being read (BLAS convention), so NaN or Inf bits in an
        # uninitialised y cannot leak into the result
        y = torch.full_like(w, float("nan"))
        y[::2] = float("inf")
        eng.vec_axpby(-3.0, w, 0.0, y)
        assert torch.equal(y, (-3.0 * w.double()).to(dt))
    # basis rows padded to a 16-byte multiple (the driver's layout): the 16-byte load paths, with the
    # trailing entries of an odd length, more vectors than one group, and an unaligned w (scalar path)
    for dt in (torch.float64, torch.float32):
        k2 = 11
        ld = (n + 63) // 64 * 64
        Vp = torch.empty((k2, ld), dtype=dt, device="cuda")[:, :n]
        Vp.copy_(torch.rand((k2, n), dtype=dt, device="cuda", generator=g) - 0.5)
        buf = torch.rand(n + 1, dtype=dt, device="cuda", generator=g) - 0.5
        for wv in (buf[:n].clone(), buf[1:]):
            h = torch.empty(64, dtype=torch.float64, device="cuda")
            eng.vec_dots(Vp, k2, wv, h)
            ref = Vp.double() @ wv.double()
            assert torch.allclose(h[:k2], ref, rtol=1e-12, atol=1e-12)
            w2 = wv.clone() if wv.data_ptr() % 16 == 0 else wv
            before = w2.double().clone()
            eng.vec_gemv(Vp, k2, h, -0.5, w2)
            ref2 = before - 0.5 * (Vp.double().T @ h[:k2])
            assert torch.allclose(w2.double(), ref2, rtol=1e-6 if dt == torch.float32 else 1e-13, atol=1e-6)
    # conditional second Gram-Schmidt pass: gs_norm against the projected norm, the flag from the
    # criterion, and the _if kernels taken or not
    for dt in (torch.float64, torch.float32):
        k3 = 9
        ld = (n + 63) // 64 * 64
        B = torch.empty((k3 + 1, ld), dtype=dt, device="cuda")[:, :n]
        Q, _ = torch.linalg.qr(torch.rand((n, k3), dtype=torch.float64, device="cuda", generator=g) - 0.5)
        B[:k3] = Q.T.to(dt)
        wv = B[k3]
        for frac, expect in ((0.3, 0), (0.999, 1)):
            # w = frac of its norm inside span(Q) (squared norm of the projection 1 - frac^2 of |w|^2)
            a = torch.rand(k3, dtype=torch.float64, device="cuda", generator=g) - 0.5
            perp = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5
            perp -= Q @ (Q.T @ perp)
            x0 = frac * (Q @ a) / (Q @ a).norm() + (1 - frac ** 2) ** 0.5 * perp / perp.norm()
            wv.copy_(x0.to(dt))
            h = torch.zeros(64, dtype=torch.float64, device="cuda")
            h2 = torch.full((64,), 7.0, dtype=torch.float64, device="cuda")
            nrm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
            flag = torch.full((1,), -1, dtype=torch.int32, device="cuda")
            eng.vec_dots(B, k3 + 1, wv, h)
            assert abs(float(h[k3]) - float(wv.double().norm() ** 2)) < 1e-6
            w_before = wv.double().clone()
            eng.vec_gemv(B, k3, h, -1.0, wv)
            eng.gs_norm(k3, h, 0.5, None, flag, nrm2)
            assert int(flag) == expect
            tol = 1e-5 if dt == torch.float32 else 1e-12
            assert abs(float(nrm2) - float(wv.double().norm() ** 2)) < tol
            w1 = wv.double().clone()
            eng.vec_dots_if(flag, B, k3 + 1, wv, h2)
            eng.vec_gemv_if(flag, B, k3, h2, -1.0, wv)
            if expect:
                assert torch.allclose(h2[:k3], B[:k3].double() @ w1, atol=1e-6)
                assert torch.allclose(wv.double(), w1 - B[:k3].double().T @ h2[:k3], atol=1e-6)
                eng.gs_norm(k3, h2, 0.0, flag, None, nrm2)
                assert abs(float(nrm2) - float(wv.double().norm() ** 2)) < tol
            else:
                assert torch.count_nonzero(h2[:k3]) == 0 and torch.equal(wv.double(), w1)
                before = float(nrm2)
                eng.gs_norm(k3, h2, 0.0, flag, None, nrm2)   # not taken: nrm2 unchanged
                assert float(nrm2) == before
    x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    x32 = torch.empty(n, dtype=torch.float32, device="cuda")
    eng.vec_convert(x, x32)
    assert torch.equal(x32, x.float())
    # mismatched tensors are refused in the binding before any device work
    V = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    w = torch.zeros(n, dtype=torch.float64, device="cuda")
    h = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        eng.vec_dots(V, 4, w, h)                                   # fewer rows than k
    with pytest.raises(ValueError):
        eng.vec_dots(V[:, : n - 1], 2, w, h)                       # rows shorter than w
    with pytest.raises(ValueError):
        eng.vec_gemv(V, 2, h.float(), 1.0, w)                      # h not float64
    with pytest.raises(ValueError):
        eng.vec_gemv(V, 2, h[:1], 1.0, w)                          # h shorter than k
    with pytest.raises(ValueError):
        eng.vec_axpby(1.0, w[:-1], 1.0, w)                         # x shorter than y
    with pytest.raises(ValueError):
        eng.vec_axpby(1.0, w.float(), 1.0, w)                      # dtype mismatch
    with pytest.raises(ValueError):
        eng.vec_mul(w.float(), w, w)                               # d not float64
    with pytest.raises(ValueError):
        eng.vec_convert(w, torch.empty(n - 1, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        eng.vec_axpby(1.0, w.cpu(), 1.0, w)                        # host tensor
    eng.close()


def test_calls_follow_the_current_stream(torch_cuda):
    """Each call enqueues its work on torch's current stream at the time of the call: applies issued
    on two different side streams, each followed by that stream's own synchronisation, give the same
    results as on the default stream."""
    torch = torch_cuda
    eng, t = setup(torch, small_case(3))
    xu, xp = (t(a) for a in small_case(3)["dirs"][0])
    ref = [v.clone() for v in eng.jacobian_apply(xu, xp)]
    torch.cuda.synchronize()
    for _ in range(2):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            yu, yp = eng.jacobian_apply(xu, xp)
            assert eng._stream == s.cuda_stream
        s.synchronize()                    # only the side stream: its work must be the apply
        assert torch.equal(yu, ref[0]) and torch.equal(yp, ref[1])
    yu, yp = eng.jacobian_apply(xu, xp)
    assert eng._stream == torch.cuda.current_stream().cuda_stream
    torch.cuda.current_stream().synchronize()
    assert torch.equal(yu, ref[0]) and torch.equal(yp, ref[1])
    eng.close()


def test_newton_fgmres_against_oracle(torch_cuda):
    """One Newton step on a small dome-like case: the driver's reported linear reduction is the
    true one (oracle Jacobian), and its next residual equals the oracle residual there."""
    torch = torch_cuda
    from oracle import StokesOracle
    from paper_1406_6573_amd.solve import NewtonKrylov
    case = small_case(2, mapped=True, nx=3, ny=3, nz=2, body=(0.0, 0.0, -1.0))
    m = case["mesh"]
    eng, t = setup(torch, case)
    u, p = t(case["u"]), t(case["p"])
    u0, p0 = u.clone(), p.clone()
    nk = NewtonKrylov(eng, restart=40, precision="fp64")
    st = nk.solve(u, p, n_newton=1, lin_tol=1e-12)
    d = nk.d64.cpu().numpy()
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"], body=(0.0, 0.0, -1.0))
    o.set_state(case["u"], case["p"])
    K = o.jacobian()
    r0 = np.concatenate([a.ravel() for a in o.residual()])
    true_red = np.linalg.norm(K @ d + r0) / np.linalg.norm(r0)
    print(f"[gpu] newton step: |r0| {st.newton_residuals[0]:.6e} (oracle {np.linalg.norm(r0):.6e}), "
          f"krylov {st.krylov_iterations[0]}, reported reduction {st.linear_reductions[0]:.3e}, true {true_red:.3e}",
          flush=True)
    assert abs(st.newton_residuals[0] - np.linalg.norm(r0)) < 1e-12 * np.linalg.norm(r0)
    assert abs(st.linear_reductions[0] - true_red) < 1e-6 * max(true_red, 1e-8) + 1e-10
    o.set_state(u.cpu().numpy(), p.cpu().numpy())
    r1 = np.linalg.norm(np.concatenate([a.ravel() for a in o.residual()]))
    assert abs(st.newton_residuals[1] - r1) < 1e-10 * r1
    assert st.newton_residuals[1] < st.newton_residuals[0]
    eng.close()


def test_newton_mixed_matches_fp64(torch_cuda):
    """Equal Krylov budgets (one FGMRES(50) cycle per Newton step): the mixed path (FP32 Krylov,
    FP64 dots and right-hand side) follows the FP64 Newton trajectory."""
    torch = torch_cuda
    from meshgen import make_config
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov
    w = make_config(5, nx=32, ny=32, nz=2)
    m = w.mesh
    res = {}
    for prec in ("fp64", "mixed"):
        eng = Engine()
        eng.upload_mesh(m)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
        eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
        u, p = t(w.u), t(w.p)
        nk = NewtonKrylov(eng, restart=50, precision=prec, refine=1)
        st = nk.solve(u, p, n_newton=3, lin_tol=1e-10, verbose=True)
        res[prec] = st.newton_residuals
        eng.close()
    a, b = np.array(res["fp64"]), np.array(res["mixed"])
    print("[gpu] newton residuals fp64", a, "mixed", b, flush=True)
    assert np.all(np.diff(a) < 0) and np.all(np.diff(b) < 0)
    assert np.max(np.abs(a - b) / a) < 1e-3


def test_mixed_refinement_reaches_fp64_accuracy(torch_cuda):
    """FP32 inner FGMRES + FP64 outer refinement solves J d = b to FP64-level accuracy (beyond what
    FP32 arithmetic alone can give), checked against a direct solve with the oracle's Jacobian."""
    torch = torch_cuda
    import scipy.sparse.linalg as spla
    from oracle import StokesOracle
    from paper_1406_6573_amd.solve import NewtonKrylov
    case = small_case(2, mapped=True, nx=2, ny=2, nz=1, frac=0.5, L=20.0)
    m = case["mesh"]
    eng, t = setup(torch, case)
    nk = NewtonKrylov(eng, restart=60, precision="mixed", refine=40)
    mu, mp = nk.split(nk.minv)
    eng.jacobi_diag(invert=True, out=(mu, mp))
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, m.n_dof)
    b[:3 * m.n_nodes][m.dmask.ravel().astype(bool)] = 0.0
    its, red = nk.linear_solve(t(b), 1e-7)
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"])
    o.set_state(case["u"], case["p"])
    K = o.jacobian().tocsc()
    d_ref = spla.spsolve(K, b)
    d = nk.d64.cpu().numpy()
    err = np.linalg.norm(d - d_ref) / np.linalg.norm(d_ref)
    true_res = np.linalg.norm(K @ d - b) / np.linalg.norm(b)
    print(f"[gpu] mixed refinement: {its} FP32 Krylov iterations, residual {red:.2e} (oracle {true_res:.2e}), "
          f"solution error vs direct solve {err:.2e}", flush=True)
    assert true_res < 1e-9 and err < 1e-6


def oracle_lines(mesh):
    """Vertical node lines of a column mesh: nodes grouped by logical (x, y), bottom to top."""
    lg = mesh.node_logical
    key = np.round(lg[:, 0] * 8).astype(np.int64) * 10 ** 7 + np.round(lg[:, 1] * 8).astype(np.int64)
    order = np.lexsort((lg[:, 2], key))
    return np.split(order, np.nonzero(np.diff(key[order]))[0] + 1)


@pytest.mark.parametrize("k,mapped", [(2, False), (3, True), (4, False)])
def test_line_blocks_match_oracle(torch_cuda, k, mapped):
    """Conforming columns: the line solve equals dense solves with the blocks of the oracle's J_c
    restricted to each vertical node line and component (Dirichlet rows included)."""
    torch = torch_cuda
    from oracle import StokesOracle
    case = small_case(k, mapped=mapped, frac=0.0, nx=3, ny=2, nz=3)
    m = case["mesh"]
    eng, t = setup(torch, case)
    n_lines = eng.line_setup()
    lines = oracle_lines(m)
    assert n_lines == len(lines)
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"])
    o.set_state(case["u"], case["p"])
    K = o.jacobian().tocsr()
    N = m.n_nodes
    rng = np.random.default_rng(4)
    r = rng.uniform(-1, 1, (3, N))
    z = eng.line_apply(t(r)).cpu().numpy()
    ref = np.zeros_like(r)
    for c in range(3):
        for ln in lines:
            idx = c * N + ln
            ref[c, ln] = np.linalg.solve(K[idx][:, idx].toarray(), r[c, ln])
    err = rel_err(z, ref)
    z32 = eng.line_apply(t(r).float()).double().cpu().numpy()
    err32 = rel_err(z32, ref)
    print(f"[gpu] line blocks k={k} mapped={mapped}: {n_lines} lines, rel err fp64 {err:.2e} fp32 {err32:.2e}",
          flush=True)
    assert err < 1e-11 and err32 < 1e-4
    eng.close()


def dependent_slots(cm, P):
    """Slots of an element on one of its hanging faces or edges, from the cmask bits (faces -x, +x,
    -y, +y, -z, +z at bits 3..8; the edge parallel to axis d with sides (s0, s1) along the other two
    axes at bit 9 + 4 d + s0 + 2 s1)."""
    a = np.arange(P ** 3)
    co = [a % P, (a // P) % P, a // (P * P)]
    side = lambda v: np.where(v == 0, 0, np.where(v == P - 1, 1, -1))
    dep = np.zeros(P ** 3, dtype=bool)
    for f in range(6):
        if (cm >> (3 + f)) & 1:
            dep |= co[f // 2] == (P - 1) * (f % 2)
    for d in range(3):
        o0, o1 = [c for c in range(3) if c != d]
        for s0 in (0, 1):
            for s1 in (0, 1):
                if (cm >> (9 + 4 * d + s0 + 2 * s1)) & 1:
                    dep |= (side(co[o0]) == s0) & (side(co[o1]) == s1)
    return dep


@pytest.mark.parametrize("k,mapped,variant", [(2, True, "zface"), (3, False, "zface"), (4, True, "zface"),
                                             (3, True, "periodic"), (2, True, "frames"), (4, True, "frames"),
                                             (3, True, "all")])
def test_line_blocks_hanging_runs(torch_cuda, k, mapped, variant):
    """Lateral and -z hanging faces: each line block is the sum, over the elements, of the oracle's
    element matrix A_e restricted to the independent slots of one element z-line (couplings through
    dependent slots left out), Dirichlet rows unit rows; the lines are the chains that these
    element z-line runs link."""
    torch = torch_cuda
    from oracle import StokesOracle
    case = small_case(k, mapped=mapped, **{**dict(frac=0.4, nx=3, ny=3, nz=2), **VARIANTS[variant]})
    m = case["mesh"]
    P, N = k + 1, m.n_nodes
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"])
    o.set_state(case["u"], case["p"])
    A, _ = o.element_matrices()
    S = P ** 3
    Qn = node_frames(m)
    up, down = {}, {}
    blocks = [dict() for _ in range(3)]
    for e in range(m.n_el):
        dep = dependent_slots(int(m.cmask[e]), P)
        for t in range(P * P):
            run = [t + P * P * z for z in range(P) if not dep[t + P * P * z]]
            for sa, sb in zip(run[:-1], run[1:]):
                na, nb = int(m.elem_nodes[e, sa]), int(m.elem_nodes[e, sb])
                assert up.get(na, nb) == nb and down.get(nb, na) == na
                up[na], down[nb] = nb, na
            for sa in run:
                for sb in run:
                    key = (int(m.elem_nodes[e, sa]), int(m.elem_nodes[e, sb]))
                    A3 = A[e][np.ix_([sa, S + sa, 2 * S + sa], [sb, S + sb, 2 * S + sb])]
                    F = Qn[key[0]].T @ A3 @ Qn[key[1]]           # in the nodes' frames
                    for c in range(3):
                        blocks[c][key] = blocks[c].get(key, 0.0) + F[c, c]
    lines = []
    for n in range(N):
        if n in down:
            continue
        ln = [n]
        while ln[-1] in up:
            ln.append(up[ln[-1]])
        lines.append(np.array(ln))
    assert sum(len(ln) for ln in lines) == N
    eng, t = setup(torch, case)
    n_lines = eng.line_setup()
    assert n_lines == len(lines)
    rng = np.random.default_rng(6)
    r = rng.uniform(-1, 1, (3, N))
    ref = np.zeros_like(r)
    for c in range(3):
        msk = m.dmask[c].astype(bool)
        for ln in lines:
            B = np.array([[blocks[c].get((a, b), 0.0) for b in ln] for a in ln])
            mk = msk[ln]
            B[mk, :] = 0.0
            B[:, mk] = 0.0
            B[mk, mk] = 1.0
            ref[c, ln] = np.linalg.solve(B, r[c, ln])
    z = eng.line_apply(t(r)).cpu().numpy()
    z32 = eng.line_apply(t(r).float()).double().cpu().numpy()
    err, err32 = rel_err(z, ref), rel_err(z32, ref)
    print(f"[gpu] hanging line runs k={k} mapped={mapped} {variant}: {n_lines} lines, rel err fp64 {err:.2e} fp32 {err32:.2e}",
          flush=True)
    assert err < 1e-11 and err32 < 1e-4
    eng.close()


@pytest.mark.parametrize("precond,variant", [("jacobi", "zface"), ("line", "zface"), ("line", "periodic"),
                                             ("line", "frames"), ("line", "all")])
def test_newton_step_variants(torch_cuda, precond, variant):
    """One Newton step on a mapped mesh with -z hanging faces, or periodic in x and y: the reported
    linear reduction is the true one (oracle Jacobian) and the next residual equals the oracle
    residual there."""
    torch = torch_cuda
    from oracle import StokesOracle
    from paper_1406_6573_amd.solve import NewtonKrylov
    case = small_case(3, mapped=True, **{**dict(frac=0.4, nx=3, ny=3, nz=2, body=(0.0, 0.0, -1.0)),
                                         **VARIANTS[variant]})
    m = case["mesh"]
    eng, t = setup(torch, case)
    u, p = t(case["u"]), t(case["p"])
    nk = NewtonKrylov(eng, restart=60, precision="fp64", precond=precond)
    st = nk.solve(u, p, n_newton=1, lin_tol=1e-10)
    d = nk.d64.cpu().numpy()
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"], body=(0.0, 0.0, -1.0))
    o.set_state(case["u"], case["p"])
    K = o.jacobian()
    r0 = np.concatenate([a.ravel() for a in o.residual()])
    true_red = np.linalg.norm(K @ d + r0) / np.linalg.norm(r0)
    print(f"[gpu] newton step {variant} ({precond}): krylov {st.krylov_iterations[0]}, reported "
          f"{st.linear_reductions[0]:.3e}, true {true_red:.3e}", flush=True)
    assert abs(st.newton_residuals[0] - np.linalg.norm(r0)) < 1e-12 * np.linalg.norm(r0)
    assert abs(st.linear_reductions[0] - true_red) < 1e-6 * max(true_red, 1e-8) + 1e-10
    o.set_state(u.cpu().numpy(), p.cpu().numpy())
    r1 = np.linalg.norm(np.concatenate([a.ravel() for a in o.residual()]))
    assert abs(st.newton_residuals[1] - r1) < 1e-10 * r1
    assert st.newton_residuals[1] < st.newton_residuals[0]
    eng.close()


@pytest.mark.parametrize("k,mapped,variant", [(2, True, ""), (3, False, "zface"), (4, True, "periodic")])
def test_picard_operator_matches_oracle(torch_cuda, k, mapped, variant):
    """The Picard operator (viscosity kept, anisotropic part of the Newton tensor dropped): FP64 and
    FP32 applies and the Jacobi diagonal against the oracle's Picard J_c; the residual is unchanged;
    the residual VJP is refused; switching back to Newton restores the Newton operator."""
    torch = torch_cuda
    from oracle import StokesOracle
    from paper_1406_6573_amd.nsmf import NsmfError
    case = small_case(k, mapped=mapped, body=(0.0, 0.1, -1.0), **VARIANTS[variant])
    m = case["mesh"]
    eng, t = setup(torch, case)
    r_newton = [a.cpu().numpy() for a in eng.residual()]
    eng.set_linearization("picard")
    with pytest.raises(NsmfError):
        eng.residual()                                   # the state was discarded
    eng.set_state(t(case["u"]), t(case["p"]))
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"], body=(0.0, 0.1, -1.0),
                     picard=True)
    o.set_state(case["u"], case["p"])
    K = o.jacobian()
    absK = abs(K)
    for (xu, xp) in case["dirs"][:2]:
        x = np.concatenate([xu.ravel(), xp.ravel()])
        yref, scale = K @ x, absK @ np.abs(x)
        yu, yp = eng.jacobian_apply(t(xu), t(xp), "fp64")
        y = np.concatenate([yu.cpu().numpy().ravel(), yp.cpu().numpy().ravel()])
        yu32, yp32 = eng.jacobian_apply(t(xu).float(), t(xp).float(), "fp32")
        y32 = np.concatenate([yu32.double().cpu().numpy().ravel(), yp32.double().cpu().numpy().ravel()])
        e64, e32 = rel_err(y, yref), float(np.max(np.abs(y32 - yref) / np.maximum(scale, 1e-300)))
        print(f"[gpu] picard k={k} mapped={mapped} {variant}: J fp64 rel {e64:.2e}, "
              f"fp32 scaled {e32:.2e}", flush=True)
        assert e64 < 1e-12 and e32 < 64 * 2.0 ** -24
    ru, rp = eng.residual()
    assert rel_err(np.concatenate([ru.cpu().numpy().ravel(), rp.cpu().numpy().ravel()]),
                   np.concatenate([a.ravel() for a in r_newton])) < 1e-15
    d_u, _ = eng.jacobi_diag()
    A, _ = o.element_matrices()
    S = o.S
    dA = np.stack([np.diagonal(A, axis1=1, axis2=2)[:, c * S:(c + 1) * S].reshape(-1) for c in range(3)])
    R2 = o.R.multiply(o.R)
    ref_u = np.stack([R2.T @ dA[c] for c in range(3)])
    ref_u[m.dmask.astype(bool)] = 1.0
    assert np.max(np.abs(d_u.cpu().numpy() - ref_u) / np.abs(ref_u)) < 1e-12
    with pytest.raises(NsmfError):
        eng.residual_vjp(t(case["dirs"][0][0]), t(case["dirs"][0][1]), "fp64")
    eng.set_linearization("newton")
    eng.set_state(t(case["u"]), t(case["p"]))
    on = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"], body=(0.0, 0.1, -1.0))
    on.set_state(case["u"], case["p"])
    xu, xp = case["dirs"][0]
    yu, yp = eng.jacobian_apply(t(xu), t(xp), "fp64")
    y = np.concatenate([yu.cpu().numpy().ravel(), yp.cpu().numpy().ravel()])
    assert rel_err(y, on.jacobian() @ np.concatenate([xu.ravel(), xp.ravel()])) < 1e-12
    eng.close()


def test_newton_converges_faster_than_picard(torch_cuda):
    """Picard steps decrease the residual monotonically from a rough start; from the state they reach,
    three Newton steps reduce the residual further than three more Picard steps (same preconditioner
    and tolerance): Newton converges quadratically near the solution, Picard linearly."""
    torch = torch_cuda
    from paper_1406_6573_amd.solve import NewtonKrylov
    case = small_case(2, mapped=True, nx=3, ny=3, nz=2, body=(0.0, 0.0, -1.0))
    eng, t = setup(torch, case)
    u, p = t(case["u"]), t(case["p"])
    st = NewtonKrylov(eng, restart=60, precision="fp64", precond="line", linearization="picard").solve(
        u, p, n_newton=6, lin_tol=1e-10)
    print("[gpu] picard from the start: " + " ".join(f"{v:.3e}" for v in st.newton_residuals), flush=True)
    assert all(b < a for a, b in zip(st.newton_residuals[:-1], st.newton_residuals[1:]))
    res = {}
    for lin in ("newton", "picard"):
        u1, p1 = u.clone(), p.clone()
        nk = NewtonKrylov(eng, restart=60, precision="fp64", precond="line", linearization=lin)
        res[lin] = nk.solve(u1, p1, n_newton=3, lin_tol=1e-12).newton_residuals
        print(f"[gpu] {lin}: residuals " + " ".join(f"{v:.3e}" for v in res[lin]), flush=True)
    eng.close()
    assert res["newton"][-1] < res["picard"][-1]


def test_line_preconditioner_beats_jacobi(torch_cuda):
    """Dome with hanging margin columns (aspect ratio ~30): one FGMRES(40) cycle reduces the Newton
    system's residual further with vertical-line blocks than with point Jacobi, and the reported
    reduction is the true one (oracle Jacobian)."""
    torch = torch_cuda
    from meshgen import make_config
    from oracle import StokesOracle
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov
    w = make_config(5, nx=12, ny=12, nz=3)
    m = w.mesh
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    o = StokesOracle(m, w.n, w.eps, w.B0, w.logA, w.beta, body=w.body)
    o.set_state(w.u, w.p)
    K = o.jacobian()
    r0 = np.concatenate([a.ravel() for a in o.residual()])
    red = {}
    for pc in ("jacobi", "line"):
        eng = Engine()
        eng.upload_mesh(m)
        eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
        eng.set_state(t(w.u), t(w.p))
        nk = NewtonKrylov(eng, restart=40, precision="fp64", precond=pc)
        nk.setup_preconditioner()
        its, rep = nk.linear_solve(t(-r0), 1e-14)
        d = nk.d64.cpu().numpy()
        true = np.linalg.norm(K @ d + r0) / np.linalg.norm(r0)
        print(f"[gpu] {pc}: {its} iterations, reported {rep:.3e}, true {true:.3e}", flush=True)
        assert abs(rep - true) < 1e-6 * true + 1e-12
        red[pc] = true
        eng.close()
    assert red["line"] < 0.1 * red["jacobi"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_upper_triangular_preconditioner(torch_cuda, precision):
    """Block upper-triangular [[F~, B^T], [0, S~]] with line blocks: within one FGMRES(40) cycle it reduces the
    true residual (oracle Jacobian) further than the block-diagonal form, in FP64 and with the FP32 Krylov
    loop under FP64 refinement."""
    torch = torch_cuda
    from meshgen import make_config
    from oracle import StokesOracle
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov
    w = make_config(5, nx=12, ny=12, nz=3)
    m = w.mesh
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    o = StokesOracle(m, w.n, w.eps, w.B0, w.logA, w.beta, body=w.body)
    o.set_state(w.u, w.p)
    K = o.jacobian()
    r0 = np.concatenate([a.ravel() for a in o.residual()])
    red = {}
    for tri in (False, True):
        eng = Engine()
        eng.upload_mesh(m)
        eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
        eng.set_state(t(w.u), t(w.p))
        nk = NewtonKrylov(eng, restart=40, precision=precision, precond="line", triangular=tri, refine=1)
        nk.setup_preconditioner()
        its, rep = nk.linear_solve(t(-r0), 1e-14)
        d = nk.d64.cpu().numpy()
        true = np.linalg.norm(K @ d + r0) / np.linalg.norm(r0)
        print(f"[gpu] {precision} triangular={tri}: {its} iterations, reported {rep:.3e}, true {true:.3e}", flush=True)
        assert abs(rep - true) < 1e-5 * true + 1e-12
        red[tri] = true
        eng.close()
    assert red[True] < 0.5 * red[False]


def test_adjoint_gradient_matches_finite_differences(torch_cuda):
    """Phi(u) = 1/2 |u - u_obs|^2 at the solved state: the adjoint gradient with respect to logA and beta
    equals central differences (h = 1e-6) of Phi at re-solved states."""
    torch = torch_cuda
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov, adjoint_gradient
    case = small_case(2, mapped=True, nx=2, ny=2, nz=1, frac=0.5, L=20.0, body=(0.0, 0.0, -1.0))
    m = case["mesh"]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    eng = Engine()
    eng.upload_mesh(m)
    nk = NewtonKrylov(eng, restart=60, precision="fp64", precond="line", triangular=True)
    rng = np.random.default_rng(9)
    u_obs = t(rng.uniform(-1, 1, (3, m.n_nodes)))

    def solve_state(logA, beta, u0, p0):
        eng.set_params(case["n"], case["eps"], case["B0"], case["body"], t(logA), t(beta))
        u, p = u0.clone(), p0.clone()
        st = nk.solve(u, p, n_newton=12, lin_tol=1e-13)
        assert st.newton_residuals[-1] < 1e-10 * st.newton_residuals[0] + 1e-12
        return u, p

    phi = lambda u: 0.5 * float(((u - u_obs) ** 2).sum())
    u, p = solve_state(case["logA"], case["beta"], t(case["u"]), t(case["p"]))
    gA, gB, its, red = adjoint_gradient(nk, u, p, u - u_obs)
    assert red < 1e-9
    h = 1e-6
    for kind, idx in (("logA", 0), ("logA", m.n_el - 1), ("beta", 0), ("beta", m.n_bface - 1)):
        vals = []
        for sgn in (1.0, -1.0):
            la, be = case["logA"].copy(), case["beta"].copy()
            (la if kind == "logA" else be)[idx] += sgn * h
            up, _ = solve_state(la, be, u, p)
            vals.append(phi(up))
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = float((gA if kind == "logA" else gB)[idx])
        print(f"[gpu] adjoint d/d{kind}[{idx}]: {ad:.10e}  FD {fd:.10e}", flush=True)
        assert abs(fd - ad) < 1e-5 * abs(ad) + 1e-9 * phi(u)
    eng.close()


def test_adjoint_gradient_matches_oracle(torch_cuda):
    """The engine's adjoint gradient (restarted FGMRES solve with J_c, then the residual VJP) against the
    oracle's (direct sparse solve with J_c^T, then the oracle's VJP) at the same state -- solved by the
    oracle's Newton iteration with direct solves -- for Phi(u) = 1/2 |u - u_obs|^2, over every entry of
    dPhi/dlogA and dPhi/dbeta."""
    torch = torch_cuda
    from oracle import StokesOracle, adjoint_gradient as oracle_adjoint, newton_solve
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov, adjoint_gradient
    case = small_case(3, mapped=True, nx=3, ny=2, nz=2, frac=0.4, L=30.0, body=(0.0, 0.0, -1.0))
    m = case["mesh"]
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"], body=case["body"])
    uh, ph, hist = newton_solve(o, case["u"], case["p"], tol=1e-13)
    assert hist[-1] <= 1e-12 * hist[0]
    rng = np.random.default_rng(11)
    u_obs = rng.uniform(-1, 1, (3, m.n_nodes))
    oA, oB, _, _ = oracle_adjoint(o, uh - u_obs)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    eng = Engine()
    eng.upload_mesh(m)
    eng.set_params(case["n"], case["eps"], case["B0"], case["body"], t(case["logA"]), t(case["beta"]))
    nk = NewtonKrylov(eng, restart=60, precision="fp64", precond="line", triangular=True, refine=20)
    u, p = t(uh), t(ph)
    gA, gB, its, red = adjoint_gradient(nk, u, p, u - t(u_obs), tol=1e-12)
    assert red < 1e-10
    eA, eB = rel_err(gA.cpu().numpy(), oA), rel_err(gB.cpu().numpy(), oB)
    mA = np.max(np.abs(gA.cpu().numpy() - oA)) / np.max(np.abs(oA))
    mB = np.max(np.abs(gB.cpu().numpy() - oB)) / np.max(np.abs(oB))
    print(f"[gpu] adjoint vs oracle: {its} iterations, logA rel {eA:.2e} (max {mA:.2e}), "
          f"beta rel {eB:.2e} (max {mB:.2e})", flush=True)
    assert eA < 1e-8 and eB < 1e-8 and mA < 1e-8 and mB < 1e-8
    eng.close()


@pytest.mark.parametrize("k,variant", [(2, "hang"), (3, "frames"), (4, "periodic"), (3, "q")])
def test_gradient_apply_matches_jacobian_at_zero_velocity(torch_cuda, k, variant):
    """nsmf_gradient_apply (B^T x_p) against the oracle's B^T in FP64, and against the velocity rows of
    the Jacobian apply at zero velocity in FP64, FP32 and with bfloat16 operators (the same arithmetic on
    the pressure term in another kernel, so equal up to the rounding order of the multiply-adds)."""
    torch = torch_cuda
    from paper_1406_6573_amd import Engine
    from oracle import StokesOracle
    kw = dict(q=dict(pspace="Q", mapped=True), hang={}, frames=dict(mapped=True, frames=True),
              periodic=dict(periodic=(True, True)))[variant]
    case = small_case(k, **kw)
    m = case["mesh"]
    eng = Engine()
    eng.upload_mesh(m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    eng.set_params(case["n"], case["eps"], case["B0"], case["body"], t(case["logA"]), t(case["beta"]))
    eng.set_state(t(case["u"]), t(case["p"]))
    rng = np.random.default_rng(3)
    xp = rng.uniform(-1, 1, (m.n_el, m.n_p))
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"], body=case["body"])
    o.set_state(case["u"], case["p"])
    K = o.jacobian()
    N = m.n_nodes
    x = np.concatenate([np.zeros(3 * N), xp.ravel()])
    ref = (K @ x)[:3 * N]
    sc = np.maximum((abs(K) @ np.abs(x))[:3 * N], 1e-300)
    got = eng.gradient_apply(t(xp)).cpu().numpy().ravel()
    assert np.max(np.abs(got - ref) / sc) < 1e-12
    # per entry, relative to (|B^T||x_p|)_i.  With the velocity part of x zero the scale holds only
    # the pressure path's terms, so the FP32 bound follows that path's depth: about 60 roundings
    # (pressure interpolation, w detJ, the geometry, three transposed sweeps, R_e^T, the assembly) with
    # a factor 4 of margin, 256 u; the Jacobian's FP32 rows are another rounding order of the same
    # arithmetic
    u32 = 2.0 ** -24
    for prec, dt, b_ref, b_jac in (("fp64", torch.float64, 1e-12, 1e-14), ("fp32", torch.float32, 256 * u32, 256 * u32),
                                   ("bf16ops", torch.float32, 16 * 2.0 ** -9, 256 * u32)):
        xpt = t(xp).to(dt)
        g = eng.gradient_apply(xpt, prec).double().cpu().numpy().ravel()
        yu, _ = eng.jacobian_apply(torch.zeros((3, N), dtype=dt, device="cuda"), xpt, prec)
        yu = yu.double().cpu().numpy().ravel()
        assert np.max(np.abs(g - ref) / sc) < b_ref, prec
        assert np.max(np.abs(g - yu) / sc) < b_jac, prec
    eng.close()
