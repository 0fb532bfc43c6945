"""Residual VJP through torch.autograd: gradcheck (central differences) on a small hanging mesh,
and the logA / beta gradients against the oracle's complex-step derivatives."""
import numpy as np
import pytest

from gpu_common import small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_gradcheck_residual(torch_cuda):
    torch = torch_cuda
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.autograd import stokes_residual
    case = small_case(2, mapped=True, nx=2, ny=2, nz=1, frac=0.5, L=20.0)
    m = case["mesh"]
    eng = Engine()
    eng.upload_mesh(m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda").requires_grad_(True)
    u, p, logA, beta = t(case["u"]), t(case["p"]), t(case["logA"]), t(case["beta"])
    print(f"[gpu] gradcheck k=2 n_el={m.n_el} n_dof={m.n_dof}", flush=True)
    fn = lambda u, p, a, b: stokes_residual(eng, u, p, a, b, body=(0.0, 0.0, -1.0))
    assert torch.autograd.gradcheck(fn, (u, p, logA, beta), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)
    eng.close()


def test_gradcheck_residual_all_variants(torch_cuda):
    """gradcheck on a mesh that is periodic in x and y, has -z hanging faces and nodal frames on
    the terrain base (the residual's u-derivative goes through the framed and periodic slots)."""
    torch = torch_cuda
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.autograd import stokes_residual
    case = small_case(2, mapped=True, nx=3, ny=3, nz=2, frac=0.4, periodic=(True, True), frames=True,
                      refine_from=1)
    m = case["mesh"]
    eng = Engine()
    eng.upload_mesh(m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda").requires_grad_(True)
    u, p, logA, beta = t(case["u"]), t(case["p"]), t(case["logA"]), t(case["beta"])
    print(f"[gpu] gradcheck all variants k=2 n_el={m.n_el} n_dof={m.n_dof}", flush=True)
    fn = lambda u, p, a, b: stokes_residual(eng, u, p, a, b, body=(0.0, 0.0, -1.0))
    assert torch.autograd.gradcheck(fn, (u, p, logA, beta), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)
    eng.close()


def test_vjp_matches_oracle_through_autograd(torch_cuda):
    torch = torch_cuda
    from oracle import StokesOracle
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.autograd import stokes_residual
    case = small_case(3, mapped=False)
    m = case["mesh"]
    eng = Engine()
    eng.upload_mesh(m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda").requires_grad_(True)
    u, p, logA, beta = t(case["u"]), t(case["p"]), t(case["logA"]), t(case["beta"])
    wu, wp = case["dirs"][0]
    r_u, r_p = stokes_residual(eng, u, p, logA, beta)
    loss = (r_u * torch.as_tensor(wu, device="cuda")).sum() + (r_p * torch.as_tensor(wp, device="cuda")).sum()
    # a second linearisation between forward and backward must not change the gradient
    eng.set_state(u.detach() * 0.5, p.detach())
    loss.backward()
    o = StokesOracle(m, case["n"], case["eps"], case["B0"], case["logA"], case["beta"])
    o.set_state(case["u"], case["p"])
    og_u, og_p, og_A, og_b = o.vjp(wu, wp)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    errs = [rel(u.grad.cpu().numpy(), og_u), rel(p.grad.cpu().numpy(), og_p), rel(logA.grad.cpu().numpy(), og_A),
            rel(beta.grad.cpu().numpy(), og_b)]
    print("[gpu] autograd VJP rel errors u, p, logA, beta:", errs, flush=True)
    assert max(errs) < 1e-12
    eng.close()
