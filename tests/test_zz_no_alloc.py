"""The allocation-free Jacobian apply (nsmf_jacobian_apply_noalloc) through the C ABI: the same result as
nsmf_jacobian_apply, bit for bit (same kernels, deterministic assembly), on two calls in a row on one GPU
(the second on a smaller mesh, which reuses the first call's scratch contents), in every precision; a
mesh whose partial sums exceed the scratch array is refused with NSMF_EINVAL."""
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


def engine(torch, mesh, n, eps, B0, body, logA, beta, u, p):
    from paper_1406_6573_amd import Engine
    eng = Engine()
    eng.upload_mesh(mesh)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    eng.set_params(n, eps, B0, body, t(logA), t(beta))
    eng.set_state(t(u), t(p))
    return eng, t


def compare(torch, eng, t, xu, xp, label):
    for prec in ("fp64", "fp32", "bf16ops"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        a, b = t(xu).to(dt), t(xp).to(dt)
        ref_u, ref_p = eng.jacobian_apply(a, b, prec)
        y_u = torch.full_like(ref_u, float("nan"))
        y_p = torch.full_like(ref_p, float("nan"))
        eng.jacobian_apply_noalloc(a, b, (y_u, y_p), prec)
        torch.cuda.synchronize()
        print(f"[gpu] no-alloc {label} {prec}: n_dof={eng.sizes['n_dof']} max|diff| "
              f"{float((y_u - ref_u).abs().max()):.1e} {float((y_p - ref_p).abs().max()):.1e}", flush=True)
        assert torch.equal(y_u, ref_u) and torch.equal(y_p, ref_p)


def test_noalloc_matches_apply_on_two_calls(torch_cuda):
    torch = torch_cuda
    from meshgen import make_config
    # first call: the slab 64x64x8 Q3 workload in FP32 (about 49 MB of partial sums) and a
    # 24x24x4 slab of the same kind in all precisions
    w = make_config(2, nx=24, ny=24, nz=4, n_dirs=1)
    eng, t = engine(torch, w.mesh, w.n, w.eps, w.B0, w.body, w.logA, w.beta, w.u, w.p)
    compare(torch, eng, t, *w.directions[0], "slab 24x24x4 Q3")
    eng.close()
    # second call, smaller mesh (hanging faces and edges, terrain-mapped)
    c = small_case(2, mapped=True, body=(0.0, 0.1, -1.0))
    eng, t = engine(torch, c["mesh"], c["n"], c["eps"], c["B0"], c["body"], c["logA"], c["beta"], c["u"], c["p"])
    compare(torch, eng, t, *c["dirs"][0], "hanging k=2 terrain")
    eng.close()


def test_noalloc_full_slab_fp32_and_size_limit(torch_cuda):
    torch = torch_cuda
    from meshgen import make_config
    from paper_1406_6573_amd import NsmfError
    w = make_config(2, n_dirs=1)
    eng, t = engine(torch, w.mesh, w.n, w.eps, w.B0, w.body, w.logA, w.beta, w.u, w.p)
    xu, xp = w.directions[0]
    a, b = t(xu).float(), t(xp).float()
    ref = eng.jacobian_apply(a, b, "fp32")
    out = (torch.empty_like(ref[0]), torch.empty_like(ref[1]))
    eng.jacobian_apply_noalloc(a, b, out, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    # FP64 partial sums of this mesh exceed the 64 MiB scratch: refused before any work
    with pytest.raises(NsmfError) as ei:
        eng.jacobian_apply_noalloc(t(xu), t(xp), (torch.empty_like(t(xu)), torch.empty_like(t(xp))), "fp64")
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    print(f"[gpu] no-alloc slab 64x64x8 Q3 fp32 equal; fp64 refused: {ei.value}", flush=True)
    eng.close()
