"""Error behaviour of the C ABI: every documented status code on the condition that raises it, and a
context that stays usable after a rejected call.  No invalid input reaches a kernel: each is rejected
on the host before any work is enqueued."""
import ctypes
from types import SimpleNamespace

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


def code_of(fn, *a, **k):
    from paper_1406_6573_amd.nsmf import NsmfError
    with pytest.raises(NsmfError) as ei:
        fn(*a, **k)
    return ei.value.code


def fake_mesh(k, n_el, n_nodes, ids=None, pspace="P"):
    P = k + 1
    en = np.zeros((n_el, P ** 3), dtype=np.int32) if ids is None else ids
    return SimpleNamespace(k=k, elem_nodes=en, cmask=np.zeros(n_el, dtype=np.uint32),
                           coords=np.zeros((3, n_nodes)), bface_elem=np.zeros(0, dtype=np.int32), dmask=None,
                           pspace=pspace)


def test_call_order_and_arguments(torch_cuda):
    torch = torch_cuda
    from paper_1406_6573_amd import Engine
    case = small_case(2, nx=2, ny=2, nz=1)
    m = case["mesh"]
    eng = Engine()
    eng.upload_mesh(m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    xu, xp = case["dirs"][0]
    # no parameters / state yet
    assert code_of(eng.jacobian_apply, t(xu), t(xp)) == -4
    assert code_of(eng.residual) == -4
    eng.set_params(case["n"], case["eps"], case["B0"], (0, 0, 0), t(case["logA"]), t(case["beta"]))
    assert code_of(eng.jacobian_apply, t(xu), t(xp)) == -4
    eng.set_state(t(case["u"]), t(case["p"]))
    yu, yp = eng.jacobian_apply(t(xu), t(xp))           # now valid
    assert torch.isfinite(yu).all() and torch.isfinite(yp).all()
    # line solve before its setup, and after a state change
    assert code_of(eng.line_apply, t(xu)) == -4
    eng.line_setup()
    eng.line_apply(t(xu))
    eng.set_state(t(case["u"]), t(case["p"]))
    assert code_of(eng.line_apply, t(xu)) == -4
    # precision out of range, through the raw entry point
    lib = eng.lib
    rc = lib.nsmf_jacobian_apply(eng.h, 7, ctypes.c_void_p(t(xu).data_ptr()), ctypes.c_void_p(t(xp).data_ptr()),
                                 ctypes.c_void_p(yu.data_ptr()), ctypes.c_void_p(yp.data_ptr()))
    assert rc == -1
    # flow-law parameters out of range
    assert code_of(eng.set_params, 0.5, case["eps"], case["B0"], (0, 0, 0), t(case["logA"]), t(case["beta"])) == -1
    assert code_of(eng.set_params, 3.0, 0.0, case["B0"], (0, 0, 0), t(case["logA"]), t(case["beta"])) == -1
    # wrong tensor shapes are rejected by the binding before the library is called
    with pytest.raises(ValueError):
        eng.jacobian_apply(t(xu)[:, :-1].contiguous(), t(xp))
    eng.close()


def test_mesh_validation(torch_cuda):
    from paper_1406_6573_amd import Engine
    eng = Engine()
    assert code_of(eng.upload_mesh, fake_mesh(5, 1, 8)) == -5                 # degree outside 2..4
    assert code_of(eng.upload_mesh, fake_mesh(2, 0, 8)) == -1                 # no elements
    ids = np.full((1, 27), 9, dtype=np.int32)
    assert code_of(eng.upload_mesh, fake_mesh(2, 1, 8, ids=ids)) == -3        # node id out of range
    good = small_case(2, nx=2, ny=2, nz=1)["mesh"]
    # inverted elements: mirror the z coordinate
    inv = SimpleNamespace(**{k: getattr(good, k) for k in ("k", "elem_nodes", "cmask", "bface_elem", "dmask")})
    inv.coords = good.coords * np.array([[1.0], [1.0], [-1.0]])
    assert code_of(eng.upload_mesh, inv) == -3
    # x depending on zeta: not column-mapped
    sh = SimpleNamespace(**{k: getattr(good, k) for k in ("k", "elem_nodes", "cmask", "bface_elem", "dmask")})
    sh.coords = good.coords.copy()
    sh.coords[0] += 0.3 * good.coords[2] ** 2
    assert code_of(eng.upload_mesh, sh) == -5
    # pressure space out of range, through the raw entry point
    from paper_1406_6573_amd.nsmf import _Mesh
    en = np.ascontiguousarray(good.elem_nodes, dtype=np.int32)
    cm = np.ascontiguousarray(good.cmask, dtype=np.uint32)
    X = np.ascontiguousarray(good.coords)
    bf = np.ascontiguousarray(good.bface_elem, dtype=np.int32)
    s = _Mesh(2, en.shape[0], X.shape[1], bf.shape[0], en.ctypes.data, cm.ctypes.data, X.ctypes.data,
              bf.ctypes.data if bf.size else None, None, 7)
    assert eng.lib.nsmf_upload_mesh(eng.h, ctypes.byref(s)) == -1
    # periods: negative -> EINVAL, periodic z -> EUNSUP
    for per, code in (((-1.0, 0.0, 0.0), -1), ((0.0, 0.0, 2.0), -5)):
        s = _Mesh(2, en.shape[0], X.shape[1], bf.shape[0], en.ctypes.data, cm.ctypes.data, X.ctypes.data,
                  bf.ctypes.data if bf.size else None, None, 0, (ctypes.c_double * 3)(*per))
        assert eng.lib.nsmf_upload_mesh(eng.h, ctypes.byref(s)) == code
    # nodal frames: n_frames < 0 -> EINVAL; a node listed twice, a frame that is not orthonormal,
    # or a framed node named by a slot above the bottom -> EMESH
    def frames_code(n, nodes, frames):
        nd = np.ascontiguousarray(nodes, dtype=np.int32)
        fr = np.ascontiguousarray(frames, dtype=np.float64)
        s = _Mesh(2, en.shape[0], X.shape[1], bf.shape[0], en.ctypes.data, cm.ctypes.data, X.ctypes.data,
                  bf.ctypes.data if bf.size else None, None, 0, (ctypes.c_double * 3)(0.0, 0.0, 0.0), n,
                  nd.ctypes.data, fr.ctypes.data)
        return eng.lib.nsmf_upload_mesh(eng.h, ctypes.byref(s))
    base = np.nonzero(good.node_logical[:, 2] == 0.0)[0][:2]
    top = np.nonzero(good.node_logical[:, 2] > 0.0)[0][:1]
    eye = np.tile(np.eye(3), (2, 1, 1))
    assert frames_code(-1, base, eye) == -1
    assert frames_code(2, [base[0], base[0]], eye) == -3
    assert frames_code(1, base[:1], 2.0 * eye[:1]) == -3
    assert frames_code(1, top, eye[:1]) == -3
    assert frames_code(2, base, eye) == 0
    # linearization kind out of range
    assert eng.lib.nsmf_set_linearization(eng.h, 2) == -1
    # the context is still usable
    eng.upload_mesh(good)
    assert eng.sizes["n_el"] == good.n_el
    eng.close()
