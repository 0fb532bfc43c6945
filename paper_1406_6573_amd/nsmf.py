"""ctypes binding of the C ABI in include/nsmf.h.

Argument marshalling only: every step of the operator runs in the HIP library.
Device vectors are torch tensors on the engine's GPU; the engine enqueues its
work on torch's current stream of that device.  If the shared library has not
been built, loading fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libnsmf.so")

FP64, FP32, FP32_BF16OPS = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16ops": FP32_BF16OPS}

STATUS = {0: "NSMF_OK", -1: "NSMF_EINVAL", -2: "NSMF_EHIP", -3: "NSMF_EMESH", -4: "NSMF_ESTATE",
          -5: "NSMF_EUNSUP", -6: "NSMF_ENOMEM"}

EXPORTED = ["nsmf_create", "nsmf_destroy", "nsmf_set_stream", "nsmf_upload_mesh", "nsmf_set_params",
            "nsmf_set_state", "nsmf_residual", "nsmf_jacobian_apply", "nsmf_residual_vjp", "nsmf_query",
            "nsmf_geometry_kind", "nsmf_set_kernel_timing", "nsmf_kernel_time", "nsmf_last_error",
            "nsmf_version", "nsmf_jacobi_diag", "nsmf_vec_dots", "nsmf_vec_gemv", "nsmf_vec_axpby", "nsmf_vec_mul",
            "nsmf_vec_convert", "nsmf_line_setup", "nsmf_line_apply", "nsmf_set_linearization",
            "nsmf_jacobian_apply_noalloc", "nsmf_lowo_apply", "nsmf_coarse_setup", "nsmf_coarse_prolong",
            "nsmf_coarse_restrict", "nsmf_vec_normalize", "nsmf_vec_dots_if", "nsmf_vec_gemv_if", "nsmf_gs_norm",
            "nsmf_gradient_apply"]


class NsmfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_el", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_bface", ctypes.c_int64), ("elem_nodes", ctypes.c_void_p), ("cmask", ctypes.c_void_p),
                ("coords", ctypes.c_void_p), ("bface_elem", ctypes.c_void_p), ("dmask", ctypes.c_void_p),
                ("pspace", ctypes.c_int32), ("period", ctypes.c_double * 3), ("n_frames", ctypes.c_int64),
                ("frame_nodes", ctypes.c_void_p), ("frames", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_double), ("eps", ctypes.c_double), ("B0", ctypes.c_double),
                ("body", ctypes.c_double * 3)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP engine library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    lib.nsmf_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.nsmf_destroy.argtypes = [vp]
    lib.nsmf_destroy.restype = None
    lib.nsmf_set_stream.argtypes = [vp, vp]
    lib.nsmf_upload_mesh.argtypes = [vp, ctypes.POINTER(_Mesh)]
    lib.nsmf_set_params.argtypes = [vp, ctypes.POINTER(_Params), vp, vp]
    lib.nsmf_set_state.argtypes = [vp, vp, vp]
    lib.nsmf_residual.argtypes = [vp, vp, vp, vp]
    lib.nsmf_jacobian_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.nsmf_gradient_apply.argtypes = [vp, ctypes.c_int, vp, vp]
    lib.nsmf_jacobian_apply_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.nsmf_residual_vjp.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp, vp]
    lib.nsmf_query.argtypes = [vp, i64p, i64p, i64p, i64p, i64p]
    lib.nsmf_geometry_kind.argtypes = [vp]
    lib.nsmf_set_kernel_timing.argtypes = [vp, ctypes.c_int]
    lib.nsmf_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64p]
    lib.nsmf_last_error.argtypes = [vp]
    lib.nsmf_last_error.restype = ctypes.c_char_p
    lib.nsmf_version.restype = ctypes.c_char_p
    i64, dbl, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.nsmf_jacobi_diag.argtypes = [vp, ci, vp, vp]
    lib.nsmf_line_setup.argtypes = [vp, i64p]
    lib.nsmf_line_apply.argtypes = [vp, ci, vp, vp]
    lib.nsmf_lowo_apply.argtypes = [vp, vp, vp]
    lib.nsmf_coarse_setup.argtypes = [vp, i64, vp, vp, vp]
    lib.nsmf_coarse_prolong.argtypes = [vp, ci, vp, vp]
    lib.nsmf_coarse_restrict.argtypes = [vp, ci, vp, vp]
    lib.nsmf_set_linearization.argtypes = [vp, ci]
    lib.nsmf_vec_dots.argtypes = [vp, ci, i64, ci, vp, i64, vp, vp]
    lib.nsmf_vec_gemv.argtypes = [vp, ci, i64, ci, vp, i64, vp, dbl, vp]
    lib.nsmf_vec_axpby.argtypes = [vp, ci, i64, dbl, vp, dbl, vp]
    lib.nsmf_vec_mul.argtypes = [vp, ci, i64, vp, vp, vp]
    lib.nsmf_vec_normalize.argtypes = [vp, ci, i64, vp, vp]
    lib.nsmf_vec_dots_if.argtypes = [vp, vp, ci, i64, ci, vp, i64, vp, vp]
    lib.nsmf_vec_gemv_if.argtypes = [vp, vp, ci, i64, ci, vp, i64, vp, dbl, vp]
    lib.nsmf_gs_norm.argtypes = [vp, ci, vp, dbl, vp, vp, vp]
    lib.nsmf_vec_convert.argtypes = [vp, i64, ci, vp, vp]
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Engine:
    """One engine context on one GPU (default: torch's current device)."""

    def __init__(self, device: Optional[int] = None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        self._check(self.lib.nsmf_create(ctypes.byref(h), self.device), None)
        self.h = h
        self.dev = torch.device("cuda", self.device)
        self.sync_stream()
        self.k = None
        self.state_version = 0
        self.linearization = "newton"

    # -------------------------------------------------------------- plumbing
    def _check(self, rc: int, h=-1):
        if rc != 0:
            msg = self.lib.nsmf_last_error(self.h if h == -1 else h)
            raise NsmfError(rc, msg.decode() if msg else "")

    def sync_stream(self):
        """Bind the context to torch's current stream of the engine's device.  Every method that
        enqueues device work calls this first, so the work always follows the caller's current
        stream (a changed stream is passed to the library before the call)."""
        s = self.torch.cuda.current_stream(self.dev).cuda_stream
        if s != getattr(self, "_stream", None):
            self._check(self.lib.nsmf_set_stream(self.h, ctypes.c_void_p(s)))
            self._stream = s

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.nsmf_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t, shape, dtype, name):
        if not (t.is_cuda and t.device.index == self.device):
            raise ValueError(f"{name} must be a CUDA tensor on device {self.device}")
        if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous {dtype} of shape {tuple(shape)}")
        return t

    def _flat(self, t, n, dtype, name):
        """A contiguous device vector of dtype with at least n entries (Krylov vector kernels)."""
        if not (t.is_cuda and t.device.index == self.device):
            raise ValueError(f"{name} must be a CUDA tensor on device {self.device}")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be a contiguous {dtype} tensor with at least {n} entries")
        return t

    def _basis(self, V, k, n, dtype, name="V"):
        """Row-major basis [rows, >= n] with at least k rows, unit stride along a row."""
        if not (V.is_cuda and V.device.index == self.device):
            raise ValueError(f"{name} must be a CUDA tensor on device {self.device}")
        if V.dtype != dtype or V.dim() != 2 or V.stride(1) != 1 or V.shape[0] < k or V.shape[1] < n:
            raise ValueError(f"{name} must be a {dtype} [rows >= {k}, cols >= {n}] tensor with unit row stride")
        return V

    # -------------------------------------------------------------- API
    def upload_mesh(self, mesh):
        """Copy a mesh (any object with k, elem_nodes, cmask, coords, bface_elem, dmask arrays, an
        optional pressure-space label pspace: "P" = P_{k-1} (default), "Q" = Q_{k-2}, an optional
        period (x, y, z) of periodic axes, 0 where not periodic, and optional nodal frames:
        frame_nodes [n] and frames [n, 3, 3] (local axes as columns, unknowns u = Q u_hat)."""
        en = np.ascontiguousarray(mesh.elem_nodes, dtype=np.int32)
        cm = np.ascontiguousarray(mesh.cmask, dtype=np.uint32)
        X = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        bf = np.ascontiguousarray(mesh.bface_elem, dtype=np.int32)
        dm = None if mesh.dmask is None else np.ascontiguousarray(mesh.dmask, dtype=np.uint8)
        fn = getattr(mesh, "frame_nodes", None)
        fn = None if fn is None or len(fn) == 0 else np.ascontiguousarray(fn, dtype=np.int32)
        fq = None if fn is None else np.ascontiguousarray(mesh.frames, dtype=np.float64).reshape(-1, 3, 3)
        if fq is not None and fq.shape[0] != fn.shape[0]:
            raise ValueError("frames must be [len(frame_nodes), 3, 3]")
        s = _Mesh(int(mesh.k), en.shape[0], X.shape[1], bf.shape[0], en.ctypes.data, cm.ctypes.data,
                  X.ctypes.data, bf.ctypes.data if bf.size else None, None if dm is None else dm.ctypes.data,
                  {"P": 0, "Q": 1}[getattr(mesh, "pspace", "P")],
                  (ctypes.c_double * 3)(*[float(v) for v in getattr(mesh, "period", (0.0, 0.0, 0.0))]),
                  0 if fn is None else fn.shape[0], None if fn is None else fn.ctypes.data,
                  None if fq is None else fq.ctypes.data)
        self.sync_stream()
        self._check(self.lib.nsmf_upload_mesh(self.h, ctypes.byref(s)))
        self.k = int(mesh.k)
        self.sizes = self.query()

    def query(self):
        vals = [ctypes.c_int64() for _ in range(5)]
        self._check(self.lib.nsmf_query(self.h, *[ctypes.byref(v) for v in vals]))
        n_nodes, n_el, n_p, n_dof, n_bface = (v.value for v in vals)
        return dict(n_nodes=n_nodes, n_el=n_el, n_p=n_p, n_dof=n_dof, n_bface=n_bface)

    def geometry_kind(self) -> str:
        kind = self.lib.nsmf_geometry_kind(self.h)
        if kind < 0:
            self._check(kind)
        return {0: "affine", 1: "column"}[kind]

    def set_params(self, n=3.0, eps=1e-10, B0=0.5, body=(0.0, 0.0, 0.0), logA=None, beta=None):
        torch = self.torch
        sz = self.sizes
        if logA is not None:
            logA = self._vec(logA, (sz["n_el"],), torch.float64, "logA")
        if beta is not None:
            beta = self._vec(beta, (sz["n_bface"],), torch.float64, "beta")
        prm = _Params(float(n), float(eps), float(B0), (ctypes.c_double * 3)(*[float(b) for b in body]))
        self.sync_stream()
        self._check(self.lib.nsmf_set_params(self.h, ctypes.byref(prm), _ptr(logA), _ptr(beta)))
        self.state_version += 1

    def set_linearization(self, kind="newton"):
        """Operator that set_state prepares: "newton" (default) or "picard" (mu kept, the
        anisotropic part of the Newton tensor dropped).  Discards the stored state."""
        codes = {"newton": 0, "picard": 1}
        if kind not in codes:
            raise ValueError("linearization must be 'newton' or 'picard'")
        self._check(self.lib.nsmf_set_linearization(self.h, codes[kind]))
        self.linearization = kind
        self.state_version += 1

    def set_state(self, u, p):
        torch = self.torch
        sz = self.sizes
        u = self._vec(u, (3, sz["n_nodes"]), torch.float64, "u")
        p = self._vec(p, (sz["n_el"], sz["n_p"]), torch.float64, "p")
        self.sync_stream()
        self._check(self.lib.nsmf_set_state(self.h, _ptr(u), _ptr(p)))
        self.state_version += 1

    def residual(self, f_u=None, out=None):
        torch = self.torch
        sz = self.sizes
        if f_u is not None:
            f_u = self._vec(f_u, (3, sz["n_nodes"]), torch.float64, "f_u")
        if out is None:
            out = (torch.empty((3, sz["n_nodes"]), dtype=torch.float64, device=self.dev),
                   torch.empty((sz["n_el"], sz["n_p"]), dtype=torch.float64, device=self.dev))
        self.sync_stream()
        self._check(self.lib.nsmf_residual(self.h, _ptr(f_u), _ptr(out[0]), _ptr(out[1])))
        return out

    def _dtype(self, prec):
        return self.torch.float64 if prec == FP64 else self.torch.float32

    def jacobian_apply(self, x_u, x_p, prec="fp64", out=None):
        prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        dt = self._dtype(prec)
        sz = self.sizes
        x_u = self._vec(x_u, (3, sz["n_nodes"]), dt, "x_u")
        x_p = self._vec(x_p, (sz["n_el"], sz["n_p"]), dt, "x_p")
        if out is None:
            out = (self.torch.empty_like(x_u), self.torch.empty_like(x_p))
        self.sync_stream()
        self._check(self.lib.nsmf_jacobian_apply(self.h, prec, _ptr(x_u), _ptr(x_p), _ptr(out[0]), _ptr(out[1])))
        return out

    def gradient_apply(self, x_p, prec="fp64", out=None):
        """y_u = B^T x_p, the velocity rows of the Jacobian apply at zero velocity (mesh only)."""
        prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        dt = self._dtype(prec)
        sz = self.sizes
        x_p = self._vec(x_p, (sz["n_el"], sz["n_p"]), dt, "x_p")
        y_u = (self.torch.empty((3, sz["n_nodes"]), dtype=dt, device=self.dev) if out is None
               else self._vec(out, (3, sz["n_nodes"]), dt, "out"))
        self.sync_stream()
        self._check(self.lib.nsmf_gradient_apply(self.h, prec, _ptr(x_p), _ptr(y_u)))
        return y_u

    def jacobian_apply_noalloc(self, x_u, x_p, out, prec="fp64"):
        """y = J_c x through the allocation-free entry point: the partial sums live in the library's
        per-GPU scratch array; the caller provides the outputs `out` = (y_u, y_p)."""
        prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        dt = self._dtype(prec)
        sz = self.sizes
        x_u = self._vec(x_u, (3, sz["n_nodes"]), dt, "x_u")
        x_p = self._vec(x_p, (sz["n_el"], sz["n_p"]), dt, "x_p")
        y_u = self._vec(out[0], (3, sz["n_nodes"]), dt, "y_u")
        y_p = self._vec(out[1], (sz["n_el"], sz["n_p"]), dt, "y_p")
        self.sync_stream()
        self._check(self.lib.nsmf_jacobian_apply_noalloc(self.h, prec, _ptr(x_u), _ptr(x_p), _ptr(y_u), _ptr(y_p)))
        return y_u, y_p

    def residual_vjp(self, w_u, w_p, prec="fp64", want=("u", "p", "logA", "beta")):
        torch = self.torch
        prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        dt = self._dtype(prec)
        sz = self.sizes
        w_u = self._vec(w_u, (3, sz["n_nodes"]), dt, "w_u")
        w_p = self._vec(w_p, (sz["n_el"], sz["n_p"]), dt, "w_p")
        g_u = torch.empty_like(w_u) if "u" in want else None
        g_p = torch.empty_like(w_p) if "p" in want else None
        g_A = torch.empty(sz["n_el"], dtype=torch.float64, device=self.dev) if "logA" in want else None
        g_b = torch.empty(sz["n_bface"], dtype=torch.float64, device=self.dev) if "beta" in want else None
        self.sync_stream()
        self._check(self.lib.nsmf_residual_vjp(self.h, prec, _ptr(w_u), _ptr(w_p), _ptr(g_u), _ptr(g_p),
                                               _ptr(g_A), _ptr(g_b)))
        return g_u, g_p, g_A, g_b

    def jacobi_diag(self, invert=False, out=None):
        """Block-Jacobi data at the state: (d_u [3, n_nodes], d_p [n_el, n_p]) in FP64, or their
        reciprocals with invert=True."""
        torch = self.torch
        sz = self.sizes
        if out is None:
            out = (torch.empty((3, sz["n_nodes"]), dtype=torch.float64, device=self.dev),
                   torch.empty((sz["n_el"], sz["n_p"]), dtype=torch.float64, device=self.dev))
        d_u, d_p = out
        self.sync_stream()
        self._check(self.lib.nsmf_jacobi_diag(self.h, 1 if invert else 0, _ptr(d_u), _ptr(d_p)))
        return d_u, d_p

    def lowo_apply(self, x_u, out=None):
        """y_u = J~_c x_u with the low-order approximation of the velocity block on the Gauss-Lobatto
        sub-grid at the state (FP64, [3, n_nodes])."""
        sz = self.sizes
        x_u = self._vec(x_u, (3, sz["n_nodes"]), self.torch.float64, "x_u")
        y_u = self.torch.empty_like(x_u) if out is None else self._vec(out, (3, sz["n_nodes"]), self.torch.float64, "out")
        self.sync_stream()
        self._check(self.lib.nsmf_lowo_apply(self.h, _ptr(x_u), _ptr(y_u)))
        return y_u

    def coarse_setup(self, n_cpts, node_cpt, node_w, node_zeta):
        """Horizontal coarse space: per node its coarse cell's 4 lattice points, bilinear weights and
        relative height (host arrays).  Coarse vectors are float64 [3, n_cpts, 3]."""
        sz = self.sizes
        cpt = np.ascontiguousarray(node_cpt, dtype=np.int32).reshape(sz["n_nodes"], 4)
        w = np.ascontiguousarray(node_w, dtype=np.float64).reshape(sz["n_nodes"], 4)
        zeta = np.ascontiguousarray(node_zeta, dtype=np.float64).reshape(sz["n_nodes"])
        self.sync_stream()
        self._check(self.lib.nsmf_coarse_setup(self.h, int(n_cpts), cpt.ctypes.data, w.ctypes.data, zeta.ctypes.data))
        self.n_cpts = int(n_cpts)

    def coarse_prolong(self, xc, out):
        """out [3, n_nodes] (float64 or float32) = masked prolongation of xc [3, n_cpts, 3] (float64)."""
        sz = self.sizes
        xc = self._vec(xc, (3, self.n_cpts, 3), self.torch.float64, "xc")
        out = self._vec(out, (3, sz["n_nodes"]), out.dtype, "out")
        self.sync_stream()
        self._check(self.lib.nsmf_coarse_prolong(self.h, self._prec_of(out), _ptr(xc), _ptr(out)))
        return out

    def coarse_restrict(self, r_u, out):
        """out [3, n_cpts, 3] (float64) = restriction of r_u [3, n_nodes] (float64 or float32)."""
        sz = self.sizes
        r_u = self._vec(r_u, (3, sz["n_nodes"]), r_u.dtype, "r_u")
        out = self._vec(out, (3, self.n_cpts, 3), self.torch.float64, "out")
        self.sync_stream()
        self._check(self.lib.nsmf_coarse_restrict(self.h, self._prec_of(r_u), _ptr(r_u), _ptr(out)))
        return out

    def line_setup(self):
        """Factor the vertical-line blocks of the velocity block at the state; returns the number of lines."""
        n = ctypes.c_int64(0)
        self.sync_stream()
        self._check(self.lib.nsmf_line_setup(self.h, ctypes.byref(n)))
        return int(n.value)

    def line_apply(self, x_u, out=None):
        """y_u = (line blocks)^{-1} x_u for x_u [3, n_nodes] (float64 or float32, contiguous)."""
        sz = self.sizes
        x_u = self._vec(x_u, (3, sz["n_nodes"]), x_u.dtype, "x_u")
        y_u = self.torch.empty_like(x_u) if out is None else self._vec(out, (3, sz["n_nodes"]), x_u.dtype, "out")
        self.sync_stream()
        self._check(self.lib.nsmf_line_apply(self.h, self._prec_of(x_u), _ptr(x_u), _ptr(y_u)))
        return y_u

    # Krylov vector kernels: 1D device tensors (float64 or float32), FP64 accumulation
    @staticmethod
    def _prec_of(t):
        import torch
        if t.dtype == torch.float64:
            return 0
        if t.dtype == torch.float32:
            return 1
        raise ValueError("vectors must be float64 or float32")

    def vec_dots(self, V, k, w, h):
        """h[:k] = V[:k] @ w  (V: [rows >= k, >= n] with unit row stride, h: float64 device [>= k])."""
        prec = self._prec_of(w)
        n = w.numel()
        self._flat(w, n, w.dtype, "w")
        self._basis(V, k, n, w.dtype)
        self._flat(h, k, self.torch.float64, "h")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_dots(self.h, prec, n, int(k), _ptr(V), V.stride(0), _ptr(w), _ptr(h)))

    def vec_gemv(self, V, k, h, alpha, w):
        """w += alpha * V[:k].T @ h[:k]."""
        prec = self._prec_of(w)
        n = w.numel()
        self._flat(w, n, w.dtype, "w")
        self._basis(V, k, n, w.dtype)
        self._flat(h, k, self.torch.float64, "h")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_gemv(self.h, prec, n, int(k), _ptr(V), V.stride(0), _ptr(h),
                                           float(alpha), _ptr(w)))

    def vec_axpby(self, a, x, b, y):
        """y = a x + b y (b == 0: y is overwritten without being read)."""
        n = y.numel()
        self._flat(y, n, y.dtype, "y")
        self._flat(x, n, y.dtype, "x")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_axpby(self.h, self._prec_of(y), n, float(a), _ptr(x), float(b), _ptr(y)))

    def vec_mul(self, d, x, z):
        """z = d * x (d float64)."""
        n = z.numel()
        self._flat(z, n, z.dtype, "z")
        self._flat(x, n, z.dtype, "x")
        self._flat(d, n, self.torch.float64, "d")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_mul(self.h, self._prec_of(z), n, _ptr(d), _ptr(x), _ptr(z)))

    def _flag(self, f, name):
        if f is None:
            return None
        if not (f.is_cuda and f.device.index == self.device) or f.dtype != self.torch.int32 or f.numel() < 1:
            raise ValueError(f"{name} must be an int32 CUDA tensor on device {self.device}")
        return f

    def vec_dots_if(self, flag, V, k, w, h):
        """vec_dots when flag[0] != 0 (a device int32), else h[:k] = 0; decided on the device."""
        prec = self._prec_of(w)
        n = w.numel()
        self._flat(w, n, w.dtype, "w")
        self._basis(V, k, n, w.dtype)
        self._flat(h, k, self.torch.float64, "h")
        self._flag(flag, "flag")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_dots_if(self.h, _ptr(flag), prec, n, int(k), _ptr(V), V.stride(0), _ptr(w),
                                              _ptr(h)))

    def vec_gemv_if(self, flag, V, k, h, alpha, w):
        """vec_gemv when flag[0] != 0 (a device int32), else w unchanged; decided on the device."""
        prec = self._prec_of(w)
        n = w.numel()
        self._flat(w, n, w.dtype, "w")
        self._basis(V, k, n, w.dtype)
        self._flat(h, k, self.torch.float64, "h")
        self._flag(flag, "flag")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_gemv_if(self.h, _ptr(flag), prec, n, int(k), _ptr(V), V.stride(0), _ptr(h),
                                              float(alpha), _ptr(w)))

    def gs_norm(self, k, h, eta2, flag_in, flag_out, nrm2):
        """nrm2[0] = h[k] - sum_{i<k} h[i]^2 and flag_out[0] = (nrm2[0] < eta2 h[k]) on the device (see
        nsmf_gs_norm); nothing is written when flag_in is given and flag_in[0] == 0."""
        self._flat(h, k + 1, self.torch.float64, "h")
        self._flat(nrm2, 1, self.torch.float64, "nrm2")
        self._flag(flag_in, "flag_in")
        self._flag(flag_out, "flag_out")
        self.sync_stream()
        self._check(self.lib.nsmf_gs_norm(self.h, int(k), _ptr(h), float(eta2), _ptr(flag_in), _ptr(flag_out),
                                          _ptr(nrm2)))

    def vec_normalize(self, nrm2, x):
        """x = x / sqrt(nrm2[0]) with nrm2 a float64 device tensor (x = 0 when nrm2[0] <= 0)."""
        n = x.numel()
        self._flat(x, n, x.dtype, "x")
        self._flat(nrm2, 1, self.torch.float64, "nrm2")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_normalize(self.h, self._prec_of(x), n, _ptr(nrm2), _ptr(x)))

    def vec_convert(self, x, out):
        """out = x converted between float64 and float32."""
        torch = self.torch
        to32 = 1 if out.dtype == torch.float32 else 0
        n = x.numel()
        self._flat(x, n, torch.float64 if to32 else torch.float32, "x")
        self._flat(out, n, torch.float32 if to32 else torch.float64, "out")
        self.sync_stream()
        self._check(self.lib.nsmf_vec_convert(self.h, n, to32, _ptr(x), _ptr(out)))

    def set_kernel_timing(self, enable: bool):
        self.sync_stream()
        self._check(self.lib.nsmf_set_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.sync_stream()
        self._check(self.lib.nsmf_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
