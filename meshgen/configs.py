"""The five synthetic workloads of the Newton-Stokes operator and their reduced variants.

Each workload stands in for a test problem of the paper (slab tests of
Sec. 4.3, ice stream of Sec. 7.1, Antarctica of Sec. 8); none of the
paper's datasets is available, so geometry, parameters and states are drawn
from seeded generators with the stated shapes (element aspect ratio, column
structure, refinement density, polynomial order).

Readings used where the workload description leaves a choice open:

* Glen law with mu = B_e (II + eps)^((1-n)/(2n)), B_e = B0 exp(-logA_e / n),
  B0 = 0.5, II = D:D / 2, eps = 1e-10, n = 3 (eq. (glen), Sec. 2.1);
* 20% refined columns = a seeded random subset, refined 2x2x2 (one level);
* flat bases carry the normal condition u_z = 0 (dmask) plus the Robin term;
  the curved terrain base carries the Robin term only;
* states: config 2/4 smooth sinusoidal field + 1e-2 uniform noise,
  config 3 Fourier fields (N = 10, gamma = 3/2) + 1e-2 noise, config 5 zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .columns import ColumnMesh, column_mesh, random_refined_columns
from .fields import FourierField, vialov_dome


@dataclass
class Workload:
    name: str
    mesh: ColumnMesh
    n: float
    eps: float
    B0: float
    logA: np.ndarray            # [n_el]
    beta: np.ndarray            # [n_bface]
    body: tuple                 # constant body-force density (b_x, b_y, b_z)
    u: np.ndarray               # [3, n_nodes]
    p: np.ndarray               # [n_el, n_p]
    directions: list = field(default_factory=list)   # [(x_u, x_p)]
    adjoint: Optional[tuple] = None                   # (w_u, w_p)
    meta: dict = field(default_factory=dict)


def _rngs(config_id: int, seed: int, n: int):
    ss = np.random.SeedSequence([config_id, seed])
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def _uniform_dirs(rng, mesh, count):
    out = []
    for _ in range(count):
        out.append((rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))))
    return out


def config1(seed: int = 0, n_dirs: int = 10, nx: int = 8, ny: int = 8, nz: int = 2, pspace: str = "P") -> Workload:
    """Unit box 8x8x2, conforming affine Q2 x P1, beta = 0, no Dirichlet mask."""
    r_u, r_p, r_d = _rngs(1, seed, 3)
    mesh = column_mesh(2, nx, ny, nz, extent=(1.0, 1.0, 1.0), pspace=pspace)
    u = r_u.uniform(-1, 1, (3, mesh.n_nodes))
    p = r_p.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    return Workload("config1", mesh, 3.0, 1e-10, 0.5, np.zeros(mesh.n_el), np.zeros(mesh.n_bface),
                    (0.0, 0.0, 0.0), u, p, _uniform_dirs(r_d, mesh, n_dirs))


def _slab_state(mesh: ColumnMesh, L: float, rng) -> tuple:
    x, y, z = mesh.coords
    w = 2.0 * np.pi / L
    sx, cx, sy, cy = np.sin(w * x), np.cos(w * x), np.sin(w * y), np.cos(w * y)
    u = np.stack([sx * cy * (1 + z), cx * sy * (1 + z), 0.1 * sx * sy * z])
    u = u + 1e-2 * rng.uniform(-1, 1, u.shape)
    p = 1e-2 * rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    return u, p


def slab(config_id: int, k: int, nx: int, ny: int, nz: int, L: float, H: float,
         frac_refined: float, seed: int, beta_lognormal: bool, n_dirs: int = 1,
         adjoint: bool = False, pspace: str = "P") -> Workload:
    r_ref, r_a, r_b, r_s, r_d, r_w = _rngs(config_id, seed, 6)
    refined = random_refined_columns(nx, ny, frac_refined, r_ref)
    mesh = column_mesh(k, nx, ny, nz, refined=refined, extent=(L, L, H), base_normal_dirichlet=True, pspace=pspace)
    logA = r_a.normal(0.0, 0.5, mesh.n_el)
    beta = np.exp(r_b.normal(0.0, 1.0, mesh.n_bface)) if beta_lognormal else np.ones(mesh.n_bface)
    u, p = _slab_state(mesh, L, r_s)
    wl = Workload(f"config{config_id}", mesh, 3.0, 1e-10, 0.5, logA, beta, (0.0, 0.0, 0.0), u, p,
                  _uniform_dirs(r_d, mesh, n_dirs))
    if adjoint:
        wl.adjoint = (r_w.uniform(-1, 1, (3, mesh.n_nodes)), r_w.uniform(-1, 1, (mesh.n_el, mesh.n_p)))
    return wl


def config2(seed: int = 0, nx: int = 64, ny: int = 64, nz: int = 8, n_dirs: int = 1, pspace: str = "P") -> Workload:
    """Slab with element size 15.625 x 15.625 x 0.125 (aspect 125), Q3 x P2, 20% refined columns."""
    return slab(2, 3, nx, ny, nz, L=15.625 * nx, H=0.125 * nz, frac_refined=0.2, seed=seed,
                beta_lognormal=False, n_dirs=n_dirs, pspace=pspace)


def config4(seed: int = 0, nx: int = 96, ny: int = 96, nz: int = 12, frac_refined: float = 0.2,
            n_dirs: int = 1, pspace: str = "P") -> Workload:
    """Config-2 geometry at 96x96x12 (element 1000/96 x 1000/96 x 1/12), beta = exp(N(0,1)), adjoint w."""
    return slab(4, 3, nx, ny, nz, L=1000.0 / 96 * nx, H=nz / 12.0, frac_refined=frac_refined, seed=seed,
                beta_lognormal=True, n_dirs=n_dirs, adjoint=True, pspace=pspace)


def config3(seed: int = 0, nx: int = 128, ny: int = 128, nz: int = 16, n_dirs: int = 1, pspace: str = "P") -> Workload:
    """Terrain-mapped slab, Q4 x P3: base b and thickness H from 8-mode Fourier fields over 500 x 500."""
    r_b, r_h, r_ux, r_uy, r_uz, r_n, r_d = _rngs(3, seed, 7)
    Lfull = 500.0
    h = Lfull / 128.0
    fb = FourierField(r_b, 2, Lfull)
    fh = FourierField(r_h, 2, Lfull)
    g = np.linspace(0.0, Lfull, 257)
    gb, gh = fb.grid(g, g), fh.grid(g, g)
    bscale = 0.5 / np.abs(gb).max()
    hmin, hmax = gh.min(), gh.max()

    def geometry(lg):
        x, y = lg[:, 0] * h, lg[:, 1] * h
        b = bscale * fb(x, y)
        H = 0.5 + 1.5 * (fh(x, y) - hmin) / (hmax - hmin)
        return np.stack([x, y, b + lg[:, 2] / nz * H], 1)

    mesh = column_mesh(4, nx, ny, nz, geometry=geometry, extent=(h * nx, h * ny, 1.0), pspace=pspace)
    fields = [FourierField(r, 10, Lfull) for r in (r_ux, r_uy, r_uz)]
    x, y, _ = mesh.coords
    u = np.stack([f(x, y) for f in fields]) + 1e-2 * r_n.uniform(-1, 1, (3, mesh.n_nodes))
    p = 1e-2 * r_n.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    return Workload("config3", mesh, 3.0, 1e-10, 0.5, np.zeros(mesh.n_el), np.ones(mesh.n_bface),
                    (0.0, 0.0, 0.0), u, p, _uniform_dirs(r_d, mesh, n_dirs))


def config5(seed: int = 0, nx: int = 256, ny: int = 256, nz: int = 8, n_dirs: int = 0, pspace: str = "P") -> Workload:
    """Dome ice sheet on a flat bed over [-500, 500]^2, Q2 x P1, refined columns along the margin r = 1."""
    r_noise, r_d = _rngs(5, seed, 2)
    half, H0 = 500.0, 2.0
    hx = 2.0 * half / nx
    vx = -half + hx * np.arange(nx + 1)
    vy = -half + (2.0 * half / ny) * np.arange(ny + 1)
    VX, VY = np.meshgrid(vx, vy, indexing="ij")
    R = np.hypot(VX, VY) / half
    Hv = np.maximum(vialov_dome(np.minimum(R, 1.0), H0) * (1.0 + 0.05 * r_noise.uniform(-1, 1, R.shape)),
                    0.05 * H0)
    inside = R < 1.0
    crossed = (inside[:-1, :-1] | inside[1:, :-1] | inside[:-1, 1:] | inside[1:, 1:]) & \
              ~(inside[:-1, :-1] & inside[1:, :-1] & inside[:-1, 1:] & inside[1:, 1:])

    def geometry(lg):
        s, t = lg[:, 0], lg[:, 1]
        i = np.clip(np.floor(s).astype(np.int64), 0, nx - 1)
        j = np.clip(np.floor(t).astype(np.int64), 0, ny - 1)
        fs, ft = s - i, t - j
        H = ((1 - fs) * (1 - ft) * Hv[i, j] + fs * (1 - ft) * Hv[i + 1, j]
             + (1 - fs) * ft * Hv[i, j + 1] + fs * ft * Hv[i + 1, j + 1])
        return np.stack([-half + s * hx, -half + t * (2.0 * half / ny), lg[:, 2] / nz * H], 1)

    mesh = column_mesh(2, nx, ny, nz, refined=crossed, geometry=geometry,
                       extent=(2 * half, 2 * half, H0), base_normal_dirichlet=True, pspace=pspace)
    u = np.zeros((3, mesh.n_nodes))
    p = np.zeros((mesh.n_el, mesh.n_p))
    return Workload("config5", mesh, 3.0, 1e-10, 0.5, np.zeros(mesh.n_el), np.ones(mesh.n_bface),
                    (0.0, 0.0, -1.0), u, p, _uniform_dirs(r_d, mesh, n_dirs))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def make_config(config_id: int, seed: int = 0, **kw) -> Workload:
    return CONFIGS[config_id](seed=seed, **kw)
