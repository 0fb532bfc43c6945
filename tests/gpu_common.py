"""Shared helpers of the GPU parity tests: seeded small cases, oracle reference, error metrics."""
import numpy as np

from meshgen.columns import column_mesh, random_refined_columns


def terrain_geometry(nx, ny, nz, L):
    def geo(lg):
        x, y = lg[:, 0] * L / nx, lg[:, 1] * L / ny
        b = 0.05 * np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L)
        H = 1.0 + 0.3 * np.cos(2 * np.pi * x / L + 0.4) * np.sin(2 * np.pi * y / L + 0.2)
        return np.stack([x, y, b + lg[:, 2] / nz * H], 1)
    return geo


def inclined_geometry(nx, ny, nz, L, a, b):
    """Planar inclined base z = a x + b y under a thickness varying linearly in x and y."""
    def geo(lg):
        x, y = lg[:, 0] * L / nx, lg[:, 1] * L / ny
        return np.stack([x, y, a * x + b * y + lg[:, 2] / nz * (1.0 + 0.004 * x - 0.003 * y)], 1)
    return geo


def small_case(k, mapped=False, frac=0.3, mask=True, seed=0, nx=4, ny=3, nz=2, L=40.0, body=(0.0, 0.0, 0.0),
               pspace="P", refine_from=0, periodic=(False, False), frames=False, incline=None):
    """A seeded case with hanging faces and edges: mesh, parameters, state, directions.  incline = (a, b)
    puts the mesh over the planar base z = a x + b y (column-mapped)."""
    rng = np.random.default_rng(1000 + 17 * k + seed)
    refined = random_refined_columns(nx, ny, frac, rng)
    geo = terrain_geometry(nx, ny, nz, L) if mapped else None
    if incline is not None:
        geo = inclined_geometry(nx, ny, nz, L, *incline)
    mesh = column_mesh(k, nx, ny, nz, refined=refined, extent=(L, L * ny / nx, 1.0), geometry=geo,
                       base_normal_dirichlet=mask and not frames, pspace=pspace, refine_from=refine_from,
                       periodic=periodic, base_frames=frames)
    case = dict(mesh=mesh, n=3.0, eps=1e-10, B0=0.5, body=body,
                logA=rng.normal(0, 0.5, mesh.n_el), beta=np.exp(rng.normal(0, 1, mesh.n_bface)))
    x, y, z = mesh.coords
    w = 2 * np.pi / L
    u = np.stack([np.sin(w * x) * np.cos(w * y) * (1 + z), np.cos(w * x) * np.sin(w * y) * (1 + z),
                  0.1 * np.sin(w * x) * np.sin(w * y) * z])
    case["u"] = u + 1e-2 * rng.uniform(-1, 1, u.shape)
    case["p"] = 1e-2 * rng.uniform(-1, 1, (mesh.n_el, mesh.n_p))
    case["dirs"] = [(rng.uniform(-1, 1, (3, mesh.n_nodes)), rng.uniform(-1, 1, (mesh.n_el, mesh.n_p)))
                    for _ in range(3)]
    return case


def rel_err(y, ref):
    return float(np.linalg.norm(np.ravel(y) - np.ravel(ref)) / max(np.linalg.norm(np.ravel(ref)), 1e-300))


def scaled_err(y, ref, scale):
    """max_i |y - ref|_i / scale_i with scale = |K||x| (rounding relative to the magnitude of the summands)."""
    s = np.ravel(scale)
    d = np.abs(np.ravel(y) - np.ravel(ref))
    keep = s > 0
    return float(np.max(d[keep] / s[keep])) if keep.any() else float(np.max(d))
