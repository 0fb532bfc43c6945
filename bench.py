"""Throughput of the Newton-Stokes Jacobian apply on one MI355X.

A step is one application y = J_c x of the Newton-linearised Stokes operator
(gather with hanging-node interpolation, sum-factorised gradients, the fused
quadrature-point Newton-tensor step, pressure terms, transposed contractions,
basal Robin term, scatter, Dirichlet rows) with inputs resident in HBM.  The
default workload is the largest single-GPU one: "terrain-mapped slab 128x128x16,
Q4 x P3, Fourier base and thickness" (56.6M DoF).  The headline value is the
mixed-precision (FP32) apply; the FP64 apply, the FP32-vs-FP64 error, the
BF16-operator trial, the linearisation (set_state), residual and VJP times are
reported beside it, and the same figures for "slab 64x64x8, Q3 x P2, aspect 125,
20% of the columns refined 2:1" under the key "slab_q3".

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s of Newton-Stokes Jacobian apply, mixed vs FP64 at stated rel. error"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(sz, geo_kind, word):
    """Bytes one Jacobian apply must move in the stored-linearisation design: per quadrature point
    the 8 values of the linearisation (mu', kappa, Sigma0) and, on column-mapped elements, 6
    geometry values (the rows of J^-1 that vary and w detJ); x read and y written once; per-element
    geometry on affine elements; the basal face data.  Connectivity, slot positions and partial sums
    are not counted (they are not part of the method's data)."""
    k = sz["k"]
    nq = sz["n_el"] * (k + 1) ** 3
    nvec = 3 * sz["n_nodes"] + sz["n_el"] * sz["n_p"]
    geo = 4 * sz["n_el"] if geo_kind == "affine" else 6 * nq
    face = sz["n_bface"] * (1 + 4 * (k + 1) ** 2)
    return word * (8 * nq + 2 * nvec + geo + face)


TRAFFIC_FILES = {2: "apply_slab64x64x8_q3_traffic.json", 3: "apply_terrain128x128x16_q4_traffic.json"}


def counter_record(config_id):
    """The committed counter summary of the workload, if it was taken with the current kernel sources
    (otherwise None)."""
    import hashlib
    if config_id not in TRAFFIC_FILES:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[config_id])
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for p in rec["sources"]:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return rec if h.hexdigest() == rec["source_sha256"] else None


def measured_traffic(config_id, prec="fp32_apply"):
    """HBM bytes per apply (every kernel of one apply) from the counter summary, or None."""
    rec = counter_record(config_id)
    return None if rec is None else 1e6 * sum(rec[prec].values())


# VALU issue: packed FP32 is not used, so a wave64 FP32 or FP64 instruction takes 4 cycles of a
# 16-lane SIMD; 256 CUs x 4 SIMDs at 2.4 GHz
N_SIMD, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4


def valu_issue(config_id, kernel_ms):
    """Compute side of the FP32 apply: the element kernel's VALU instruction count from the counter
    summary, the time their issue alone takes on the whole chip, and its share of the apply's measured
    device time (None without a current summary)."""
    rec = counter_record(config_id)
    if rec is None or "fp32_element_kernel_valu" not in rec:
        return None
    v = rec["fp32_element_kernel_valu"]
    floor_ms = v["valu_instructions"] * CYCLES_PER_VALU / (N_SIMD * CLOCK_HZ) * 1e3
    return {"kernel": v["kernel"], "valu_instructions": v["valu_instructions"],
            "valu_instructions_per_wavefront": round(v["valu_instructions"] / v["wavefronts"]),
            "issue_floor_ms": floor_ms, "frac_of_apply": floor_ms / kernel_ms}


def cpu_baseline(seed=0):
    """The FP64 oracle as it stands: assemble the Jacobian and apply it once, on a reduced
    sample of the same workload (terrain 16x16x4, Q4 x P3, same construction)."""
    import threadpoolctl
    from meshgen import make_config
    from oracle import StokesOracle
    w = make_config(3, seed=seed, nx=16, ny=16, nz=4)
    m = w.mesh
    t0 = time.perf_counter()
    o = StokesOracle(m, w.n, w.eps, w.B0, w.logA, w.beta)
    o.set_state(w.u, w.p)
    xu, xp = w.directions[0]
    o.jacobian_apply(xu, xp)
    t1 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        o.jacobian_apply(xu, xp)
    t2 = time.perf_counter()
    threads = max([p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()] + [1])
    return {"value": m.n_dof / (t1 - t0) / 1e9, "unit": "GDoF/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"terrain 16x16x4 Q4xP3 (same construction as the 128x128x16 workload), {m.n_el} elements, "
                       f"{m.n_dof} DoF: dense-quadrature element matrices + CSR assembly + one SpMV = "
                       f"{t1 - t0:.2f} s; SpMV alone with the assembled matrix {(t2 - t1) / reps * 1e3:.2f} ms "
                       f"({m.n_dof / ((t2 - t1) / reps) / 1e9:.4f} GDoF/s)")}


def run_newton(args, w, dev, n_newton=5, restart=50):
    """Newton driver on the workload: FP64 and mixed precision with equal Krylov budgets."""
    import torch
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov
    m = w.mesh
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    out = {}
    for prec in ("fp64", "mixed"):
        eng = Engine(0)
        eng.upload_mesh(m)
        eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
        u, p = t(w.u), t(w.p)
        nk = NewtonKrylov(eng, restart=restart, precision=prec, refine=1, precond=args.precond,
                          triangular=not args.block_diagonal, linearization=args.linearization,
                          coarse=(m, (args.coarse, args.coarse)) if args.coarse > 0 else None,
                          coarse_mode=args.coarse_mode)
        st = nk.solve(u, p, n_newton=n_newton, lin_tol=1e-8, verbose=True)
        out[prec] = dict(seconds=st.seconds, newton_residuals=st.newton_residuals,
                         linear_reductions=st.linear_reductions, krylov_iterations=st.krylov_iterations,
                         step_lengths=st.step_lengths)
        eng.close()
        del nk
        torch.cuda.empty_cache()
    a, b = np.array(out["fp64"]["newton_residuals"]), np.array(out["mixed"]["newton_residuals"])
    pc = {"jacobi": "point-Jacobi", "line": "vertical-line-block"}[args.precond] + \
        (f" + F~ coarse correction ({args.coarse}x{args.coarse} lattice, {args.coarse_mode})" if args.coarse > 0 else "") + \
        " velocity block, " + ("block-diagonal" if args.block_diagonal else "block upper-triangular")
    steps = "Newton" if args.linearization == "newton" else "Picard"
    rec = {"metric": f"Newton-Krylov solve: 5 {steps} steps x FGMRES(50), {pc}, FP64 vs mixed",
           "value": out["fp64"]["seconds"] / out["mixed"]["seconds"], "unit": "speedup mixed vs fp64",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": f"config{args.config}", "n_dof": m.n_dof, "n_el": m.n_el, "k": m.k,
                      "preconditioner": args.precond, "triangular": not args.block_diagonal,
                      "linearization": args.linearization, "coarse_cells": args.coarse,
                      "coarse_mode": args.coarse_mode},
           "residual_reduction_fp64": float(a[-1] / a[0]), "residual_reduction_mixed": float(b[-1] / b[0]),
           "max_rel_diff_newton_residuals": float(np.max(np.abs(a - b) / a)), "fp64": out["fp64"],
           "mixed": out["mixed"]}
    print(json.dumps(rec), flush=True)


def run_solve(args, w, dev, target=1e-6, inner_tol=1e-3, max_cycles=10, restart=50):
    """Linear solve J d = b at the workload's state to a relative FP64 residual of 1e-6: cycles of
    FGMRES(50) on the FP64 residual r = b - J_64 d (restarted FGMRES in FP64; FP32 Krylov cycles with
    FP64 outer refinement in mixed precision), b = J x for a seeded random x."""
    import torch
    from paper_1406_6573_amd import Engine
    from paper_1406_6573_amd.solve import NewtonKrylov
    m = w.mesh
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    eng = Engine(0)
    eng.upload_mesh(m)
    eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
    eng.set_state(t(w.u), t(w.p))
    N = m.n_nodes
    xr = np.random.default_rng(5).uniform(-1, 1, m.n_dof)
    xr[:3 * N][m.dmask.ravel().astype(bool)] = 0.0
    yu, yp = eng.jacobian_apply(t(xr[:3 * N].reshape(3, N)), t(xr[3 * N:].reshape(m.n_el, m.n_p)), "fp64")
    b = torch.cat([yu.reshape(-1), yp.reshape(-1)])
    bn = float(b.norm())
    out = {}
    for prec in ("fp64", "mixed"):
        nk = NewtonKrylov(eng, restart=restart, precision=prec, refine=1, precond=args.precond,
                          triangular=not args.block_diagonal,
                          coarse=(m, (args.coarse, args.coarse)) if args.coarse > 0 else None,
                          coarse_mode=args.coarse_mode)
        d = torch.zeros_like(b)
        r = torch.empty_like(b)
        b32 = torch.empty(nk.n, dtype=torch.float32, device=dev) if prec == "mixed" else None
        hist, its = [1.0], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nk.setup_preconditioner()
        r.copy_(b)
        for _ in range(max_cycles):
            # one FGMRES cycle on the FP64 residual: in FP64, or in FP32 on its rounding (refinement)
            if prec == "fp64":
                nk.d64.zero_()
                k, _ = nk.fgmres(r, nk.d64, inner_tol)
                d += nk.d64
            else:
                eng.vec_convert(r, b32)
                nk.tmp.zero_()
                k, _ = nk.fgmres(b32, nk.tmp, inner_tol)
                eng.vec_convert(nk.tmp, nk.w64)
                d += nk.w64
            its += k
            du, dp = nk.split(d)
            ru, rp = eng.jacobian_apply(du.contiguous(), dp.contiguous(), "fp64")
            torch.sub(b, torch.cat([ru.reshape(-1), rp.reshape(-1)]), out=r)
            hist.append(float(r.norm()) / bn)
            if hist[-1] <= target:
                break
        torch.cuda.synchronize()
        out[prec] = dict(seconds=time.perf_counter() - t0, krylov_iterations=its, residual_history=hist)
        print(f"[bench] solve {prec}: {its} iterations, residuals " + " ".join(f"{v:.2e}" for v in hist),
              file=sys.stderr, flush=True)
        del nk
    eng.close()
    pc = {"jacobi": "point-Jacobi", "line": "vertical-line-block"}[args.precond] + \
        (f" + F~ coarse correction ({args.coarse}x{args.coarse} lattice, {args.coarse_mode})" if args.coarse > 0 else "") + \
        " velocity block, " + ("block-diagonal" if args.block_diagonal else "block upper-triangular")
    rec = {"metric": f"Linear solve J d = b to relative residual {target:g}: FGMRES({restart}) cycles on the FP64 "
                     f"residual, {pc}, FP64 vs mixed",
           "value": out["fp64"]["seconds"] / out["mixed"]["seconds"], "unit": "speedup mixed vs fp64",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": f"config{args.config}", "n_dof": m.n_dof, "n_el": m.n_el, "k": m.k,
                      "pressure": args.pspace, "preconditioner": args.precond,
                      "triangular": not args.block_diagonal, "coarse_cells": args.coarse,
                      "coarse_mode": args.coarse_mode},
           "reached_fp64": out["fp64"]["residual_history"][-1] <= target,
           "reached_mixed": out["mixed"]["residual_history"][-1] <= target,
           "fp64": out["fp64"], "mixed": out["mixed"]}
    print(json.dumps(rec), flush=True)


WORKLOADS = {1: "unit box 8x8x2 {pair}", 2: "slab 64x64x8 {pair}, aspect 125, 20% columns refined 2:1",
             3: "terrain slab 128x128x16 {pair}, Fourier base and thickness", 4: "slab 96x96x12 {pair}, 20% refined",
             5: "dome 256x256x8 {pair}, margin refined"}


def measure_applies(config_id, pspace, steps, warmup, dev, with_aux=True):
    """Build the workload, then time `steps` Jacobian applies in FP64, FP32 and FP32 with bfloat16
    operators (after `warmup` untimed ones each), with inputs resident in HBM.  Returns a dict."""
    import torch
    from meshgen import make_config
    from paper_1406_6573_amd import Engine

    print(f"[bench] building workload config{config_id}", file=sys.stderr, flush=True)
    w = make_config(config_id, n_dirs=1, pspace=pspace)
    m = w.mesh
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    eng = Engine(0)
    eng.upload_mesh(m)
    eng.set_params(w.n, w.eps, w.B0, w.body, t(w.logA), t(w.beta))
    u, p = t(w.u), t(w.p)
    xu, xp = w.directions[0]
    x64u, x64p = t(xu), t(xp)
    x32u, x32p = x64u.float(), x64p.float()
    y64 = (torch.empty_like(x64u), torch.empty_like(x64p))
    y32 = (torch.empty_like(x32u), torch.empty_like(x32p))
    sz = dict(eng.sizes)
    sz["k"] = m.k
    geo = eng.geometry_kind()
    print(f"[bench] n_el={sz['n_el']} n_dof={sz['n_dof']} geometry={geo}", file=sys.stderr, flush=True)

    def timed(fn, n, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n * 1e3

    eng.set_state(u, p)
    res = {}
    if with_aux:
        res["set_state_ms"] = timed(lambda: eng.set_state(u, p), 5, 1)
        res["residual_ms"] = timed(lambda: eng.residual(), 10, 2)
        res["vjp_fp64_ms"] = timed(lambda: eng.residual_vjp(x64u, x64p), 10, 2)
    out = {}
    for prec, (xa, xb, yy) in (("fp64", (x64u, x64p, y64)), ("fp32", (x32u, x32p, y32)),
                              ("bf16ops", (x32u, x32p, y32))):
        fn = lambda: eng.jacobian_apply(xa, xb, prec, out=yy)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        eng.set_kernel_timing(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        kms, nk = eng.kernel_time()
        eng.set_kernel_timing(False)
        out[prec] = dict(ms=ms, kernel_ms=kms / max(nk, 1))
        print(f"[bench] config{config_id} {prec}: {ms:.4f} ms/apply, device time {kms / max(nk, 1):.4f} ms",
              file=sys.stderr, flush=True)
    # accuracy of the mixed paths against the FP64 apply (which matches the FP64 oracle to ~1e-13)
    r64u, r64p = eng.jacobian_apply(x64u, x64p, "fp64")
    ref = torch.cat([r64u.reshape(-1), r64p.reshape(-1)])
    errs = {}
    for prec in ("fp32", "bf16ops"):
        a, b = eng.jacobian_apply(x32u, x32p, prec)
        got = torch.cat([a.reshape(-1), b.reshape(-1)]).double()
        errs[prec] = float((got - ref).norm() / ref.norm())
    eng.close()
    del eng, u, p, x64u, x64p, x32u, x32p, y64, y32, r64u, r64p, ref
    torch.cuda.empty_cache()
    n_dof = sz["n_dof"]
    res.update(sz=sz, geo=geo, k=m.k, out=out, errs=errs,
               gdofs={k: n_dof / (v["ms"] * 1e-3) / 1e9 for k, v in out.items()},
               bytes32=algorithmic_bytes(sz, geo, 4), bytes64=algorithmic_bytes(sz, geo, 8))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the second (slab Q3) workload")
    ap.add_argument("--pspace", choices=["P", "Q"], default="P",
                    help="pressure space: P = P_{k-1} (the workloads as stated), Q = Q_{k-2} (Gauss-point Lagrange)")
    ap.add_argument("--newton", action="store_true",
                    help="instead of the apply benchmark, run the Newton/FGMRES driver (5 steps x FGMRES(50)) "
                         "in FP64 and in mixed precision and print one JSON line")
    ap.add_argument("--precond", choices=["jacobi", "line"], default="line",
                    help="velocity block of the Newton driver's preconditioner (with --newton)")
    ap.add_argument("--block-diagonal", action="store_true",
                    help="block-diagonal instead of block upper-triangular preconditioner (with --newton)")
    ap.add_argument("--linearization", choices=["newton", "picard"], default="newton",
                    help="operator of the nonlinear steps (with --newton)")
    ap.add_argument("--coarse", type=int, default=0,
                    help="with --newton/--solve: add the F~-based horizontal coarse correction on a lattice of this "
                         "many cells per direction (0: none)")
    ap.add_argument("--coarse-mode", choices=["mult", "add"], default="mult",
                    help="coarse correction combined with the line blocks multiplicatively or additively")
    ap.add_argument("--solve", action="store_true",
                    help="time a linear solve to 1e-6 at the workload's state, FP64 vs mixed, instead of the applies")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (multi-GPU sharding is "
              f"not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from meshgen import make_config

    dev = torch.device("cuda", 0)
    if args.calibration_copy_mib > 0:
        src = torch.ones(args.calibration_copy_mib * 2 ** 18, dtype=torch.float32, device=dev)
        dst = src.clone()
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.calibration_copy_mib} MiB done ({float(dst[0])})", file=sys.stderr)
        del src, dst
    if args.newton or args.solve:
        print(f"[bench] building workload config{args.config}", file=sys.stderr, flush=True)
        w = make_config(args.config, n_dirs=1, pspace=args.pspace)
        (run_newton if args.newton else run_solve)(args, w, dev)
        return

    r = measure_applies(args.config, args.pspace, args.steps, args.warmup, dev)
    sz, geo, k, out, errs, gdofs = r["sz"], r["geo"], r["k"], r["out"], r["errs"], r["gdofs"]
    ach32 = r["bytes32"] / (out["fp32"]["kernel_ms"] * 1e-3) / 1e9
    ach64 = r["bytes64"] / (out["fp64"]["kernel_ms"] * 1e-3) / 1e9
    pair = f"Q{k}xP{k - 1}" if args.pspace == "P" else f"Q{k}xQ{k - 2}"
    traffic = measured_traffic(args.config) if args.pspace == "P" else None
    rec = {
        "metric": METRIC, "value": gdofs["fp32"], "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["fp32"]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"config{args.config}: " + WORKLOADS[args.config].format(pair=pair),
                   "k": k, "n_el": sz["n_el"], "n_dof": sz["n_dof"], "geometry": geo, "pressure": pair.split("x")[1]},
        "rel_err_vs_fp64": errs["fp32"],
        "fp64": {"value": gdofs["fp64"], "ms_per_step": out["fp64"]["ms"],
                 "roofline_frac": ach64 / HBM_PEAK_GBS},
        "speedup_mixed_vs_fp64": out["fp64"]["ms"] / out["fp32"]["ms"],
        "bf16ops_trial": {"value": gdofs["bf16ops"], "rel_err_vs_fp64": errs["bf16ops"]},
        "set_state_ms": r["set_state_ms"], "residual_ms": r["residual_ms"], "vjp_fp64_ms": r["vjp_fp64_ms"],
        "roofline": {"bound": "hbm", "achieved": ach32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach32 / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / 1e9,
                     "compute": valu_issue(args.config, out["fp32"]["kernel_ms"]) if args.pspace == "P" else None,
                     "traffic_unit": "GB per apply",
                     "kernel": f"one FP32 apply (all its kernels), Q{k} {geo}",
                     "kernel_ms": out["fp32"]["kernel_ms"], "algorithmic_bytes": r["bytes32"]},
    }
    if not args.no_extra and args.config != 2:
        r2 = measure_applies(2, args.pspace, args.steps, args.warmup, dev, with_aux=False)
        pair2 = "Q3xP2" if args.pspace == "P" else "Q3xQ1"
        rec["slab_q3"] = {
            "workload": "config2: " + WORKLOADS[2].format(pair=pair2), "n_dof": r2["sz"]["n_dof"],
            "fp32": {"value": r2["gdofs"]["fp32"], "ms_per_step": r2["out"]["fp32"]["ms"],
                     "roofline_frac": r2["bytes32"] / (r2["out"]["fp32"]["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "fp64": {"value": r2["gdofs"]["fp64"], "ms_per_step": r2["out"]["fp64"]["ms"],
                     "roofline_frac": r2["bytes64"] / (r2["out"]["fp64"]["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "bf16ops_trial": {"value": r2["gdofs"]["bf16ops"], "rel_err_vs_fp64": r2["errs"]["bf16ops"]},
            "rel_err_vs_fp64": r2["errs"]["fp32"],
            "traffic_GB_per_apply": (lambda v: None if v is None else v / 1e9)(measured_traffic(2)),
        }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a reduced sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
