#!/usr/bin/env python3
"""Benchmark of the per-time-step Newton–Krylov–Schwarz solve of scheme (2.20).

Workload (one "step" = one accepted time step, all Newton iterations included):
2D periodic [0,1]^2, 512 x 512 cells, alpha = beta = 1.2, theta = 0.1, gamma = 1e-3,
rho = 1, seeded initial data u0 = 0.5 + 0.05 U(-1,1), v0 = 0.05 U(-1,1); adaptive
dt in [1e-4, 1e-1] (eta0 = 1e4); FP64 Newton (tol 1e-8) with right-preconditioned
GMRES(30) and left-restricted additive Schwarz on 8 x 8 subdomains, overlap 2,
subdomain ILU(0) (shifted by 0.02 diag, factored once per step attempt).  The
default run is the workload's 200 steps from the initial data.

Metric: dof * Newton iterations / s with dof = 2 * cells, counting every Newton
iteration of every attempt, over the timed steps (inputs resident in HBM).

Also printed: the roofline of the dominant kernel (algorithmic bytes per launch
over its average duration, measured live with HIP events on the library's stream)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # the headline configuration (one accepted step = one bench step)
    "periodic512": dict(name="periodic512", shape=(512, 512), bc="periodic", sub=(8, 8), overlap=2,
                        adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4, newton_rtol=1e-8, newton_atol=1e-13,
                        gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.02, precision="fp64",
                        seed=0, steps=200,
                        text="periodic512: 2D periodic 512x512, 200 adaptive steps dt in [1e-4,1e-1], FP64 NKS, "
                             "left-RAS 8x8 overlap 2, ILU(0) shift 0.02, GMRES(30), tol 1e-8"),
    # the same run with the subdomain ILU(0) on the width-2 box pattern (no shift) over 32x32
    # subdomains, its fastest layout at this size
    "periodic512_box32": dict(name="periodic512_box32", shape=(512, 512), bc="periodic", sub=(32, 32), overlap=2,
                              adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4, newton_rtol=1e-8,
                              newton_atol=1e-13, gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.0,
                              precision="fp64", seed=0, steps=200, subsolver="iluk_box", fill_level=0,
                              text="periodic512_box32: 2D periodic 512x512, 200 adaptive steps dt in [1e-4,1e-1], "
                                   "FP64 NKS, left-RAS 32x32 overlap 2, ILU(0) on the width-2 box pattern (no "
                                   "shift), GMRES(30), tol 1e-8"),
    # the 2048^2 Neumann configuration with FP32 subdomain factors and solves
    "neumann2048": dict(name="neumann2048", shape=(2048, 2048), bc="neumann", sub=(16, 16), overlap=2,
                        adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4, newton_rtol=1e-8, newton_atol=1e-13,
                        gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.02, precision="mixed",
                        seed=0, steps=50,
                        text="neumann2048: 2D Neumann 2048x2048, 50 adaptive steps dt in [1e-4,1e-1], FP64 NKS "
                             "with FP32 subdomain ILU(0) factors/solves, left-RAS 16x16 overlap 2, shift 0.02, "
                             "GMRES(30), tol 1e-8"),
    # the 3D Neumann configuration; 512 subdomains of 16^3 as in the paper's 128^3 solver
    # study on 512 processors (Section 4)
    "neumann128_3d": dict(name="neumann128_3d", shape=(128, 128, 128), bc="neumann", sub=(8, 8, 8), overlap=1,
                          adaptive=True, dt_min=1e-4, dt_max=2.0, eta0=100.0, newton_rtol=1e-8, newton_atol=1e-13,
                          gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.02, precision="fp64",
                          seed=0, steps=20,
                          text="neumann128_3d: 3D Neumann 128^3, 20 adaptive steps dt in [1e-4,2] (eta0 = 100), FP64 "
                               "NKS, left-RAS 8x8x8 overlap 1, ILU(0) shift 0.02, GMRES(30), tol 1e-8"),
    # the paper's long adaptive 2D run (Section 4.2: alpha 4, beta 2, gamma 5e-3, theta 0.1,
    # rho 1e-3, u0 = 0.55 + 0.05 U(-1,1), dt in [1e-4, 10], eta = 1e4), its first steps
    "long128": dict(name="long128", shape=(128, 128), bc="periodic", sub=(8, 8), overlap=1,
                    adaptive=True, dt_min=1e-4, dt_max=10.0, eta0=1e4, newton_rtol=1e-8, newton_atol=1e-13,
                    gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.02, precision="fp64",
                    seed=0, steps=2000, u_mean=0.55,
                    phys=dict(alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001),
                    text="long128: the paper's long adaptive 2D run, 128x128 periodic, alpha 4, beta 2, gamma 5e-3, "
                         "theta 0.1, rho 1e-3, u0 = 0.55 + 0.05 U(-1,1), dt in [1e-4,10] (eta0 = 1e4), first 2000 "
                         "steps, FP64 NKS, left-RAS 8x8 overlap 1, ILU(0) shift 0.02, GMRES(30), tol 1e-8"),
    # the same run carried on to late times: exact subdomain LU (ILU(0) forces dt retries
    # once dt grows) and an absolute Newton tolerance above the residual's FP64 rounding
    # floor (about 2e-7 on this grid), which the late, slowly changing states reach
    "long128_lu": dict(name="long128_lu", shape=(128, 128), bc="periodic", sub=(8, 8), overlap=1,
                       adaptive=True, dt_min=1e-4, dt_max=10.0, eta0=1e4, newton_rtol=1e-8, newton_atol=1e-6,
                       gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.0, precision="fp64",
                       seed=0, steps=6000, u_mean=0.55, subsolver="lu",
                       phys=dict(alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001),
                       text="long128_lu: the paper's long adaptive 2D run (Section 4.2 parameters, 128x128 periodic, "
                            "dt in [1e-4,10], eta0 = 1e4) to late times: 6000 steps, FP64 NKS, left-RAS 8x8 overlap 1, "
                            "exact subdomain LU, GMRES(30), Newton eps_r 1e-8 with eps_a 1e-6"),
    # the 2048^2 Neumann configuration's coefficients and form (FP32 subdomain solves, adaptive
    # dt, 50 steps) at the largest grid where a one-level Schwarz method converges here:
    # 1024^2 with exact subdomain LU on 32x8 boxes with overlap 8 (19 GMRES per Newton step)
    "neumann1024_lu": dict(name="neumann1024_lu", shape=(1024, 1024), bc="neumann", sub=(32, 8), overlap=8,
                           adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4, newton_rtol=1e-8, newton_atol=1e-13,
                           gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.0, precision="mixed",
                           seed=0, steps=50, subsolver="lu",
                           text="neumann1024_lu: 2D Neumann 1024x1024, 50 adaptive steps dt in [1e-4,1e-1], FP64 NKS "
                                "with FP32 exact subdomain LU factors/solves, left-RAS 32x8 overlap 8, GMRES(30), "
                                "tol 1e-8"),
    "long128_lu_neumann": dict(name="long128_lu_neumann", shape=(128, 128), bc="neumann", sub=(8, 8), overlap=1,
                               adaptive=True, dt_min=1e-4, dt_max=10.0, eta0=1e4, newton_rtol=1e-8,
                               newton_atol=1e-6, gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30, ilu_shift=0.0,
                               precision="fp64", seed=0, steps=6000, u_mean=0.55, subsolver="lu",
                               phys=dict(alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001),
                               text="long128_lu_neumann: as long128_lu with homogeneous Neumann boundaries"),
}
# 96 independent periodic instances of uneven size (N in {96,128,192,256}), theta and
# gamma drawn per instance, 10 steps at dt = 1e-3, all instances in one batched solve
BATCH = dict(name="batch96", count=96, base_seed=1000, steps=10, overlap=2, boxes=(32, 48, 64),
             common=dict(dt_fixed=1e-3, overlap=2, ilu_shift=0.02, newton_rtol=1e-8, newton_atol=1e-13,
                         gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30),
             text="batch96: 96 independent 2D periodic instances, N uniform in {96,128,192,256}, theta~U(0.08,0.12), "
                  "gamma~U(5e-4,2e-3), 10 fixed steps dt=1e-3, one batched NKS per step (left-RAS ILU(0) shift 0.02, "
                  "overlap 2, autotuned boxes, GMRES(30) cycles replayed from HIP graphs), tol 1e-8")
# the same batch with the subdomain ILU(0) on the width-2 box pattern (no shift)
BATCH_BOX = dict(BATCH, name="batch96_box", boxes=(24, 32, 48, 64),
                 common=dict(BATCH["common"], ilu_shift=0.0, subsolver="iluk_box", fill_level=0),
                 text="batch96_box: the batch96 instances and steps with the subdomain ILU(0) on the width-2 box "
                      "pattern (no shift), autotuned boxes, one batched NKS per step, tol 1e-8")
WORKLOAD = WORKLOADS["periodic512"]


def ras_bytes_per_cell(box_cells: float, owned_cells: float, nslot: int = 24, sp: int = 8) -> float:
    """Algorithmic bytes of one left-RAS apply per owned cell: read r on the extended
    box (16 B per box cell), read the factors (nslot * sp per box cell), write z on the
    owned cells (16 B)."""
    omega = box_cells / owned_cells
    return omega * 16.0 + omega * nslot * sp + 16.0


def spmv_dots_bytes_per_cell(j_avg: float) -> float:
    """J z (24 coefficients + z) written to w, plus one read of j+1 basis vectors."""
    return 24 * 8 + 16 + 16 + 16 * (j_avg + 1)


def arnoldi_bytes_per_cell(k: float, m: int = 30) -> float:
    """Sum over the k Arnoldi steps of one Newton solve (cycles of m) of B_arn(j) =
    32 (j + 1) + 64 per cell (CGS: one read of basis vectors 0..j for the dots, one for
    the update, plus the new vector); k may be fractional (a mean over Newton solves)."""
    total, left = 0.0, k
    while left > 0:
        kk = min(left, m)
        total += 32.0 * kk * (kk + 1) / 2.0 + 64.0 * kk
        left -= kk
    return total


def step_bytes_per_cell(newton: int, gmres: int, steps: int, nnz: int, omega: float, sp: int, m: int = 30,
                        fac_slots: int = 0, ras_slots: int = 0) -> float:
    """Algorithmic bytes per cell of a run (the minimum the method moves: one read of
    each operand and one write of each result): per Newton iteration B_res (two
    evaluations: the iteration's residual and an accepted full step) + B_jac + B_fact
    (one factorisation per step, factor reuse) + sum over its GMRES iterations of B_spmv
    + B_ras + B_arn(j) + B_upd, with the mean GMRES count per Newton iteration.
    fac_slots / ras_slots: factor values per box cell written by the factorisation and
    read (with the box vector) by one Schwarz apply; default nnz (the stencil-pattern
    ILU(0), whose records have the Jacobian's slots)."""
    if newton <= 0:
        return 0.0
    k = gmres / newton
    b_res, b_jac, b_spmv = 48.0, 32.0 + 8.0 * nnz, 8.0 * nnz + 32.0
    b_ras = omega * 16.0 + omega * (ras_slots or nnz) * sp + 16.0
    b_fact = omega * (nnz * 8.0 + (fac_slots or nnz) * sp) * steps / newton
    per_newton = 2 * b_res + b_jac + b_fact + k * (b_spmv + b_ras) + arnoldi_bytes_per_cell(k, m) + 16.0 * (k + 1)
    return newton * per_newton


# The dominant (Schwarz) kernel of each workload, as rocprofv3 names it, and its source.
RAS_KERNELS = {
    "periodic512": ("void k_ras_apply2d<double, 1, 5, false>", "schwarz2d.hip"),
    "neumann128_3d": ("void k_ras_apply3d_win<double, 3>", "schwarz3d.hip"),
    "periodic512_box32": ("void k_boxilu_apply2d<double, 3, 4, 64, false>", "boxilu2d.hip"),
}


def code_sha256(text: str) -> str:
    """SHA-256 of a C++ source without its // comments, blank lines and indentation:
    changes only when the code does."""
    import hashlib
    import re
    lines = [re.sub(r"//.*$", "", line).strip() for line in text.splitlines()]
    return hashlib.sha256("\n".join(line for line in lines if line).encode()).hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the workload's Schwarz kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (profiles/traffic_<workload>.json, scaled by a
    plain-copy calibration), or None when the kernel's source code changed since the
    counters were taken (or none were taken)."""
    if workload not in RAS_KERNELS:
        return None
    kernel, source = RAS_KERNELS[workload]
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")))
        src = open(os.path.join(ROOT, "paper_2007_04560_amd", "csrc", source)).read()
    except OSError:
        return None
    if code_sha256(src) != prof.get("source_code_sha256"):
        return None
    k = prof["kernels"].get(kernel)
    return k["hbm_bytes_per_launch"] if k else None


def run_gpu(steps: int, warmup: int, timing: bool, w=None):
    import numpy as np
    import torch
    from acch_inputs import random_ic
    from paper_2007_04560_amd import Solver

    w = w or WORKLOAD
    u0, v0 = random_ic(w["shape"], w["seed"], u_mean=w.get("u_mean", 0.5))
    kw = dict(bc=w["bc"], sub=w["sub"], overlap=w["overlap"], adaptive=w["adaptive"], dt_min=w["dt_min"],
              dt_max=w["dt_max"], eta0=w["eta0"], newton_rtol=w["newton_rtol"], newton_atol=w["newton_atol"],
              gmres_rtol=w["gmres_rtol"], gmres_atol=w["gmres_atol"], gmres_restart=w["gmres_restart"],
              ilu_shift=w["ilu_shift"], precision=w["precision"], subsolver=w.get("subsolver", "ilu0"),
              fill_level=w.get("fill_level", 0),
              **w.get("phys", {}))
    if warmup > 0:
        with Solver(u0, v0, **kw) as s:
            s.step(warmup)
    s = Solver(u0, v0, **kw)
    E0, M0 = s.energy()
    # sampled: HIP events around one Schwarz launch in 16 and none elsewhere (an event
    # pair around every launch costs ~20 % of the step time on this workload)
    s.timing(2 if timing else False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if steps <= 1000:
        recs = s.step(steps)
    else:   # long runs: chunks of 500 steps, a progress line on stderr after each
        recs = []
        while len(recs) < steps:
            recs += s.step(min(500, steps - len(recs)))
            print(json.dumps({"progress_steps": len(recs), "t": recs[-1]["t"], "dt": recs[-1]["dt"],
                              "wall_s": round(time.perf_counter() - t0, 1)}), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = s.kernel_stats() if timing else {}
    launches, syncs = s.counters()
    info = s.info()
    E1, M1 = s.energy()
    fields = s.fields()
    s.close()
    return dict(elapsed=t1 - t0, recs=recs, stats=stats, info=info, launches=launches, syncs=syncs,
                E0=E0, E1=E1, M0=M0, M1=M1, ncell=u0.size, fields=fields)


def batch_inputs():
    from acch_inputs import batched_instances
    insts = batched_instances(BATCH["count"], BATCH["base_seed"])
    fields = [w.initial() for w in insts]
    params = [dict(bc="periodic", theta=w.theta, gamma=w.gamma) for w in insts]
    return fields, params


def run_batch(steps: int, warmup: int, with_sequential: bool = True, B=BATCH):
    """The batched workload: autotune the box size, then time `steps` batched steps in
    FP64 and in mixed precision (fresh batches from the initial data), the batched
    preconditioner launch with HIP events on the batch stream, and the same instances
    solved one after another by the single-instance solver (FP64)."""
    import numpy as np
    import torch
    from paper_2007_04560_amd import BatchSolver, Solver
    from paper_2007_04560_amd.batch import autotune, with_boxes

    fields, params = batch_inputs()
    common = B["common"]
    shapes = [u.shape for u, _ in fields]
    dof = np.array([2 * u.size for u, _ in fields])
    out = {"box": {}, "autotune_s_per_step": {}}
    cache = os.path.join(tempfile.gettempdir(), "acch_batch_tune_%s.json" % B["name"])
    for prec in ("fp64", "mixed"):
        # box width tuned per precision (cached per instance-size mix, precision, overlap)
        best, tune = autotune(fields, params, boxes=B["boxes"], steps=1, cache=cache, precision=prec, **common)
        out["box"][prec] = best
        out["autotune_s_per_step"][prec] = {str(k): round(v, 4) for k, v in tune.items()}
        sub_params = with_boxes(shapes, params, best, B["overlap"])
        out.setdefault("sub_params_by_precision", {})[prec] = sub_params
        if warmup > 0:
            with BatchSolver(fields, sub_params, precision=prec, **common) as b:
                b.step(warmup)
        b = BatchSolver(fields, sub_params, precision=prec, **common)
        b.stream.synchronize()
        t0 = time.perf_counter()
        nit, git = b.step(steps)
        b.stream.synchronize()
        el = time.perf_counter() - t0
        r = {"elapsed": el, "newton": int(nit.sum()), "gmres": int(git.sum()),
             "dof_newton": float((dof * nit).sum()), "counters": b.counters(),
             "fields": [b.fields(i) for i in range(len(fields))]}   # after the timed region
        if prec == "fp64":
            info = b.info()
            x = torch.randn(2 * info["ncell"], dtype=torch.float64, device=b.device)
            z = b.precondition(x)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            with torch.cuda.stream(b.stream):
                e0.record()
                for _ in range(reps):
                    b.precondition(x, z)
                e1.record()
            e1.synchronize()
            r["ras_avg_s"] = e0.elapsed_time(e1) / reps * 1e-3
            r["info"] = info
        b.close()
        out[prec] = r
    sub_params = out.pop("sub_params_by_precision")["fp64"]   # the FP64 batch's boxes
    # Form 1 on the batch: the mixed-precision batch's final fields against the FP64 batch's
    out["mixed_vs_fp64_max_rel_l2"] = max(_rel_l2(m, f) for m, f in zip(out["mixed"].pop("fields"),
                                                                         out["fp64"].pop("fields")))
    if with_sequential:
        t_seq = 0.0
        n_seq = 0
        for (u, v), p in zip(fields, sub_params):
            kw = dict(common)
            kw.update(p)
            with Solver(u, v, **kw) as s:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                recs = s.step(steps)
                torch.cuda.synchronize()
                t_seq += time.perf_counter() - t0
                n_seq += sum(int(x["newton_its"]) for x in recs)
        out["sequential"] = {"elapsed": t_seq, "newton": n_seq}
    out["dof_total"] = int(dof.sum())
    out["sub_params"] = sub_params
    out["shapes"] = shapes
    return out


def batch_line(args, B=BATCH):
    r = run_batch(args.steps, args.warmup, with_sequential=not args.no_sequential, B=B)
    f = r["fp64"]
    value = f["dof_newton"] / f["elapsed"]
    # algorithmic bytes of one batched Schwarz launch per instance: stencil pattern omega*16 +
    # omega*24*8 + 16 per owned cell; box pattern (2*52 + 4)*8 + 16 per box cell (the L and U
    # records, the box vector written and read in each sweep) + 16 per owned cell
    box = B["common"].get("subsolver") == "iluk_box"
    d = B["overlap"]
    bytes_launch = 0.0
    for (ny, nx), p in zip(r["shapes"], r["sub_params"]):
        kx, ky = p["sub"]
        box_cells = (nx + 2 * d * kx) * (ny + 2 * d * ky)
        bytes_launch += box_cells * ((108 * 8 + 16) if box else (16 + 24 * 8)) + 16 * nx * ny
    achieved = bytes_launch / f["ras_avg_s"] / 1e9
    line = {
        "metric": "dof*Newton-steps/s at 1e-8 tol",
        "value": round(value, 1),
        "unit": "dof*Newton/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f["elapsed"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": B["text"], "instances": B["count"], "dof": r["dof_total"],
                   "box": r["box"], "autotune_s_per_step": r["autotune_s_per_step"],
                   "newton_its": f["newton"], "gmres_its": f["gmres"],
                   "batched_fp64_s": round(f["elapsed"], 4),
                   "batched_mixed_s": round(r["mixed"]["elapsed"], 4),
                   "mixed_value": round(r["mixed"]["dof_newton"] / r["mixed"]["elapsed"], 1),
                   "mixed_vs_fp64_final_fields_max_rel_l2": r["mixed_vs_fp64_max_rel_l2"],
                   "counters_fp64": f["counters"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": ("k_boxilu_apply2d" if box else "k_ras_apply2d") + " (all subdomains of all instances)",
                     "avg_us": round(f["ras_avg_s"] * 1e6, 2), "bytes_per_launch": int(bytes_launch)},
    }
    if "sequential" in r:
        sq = r["sequential"]
        line["config"]["sequential_fp64_s"] = round(sq["elapsed"], 4)
        line["config"]["speedup_batched_vs_sequential"] = round(sq["elapsed"] / f["elapsed"], 2)
        line["config"]["speedup_mixed_vs_sequential"] = round(sq["elapsed"] / r["mixed"]["elapsed"], 2)
    print(json.dumps(line), flush=True)
    return 0


def adjoint_line(args, w=None):
    """Gradient of the final energy after `steps` accepted steps of a workload (512x512
    periodic or the 128^3 Neumann one) with respect to (u0, v0, alpha, beta, theta,
    gamma), checkpoints every 5 steps: the forward run, then the backward pass
    (segment recomputation + transposed solves)."""
    import numpy as np
    import torch
    from acch_inputs import random_ic
    from paper_2007_04560_amd import Solver
    from paper_2007_04560_amd.adjoint import final_energy
    w = w or WORKLOAD
    u0, v0 = random_ic(w["shape"], w["seed"])
    kw = dict(bc=w["bc"], sub=w["sub"], overlap=w["overlap"], adaptive=w["adaptive"], dt_min=w["dt_min"],
              dt_max=w["dt_max"], eta0=w["eta0"], newton_rtol=w["newton_rtol"], newton_atol=w["newton_atol"],
              gmres_rtol=w["gmres_rtol"], gmres_atol=w["gmres_atol"], gmres_restart=w["gmres_restart"],
              ilu_shift=w["ilu_shift"], subsolver=w.get("subsolver", "ilu0"), fill_level=w.get("fill_level", 0))
    boxilu = w.get("subsolver") == "iluk_box"
    steps = args.steps
    params = torch.tensor([1.2, 1.2, 0.1, 1e-3], dtype=torch.float64, requires_grad=True)
    tu = torch.tensor(u0, requires_grad=True)
    tv = torch.tensor(v0, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E = final_energy(tu, tv, params, steps, checkpoint_every=5, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    E.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # the transposed Schwarz apply, timed with HIP events on the library's stream
    s = Solver(u0, v0, **kw)
    X = s.vector(np.concatenate([u0.ravel(), v0.ravel()]))
    s.jacobian(X, X, 1e-3)
    s.factor()
    r = torch.randn(2 * u0.size, dtype=torch.float64, device="cuda")
    s.timing(True)
    for _ in range(20):
        s.precondition_transpose(r)
    ras_ms, ras_n = s.kernel_stats()["ras"]
    info = s.info()
    s.close()
    avg_s = ras_ms / ras_n * 1e-3
    owned = u0.size / info["nsub"]
    if u0.ndim == 3:
        box = 1.0
        for n_a, p_a in zip(reversed(w["shape"]), w["sub"]):
            box *= n_a / p_a + 2 * w["overlap"]
        bytes_launch = ras_bytes_per_cell(box, owned, nslot=40) * u0.size
    elif boxilu:   # transposed records of every box cell, the box vector written and read back, r, z
        bytes_launch = info["nsub"] * info["box_w"] * info["box_h"] * (108 * 8 + 16) + 16 * u0.size
    else:
        bytes_launch = ras_bytes_per_cell(info["box_w"] * info["box_h"], owned) * u0.size
    achieved = bytes_launch / avg_s / 1e9
    line = {"metric": "gradient time of the final energy (forward + adjoint)", "value": round(t2 - t0, 4),
            "unit": "s", "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round((t2 - t0) / steps * 1e3, 3),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"adjoint of {w['name']}: dE/d(u0, v0, alpha, beta, theta, gamma) after {steps} "
                                   "adaptive steps, dt frozen, checkpoints every 5 steps",
                       "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
                       "energy": float(E.detach()), "grad_params": [float(x) for x in params.grad],
                       "grad_v0_norm": float(tv.grad.norm())},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "k_boxilu_apply2d (transposed records)" if boxilu else
                                   "transposed Schwarz (sweep + gather)",
                         "avg_us": round(avg_s * 1e6, 2), "bytes_per_launch": int(bytes_launch)}}
    print(json.dumps(line), flush=True)
    return 0


# The paper's 2D solver study (Section 4.3, Tables 2 and 3): 128 x 128 Neumann, the
# Section 4.2 coefficients and random initial data, the first 10 steps at dt = 1e-4,
# Newton eps_r = 1e-6 (Section 4), 24 subdomains (6 x 4), one-level Schwarz.
STUDY2D = dict(shape=(128, 128), bc="neumann", sub=(6, 4), dt_fixed=1e-4, steps=10, u_mean=0.55, seed=0,
               newton_rtol=1e-6, newton_atol=1e-13, gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30,
               phys=dict(alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001))


STUDY3D = dict(shape=(128, 128, 128), bc="neumann", sub=(8, 8, 8), dt_fixed=1e-4, steps=10, u_mean=0.55, seed=0,
               newton_rtol=1e-6, newton_atol=1e-13, gmres_rtol=1e-8, gmres_atol=1e-14, gmres_restart=30,
               phys=dict(alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001))


def study3d_line(args):
    """Table 3's 3D half (128^3 Neumann, 512 subdomains): the Schwarz variants x overlap
    with ILU(0) (shift 0.02, factored once per step): Newton iterations, GMRES iterations
    per Newton iteration and time for 10 steps at dt = 1e-4."""
    import torch
    from acch_inputs import random_ic
    from paper_2007_04560_amd import Solver
    w = STUDY3D
    u0, v0 = random_ic(w["shape"], w["seed"], u_mean=w["u_mean"])
    base = dict(bc=w["bc"], sub=w["sub"], dt_fixed=w["dt_fixed"], newton_rtol=w["newton_rtol"],
                newton_atol=w["newton_atol"], gmres_rtol=w["gmres_rtol"], gmres_atol=w["gmres_atol"],
                gmres_restart=w["gmres_restart"], ilu_shift=0.02, **w["phys"])
    table3 = {}
    for kind in ("classical", "left", "right"):
        for ov in (0, 1, 2):
            if kind != "classical" and ov == 0:
                continue
            try:
                s = Solver(u0, v0, schwarz=kind, overlap=ov, **base)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                recs = s.step(w["steps"])
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                s.close()
                nit = sum(int(x["newton_its"]) for x in recs)
                git = sum(int(x["gmres_its"]) for x in recs)
                table3[f"{kind} overlap {ov}"] = {"newton": nit, "gmres_per_newton": round(git / max(nit, 1), 2),
                                                  "seconds": round(el, 4)}
            except Exception as e:
                table3[f"{kind} overlap {ov}"] = {"failed": str(e)[:160]}
            print(json.dumps({"study3d": kind, "overlap": ov, **table3[f"{kind} overlap {ov}"]}), file=sys.stderr,
                  flush=True)
    best = table3.get("left overlap 1", {})
    line = {"metric": "time of the first 10 steps (paper's 3D solver study)", "value": best.get("seconds"),
            "unit": "s", "n_gpus": 1, "steps": w["steps"], "warmup": 0,
            "ms_per_step": round(best["seconds"] / w["steps"] * 1e3, 3) if "seconds" in best else None,
            "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "study3d: 3D Neumann 128^3, alpha 4, beta 2, gamma 5e-3, theta 0.1, rho 1e-3, "
                                   "u0 = 0.55 + 0.05 U(-1,1), 10 steps dt = 1e-4, Newton eps_r 1e-6, GMRES(30) "
                                   "xi_r 1e-8, 8x8x8 subdomains, ILU(0) shift 0.02 reuse; value = left-RAS overlap 1",
                       "table3_ilu0_reuse": table3},
            "roofline": None}
    print(json.dumps(line), flush=True)
    return 0


def study_line(args):
    """Table 2 (subdomain solvers under classical AS, overlap 1, with and without the
    factor reuse) and Table 3 (Schwarz variants x overlap, ILU(0) reuse) on one GPU:
    Newton iterations, GMRES iterations per Newton iteration and time for 10 steps."""
    import torch
    from acch_inputs import random_ic
    from paper_2007_04560_amd import Solver
    w = STUDY2D
    u0, v0 = random_ic(w["shape"], w["seed"], u_mean=w["u_mean"])
    base = dict(bc=w["bc"], sub=w["sub"], dt_fixed=w["dt_fixed"], newton_rtol=w["newton_rtol"],
                newton_atol=w["newton_atol"], gmres_rtol=w["gmres_rtol"], gmres_atol=w["gmres_atol"],
                gmres_restart=w["gmres_restart"], **w["phys"])

    def run(**kw):
        k = dict(base)
        k.update(kw)
        try:
            with Solver(u0, v0, **k) as s:
                s.step(1)          # warm-up on a separate instance below; this one is discarded
            s = Solver(u0, v0, **k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs = s.step(w["steps"])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            s.close()
            nit = sum(int(x["newton_its"]) for x in recs)
            git = sum(int(x["gmres_its"]) for x in recs)
            return {"newton": nit, "gmres_per_newton": round(git / max(nit, 1), 2), "seconds": round(el, 4)}
        except Exception as e:   # a configuration that diverges is reported, not fatal
            return {"failed": str(e)[:160]}

    table2 = {}
    for name, kw in [("ILU(0)", dict(subsolver="ilu0")), ("ILU(0) shift 0.02", dict(subsolver="ilu0", ilu_shift=0.02)),
                     ("ILU(1)", dict(subsolver="iluk", fill_level=1)), ("ILU(2)", dict(subsolver="iluk", fill_level=2)),
                     ("LU", dict(subsolver="lu")),
                     ("ILU(0) box pattern", dict(subsolver="iluk_box", fill_level=0)),
                     ("ILU(1) box pattern", dict(subsolver="iluk_box", fill_level=1)),
                     ("ILU(2) box pattern", dict(subsolver="iluk_box", fill_level=2))]:
        table2[name] = {"refactor": run(schwarz="classical", overlap=1, ilu_reuse=False, **kw),
                        "reuse": run(schwarz="classical", overlap=1, ilu_reuse=True, **kw)}
    table3, table3_box = {}, {}
    for kind in ("classical", "left", "right"):
        for ov in (0, 1, 2):
            if kind != "classical" and ov == 0:
                continue   # without overlap both restricted variants are classical AS
            table3[f"{kind} overlap {ov}"] = run(schwarz=kind, overlap=ov, ilu_shift=0.02)
            table3_box[f"{kind} overlap {ov}"] = run(schwarz=kind, overlap=ov, subsolver="iluk_box", fill_level=0)
    best = table3.get("left overlap 1", {})
    line = {"metric": "time of the first 10 steps (paper's 2D solver study)", "value": best.get("seconds"),
            "unit": "s", "n_gpus": 1, "steps": w["steps"], "warmup": 1,
            "ms_per_step": round(best["seconds"] / w["steps"] * 1e3, 3) if "seconds" in best else None,
            "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "study2d: 2D Neumann 128x128, alpha 4, beta 2, gamma 5e-3, theta 0.1, rho 1e-3, "
                                   "u0 = 0.55 + 0.05 U(-1,1), 10 steps dt = 1e-4, Newton eps_r 1e-6, GMRES(30) "
                                   "xi_r 1e-8, 6x4 subdomains; value = left-RAS overlap 1, ILU(0) shift 0.02, reuse",
                       "table2_classical_overlap1": table2, "table3_ilu0_reuse": table3,
                       "table3_box_ilu0_reuse": table3_box},
            "roofline": None}
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline(budget_s: float = 20.0):
    """The FP64 oracle (NumPy residual/Jacobian, SuperLU direct Newton solves, same dt
    controller) on a bounded sample: the same workload's physics, controller and
    initial-data recipe on a 128 x 128 grid, stepped until about budget_s seconds."""
    import numpy as np
    from acch_inputs import random_ic
    from oracle import controller, newton
    from oracle.params import Problem

    w = WORKLOAD
    shape = (128, 128)
    u0, v0 = random_ic(shape, w["seed"])
    run = controller.Run(Problem(bc=w["bc"]), u0, v0, adaptive=True, dt_min=w["dt_min"], dt_max=w["dt_max"],
                         eta=w["eta0"], newton=newton.NewtonOptions(rtol=w["newton_rtol"], atol=w["newton_atol"]))
    t0 = time.perf_counter()
    its = 0
    steps = 0
    while time.perf_counter() - t0 < budget_s and steps < 50:
        its += run.step().newton_its
        steps += 1
    el = time.perf_counter() - t0
    dof = 2 * u0.size
    return {"value": dof * its / el, "unit": "dof*Newton/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle on the same workload at 128x128 (2D periodic, same parameters, controller and "
                      f"seeded initial data): {steps} time steps, {its} Newton iterations in {el:.1f} s; "
                      f"SuperLU and NumPy single-threaded, host has {os.cpu_count()} logical CPUs"}


def _rel_l2(a, b):
    import numpy as np
    return float(np.sqrt(np.sum((a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2) / np.sum(b[0] ** 2 + b[1] ** 2)))


def forms_summary(args, w, fp64_run):
    """The chosen forms next to the plain FP64 run: (1) mixed precision on the same
    workload (time, speedup, final-field difference to the FP64 run), (2) the batched
    workload (batched FP64 and mixed against the instances solved one by one, and the same
    batch with box-pattern ILU(0)), and the
    error of the GPU's FP64 and mixed results against the FP64 oracle on the 64 x 64
    periodic workload (10 steps at dt = 1e-3, both sides at Newton tolerance 1e-8)."""
    import numpy as np
    from acch_inputs import random_ic
    from oracle import controller, newton, scheme
    from oracle.params import Problem
    from paper_2007_04560_amd import Solver
    out = {}
    wm = dict(w)
    wm["precision"] = "mixed"
    rm = run_gpu(args.steps, 0, timing=False, w=wm)
    nm = sum(int(x["newton_its"]) for x in rm["recs"])
    out["mixed"] = {"seconds": round(rm["elapsed"], 4), "fp64_seconds": round(fp64_run["elapsed"], 4),
                    "value": round(2 * rm["ncell"] * nm / rm["elapsed"], 1),
                    "speedup_vs_fp64": round(fp64_run["elapsed"] / rm["elapsed"], 3),
                    "newton_its": nm, "gmres_its": sum(int(x["gmres_its"]) for x in rm["recs"]),
                    "final_fields_rel_l2_vs_fp64": _rel_l2(rm["fields"], fp64_run["fields"]),
                    "mass_drift_rel": abs(rm["M1"] - rm["M0"]) / rm["M0"]}
    b = run_batch(BATCH["steps"], 1, with_sequential=True)
    out["batched"] = {"workload": BATCH["text"], "batched_fp64_s": round(b["fp64"]["elapsed"], 4),
                      "batched_mixed_s": round(b["mixed"]["elapsed"], 4),
                      "sequential_fp64_s": round(b["sequential"]["elapsed"], 4),
                      "speedup_batched_vs_sequential": round(b["sequential"]["elapsed"] / b["fp64"]["elapsed"], 3),
                      "speedup_mixed_batched_vs_sequential": round(b["sequential"]["elapsed"] / b["mixed"]["elapsed"],
                                                                   3),
                      "value_fp64": round(b["fp64"]["dof_newton"] / b["fp64"]["elapsed"], 1),
                      "mixed_vs_fp64_final_fields_max_rel_l2": b["mixed_vs_fp64_max_rel_l2"]}
    # the same batch with ILU(0) on the box pattern (its own autotuned widths)
    bb = run_batch(BATCH_BOX["steps"], 1, with_sequential=False, B=BATCH_BOX)
    out["batched_box"] = {"workload": BATCH_BOX["text"], "box": bb["box"],
                          "batched_fp64_s": round(bb["fp64"]["elapsed"], 4),
                          "batched_mixed_s": round(bb["mixed"]["elapsed"], 4),
                          "gmres_per_newton_fp64": round(bb["fp64"]["gmres"] / max(1, bb["fp64"]["newton"]), 2),
                          "value_fp64": round(bb["fp64"]["dof_newton"] / bb["fp64"]["elapsed"], 1),
                          "value_mixed": round(bb["mixed"]["dof_newton"] / bb["mixed"]["elapsed"], 1),
                          "time_vs_stencil_batch_fp64": round(bb["fp64"]["elapsed"] / b["fp64"]["elapsed"], 3),
                          "time_vs_stencil_batch_mixed": round(bb["mixed"]["elapsed"] / b["mixed"]["elapsed"], 3),
                          "mixed_vs_fp64_final_fields_max_rel_l2": bb["mixed_vs_fp64_max_rel_l2"]}
    shape = (64, 64)
    u0, v0 = random_ic(shape, 0)
    P = Problem(bc="periodic")
    run = controller.Run(P, u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-8, atol=1e-13))
    ref = []
    for _ in range(10):
        run.step()
        ref.append((run.u.copy(), run.v.copy()))
    M0 = scheme.mass(u0, P)
    par = {}
    for prec in ("fp64", "mixed"):
        with Solver(u0, v0, bc="periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3, precision=prec) as s:
            errs, drift = [], 0.0
            for k in range(10):
                info = s.step(1)[0]
                errs.append(_rel_l2(s.fields(), ref[k]))
                drift = max(drift, abs(info["mass"] - M0) / M0)
        par[prec] = {"max_step_rel_l2_vs_oracle": max(errs), "mass_drift_rel": drift}
    out["error_vs_oracle_64x64"] = par
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="default: the workload's step count")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="default workload: skip the mixed-precision, batched and 64x64 oracle comparisons")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel HIP-event timers")
    ap.add_argument("--workload", default="periodic512",
                    choices=sorted(WORKLOADS) + ["batch96", "batch96_box", "adjoint512", "adjoint3d128",
                                                 "adjoint512_box32", "study2d", "study3d"])
    ap.add_argument("--no-sequential", action="store_true", help="batch96: skip the one-by-one FP64 comparison")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 64 MiB FP64 tensor 3 times (reference for the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--sub", default=None, help="subdomains per axis, x,y[,z] (default: the workload's)")
    ap.add_argument("--overlap", type=int, default=None, help="subdomain overlap (default: the workload's)")
    ap.add_argument("--subsolver", default=None, choices=["ilu0", "ilu1", "ilu2", "lu", "ilu0box", "ilu1box", "ilu2box"],
                    help="subdomain solver (Table 2; default: the workload's); the *box solvers take the width-2 "
                         "box of cell couplings as the level-0 pattern")
    ap.add_argument("--ilu-shift", type=float, default=None, help="diagonal shift of the subdomain matrices")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copied 64 MiB FP64 three times"}), flush=True)
        return 0
    if args.workload in ("adjoint512", "adjoint3d128", "adjoint512_box32"):
        if args.gpus != 1:
            print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus})", file=sys.stderr)
            return 2
        if args.steps is None:
            args.steps = 20
        return adjoint_line(args, WORKLOADS[{"adjoint512": "periodic512", "adjoint3d128": "neumann128_3d",
                                             "adjoint512_box32": "periodic512_box32"}[args.workload]])
    if args.workload in ("study2d", "study3d"):
        if args.gpus != 1:
            print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus})", file=sys.stderr)
            return 2
        return study_line(args) if args.workload == "study2d" else study3d_line(args)
    if args.workload in ("batch96", "batch96_box"):
        if args.gpus != 1:
            print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus})", file=sys.stderr)
            return 2
        B = BATCH if args.workload == "batch96" else BATCH_BOX
        if args.steps is None:
            args.steps = B["steps"]
        return batch_line(args, B)
    w = dict(WORKLOADS[args.workload])
    if args.precision:
        w["precision"] = args.precision
    if args.sub or args.overlap is not None:
        w["sub"] = tuple(int(x) for x in args.sub.split(",")) if args.sub else w["sub"]
        w["overlap"] = w["overlap"] if args.overlap is None else args.overlap
        w["text"] += f" [subdomains {'x'.join(map(str, w['sub']))}, overlap {w['overlap']}]"
    if args.subsolver or args.ilu_shift is not None:
        if args.subsolver:
            w["subsolver"] = {"ilu1": "iluk", "ilu2": "iluk", "ilu0box": "iluk_box", "ilu1box": "iluk_box",
                              "ilu2box": "iluk_box"}.get(args.subsolver, args.subsolver)
            w["fill_level"] = {"ilu1": 1, "ilu2": 2, "ilu1box": 1, "ilu2box": 2}.get(args.subsolver, 0)
            if args.subsolver == "lu" and args.ilu_shift is None:
                w["ilu_shift"] = 0.0
        if args.ilu_shift is not None:
            w["ilu_shift"] = args.ilu_shift
        w["text"] += f" [subdomain solver {args.subsolver or w.get('subsolver', 'ilu0')}, shift {w['ilu_shift']}]"
    if args.steps is None:
        args.steps = w["steps"]
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU runs are not implemented",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    r = run_gpu(args.steps, args.warmup, timing=not args.no_timing, w=w)
    recs = r["recs"]
    newton_its = sum(int(x["newton_its"]) for x in recs)
    gmres_its = sum(int(x["gmres_its"]) for x in recs)
    dof = 2 * r["ncell"]
    value = dof * newton_its / r["elapsed"]
    info = r["info"]
    if len(w["shape"]) == 3:   # boxes of (n/p + 2 overlap)^3 cells, 40 slots per cell
        box = 1.0
        for n_a, p_a in zip(reversed(w["shape"]), w["sub"]):
            box *= n_a / p_a + 2 * w["overlap"]
    else:
        box = info["box_w"] * info["box_h"]
    owned = r["ncell"] / info["nsub"]
    nslot = 40 if len(w["shape"]) == 3 else 24
    roofline = None
    stats = r["stats"]
    boxilu = w.get("subsolver") == "iluk_box" and w.get("fill_level", 0) == 0
    band = w.get("subsolver", "ilu0") != "ilu0" and not boxilu
    if stats and stats["ras"][1] > 0:
        ras_ms, ras_n = stats["ras"]
        avg_s = ras_ms / ras_n * 1e-3
        sp = 4 if w["precision"] == "mixed" else 8
        if band:   # the band solve reads every stored diagonal of each box once
            bw, bh = info["box_w"], info["box_h"]
            nrow = 2 * bw * bh
            nd = 8 * bw + 1 + (10 if w.get("subsolver") == "iluk_box" else 0)   # stored diagonals
            bytes_launch = info["nsub"] * (nrow * nd * sp + 16 * bw * bh) + 16 * r["ncell"]
        elif boxilu:   # both records of every box cell, its y written and read back, r read; z written
            bytes_launch = info["nsub"] * info["box_w"] * info["box_h"] * (108 * sp + 16) + 16 * r["ncell"]
        else:
            bytes_launch = ras_bytes_per_cell(box, owned, nslot=nslot, sp=sp) * r["ncell"]
        achieved = bytes_launch / avg_s / 1e9
        same_kernel = w.get("subsolver", "ilu0") == WORKLOADS[w["name"]].get("subsolver", "ilu0")
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(w["name"])
                    if sp == 8 and w["sub"] == WORKLOADS[w["name"]]["sub"] and same_kernel else None,
                    "kernel": "k_band_solve2d" if band else "k_boxilu_apply2d" if boxilu else
                              ("k_ras_apply3d_win" if len(w["shape"]) == 3 else "k_ras_apply2d"),
                    "avg_us": round(avg_s * 1e6, 2), "timed_launches": ras_n,
                    "timing": "HIP events on the library stream around 1 in 16 Schwarz launches of the timed region",
                    "bytes_per_launch": int(bytes_launch)}
    line = {
        "metric": "dof*Newton-steps/s at 1e-8 tol",
        "value": round(value, 1),
        "unit": "dof*Newton/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["elapsed"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["precision"] == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": w["text"] if w["precision"] == WORKLOADS[w["name"]]["precision"]
                   else w["text"] + f" (precision {w['precision']})",
                   "cells": r["ncell"], "dof": dof, "newton_its": newton_its, "gmres_its": gmres_its,
                   "gmres_per_newton": round(gmres_its / max(1, newton_its), 2),
                   "t_final": recs[-1]["t"] if recs else 0.0,
                   "dt_last": recs[-1]["dt"] if recs else 0.0,
                   "energy_first_last": [r["E0"], r["E1"]],
                   "mass_drift_rel": abs(r["M1"] - r["M0"]) / r["M0"],
                   "dt_range": [min(x["dt"] for x in recs), max(x["dt"] for x in recs)] if recs else None,
                   "energy_max_rel_increase": max([0.0] + [(b["energy"] - a["energy"]) / abs(a["energy"])
                                                          for a, b in zip(recs, recs[1:])]),
                   "dt_growth_orders": round(math.log10(max(x["dt"] for x in recs) / min(x["dt"] for x in recs)), 3)
                   if recs else None,
                   "retries": sum(int(x["retries"]) for x in recs),
                   "launches": r["launches"], "host_syncs": r["syncs"],
                   "kernel_ms": {k: round(v[0], 3) for k, v in stats.items() if v[1]}},
        "roofline": roofline,
    }
    if not band:   # the whole run against the HBM roofline (ILU(0) subdomain solver)
        omega = box / owned
        # box-pattern ILU(0): 2 x 52 record slots per box cell, and the box vector written and
        # read back by the sweeps (4 more values)
        slots = dict(fac_slots=104, ras_slots=108) if boxilu else {}
        tot = step_bytes_per_cell(newton_its, gmres_its, len(recs), nslot, omega, 4 if w["precision"] == "mixed" else 8,
                                  w["gmres_restart"], **slots) * r["ncell"]
        line["config"]["whole_run_roofline"] = {
            "algorithmic_bytes": int(tot), "achieved_GBps": round(tot / r["elapsed"] / 1e9, 1),
            "frac": round(tot / r["elapsed"] / 1e9 / HBM_PEAK_GBS, 4),
            "model": "per Newton iteration: 2 residuals + Jacobian + factorisation/step + per GMRES iteration "
                     "(SpMV + left-RAS + CGS Arnoldi) + update, mean GMRES count per Newton iteration"}
    if w["adaptive"] and recs:
        # the same interval at the smallest step would take t_final / dt_min steps
        fixed = recs[-1]["t"] / w["dt_min"]
        line["config"]["fixed_dt_min_steps"] = round(fixed)
        line["config"]["adaptive_step_saving"] = round(1.0 - len(recs) / fixed, 4)
    if not args.no_forms and args.workload == "periodic512" and w["precision"] == "fp64":
        line["config"]["forms"] = forms_summary(args, w, r)
    if not args.no_forms and args.workload == "neumann1024_lu" and w["precision"] == "mixed":
        # the same run in plain FP64: time-to-solution and the difference of the results
        wd = dict(w)
        wd["precision"] = "fp64"
        rd = run_gpu(args.steps, 0, timing=False, w=wd)
        line["config"]["fp64"] = {"seconds": round(rd["elapsed"], 4), "mixed_seconds": round(r["elapsed"], 4),
                                  "mixed_speedup": round(rd["elapsed"] / r["elapsed"], 3),
                                  "final_fields_rel_l2_mixed_vs_fp64": _rel_l2(r["fields"], rd["fields"]),
                                  "newton_its": sum(int(x["newton_its"]) for x in rd["recs"]),
                                  "gmres_its": sum(int(x["gmres_its"]) for x in rd["recs"])}
    if not args.no_cpu_baseline and args.workload == "periodic512":
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
