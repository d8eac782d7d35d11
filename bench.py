#!/usr/bin/env python3
"""Benchmark of the GSIS / DVM hot path on one MI355X.

Workload: 2D radiative lid-driven, heated cavity with a concentric square obstacle on ~20k unstructured
triangles (Delaunay of seeded jittered points), 32x32 Gauss-Hermite reduced velocity grid, 32 gray
ordinates (4 x 8, z-mirrored), Kn = 0.1, optical thickness 1, FP32 distributions with FP64 moments and
macro solve.  Synthetic inputs, no data files.

One step = one GSIS outer iteration: kinetic step (gradients, residual with upwind fluxes and the
relaxation source, Jacobi sweeps), moments, boundary flux moments, synthetic-equation solve,
synchronisation, moments and residual.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# measured HBM traffic of the dominant kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated on a copy)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_cavity20k_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2601_03935_amd", "csrc", "kinetic.hip")


def measured_traffic():
    """HBM bytes per launch of the sweep kernel from the committed counter summary, or None when the kernel
    source has changed since the counters were taken."""
    import hashlib

    try:
        t = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    return t["bytes_per_launch"] if t.get("kernel_source_sha256") == sha else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--Kn", type=float, default=0.1)
    ap.add_argument("--tau", type=float, default=1.0, help="optical thickness (= 1 / Kn_photon)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="bound of the oracle baseline run")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-outer", type=int, default=600)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibration of the HBM byte counters)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if a.copy_probe:
        n = 1 << 28  # 1 GiB of float32
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": 4 * n, "copies": 3}), flush=True)
        return

    from paper_2601_03935_amd.gsis import KERNEL_KINDS, Solver, oracle_opts
    from workloads import case_cavity

    case = case_cavity(Kn=a.Kn, tau_opt=a.tau)
    nc, nv, no = case.mesh.nc, case.vgrid.nv, case.ords.no
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    s = Solver(case, device=0, stream=stream.cuda_stream, precision=a.precision)
    # warm-up: two conventional iterations from the equilibrium start, then GSIS iterations
    s.iterate(gsis=False, n=2)
    for _ in range(a.warmup):
        s.iterate(gsis=True)
    torch.cuda.synchronize()
    s.set_profiling(True)
    s.counters()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    inner = []
    eps = []
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(a.steps):
        e, it = s.iterate(gsis=True)
        eps.append(e)
        inner.append(it)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    stats = s.kernel_stats()
    s.set_profiling(False)
    step_ms = ms / a.steps
    value = nc * nv * a.steps / (ms * 1e-3)
    kernels = {}
    for k in KERNEL_KINDS:
        tms, n, by = stats[k]
        if n == 0:
            continue
        kernels[k] = dict(ms_per_step=tms / a.steps, launches_per_step=n / a.steps,
                          gbs=(by / (tms * 1e-3) / 1e9) if by > 0 and tms > 0 else None)
    dom = max((k for k in kernels if stats[k][2] > 0), key=lambda k: stats[k][0])
    tms, n, by = stats[dom]
    achieved = by / n / (tms / n * 1e-3) / 1e9
    kin_ms = sum(stats[k][0] for k in ("grad", "residual", "sweep", "rad", "boundary")) / a.steps
    kin_bytes_ideal = nc * (2 * 4 * nv + 2 * no) * (4 if a.precision == "fp32" else 8)
    out = {
        "metric": "DVM cell·velocity updates/s + HBM GB/s; wall time to 1e-6 residual",
        "value": value,
        "unit": "cell-velocity updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "2D radiative lid-driven heated cavity with square obstacle",
            "cells": nc, "velocities": nv, "distributions_per_velocity": 4, "ordinates": no,
            "Kn_gas": a.Kn, "optical_thickness": a.tau, "scheme": "GSIS",
            "kinetic_sweeps": s.opts.kin_sweeps, "max_inner": s.opts.max_inner,
            "storage": a.precision + " distributions, fp64 moments and macro solve",
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if dom == "sweep" and a.precision == "fp32" else None,
                     "algorithmic_bytes_per_launch": by / n},
        "kinetic_step": {"ms": kin_ms, "ideal_bytes": kin_bytes_ideal,
                         "ideal_gbs": kin_bytes_ideal / (kin_ms * 1e-3) / 1e9},
        "kernels": kernels,
        "inner_iterations_per_step": float(np.mean(inner)),
        "eps_last": eps[-1],
    }
    if not a.no_time_to_tol:
        # wall time to the residual tolerance from the equilibrium start (10 conventional iterations first),
        # the configured precision and plain FP64 GSIS on the same GPU
        out["time_to_tol"] = {}
        for prec in dict.fromkeys((a.precision, "fp64")):
            s2 = Solver(case, device=0, stream=stream.cuda_stream, precision=prec, tol=a.tol, max_outer=a.max_outer)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, rep, hist = s2.solve()
            torch.cuda.synchronize()
            out["time_to_tol"][prec] = {"tol": a.tol, "seconds": time.perf_counter() - t0, "iterations": int(rep.iters),
                                        "converged": bool(rc == 0), "eps_final": float(rep.eps_final),
                                        "t_kinetic_s": rep.t_kinetic_s, "t_macro_s": rep.t_macro_s}
            s2.close()
    if not a.no_cpu_baseline:
        from oracle import Oracle

        o = Oracle(case, **oracle_opts(s.opts))
        o.iterate(gsis=False)
        o.iterate(gsis=False)
        t0 = time.perf_counter()
        k = 0
        while True:
            o.iterate(gsis=True)
            k += 1
            if time.perf_counter() - t0 > a.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": nc * nv * k / dt, "unit": "cell-velocity updates/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())), "kind": "oracle",
                               "sample": f"{k} FP64 GSIS iterations of the same workload ({dt:.1f} s)"}
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
