#!/usr/bin/env python3
"""Benchmark of the GSIS / DVM hot path on one MI355X.

Default workload: the 3D radiative Mach-10 blunt capsule (spherical-cap forebody of radius 1, 33 degree
cone) on 213,976 tetrahedra with a 24^3 velocity grid (three distributions per node) and 96 gray
ordinates, Kn 0.01, optical thickness 1, sigma_R 0.045: FP32 distributions (35.5 GB per copy) with FP64
moments, synthetic-equation solve and residual.  Synthetic inputs, no data files.

One step = one GSIS outer iteration: per-cell prologue, kinetic step (limited gradients, wall densities,
residual with upwind fluxes and the relaxation source, Jacobi sweeps, radiation), moments, boundary flux
moments, synthetic-equation solve, synchronisation, moments and residual.  Prints one JSON line.  Other
workloads (--workload): the 2D cavity, the Ma 5 cylinder, the normal shock, one velocity shard of the
capsule.
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
KERNEL_SOURCE = os.path.join(ROOT, "paper_2601_03935_amd", "csrc", "kinetic.hip")


def kernel_source_sha256(path=KERNEL_SOURCE, name="k_sweep_v"):
    """Hash of one kernel's definition text (from its template line to the closing brace at column 0)."""
    import hashlib

    src = open(path).read()
    i = src.index(f"void {name}(")
    i = src.rindex("template <", 0, i)
    j = src.index("\n}\n", i) + 3
    return hashlib.sha256(src[i:j].encode()).hexdigest()


KERNEL_NAMES = {"sweep": "k_sweep_v", "residual": "k_residual_v", "grad": "k_grad_v"}


def measured_traffic(kind="sweep", workload="capsule"):
    """HBM bytes per launch of a DVM kernel from the committed counter summary of the workload, or None when
    there is none or the kernel definition has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{KERNEL_NAMES.get(kind, kind)}_{workload}_traffic.json")
    try:
        t = json.load(open(path))
        sha = kernel_source_sha256(name=KERNEL_NAMES[kind])
    except (OSError, ValueError, KeyError):
        return None
    return t["bytes_per_launch"] if t.get("kernel_source_sha256") == sha else None


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed GSIS iterations (capsule 10, cavity 20)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed iterations before (capsule 3: two conventional and one GSIS; cavity 5)")
    ap.add_argument("--Kn", type=float, default=0.1)
    ap.add_argument("--tau", type=float, default=1.0, help="optical thickness (= 1 / Kn_photon)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="bound of the oracle baseline run")
    ap.add_argument("--no-oracle-timings", action="store_true",
                    help="capsule: skip the oracle timings of the 1D, cavity and cylinder configurations")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-outer", type=int, default=600)
    ap.add_argument("--kin-relax", default="jacobi", choices=["jacobi", "sgs"],
                    help="capsule, cylinder: kinetic point relaxation (Jacobi sweeps or colored symmetric Gauss-Seidel)")
    ap.add_argument("--kin-sweeps", type=int, default=None, help="capsule, cylinder: sweeps per kinetic step (8 Jacobi, 1 SGS)")
    ap.add_argument("--max-inner", type=int, default=100,
                    help="capsule: inner iterations of each synthetic solve (tolerance 1e-7 or this many)")
    ap.add_argument("--workload", default="capsule",
                    choices=["capsule", "cavity", "capsule-shard", "capsule-ma5", "cylinder", "shock", "c5-gen",
                             "c5-eval"],
                    help="capsule: GSIS iterations of the 3D Ma 10 capsule at full size (default); cavity: GSIS "
                         "iterations of the 2D radiative cavity; capsule-shard: kinetic steps "
                         "of the 3D capsule on one eighth of its velocity space (one GPU's share); capsule-ma5: "
                         "the full-size capsule mesh converged at Mach 5 by Mach continuation (use --tol 1e-5); "
                         "cylinder: the "
                         "Ma 5 cylinder solved from the free stream to the tolerance; shock: iterations to 2e-6 of "
                         "the Ma 5 normal shock, GSIS and conventional")
    ap.add_argument("--cyl-Kn", type=float, default=0.01, help="Kn of the cylinder workload")
    ap.add_argument("--max-stage", type=int, default=400, help="iteration limit per Mach stage (cylinder, capsule-ma5)")
    ap.add_argument("--no-warmstart", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--ws-cases", type=int, default=24, help="training cases of the warm-start network")
    ap.add_argument("--no-fp64", action="store_true", help="capsule: skip the FP64 leg")
    ap.add_argument("--c5-cases", type=int, default=256, help="c5: cases of the warm-start data set")
    ap.add_argument("--c5-train", type=int, default=224, help="c5: the first this many cases train, the rest test")
    ap.add_argument("--c5-shard", default="0/1", help="c5-gen: k/n solves cases k, k + n, ...")
    ap.add_argument("--c5-dir", default="c5_cases", help="c5: directory of the per-case solutions")
    ap.add_argument("--c5-seconds", type=float, default=1000.0, help="c5-gen: stop starting cases after this")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibration of the HBM byte counters)")
    a = ap.parse_args(argv)
    if a.steps is None:
        a.steps = 10 if a.workload == "capsule" else 20
    if a.warmup is None:
        a.warmup = 3 if a.workload == "capsule" else 5
    return a


def capsule_case(nvx=24, mesh_kw=None):
    """The 3D capsule workload: Ma 10, Kn 0.01, optical thickness 1, sigma_R 0.045, 96 ordinates (8
    Gauss-Legendre polar x 12 azimuths), nvx^3 velocities on the box [-15, u_inf + 9] x [-15, 15]^2."""
    from workloads import case_capsule

    return case_capsule(Kn=0.01, tau_opt=1.0, Ma=10.0, nvx=nvx, n_theta=8, n_phi=12, sigma_R=0.045,
                        mesh_kw=mesh_kw or dict(n_s=46, n_phi=28, n_r=28), vgrid="box")


def capsule_case_ma(Ma, nvx=24):
    """The capsule workload at another far-field Mach number (box velocity grid sized for it)."""
    from workloads import case_capsule

    return case_capsule(Kn=0.01, tau_opt=1.0, Ma=Ma, nvx=nvx, n_theta=8, n_phi=12, sigma_R=0.045,
                        mesh_kw=dict(n_s=46, n_phi=28, n_r=28), vgrid="box")


# Limiter constant of the capsule runs: the limiter acts through (K h)^1.5 and the tetrahedra of the capsule
# mesh are ~10x larger than the cavity's triangles; K = 1 keeps (K h)^1.5 near the cavity's value, where the
# default K = 10 leaves the reconstruction unlimited and the second-order iteration unstable on tetrahedra.
CAPSULE_K = 1.0
# longest run of timed iterations from one start (the start-up transient on the 24^3 box grid stays admissible
# for ~15 iterations from the start from rest)
CAPSULE_SEGMENT = 10


def _start_capsule(s, case):
    """Gas at rest (rho = T = 1) inside, the Ma 10 free stream at the far field: the impulsive start from the
    uniform free stream empties the wake within two iterations on this velocity grid, the start from rest
    keeps every cell a gas state for the ~15 iterations the benchmark runs."""
    import numpy as np

    n = case.mesh.nc
    s.init_equilibrium(np.ones(n), np.zeros((n, 3)), np.ones(n))


def kernel_table(stats, steps):
    out = {}
    for k, (tms, n, by) in stats.items():
        if n:
            out[k] = dict(ms_per_step=tms / steps, launches_per_step=n / steps,
                          alg_gbs=(by / (tms * 1e-3) / 1e9) if by > 0 and tms > 0 else None)
    return out


def bench_capsule(a):
    """GSIS iterations of the 3D capsule at full size (see capsule_case): two conventional and a.warmup - 2 GSIS
    warm-up iterations from the start from rest, then timed GSIS iterations run back to back (one host wait),
    with HIP events around every kernel kind on the library's stream.  The start-up transient of the 24^3 box
    grid stays admissible for ~15 iterations (the cold wake is not resolved by it), so the timed iterations
    run in segments of at most CAPSULE_SEGMENT, each from a fresh start and warm-up that are not timed."""
    import numpy as np
    import torch

    from paper_2601_03935_amd.gsis import Solver

    case = capsule_case()
    nc, nv, no = case.mesh.nc, case.vgrid.nv, case.ords.no
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ksw = a.kin_sweeps if a.kin_sweeps is not None else (8 if a.kin_relax == "jacobi" else 1)
    s = Solver(case, device=0, stream=stream.cuda_stream, precision=a.precision, limiter_K=CAPSULE_K,
               max_inner=a.max_inner, sweep=a.kin_relax, kin_sweeps=ksw)
    free, total = torch.cuda.mem_get_info()
    mem_gb = (total - free) / 1e9
    ms, left, segments = 0.0, a.steps, 0
    stats = None
    while left > 0:
        seg = min(left, CAPSULE_SEGMENT)
        _start_capsule(s, case)
        s.iterate(gsis=False, n=2)
        if a.warmup > 2:
            s.iterate(gsis=True, n=a.warmup - 2)
        torch.cuda.synchronize()
        s.set_profiling(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        eps, inner = s.iterate(gsis=True, n=seg)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms += ev0.elapsed_time(ev1)
        st = s.kernel_stats()
        stats = st if stats is None else {k: tuple(x + y for x, y in zip(stats[k], st[k])) for k in st}
        s.set_profiling(False)
        left -= seg
        segments += 1
    F = s.fields()
    s.close()
    del s
    torch.cuda.empty_cache()
    kernels = kernel_table(stats, a.steps)
    es = 4 if a.precision == "fp32" else 8
    unit_bytes = 2 * 3 * es  # per cell-velocity per kinetic step: read and write f once, three distributions
    units = nc * nv
    # dominant DVM kernel by time; its launches each cover every cell and velocity
    dom = max(("grad", "residual", "sweep"), key=lambda k: stats[k][0])
    tms, n, _ = stats[dom]
    sgs = a.kin_relax == "sgs"
    if dom == "sweep" and sgs:
        # a colored sweep launch covers one colour; a forward or backward pass covers every cell once
        passes = 2 * ksw * a.steps
        achieved = unit_bytes * units / (tms / passes * 1e-3) / 1e9
    else:
        achieved = unit_bytes * units / (tms / n * 1e-3) / 1e9
    kin_ms = sum(stats[k][0] for k in ("grad", "residual", "sweep", "rad", "boundary")) / a.steps
    kin_gbs = unit_bytes * units / (kin_ms * 1e-3) / 1e9
    out = {
        "metric": "DVM cell·velocity updates/s + HBM GB/s; wall time to 1e-6 residual",
        "value": units * a.steps / (ms * 1e-3), "unit": "cell-velocity updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if a.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "3D Ma 10 blunt capsule (spherical cap radius 1 + 33 deg cone), full size",
                   "cells": nc, "cell_type": "tetrahedra", "velocities": nv, "velocity_grid": "24^3 uniform box",
                   "distributions_per_velocity": 3, "ordinates": no, "Kn_gas": 0.01, "Mach": 10.0,
                   "optical_thickness": 1.0, "sigma_R": 0.045, "scheme": "GSIS",
                   "kinetic_relaxation": (f"{ksw} colored symmetric Gauss-Seidel sweep{'s' if ksw > 1 else ''}" if sgs
                                          else f"{ksw} Jacobi sweeps"),
                   "max_inner": a.max_inner, "limiter_K": CAPSULE_K, "start": "gas at rest, Ma 10 far field",
                   "storage": a.precision + " distributions, fp64 moments, synthetic solve and residual",
                   "device_memory_gb": mem_gb},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if (sgs and dom == "sweep") else measured_traffic(dom),
                     "algorithmic_bytes_per_launch": unit_bytes * units,
                     "accounting": "24 B per cell-velocity (f read and written once, 3 distributions, FP32) x "
                                   "cells x velocities per launch / mean launch time"
                                   + (" (per forward or backward pass of the colored sweep)" if sgs and dom == "sweep"
                                      else "")},
        "kinetic_step": {"ms": kin_ms, "algorithmic_bytes": unit_bytes * units, "gbs": kin_gbs,
                         "frac": kin_gbs / HBM_PEAK_GBS},
        "kernels": kernels,
        "inner_iterations_last_step": int(inner), "eps_last": eps, "timed_segments": segments,
        "fields_finite": bool(np.isfinite(F).all()),
    }
    return out



def unit_roofline(unit_bytes, units, stat, traffic, ndist, es):
    """HBM roofline of the sweep kernel by the per-cell-velocity accounting: every reduced distribution read and
    written once per kinetic step (unit_bytes per cell-velocity) x the cell-velocities one launch covers, over
    the mean launch time.  The kernel's own byte rate (its operand arrays, each once) is reported beside it."""
    tms, n, by = stat
    mean_s = tms / n * 1e-3
    achieved = unit_bytes * units / mean_s / 1e9
    return {"bound": "hbm", "kernel": "sweep", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": unit_bytes * units,
            "accounting": f"{unit_bytes} B per cell-velocity (f read and written once, {ndist} distributions, "
                          f"{'FP32' if es == 4 else 'FP64'}) x cells x velocities per launch / mean launch time",
            "kernel_operand_gbs": by / n / mean_s / 1e9}

def bench_capsule_converge(a):
    """The full-size capsule mesh and 24^3 box velocities (box sized for Mach 5) converged on one GPU, FP32:
    from a Mach 2 uniform start, Mach continuation 2 -> 3 -> 4 -> 5 of the far field (40 conventional and 60
    first-order iterations in the first stage, 20 first-order after each jump; stages to epsilon < 1e-4,
    the last to --tol), limiter K = 1.  Wall time, iterations per stage and the per-iteration cost."""
    import numpy as np
    import torch

    from paper_2601_03935_amd.gsis import Solver

    case = capsule_case_ma(5.0)
    nc, nv = case.mesh.nc, case.vgrid.nv
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    s = Solver(case, device=0, stream=stream.cuda_stream, precision=a.precision, limiter_K=CAPSULE_K,
               max_inner=a.max_inner)
    g = np.sqrt(case.gas.gamma)
    u0 = np.zeros((nc, 3))
    u0[:, 0] = 2.0 * g
    s.init_equilibrium(np.ones(nc), u0, np.ones(nc))
    states = [(1.0, 1.0, (Ma * g, 0.0, 0.0)) for Ma in (2.0, 3.0, 4.0, 5.0)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, hist, ok = s.solve_continuation(1, states, stage_tol=1e-4, tol=a.tol, max_stage=a.max_stage,
                                         first_order_jump=20)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    F = s.fields()
    s.close()
    iters = int(sum(its))
    return {
        "metric": "wall time to the residual tolerance from a Mach 2 start (3D Ma 5 capsule, Mach continuation)",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": iters, "warmup": 0, "ms_per_step": 1e3 * sec / iters,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "3D Ma 5 blunt capsule (spherical cap radius 1 + 33 deg cone), full-size mesh",
                   "cells": nc, "cell_type": "tetrahedra", "velocities": nv, "velocity_grid": "24^3 uniform box",
                   "distributions_per_velocity": 3, "ordinates": case.ords.no, "Kn_gas": 0.01, "Mach": 5.0,
                   "optical_thickness": 1.0, "sigma_R": 0.045, "tol": a.tol, "mach_steps": [2, 3, 4, 5],
                   "limiter_K": CAPSULE_K, "kinetic_relaxation": "8 Jacobi sweeps", "max_inner": a.max_inner},
        "converged": ok, "iterations_per_stage": its, "eps_final": float(hist[-1]),
        "eps_tail": [float(x) for x in hist[-5:]],
        "cell_velocity_updates_per_s": nc * nv * iters / sec,
        "fields_finite": bool(np.isfinite(F).all()), "min_density": float(F[:, 0].min()),
    }


def bench_capsule_fp64(a):
    """FP64 distributions on the full capsule (same mesh, velocities, physics and start): with one symmetric
    Gauss-Seidel sweep in place and the gradients recomputed inside the residual the state fits in 152 GB
    (f and r, 71 GB each; eight Jacobi sweeps with stored gradients would need ~500 GB).  Two conventional
    and one GSIS warm-up iteration, then four timed GSIS iterations (inside the ten iterations this
    relaxation keeps the start-up admissible)."""
    import torch

    from paper_2601_03935_amd.gsis import GsisError, Solver

    case = capsule_case()
    nc, nv = case.mesh.nc, case.vgrid.nv
    stream = torch.cuda.current_stream()
    s = Solver(case, device=0, stream=stream.cuda_stream, precision="fp64", limiter_K=CAPSULE_K, sweep="sgs",
               kin_sweeps=1, kin_fused=1)
    free, total = torch.cuda.mem_get_info()
    _start_capsule(s, case)
    s.iterate(gsis=False, n=2)
    s.iterate(gsis=True, n=1)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = 4
    ev0.record(stream)
    try:
        s.iterate(gsis=True, n=steps)
    except GsisError as ex:
        s.close()
        return {"velocities": nv, "cells": nc, "failed": str(ex)}
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s.close()
    torch.cuda.empty_cache()
    return {"cells": nc, "velocities": nv, "relaxation": "1 symmetric Gauss-Seidel sweep",
            "gradients": "recomputed in the residual", "device_memory_gb": (total - free) / 1e9, "steps": steps,
            "ms_per_step": ms / steps, "cell_velocity_updates_per_s": nc * nv * steps / (ms * 1e-3)}


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def capsule_cpu_baseline(a):
    """The FP64 oracle (OpenMP over cells, OMP_NUM_THREADS threads) on a bounded sample of the capsule
    workload: a reduced mesh (10 x 8 x 8 structured cells split into 3,632 tetrahedra) with the same 24^3
    velocities, physics and start; two untimed conventional iterations, then GSIS iterations timed until
    a.cpu_seconds."""
    import time as _t

    from oracle import Oracle
    from paper_2601_03935_amd.gsis import oracle_opts, default_opts

    case = capsule_case(nvx=24, mesh_kw=dict(n_s=10, n_phi=8, n_r=8))
    import numpy as np

    o = Oracle(case, **oracle_opts(default_opts(limiter_K=CAPSULE_K)))
    n = case.mesh.nc
    o.init_equilibrium(np.ones(n), np.zeros((n, 3)), np.ones(n))
    o.iterate(gsis=False)
    o.iterate(gsis=False)
    t0 = _t.perf_counter()
    k = 0
    while True:
        o.iterate(gsis=True)
        k += 1
        if _t.perf_counter() - t0 > a.cpu_seconds:
            break
    dt = _t.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    return {"value": n * case.vgrid.nv * k / dt, "unit": "cell-velocity updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_info(),
            "sample": f"{k} FP64 GSIS iterations (after 2 untimed conventional ones) of the capsule on {n} "
                      f"tetrahedra x {case.vgrid.nv} velocities ({dt:.1f} s)"}


def oracle_timings(a):
    """The FP64 oracle on the host cores for the other configurations (context beside the capsule baseline):
    the 1D Fourier flow to epsilon < 1e-6 (10 conventional iterations, then GSIS), one kinetic step and one
    GSIS iteration of the full-size cavity (Kn 0.1, optical thickness 1) from its start, and one kinetic step
    of the full-size Ma 5 cylinder from the free stream."""
    import time as _t

    from oracle import Oracle
    from workloads import case_cavity, case_cylinder, case_fourier_1d

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    out = {"kind": "oracle", "cores": cores, "cpu_model": cpu_info()}
    c = case_fourier_1d()
    o = Oracle(c)
    t0 = _t.perf_counter()
    n, hist = o.solve(gsis=True, n_precond=10, tol=1e-6, max_outer=1000)
    dt = _t.perf_counter() - t0
    out["fourier_1d"] = {"cells": c.mesh.nc, "velocities": c.vgrid.nv, "iterations_to_1e-6": int(n),
                         "seconds_to_1e-6": dt}
    del o
    for name, c in (("cavity", case_cavity()), ("cylinder", case_cylinder())):
        o = Oracle(c)
        t0 = _t.perf_counter()
        o.kinetic_step()
        tk = _t.perf_counter() - t0
        rec = {"cells": c.mesh.nc, "velocities": c.vgrid.nv, "kinetic_step_s": tk,
               "cell_velocity_updates_per_s": c.mesh.nc * c.vgrid.nv / tk}
        if name == "cavity":
            t0 = _t.perf_counter()
            o.iterate(gsis=True)
            rec["gsis_iteration_s"] = _t.perf_counter() - t0
        out[name] = rec
        del o
    return out


def bench_capsule_shard(a):
    """Kinetic steps (moments, prologue, gradients, wall densities, residual with the relaxation source,
    Jacobi sweeps, radiation) of the 3D capsule on ~213k tetrahedra with 12^3 velocities -- one eighth of the
    24^3 grid, i.e. one GPU's share when velocity space is split over eight -- and 96 ordinates, FP32."""
    import torch

    from paper_2601_03935_amd.gsis import KERNEL_KINDS, Solver
    from workloads import case_capsule

    case = case_capsule(Kn=0.01, tau_opt=1.0, Ma=10.0, nvx=12, xmax=20.0, n_theta=8, n_phi=12, sigma_R=0.045,
                        mesh_kw=dict(n_s=46, n_phi=28, n_r=28))
    nc, nv, no = case.mesh.nc, case.vgrid.nv, case.ords.no
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    s = Solver(case, device=0, stream=stream.cuda_stream, precision=a.precision)
    for _ in range(a.warmup):
        s.kinetic_step()
    torch.cuda.synchronize()
    s.set_profiling(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(a.steps):
        s.kinetic_step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    stats = s.kernel_stats()
    s.set_profiling(False)
    s.close()
    kernels = {}
    for k in KERNEL_KINDS:
        tms, n, by = stats[k]
        if n:
            kernels[k] = dict(ms_per_step=tms / a.steps, launches_per_step=n / a.steps,
                              gbs=(by / (tms * 1e-3) / 1e9) if by > 0 and tms > 0 else None)
    es = 4 if a.precision == "fp32" else 8
    return {
        "metric": "DVM cell-velocity updates/s of the kinetic step (3D capsule, one velocity-space shard)",
        "value": nc * nv * a.steps / (ms * 1e-3), "unit": "cell-velocity updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if a.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "3D blunt capsule (spherical cap + 33 deg cone), kinetic step on 1/8 of velocity space",
                   "cells": nc, "velocities": nv, "velocities_full_grid": 24 ** 3, "distributions_per_velocity": 3,
                   "ordinates": no, "Kn_gas": 0.01, "Mach": 10.0, "optical_thickness": 1.0},
        "roofline": unit_roofline(2 * 3 * es, nc * nv, stats["sweep"], None, 3, es),
        "kernels": kernels,
    }


def bench_cylinder(a):
    """Ma 5 flow past a cylinder on 40,960 triangles with 64 x 64 Newton-Cotes velocities (|xi| <= 12) and 64
    ordinates, Kn 0.01 (--cyl-Kn), optical thickness 1, sigma_R 0.1, FP32, from the uniform free stream: Mach
    continuation 2 -> 3 -> 4 -> 5 (each stage to 1e-4, the last to the tolerance; 40 conventional and 60
    first-order iterations at the start, 10 first-order iterations after each Mach step);
    then 5 profiled GSIS iterations at the converged state for the kernel table."""
    import numpy as np
    import torch

    from paper_2601_03935_amd.gsis import KERNEL_KINDS, Solver
    from workloads import case_cylinder

    Kn = a.cyl_Kn
    case = case_cylinder(Kn=Kn, tau_opt=1.0, Ma=2.0, nvx=64, xmax=12.0, n_theta=4, n_phi=16, sigma_R=0.1)
    nc, nv, no = case.mesh.nc, case.vgrid.nv, case.ords.no
    gam = case.gas.gamma
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ksw = a.kin_sweeps if a.kin_sweeps is not None else (8 if a.kin_relax == "jacobi" else 1)
    s = Solver(case, device=0, stream=stream.cuda_stream, precision=a.precision, sweep=a.kin_relax, kin_sweeps=ksw)
    states = [(1.0, 1.0, (Ma * np.sqrt(gam), 0.0, 0.0)) for Ma in (2.0, 3.0, 4.0, 5.0)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # 20 first-order iterations after each Mach jump: with 10, the jump to Mach 5 leaves one cell of the moving
    # shock with a negative translational temperature (the iteration stops as diverged)
    its, hist, ok = s.solve_continuation(1, states, stage_tol=1e-4, tol=a.tol, max_stage=a.max_stage,
                                         first_order_jump=20)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    plain_fields = s.fields()
    s.set_profiling(True)
    for _ in range(5):
        s.iterate(gsis=True)
    stats = s.kernel_stats()
    s.set_profiling(False)
    s.close()
    kernels = {}
    for k in KERNEL_KINDS:
        tms, n, by = stats[k]
        if n:
            kernels[k] = dict(ms_per_step=tms / 5, launches_per_step=n / 5,
                              gbs=(by / (tms * 1e-3) / 1e9) if by > 0 and tms > 0 else None)
    es = 4 if a.precision == "fp32" else 8
    iters = int(sum(its))
    ws = None if a.no_warmstart else cylinder_warmstart_leg(a, case, stream, plain_fields)
    return {
        "metric": "wall time to the residual tolerance from the free stream (Ma 5 cylinder, Mach continuation)",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": iters, "warmup": 0, "ms_per_step": 1e3 * sec / iters,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "2D Ma 5 cylinder, radius 1, annulus to r = 6", "cells": nc, "velocities": nv,
                   "distributions_per_velocity": 4, "ordinates": no, "Kn_gas": Kn, "Mach": 5.0,
                   "optical_thickness": 1.0, "sigma_R": 0.1, "tol": a.tol, "mach_steps": [2, 3, 4, 5],
                   "kinetic_relaxation": (f"{ksw} colored symmetric Gauss-Seidel sweep{'s' if ksw > 1 else ''}"
                                          if a.kin_relax == "sgs" else f"{ksw} Jacobi sweeps")},
        "converged": ok, "iterations_per_stage": its, "eps_final": float(hist[-1]),
        "cell_velocity_updates_per_s": nc * nv * iters / sec,
        "roofline": unit_roofline(2 * 4 * es, nc * nv, stats["sweep"], None, 4, es),
        "kernels": kernels,
        "warmstart": ws,
    }


def bench_shock(a):
    """Ma 5 normal shock (Sec. 4.1), FP64 like the paper's runs: for (Z_r, Z_v) = (2.6, 26) on [-60, 140]
    and (8, 100) on [-60, 290] (dx = 0.25: 800 and 1,400 cells), 64 uniform velocities on [-15, 15] and
    48 ordinates, outer iterations and wall time to epsilon < 2e-6 from the discontinuous start for GSIS
    (10 conventional iterations first, the paper's inner settings: at most 100 inner iterations, tolerance
    1e-7) and for the conventional iteration alone; GSIS once more with up to 400 inner iterations, which
    isolates the inner solver's share of the difference to the paper's counts."""
    import numpy as np
    import torch

    from paper_2601_03935_amd.gsis import Solver
    from workloads import case_normal_shock

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    out = []
    total = 0.0
    for Zr, Zv, x1, paper in ((2.6, 26.0, 140.0, (68, 991)), (8.0, 100.0, 290.0, (90, 2566))):
        case = case_normal_shock(Z_r=Zr, Z_v=Zv, x0=-60.0, x1=x1)
        row = {"Z_r": Zr, "Z_v": Zv, "cells": case.mesh.nc, "paper_iterations": {"gsis": paper[0], "cis": paper[1]}}
        for name, kw in (("gsis", dict(scheme="gsis", max_outer=1500)), ("cis", dict(scheme="cis", max_outer=6000)),
                         ("gsis_max_inner_400", dict(scheme="gsis", max_outer=1500, max_inner=400))):
            s = Solver(case, device=0, stream=stream.cuda_stream, precision="fp64", tol=2e-6, n_precond=10, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, rep, hist = s.solve()
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            s.close()
            row[name] = {"iterations": int(len(hist)), "converged": bool(hist[-1] < 2e-6), "seconds": sec,
                         "eps_final": float(hist[-1]), "eps_min": float(np.min(hist))}
            if name == "gsis":
                total += sec
        out.append(row)
    r0 = out[0]
    return {
        "metric": "outer iterations to epsilon < 2e-6, Ma 5 normal shock, GSIS (Z_r, Z_v) = (2.6, 26)",
        "value": r0["gsis"]["iterations"], "unit": "iterations", "n_gpus": 1, "steps": r0["gsis"]["iterations"],
        "warmup": 0, "ms_per_step": 1e3 * r0["gsis"]["seconds"] / r0["gsis"]["iterations"],
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1D Ma 5 normal shock, Rankine-Hugoniot far fields", "dx": 0.25, "velocities": 64,
                   "ordinates": 48, "Kn_gas": 5 * np.pi / 16, "Kn_photon": 10.0, "sigma_R": 0.01, "tol": 2e-6},
        "cases": out, "gsis_seconds_total": total,
    }


def cylinder_warmstart_leg(a, case, stream, plain_fields):
    """Learned warm start for the cylinder: 12 seeded cylinders (Mach 3-5, Kn 0.01-0.1, optical thickness
    0.3-3) on 6,144 triangles with 32 x 32 velocities, solved by Mach continuation, train the network on
    the GPU; the benchmark cylinder then starts at Mach 5 from its prediction (no continuation: 10
    conventional and 20 first-order iterations, then GSIS).  Reported against the continuation solve."""
    import numpy as np
    import torch

    from paper_2601_03935_amd import warmstart as WS
    from paper_2601_03935_amd.gsis import Solver
    from workloads import case_cylinder, mesh_annulus, warmstart_cylinder_params

    st = stream.cuda_stream
    coarse = mesh_annulus(n_theta=96, n_r=32)
    P = warmstart_cylinder_params(12, seed=3)
    cases = [case_cylinder(mesh=coarse, Ma=m, Kn=k, tau_opt=t, nvx=32, xmax=12.0, sigma_R=0.1, n_theta=2, n_phi=8)
             for m, k, t in P]
    t0 = time.perf_counter()
    X, Y, info = WS.cylinder_training_set(cases, stream=st, precision=a.precision)
    t_data = time.perf_counter() - t0
    ws = WS.WarmStart(width=256, bf16=True, seed=0, stream=st, family="cylinder")
    t0 = time.perf_counter()
    loss = ws.fit(X, Y, epochs=200, batch=2048, lr=2e-3)
    t_train = time.perf_counter() - t0
    target = case_cylinder(mesh=case.mesh, Ma=5.0, Kn=case.flow.Kn_gas, tau_opt=case.flow.k_eff, nvx=64, xmax=12.0,
                           n_theta=4, n_phi=16, sigma_R=case.gas.sigma_R)
    s = Solver(target, device=0, stream=st, precision=a.precision, n_precond=10, first_order_iters=20,
               tol=a.tol, max_outer=a.max_outer)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = ws.init_solver(s, target)
    rc, rep, _ = s.solve()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    F = s.fields()
    s.close()
    w = case.mesh.vol
    err = {}
    for name, pv, i in (("rho", pred["rho"], 0), ("Tt", pred["Tt"], 3), ("TR", pred["TR"], 6)):
        ref = plain_fields[:, i]
        err[name] = float(np.sqrt((w * (pv - ref) ** 2).sum() / (w * ref ** 2).sum()))
    err["converged_vs_plain_T"] = float(np.sqrt((w * (F[:, 7] - plain_fields[:, 7]) ** 2).sum() /
                                                (w * plain_fields[:, 7] ** 2).sum()))
    return {"tol": a.tol, "seconds": sec, "iterations": int(rep.iters), "converged": bool(rc == 0),
            "eps_final": float(rep.eps_final), "prediction_rel_l2_vs_plain": err,
            "train_cases": len(cases), "train_cases_converged": int(sum(r["ok"] for r in info)),
            "train_cases_first_order": int(sum(r["ok"] and r.get("order") == 1 for r in info)),
            "train_rows": int(X.shape[0]), "train_data_s": t_data, "train_s": t_train, "train_loss": loss,
            "network": "4-layer MLP 8-256-256-256-7, tanh, BF16 operands on MFMA, FP32 accumulation, Adam"}


def warmstart_leg(a, case, stream, plain_fields):
    """Learned warm start: converged solutions of seeded coarse cavities (Kn, optical thickness and lid speed
    drawn around the benchmark case) train the network on the GPU; the benchmark case then starts from its
    prediction.  Reported: time and iterations to tolerance (inference included), data and training cost,
    and the prediction error against the converged plain solve of the same case."""
    import numpy as np
    import torch

    from paper_2601_03935_amd import warmstart as WS
    from paper_2601_03935_amd.gsis import Solver
    from workloads import case_cavity, mesh_cavity, warmstart_cavity_params

    st = stream.cuda_stream
    coarse = mesh_cavity(h=0.025)
    P = warmstart_cavity_params(a.ws_cases, seed=2)
    cases = [case_cavity(Kn=k, tau_opt=t, u_lid=u, mesh=coarse, nvx=16) for k, t, u in P]
    t0 = time.perf_counter()
    X, Y = WS.training_set(cases, stream=st, precision="fp32", tol=1e-5, max_outer=a.max_outer)
    t_data = time.perf_counter() - t0
    ws = WS.WarmStart(width=256, bf16=True, seed=0, stream=st)
    t0 = time.perf_counter()
    loss = ws.fit(X, Y, epochs=60, batch=4096, lr=2e-3)
    t_train = time.perf_counter() - t0
    s = Solver(case, device=0, stream=st, precision=a.precision, tol=a.tol, max_outer=a.max_outer)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = ws.init_solver(s, case)
    rc, rep, _ = s.solve()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    F = s.fields()
    s.close()
    err = {}
    if plain_fields is not None:
        w = case.mesh.vol
        for name, pv, i in (("rho", pred["rho"], 0), ("Tt", pred["Tt"], 3), ("TR", pred["TR"], 6)):
            ref = plain_fields[:, i]
            err[name] = float(np.sqrt((w * (pv - ref) ** 2).sum() / (w * ref ** 2).sum()))
        uref = plain_fields[:, 1:3]
        err["u"] = float(np.sqrt((w[:, None] * (pred["u"] - uref) ** 2).sum() / (w[:, None] * uref ** 2).sum()))
        err["converged_vs_plain_T"] = float(np.sqrt((w * (F[:, 7] - plain_fields[:, 7]) ** 2).sum() /
                                                    (w * plain_fields[:, 7] ** 2).sum()))
    return {"tol": a.tol, "seconds": sec, "iterations": int(rep.iters), "converged": bool(rc == 0),
            "eps_final": float(rep.eps_final), "t_kinetic_s": rep.t_kinetic_s, "t_macro_s": rep.t_macro_s,
            "prediction_rel_l2_vs_plain": err, "train_cases": len(cases), "train_rows": int(X.shape[0]),
            "train_data_s": t_data, "train_s": t_train, "train_loss": loss,
            "network": "4-layer MLP 7-256-256-256-7, tanh, BF16 weights, FP32 accumulation, Adam"}


def bench_c5_gen(a):
    """Warm-start data set of hypersonic cylinders (Mach 3-10, Kn 1e-3-1, optical thickness 1e-2-1e2, 20,160
    triangles, 64^2 velocities, 64 ordinates): this shard's cases solved from the free stream by Mach
    continuation (first-order fallback), each written to a.c5_dir as case_NNN.npz with its targets (log
    rho, u, log T_t, log T_r, log T_v, log T_R; float16), the continuation's iteration count and time."""
    import numpy as np
    import torch

    from paper_2601_03935_amd import warmstart as WS
    from workloads import case_c5_cylinder, mesh_annulus, warmstart_c5_params

    k, n = (int(x) for x in a.c5_shard.split("/"))
    os.makedirs(a.c5_dir, exist_ok=True)
    P = warmstart_c5_params(a.c5_cases, seed=2)
    mesh = mesh_annulus(n_theta=180, n_r=56, seed=1)
    st = torch.cuda.current_stream().cuda_stream
    t_start = time.perf_counter()
    done = []
    for i in range(k, a.c5_cases, n):
        if time.perf_counter() - t_start > a.c5_seconds:
            break
        Ma, Kn, tau = P[i]
        c = case_c5_cylinder(Ma, Kn, tau, mesh=mesh)
        Y, rec = WS.cylinder_case_solution(c, stream=st, precision=a.precision, tol=a.tol)
        np.savez_compressed(os.path.join(a.c5_dir, f"case_{i:03d}.npz"), index=i, Ma=Ma, Kn=Kn, tau=tau,
                            ok=bool(rec["ok"]), order=int(rec.get("order", 0)),
                            iterations=int(rec.get("iterations", -1)), seconds=float(rec.get("seconds", -1.0)),
                            targets=(Y if Y is not None else np.zeros((0, 7))).astype(np.float16))
        done.append(dict(i=i, **{q: (float(v) if isinstance(v, (float, np.floating)) else v) for q, v in rec.items()}))
        print(json.dumps(done[-1]), file=sys.stderr, flush=True)
    return {"workload": "c5-gen", "shard": a.c5_shard, "cases": len(done),
            "converged": int(sum(d["ok"] for d in done)), "seconds": time.perf_counter() - t_start}


def bench_c5_eval(a):
    """Train the warm-start network on the solved training cases of the data set (cases below a.c5_train)
    and start each solved test case from its prediction (10 conventional and 20 first-order iterations, then
    GSIS to the tolerance): iterations and wall time against the continuation from the free stream."""
    import glob

    import numpy as np
    import torch

    from paper_2601_03935_amd import warmstart as WS
    from paper_2601_03935_amd.gsis import GsisError, Solver
    from workloads import case_c5_cylinder, mesh_annulus

    mesh = mesh_annulus(n_theta=180, n_r=56, seed=1)
    st = torch.cuda.current_stream().cuda_stream
    recs = [dict(np.load(f)) for f in sorted(glob.glob(os.path.join(a.c5_dir, "case_*.npz")))]
    train = [r for r in recs if int(r["index"]) < a.c5_train and bool(r["ok"])]
    test = [r for r in recs if int(r["index"]) >= a.c5_train and bool(r["ok"])]
    X = np.concatenate([WS.cylinder_features(case_c5_cylinder(float(r["Ma"]), float(r["Kn"]), float(r["tau"]),
                                                              mesh=mesh)) for r in train])
    Y = np.concatenate([r["targets"].astype(np.float64) for r in train])
    rows_all = int(X.shape[0])
    if rows_all > 2_000_000:  # one training call takes at most ~2.1M rows: a seeded subset of the cells
        keep = np.sort(np.random.default_rng(0).choice(rows_all, 2_000_000, replace=False))
        X, Y = X[keep], Y[keep]
    ws = WS.WarmStart(width=256, bf16=True, seed=0, stream=st, family="cylinder")
    t0 = time.perf_counter()
    loss = ws.fit(X, Y, epochs=40, batch=8192, lr=2e-3)
    t_train = time.perf_counter() - t0
    rows = []
    for r in test:
        c = case_c5_cylinder(float(r["Ma"]), float(r["Kn"]), float(r["tau"]), mesh=mesh)
        # second order after 20 first-order iterations; where that fails, first order throughout (the order the
        # data set falls back to for cases whose second-order shock does not settle on this mesh)
        t0 = time.perf_counter()
        it, ok, order = -1, False, 0
        for so in (1, 0):
            s = Solver(c, device=0, stream=st, precision=a.precision, n_precond=10, first_order_iters=20,
                       second_order=so, tol=a.tol, max_outer=1500)
            try:
                ws.init_solver(s, c)
                rc, rep, _ = s.solve()
                it, ok, order = int(rep.iters), bool(rc == 0), 2 if so else 1
            except GsisError:
                it, ok = -1, False
            torch.cuda.synchronize()
            s.close()
            if ok:
                break
        rows.append(dict(index=int(r["index"]), Ma=float(r["Ma"]), Kn=float(r["Kn"]), tau=float(r["tau"]),
                         warm_iterations=it, warm_seconds=time.perf_counter() - t0, warm_converged=ok,
                         warm_order=order, continuation_order=int(r["order"]),
                         continuation_iterations=int(r["iterations"]), continuation_seconds=float(r["seconds"])))
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    good = [x for x in rows if x["warm_converged"]]
    out = {"workload": "c5-eval", "cases_solved": len(recs), "train_cases": len(train), "test_cases": len(test),
           "train_rows": int(X.shape[0]), "train_rows_available": rows_all, "train_s": t_train, "train_loss": loss,
           "warm_converged": len(good), "per_case": rows}
    # freestream start (the continuation) as the fallback where the warm start does not converge
    out["total_seconds_warm_with_fallback"] = float(sum(x["warm_seconds"] +
                                                        (0.0 if x["warm_converged"] else x["continuation_seconds"])
                                                        for x in rows))
    out["total_seconds_continuation_all"] = float(sum(x["continuation_seconds"] for x in rows))
    if good:
        out["median_iterations_warm"] = float(np.median([x["warm_iterations"] for x in good]))
        out["median_iterations_continuation"] = float(np.median([x["continuation_iterations"] for x in good]))
        out["total_seconds_warm"] = float(sum(x["warm_seconds"] for x in good))
        out["total_seconds_continuation"] = float(sum(x["continuation_seconds"] for x in good))
    return out


def cavity_time_to_tol(a, case=None, stream=None):
    """Wall time to the residual tolerance on the 2D cavity from the uniform start (10 conventional iterations
    first): the configured precision, plain FP64 GSIS, and the configured precision started from the
    warm-start network's prediction."""
    import torch

    from paper_2601_03935_amd.gsis import Solver
    from workloads import case_cavity

    case = case or case_cavity(Kn=a.Kn, tau_opt=a.tau)
    stream = stream or torch.cuda.current_stream()
    out = {"workload": f"2D radiative cavity, {case.mesh.nc} triangles x {case.vgrid.nv} velocities, Kn {a.Kn}"}
    plain_fields = None
    for prec in dict.fromkeys((a.precision, "fp64")):
        s2 = Solver(case, device=0, stream=stream.cuda_stream, precision=prec, tol=a.tol, max_outer=a.max_outer)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep, hist = s2.solve()
        torch.cuda.synchronize()
        out[prec] = {"tol": a.tol, "seconds": time.perf_counter() - t0, "iterations": int(rep.iters),
                     "converged": bool(rc == 0), "eps_final": float(rep.eps_final),
                     "t_kinetic_s": rep.t_kinetic_s, "t_macro_s": rep.t_macro_s}
        if prec == a.precision:
            plain_fields = s2.fields()
        out[prec]["fields_rel_l2_vs_oracle"] = fields_vs_fixture(s2.fields(), case, a)
        s2.close()
    if not a.no_warmstart:
        out[a.precision + "+warmstart"] = warmstart_leg(a, case, stream, plain_fields)
    return out


FIELDS_2D = ("rho", "ux", "uy", "Tt", "Tr", "Tv", "TR", "T", "qtx", "qty", "qrx", "qry", "qvx", "qvy", "qRx", "qRy",
             "sigxx", "sigxy", "sigyy")


def fields_vs_fixture(F, case, a):
    """Relative L2 (volume weights; velocities against the lid speed 0.18, other fields floored at 1e-2) of
    converged cavity fields against the FP64 oracle's converged fields stored under tests/golden (written by
    tests/golden/make_cavity_fixtures.py), or None when there is no fixture for this case."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"cavity_conv_Kn{a.Kn:g}_tau{a.tau:g}.npz")
    if not os.path.exists(path) or a.tol != 1e-6:
        return None
    Fo = np.load(path)["fields"].astype(np.float64)
    if Fo.shape[0] != F.shape[0]:
        return None
    w = case.mesh.vol / case.mesh.vol.sum()
    out = {}
    for i, n in enumerate(FIELDS_2D[: Fo.shape[1]]):
        num = np.sqrt((w * (F[:, i] - Fo[:, i]) ** 2).sum())
        den = max(np.sqrt((w * Fo[:, i] ** 2).sum()), 0.18 if n[0] == "u" else 1e-2)
        out[n] = float(num / den)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if a.copy_probe:
        # plain device copies: the calibration kernel of the HBM byte counters, and the bandwidth a
        # streaming copy reaches on this GPU (context for the roofline fractions)
        n = 1 << 28  # 1 GiB of float32
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_bytes_each": 4 * n, "copies": 13, "copy_ms": ms,
                          "copy_gbs_read_plus_write": 2 * 4 * n / (ms * 1e-3) / 1e9}), flush=True)
        return
    if a.workload == "capsule":
        out = bench_capsule(a)
        if not a.no_fp64:
            out["fp64_full_size"] = bench_capsule_fp64(a)
        if not a.no_time_to_tol:
            out["time_to_tol_cavity"] = cavity_time_to_tol(a)
        if not a.no_cpu_baseline:
            out["cpu_baseline"] = capsule_cpu_baseline(a)
            if not a.no_oracle_timings:
                out["oracle_timings"] = oracle_timings(a)
        print(json.dumps(out), flush=True)
        return
    if a.workload == "c5-gen":
        print(json.dumps(bench_c5_gen(a)), flush=True)
        return
    if a.workload == "c5-eval":
        print(json.dumps(bench_c5_eval(a)), flush=True)
        return
    if a.workload == "capsule-shard":
        print(json.dumps(bench_capsule_shard(a)), flush=True)
        return
    if a.workload == "cylinder":
        print(json.dumps(bench_cylinder(a)), flush=True)
        return
    if a.workload == "capsule-ma5":
        print(json.dumps(bench_capsule_converge(a)), flush=True)
        return
    if a.workload == "shock":
        print(json.dumps(bench_shock(a)), flush=True)
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
    # events in the timed region around the dominant kernel only (the Jacobi sweep): timing every kind
    # adds ~52 event records per iteration (about 0.18 ms of 4.8); the table of all kinds comes from a
    # separate profiled pass after the timed region
    s.set_profiling(True, kinds=["sweep"])
    s.counters()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    inner = []
    eps = []
    torch.cuda.synchronize()
    ev0.record(stream)
    # one batch of a.steps whole GSIS iterations (each computes its residual; the host waits once)
    e, it = s.iterate(gsis=True, n=a.steps)
    eps.append(e)
    inner.append(it)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    stats_timed = s.kernel_stats()
    nprof = 5
    s.set_profiling(True)
    s.iterate(gsis=True, n=nprof)
    stats = s.kernel_stats()
    s.set_profiling(False)
    step_ms = ms / a.steps
    value = nc * nv * a.steps / (ms * 1e-3)
    kernels = {}
    for k in KERNEL_KINDS:
        tms, n, by = stats[k]
        if n == 0:
            continue
        kernels[k] = dict(ms_per_step=tms / nprof, launches_per_step=n / nprof,
                          gbs=(by / (tms * 1e-3) / 1e9) if by > 0 and tms > 0 else None)
    es = 4 if a.precision == "fp32" else 8
    kin_ms = sum(stats[k][0] for k in ("grad", "residual", "sweep", "rad", "boundary")) / nprof
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
        "roofline": unit_roofline(2 * 4 * es, nc * nv, stats_timed["sweep"],
                                  measured_traffic("sweep", "cavity20k") if a.precision == "fp32" else None, 4, es),
        "kinetic_step": {"ms": kin_ms, "ideal_bytes": kin_bytes_ideal,
                         "ideal_gbs": kin_bytes_ideal / (kin_ms * 1e-3) / 1e9},
        "kernels": kernels,
        "inner_iterations_last_step": int(inner[-1]),
        "eps_last": eps[-1],
    }
    if not a.no_time_to_tol:
        out["time_to_tol"] = cavity_time_to_tol(a, case, stream)
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
