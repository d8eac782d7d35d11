"""ctypes binding of libgsis.so: argument marshalling only.

Every function of ``include/gsis.h`` is exposed under the same name on the object returned by
:func:`lib`; :class:`Solver` wraps one handle for a case built from plain arrays.  No computation
happens here: every step of the method runs in the library's HIP kernels.  Importing works without
a GPU; creating a handle needs one, and a missing library raises instead of falling back.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsis.so")

GSIS_OK, GSIS_E_ARG, GSIS_E_OOM, GSIS_E_DEVICE, GSIS_E_STATE, GSIS_E_DIVERGED = 0, -1, -2, -3, -4, -5
GSIS_W_NOT_CONVERGED = 1
GSIS_BC_WALL, GSIS_BC_FARFIELD = 0, 1
GSIS_CIS, GSIS_GSIS = 0, 1
GSIS_FP64, GSIS_FP32 = 0, 1
GSIS_SWEEP_JACOBI, GSIS_SWEEP_SGS = 0, 1

# every entry point declared in include/gsis.h
EXPORTS = [
    "gsis_create", "gsis_destroy", "gsis_last_error", "gsis_default_opts", "gsis_set_stream", "gsis_set_mesh",
    "gsis_set_velocity_grid", "gsis_set_boundary", "gsis_set_ordinates", "gsis_set_gas", "gsis_set_flow", "gsis_set_opts",
    "gsis_init_equilibrium", "gsis_init_fields", "gsis_set_state", "gsis_get_state", "gsis_get_state_cells", "gsis_iterate", "gsis_solve",
    "gsis_kinetic_step", "gsis_macro_solve", "gsis_sync", "gsis_nfields", "gsis_get_fields",
    "gsis_get_residual_history", "gsis_get_surface_flux", "gsis_get_counters", "gsis_set_profiling",
    "gsis_get_kernel_stats", "gsis_checkpoint", "gsis_restore",
]
KERNEL_KINDS = ["grad", "residual", "sweep", "rad", "moments", "boundary", "sync", "macro"]


class gsis_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rho", C.c_double), ("T", C.c_double), ("u", C.c_double * 3)]


class gsis_gas(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("d_r", "d_v", "Z_r", "Z_v", "omega", "Sc", "sigma_R", "Tv_ref")]


class gsis_flow(C.Structure):
    _fields_ = [("Kn_gas", C.c_double), ("k_eff", C.c_double)]


class gsis_opts(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("precision", C.c_int32), ("tol", C.c_double), ("max_outer", C.c_int32),
                ("n_precond", C.c_int32), ("cfl_meso", C.c_double), ("cfl_v", C.c_double),
                ("kin_sweeps", C.c_int32), ("kin_omega", C.c_double), ("limiter_K", C.c_double),
                ("second_order", C.c_int32), ("cfl_macro", C.c_double), ("inner_tol", C.c_double),
                ("max_inner", C.c_int32), ("n_sweeps", C.c_int32), ("first_order_iters", C.c_int32),
                ("sweep", C.c_int32), ("kin_fused", C.c_int32), ("conservative", C.c_int32)]


class gsis_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("eps_final", C.c_double), ("t_total_s", C.c_double),
                ("t_kinetic_s", C.c_double), ("t_macro_s", C.c_double), ("t_other_s", C.c_double),
                ("inner_total", C.c_int64)]


_lib = None


def lib():
    """Load libgsis.so (built in-tree by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2601_03935_amd/build.py")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same soname), and a process that loads
    # both cannot use the GPU through the second.  Loading torch first makes the library bind to torch's
    # runtime, so torch streams and device memory can be handed to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "gsis_create": ([I32, C.POINTER(P)], I32),
        "gsis_destroy": ([P], None),
        "gsis_last_error": ([P], C.c_char_p),
        "gsis_default_opts": ([C.POINTER(gsis_opts)], None),
        "gsis_set_stream": ([P, P], I32),
        "gsis_set_mesh": ([P, I32, I64, I64, P, P, P, P, P, P, I32, P], I32),
        "gsis_set_velocity_grid": ([P, I64, P, P], I32),
        "gsis_set_ordinates": ([P, I64, P, P], I32),
        "gsis_set_gas": ([P, C.POINTER(gsis_gas)], I32),
        "gsis_set_flow": ([P, C.POINTER(gsis_flow)], I32),
        "gsis_set_opts": ([P, C.POINTER(gsis_opts)], I32),
        "gsis_init_equilibrium": ([P, P, P, P], I32),
        "gsis_set_state": ([P, P, P], I32),
        "gsis_get_state": ([P, P, P], I32),
        "gsis_get_state_cells": ([P, P, C.c_int64, P, P], I32),
        "gsis_iterate": ([P, I32, I32, C.POINTER(D), C.POINTER(I32)], I32),
        "gsis_solve": ([P, C.POINTER(gsis_report)], I32),
        "gsis_kinetic_step": ([P], I32),
        "gsis_macro_solve": ([P, P, C.POINTER(I32)], I32),
        "gsis_sync": ([P, P], I32),
        "gsis_init_fields": ([P, P, P, P, P, P, P], I32),
        "gsis_set_boundary": ([P, I32, C.POINTER(gsis_bc)], I32),
        "gsis_nfields": ([P], I32),
        "gsis_get_fields": ([P, P], I32),
        "gsis_get_residual_history": ([P, P, I64, C.POINTER(I64)], I32),
        "gsis_get_surface_flux": ([P, P, P, P], I32),
        "gsis_get_counters": ([P, C.POINTER(D), C.POINTER(D), C.POINTER(D)], I32),
        "gsis_set_profiling": ([P, I32], I32),
        "gsis_get_kernel_stats": ([P, I32, C.POINTER(D), C.POINTER(I64), C.POINTER(D)], I32),
        "gsis_checkpoint": ([P, C.c_char_p], I32),
        "gsis_restore": ([P, C.c_char_p], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw) -> gsis_opts:
    o = gsis_opts()
    lib().gsis_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp32": GSIS_FP32, "fp64": GSIS_FP64}[v]
        if k == "scheme" and isinstance(v, str):
            v = {"cis": GSIS_CIS, "gsis": GSIS_GSIS}[v]
        if k == "sweep" and isinstance(v, str):
            v = {"jacobi": GSIS_SWEEP_JACOBI, "sgs": GSIS_SWEEP_SGS}[v]
        setattr(o, k, v)
    return o


class GsisError(RuntimeError):
    pass


class Solver:
    """One library handle set up for a case (mesh, grids, gas, flow, boundary tags, initial fields)."""

    def __init__(self, case, device: int = 0, stream=None, **opts):
        self.L = lib()
        h = C.c_void_p()
        self._check(self.L.gsis_create(device, C.byref(h)), "gsis_create", handle=None)
        self.h = h
        self.case = case
        m, g, q = case.mesh, case.vgrid, case.ords
        self.D, self.nc, self.nv, self.no = m.dim, m.nc, g.nv, q.no
        self.ND = 3 if self.D == 3 else 4
        self.NW = self.D + 5
        if stream is not None:
            self._check(self.L.gsis_set_stream(self.h, C.c_void_p(stream)), "gsis_set_stream")
        kind, rho, T, u = case.bc_arrays()
        bcs = (gsis_bc * max(1, len(kind)))()
        for i in range(len(kind)):
            bcs[i].kind = int(kind[i])
            bcs[i].rho = float(rho[i])
            bcs[i].T = float(T[i])
            for a in range(3):
                bcs[i].u[a] = float(u[i, a])
        self._keep = [_f64(m.vol), _f64(m.ctr), np.ascontiguousarray(m.face_cells, dtype=np.int64), _f64(m.face_n),
                      _f64(m.face_area), _f64(m.face_ctr)]
        k = self._keep
        self._check(self.L.gsis_set_mesh(self.h, m.dim, m.nc, m.nf, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]),
                                         _p(k[4]), _p(k[5]), len(kind), C.cast(bcs, C.c_void_p)), "gsis_set_mesh")
        self._check(self.L.gsis_set_velocity_grid(self.h, g.nv, _p(_f64(g.xi)), _p(_f64(g.w))),
                    "gsis_set_velocity_grid")
        self._check(self.L.gsis_set_ordinates(self.h, q.no, _p(_f64(q.omega)), _p(_f64(q.w))), "gsis_set_ordinates")
        gs = case.gas
        self._check(self.L.gsis_set_gas(self.h, C.byref(gsis_gas(gs.d_r, gs.d_v, gs.Z_r, gs.Z_v, gs.omega, gs.Sc,
                                                                  gs.sigma_R, getattr(gs, "Tv_ref", 0.0)))),
                    "gsis_set_gas")
        self._check(self.L.gsis_set_flow(self.h, C.byref(gsis_flow(case.flow.Kn_gas, case.flow.k_eff))),
                    "gsis_set_flow")
        self.opts = default_opts(**opts)
        self._check(self.L.gsis_set_opts(self.h, C.byref(self.opts)), "gsis_set_opts")
        self.init_equilibrium(case.init_rho, case.init_u, case.init_T)

    def set_boundary(self, tag, kind, rho, T, u):
        """New state for a boundary tag (same kind), e.g. a Mach-number continuation step."""
        b = gsis_bc()
        b.kind, b.rho, b.T = int(kind), float(rho), float(T)
        for a in range(3):
            b.u[a] = float(u[a]) if a < len(u) else 0.0
        self._check(self.L.gsis_set_boundary(self.h, int(tag), C.byref(b)), "gsis_set_boundary")

    def solve_continuation(self, tag, states, stage_tol=1e-4, tol=1e-6, max_stage=400, n_precond=40,
                           first_order_iters=60, first_order_jump=10):
        """Continuation in the boundary state of `tag` (e.g. free-stream Mach 2, 3, 4, 5): each (rho, T, u)
        in `states` is imposed in turn and GSIS iterated until epsilon < stage_tol (tol for the last one)
        or max_stage iterations.  The first stage starts with n_precond conventional iterations and uses
        first-order reconstruction for its first `first_order_iters` iterations; later stages for their
        first `first_order_jump`.  Returns (iterations per stage, epsilon history, converged)."""
        so = int(self.opts.second_order)
        kind = self.case.bcs[tag]["kind"]
        its, hist = [], []
        ok = False
        for i, (rho, T, u) in enumerate(states):
            self.set_boundary(tag, kind, rho, T, u)
            last = i == len(states) - 1
            thr = tol if last else stage_tol
            k = 0
            while k < max_stage:
                nfo = first_order_iters if i == 0 else first_order_jump
                self.set_opts(second_order=0 if k < nfo else so)
                e, _ = self.iterate(gsis=(i > 0 or k >= n_precond))
                hist.append(e)
                k += 1
                if e < thr and k > nfo:
                    break
            its.append(k)
            ok = bool(hist[-1] < thr)
        self.set_opts(second_order=so)
        return its, np.asarray(hist), ok

    def set_opts(self, **kw):
        """Change options between iterations; the state is kept unless the precision changes (that
        reallocates and needs a new initial state)."""
        o = self.opts
        for k, v in kw.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp32": GSIS_FP32, "fp64": GSIS_FP64}[v]
            if k == "scheme" and isinstance(v, str):
                v = {"cis": GSIS_CIS, "gsis": GSIS_GSIS}[v]
            if k == "sweep" and isinstance(v, str):
                v = {"jacobi": GSIS_SWEEP_JACOBI, "sgs": GSIS_SWEEP_SGS}[v]
            setattr(o, k, v)
        self._check(self.L.gsis_set_opts(self.h, C.byref(o)), "gsis_set_opts")

    def _check(self, rc, what, handle="self"):
        if rc < 0:
            msg = ""
            if handle == "self" and getattr(self, "h", None):
                msg = self.L.gsis_last_error(self.h).decode()
            raise GsisError(f"{what} failed with code {rc}: {msg}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.L.gsis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state -----------------------------------------------------------------
    def init_equilibrium(self, rho, u, T):
        self._check(self.L.gsis_init_equilibrium(self.h, _p(_f64(rho)), _p(_f64(u)), _p(_f64(T))),
                    "gsis_init_equilibrium")

    def init_fields(self, rho, u, Tt, Tr, Tv, TR):
        """Multi-temperature equilibrium start from fields (e.g. a learned warm start)."""
        a = [_f64(v) for v in (rho, u, Tt, Tr, Tv, TR)]
        self._check(self.L.gsis_init_fields(self.h, *[_p(v) for v in a]), "gsis_init_fields")

    def set_state(self, f, I):
        f, I = _f64(f), _f64(I)
        assert f.size == self.nc * self.ND * self.nv and I.size == self.nc * self.no
        self._check(self.L.gsis_set_state(self.h, _p(f), _p(I)), "gsis_set_state")

    def get_state(self):
        f = np.empty((self.nc, self.ND, self.nv))
        I = np.empty((self.nc, self.no))
        self._check(self.L.gsis_get_state(self.h, _p(f), _p(I)), "gsis_get_state")
        return f, I

    def get_state_cells(self, cells):
        """State rows (f [n, ND, nv], I [n, no]) of the listed cells."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        f = np.empty((len(cells), self.ND, self.nv))
        I = np.empty((len(cells), self.no))
        self._check(self.L.gsis_get_state_cells(self.h, _p(cells), len(cells), _p(f), _p(I)), "gsis_get_state_cells")
        return f, I

    def checkpoint(self, path):
        self._check(self.L.gsis_checkpoint(self.h, str(path).encode()), "gsis_checkpoint")

    def restore(self, path):
        self._check(self.L.gsis_restore(self.h, str(path).encode()), "gsis_restore")

    def fields(self):
        n = self.L.gsis_nfields(self.h)
        out = np.empty((self.nc, n))
        self._check(self.L.gsis_get_fields(self.h, _p(out)), "gsis_get_fields")
        return out

    # stages ------------------------------------------------------------------
    def kinetic_step(self):
        self._check(self.L.gsis_kinetic_step(self.h), "gsis_kinetic_step")

    def macro_solve(self):
        W = np.empty((self.nc, self.NW))
        it = C.c_int32(0)
        self._check(self.L.gsis_macro_solve(self.h, _p(W), C.byref(it)), "gsis_macro_solve")
        return W, it.value

    def sync(self, W):
        self._check(self.L.gsis_sync(self.h, _p(_f64(W))), "gsis_sync")

    def iterate(self, gsis=True, n=1):
        e = C.c_double(0)
        it = C.c_int32(0)
        self._check(self.L.gsis_iterate(self.h, GSIS_GSIS if gsis else GSIS_CIS, n, C.byref(e), C.byref(it)),
                    "gsis_iterate")
        return e.value, it.value

    def solve(self):
        rep = gsis_report()
        rc = self._check(self.L.gsis_solve(self.h, C.byref(rep)), "gsis_solve")
        n = C.c_int64(0)
        self.L.gsis_get_residual_history(self.h, None, 0, C.byref(n))
        hist = np.zeros(max(1, n.value))
        self.L.gsis_get_residual_history(self.h, _p(hist), n.value, C.byref(n))
        return rc, rep, hist[: n.value]

    def surface_flux(self):
        nf = self.case.mesh.nf
        qc, qr, pw = np.empty(nf), np.empty(nf), np.empty(nf)
        self._check(self.L.gsis_get_surface_flux(self.h, _p(qc), _p(qr), _p(pw)), "gsis_get_surface_flux")
        return qc, qr, pw

    def set_profiling(self, on=True, kinds=None):
        """Per-kernel event timing: every kind, or only the named kinds (e.g. ["sweep"])."""
        v = int(bool(on))
        if on and kinds is not None:
            v = 0x100
            for k in kinds:
                v |= 1 << KERNEL_KINDS.index(k)
        self._check(self.L.gsis_set_profiling(self.h, v), "gsis_set_profiling")

    def kernel_stats(self):
        """{kind: (ms_total, launches, bytes_total)} of the kernels timed since profiling was enabled."""
        out = {}
        for i, name in enumerate(KERNEL_KINDS):
            ms, n, by = C.c_double(0), C.c_int64(0), C.c_double(0)
            self._check(self.L.gsis_get_kernel_stats(self.h, i, C.byref(ms), C.byref(n), C.byref(by)),
                        "gsis_get_kernel_stats")
            out[name] = (ms.value, n.value, by.value)
        return out

    def counters(self):
        a, b, c = C.c_double(0), C.c_double(0), C.c_double(0)
        self.L.gsis_get_counters(self.h, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value


def oracle_opts(opts: gsis_opts) -> dict:
    """The oracle option set equivalent to a library option set (for parity runs)."""
    return dict(cfl_meso=opts.cfl_meso, cfl_macro=opts.cfl_macro, limiter_K=opts.limiter_K, inner_tol=opts.inner_tol,
                max_inner=opts.max_inner, n_sweeps=opts.n_sweeps, second_order=opts.second_order, cfl_v=opts.cfl_v,
                kin_sweeps=opts.kin_sweeps, kin_omega=opts.kin_omega, diss_ref=1, macro_order2=0, sweep=opts.sweep,
                conservative=opts.conservative)
