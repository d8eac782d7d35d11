"""FP64 CPU oracle of the GSIS / DVM method: TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It wraps ``gsis_oracle.c`` (plain double-precision
loops written from the paper) through ctypes and shares no code with the HIP
library; inputs come from the ``workloads`` generators.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

# option vector layout of orc_create
DEFAULT_OPTS = dict(cfl_meso=1e5, cfl_macro=1e3, limiter_K=10.0, inner_tol=1e-7, max_inner=100, n_sweeps=2,
                    second_order=1, cfl_v=5.0, kin_sweeps=8, kin_omega=1.0, diss_ref=1, macro_order2=0, sweep=0, period=0.0,
                    rad_implicit=1, conservative=0)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [C.c_int, C.c_int64, C.c_int64] + [P] * 6 + [C.c_int] + [P] * 4 + \
            [C.c_int64, P, P, C.c_int64, P, P, P, P, P]
        lib.orc_destroy.argtypes = [P]
        lib.orc_set_state.argtypes = [P, P, P]
        lib.orc_get_state.argtypes = [P, P, P]
        lib.orc_init_equilibrium.argtypes = [P, P, P, P]
        lib.orc_nfields.argtypes = [C.c_int]
        lib.orc_nfields.restype = C.c_int
        lib.orc_fields.argtypes = [P, P]
        lib.orc_collision.argtypes = [P, P]
        lib.orc_rad_source.argtypes = [P, P]
        lib.orc_kinetic_step.argtypes = [P, P]
        lib.orc_boundary.argtypes = [P, P, P]
        lib.orc_hot.argtypes = [P, P]
        lib.orc_macro_solve.argtypes = [P, P]
        lib.orc_macro_solve.restype = C.c_int
        lib.orc_sync.argtypes = [P, P]
        lib.orc_macro_residual.argtypes = [P, P, P]
        lib.orc_face_hot.argtypes = [P, P]
        lib.orc_macro_state.argtypes = [P, P]
        lib.orc_macro_sources.argtypes = [P, P, P]
        lib.orc_iterate.argtypes = [P, C.c_int, P]
        lib.orc_iterate.restype = C.c_double
        lib.orc_solve.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_int, P]
        lib.orc_solve.restype = C.c_int
        lib.orc_set_second_order.argtypes = [P, C.c_int]
        lib.orc_safeguard_hits.argtypes = [P]
        lib.orc_safeguard_hits.restype = C.c_int64
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Oracle state for one case.  Distributions are [nc, ND, nv] (G, R, V[, H]); intensity [nc, no]."""

    NHOT = 21

    def __init__(self, case, **opts):
        lib = _load()
        o = dict(DEFAULT_OPTS)
        o.update(opts)
        self.opts = o
        self.case = case
        m, g, q = case.mesh, case.vgrid, case.ords
        self.D = m.dim
        assert g.dimv == m.dim, "the velocity grid dimension must match the mesh dimension"
        self.ND = 3 if self.D == 3 else 4
        self.nc, self.nv, self.no = m.nc, g.nv, q.no
        self.NW = self.D + 5
        self.nfields = lib.orc_nfields(self.D)
        kind, rho, T, u = case.bc_arrays()
        gas = case.gas
        gasv = _f64([gas.d_r, gas.d_v, gas.Z_r, gas.Z_v, gas.omega, gas.Sc, gas.sigma_R, gas.Tv_ref])
        flowv = _f64([case.flow.Kn_gas, case.flow.k_eff])
        optv = _f64([o["cfl_meso"], o["cfl_macro"], o["limiter_K"], o["inner_tol"], o["max_inner"], o["n_sweeps"],
                     o["second_order"], o["cfl_v"], o["kin_sweeps"], o["kin_omega"], o["diss_ref"],
                     o["macro_order2"], o["sweep"], o["period"], o["rad_implicit"], o["conservative"]])
        self._keep = [_f64(m.vol), _f64(m.ctr), np.ascontiguousarray(m.face_cells, dtype=np.int64), _f64(m.face_n),
                      _f64(m.face_area), _f64(m.face_ctr), np.ascontiguousarray(kind, dtype=np.int32), _f64(rho),
                      _f64(T), _f64(u), _f64(g.xi), _f64(g.w), _f64(q.omega), _f64(q.w), gasv, flowv, optv]
        k = self._keep
        self.h = lib.orc_create(self.D, m.nc, m.nf, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]),
                                len(kind), _p(k[6]), _p(k[7]), _p(k[8]), _p(k[9]), g.nv, _p(k[10]), _p(k[11]),
                                q.no, _p(k[12]), _p(k[13]), _p(k[14]), _p(k[15]), _p(k[16]))
        self.lib = lib
        lib.orc_init_equilibrium(self.h, _p(_f64(case.init_rho)), _p(_f64(case.init_u)), _p(_f64(case.init_T)))

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_destroy(self.h)
            self.h = None

    # state -----------------------------------------------------------------
    def get_state(self):
        f = np.empty((self.nc, self.ND, self.nv))
        I = np.empty((self.nc, self.no))
        self.lib.orc_get_state(self.h, _p(f), _p(I))
        return f, I

    def set_state(self, f, I):
        f = _f64(f)
        I = _f64(I)
        assert f.size == self.nc * self.ND * self.nv and I.size == self.nc * self.no
        self.lib.orc_set_state(self.h, _p(f), _p(I))

    def init_equilibrium(self, rho, u, T):
        self.lib.orc_init_equilibrium(self.h, _p(_f64(rho)), _p(_f64(u)), _p(_f64(T)))

    # operators ---------------------------------------------------------------
    def fields(self):
        out = np.empty((self.nc, self.nfields))
        self.lib.orc_fields(self.h, _p(out))
        return out

    def collision(self):
        J = np.empty((self.nc, self.ND, self.nv))
        self.lib.orc_collision(self.h, _p(J))
        return J

    def rad_source(self):
        J = np.empty((self.nc, self.no))
        self.lib.orc_rad_source(self.h, _p(J))
        return J

    def kinetic_step(self, want_residual=False):
        r = np.empty((self.nc, self.ND, self.nv)) if want_residual else None
        self.lib.orc_kinetic_step(self.h, _p(r))
        return r

    def boundary(self):
        nf = self.case.mesh.nf
        bf = np.empty((nf, self.NW))
        bs = np.empty((nf, 3))
        self.lib.orc_boundary(self.h, _p(bf), _p(bs))
        return bf, bs

    def hot(self):
        out = np.empty((self.nc, self.NHOT))
        self.lib.orc_hot(self.h, _p(out))
        return out

    def macro_solve(self):
        W = np.empty((self.nc, self.NW))
        it = self.lib.orc_macro_solve(self.h, _p(W))
        return W, it

    def face_hot(self):
        out = np.empty((self.case.mesh.nf, self.NHOT))
        self.lib.orc_face_hot(self.h, _p(out))
        return out

    def macro_residual(self, W):
        R = np.empty((self.nc, self.NW))
        self.lib.orc_macro_residual(self.h, _p(_f64(W)), _p(R))
        return R

    def macro_state(self):
        W = np.empty((self.nc, self.NW))
        self.lib.orc_macro_state(self.h, _p(W))
        return W

    def macro_sources(self, W):
        Q = np.empty((self.nc, self.NW))
        self.lib.orc_macro_sources(self.h, _p(_f64(W)), _p(Q))
        return Q

    def sync(self, W):
        self.lib.orc_sync(self.h, _p(_f64(W)))

    def iterate(self, gsis=True):
        inner = C.c_int(0)
        e = self.lib.orc_iterate(self.h, int(bool(gsis)), C.byref(inner))
        return e, inner.value

    def safeguard_hits(self):
        """Cell updates of the last synthetic solve that the positivity / trust-region safeguard shortened."""
        return int(self.lib.orc_safeguard_hits(self.h))

    def set_second_order(self, so: int):
        """Switch the face reconstruction order between iterations (start-up protocols)."""
        self.lib.orc_set_second_order(self.h, int(so))

    def solve(self, gsis=True, n_precond=10, tol=1e-6, max_outer=1000, first_order_iters=0):
        """n_precond conventional iterations then GSIS, the first `first_order_iters` iterations with first-order
        reconstruction.  Returns (iterations, eps history); negative iterations flag a NaN residual."""
        if first_order_iters <= 0:
            hist = np.zeros(max_outer)
            n = self.lib.orc_solve(self.h, int(bool(gsis)), int(n_precond), float(tol), int(max_outer), _p(hist))
            return n, hist[: abs(n)]
        so = int(self.opts["second_order"])
        hist = []
        for k in range(max_outer):
            self.set_second_order(0 if k < first_order_iters else so)
            e, _ = self.iterate(gsis=gsis and k >= n_precond)
            hist.append(e)
            if e != e:
                return -(k + 1), np.array(hist)
            if e < tol:
                return k + 1, np.array(hist)
        self.set_second_order(so)
        return max_outer, np.array(hist)


def field_names(D: int):
    ax = "xyz"[:D]
    names = ["rho"] + [f"u{a}" for a in ax] + ["Tt", "Tr", "Tv", "TR", "T"]
    for q in ("qt", "qr", "qv", "qR"):
        names += [f"{q}{a}" for a in ax]
    names += [f"sig{ax[a]}{ax[b]}" for a in range(D) for b in range(a, D)]
    return names
