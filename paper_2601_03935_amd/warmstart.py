"""Learned warm start (ctypes binding of include/gsis_warmstart.h plus feature plumbing).

A 4-layer perceptron maps case parameters and cell geometry to initial macroscopic fields; it is trained
on the GPU, by the library's own forward/backward/Adam kernels, on converged solutions the solver itself
produced.  The solver then starts from the multi-temperature equilibrium of the predicted fields
(``gsis_init_warmstart``: standardisation, network, de-standardisation, the exponential of the log targets,
the closed-domain mass scaling and the equilibrium fill all run on the device) instead of the uniform start;
the converged answer is unchanged (same fixed point), only the number of iterations to reach it.  This
module only builds the per-cell features (inputs) and marshals arguments.

Features here are for the lid-driven cavity family (unit square with the concentric square obstacle):
log10 Kn, log10 optical thickness, lid speed, x, y, distance to the nearest wall, distance to the lid.
Targets: log rho, u_x, u_y, log T_t, log T_r, log T_v, log T_R.  Inputs and targets are standardised
with the training-set mean and spread, stored with the weights.
"""

from __future__ import annotations

import ctypes as C
import time

import numpy as np

from .gsis import GsisError, Solver, lib

EXPORTS = [
    "gsis_mlp_create", "gsis_mlp_destroy", "gsis_mlp_last_error", "gsis_mlp_set_stream", "gsis_mlp_num_params",
    "gsis_mlp_get_params", "gsis_mlp_set_params", "gsis_mlp_forward", "gsis_mlp_forward_noalloc",
    "gsis_mlp_loss_grad", "gsis_mlp_adam_step",
    "gsis_mlp_train", "gsis_ws_fit_norm", "gsis_ws_train", "gsis_ws_predict", "gsis_ws_save", "gsis_ws_load",
    "gsis_ws_targets", "gsis_init_warmstart",
]

N_IN, N_OUT = 7, 7
HOLE = (0.35, 0.65)
FEATURES = {}


class gsis_mlp_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64)]


class gsis_ws_norm(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_out", C.c_int32), ("x_mean", C.c_double * 64), ("x_scale", C.c_double * 64),
                ("y_mean", C.c_double * 64), ("y_scale", C.c_double * 64)]


_registered = False


def _lib():
    global _registered
    L = lib()
    if not _registered:
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "gsis_mlp_create": ([I32, I32, I32, I32, I32, C.c_uint64, C.POINTER(C.c_void_p)], I32),
            "gsis_mlp_destroy": ([P], None),
            "gsis_mlp_last_error": ([P], C.c_char_p),
            "gsis_mlp_set_stream": ([P, P], I32),
            "gsis_mlp_num_params": ([P], I64),
            "gsis_mlp_get_params": ([P, P], I32),
            "gsis_mlp_set_params": ([P, P], I32),
            "gsis_mlp_forward": ([P, I64, P, P], I32),
            "gsis_mlp_forward_noalloc": ([P, I64, P, P], I32),
            "gsis_mlp_loss_grad": ([P, I64, P, P, C.POINTER(C.c_double), P], I32),
            "gsis_mlp_adam_step": ([P, C.POINTER(gsis_mlp_train_opts), I64, P, P, C.POINTER(C.c_double)], I32),
            "gsis_mlp_train": ([P, I64, P, P, C.POINTER(gsis_mlp_train_opts), C.POINTER(C.c_double)], I32),
            "gsis_ws_fit_norm": ([I64, I32, P, I32, P, C.POINTER(gsis_ws_norm)], I32),
            "gsis_ws_train": ([P, C.POINTER(gsis_ws_norm), I64, P, P, C.POINTER(gsis_mlp_train_opts),
                               C.POINTER(C.c_double)], I32),
            "gsis_ws_predict": ([P, C.POINTER(gsis_ws_norm), I64, P, P], I32),
            "gsis_ws_save": ([P, C.POINTER(gsis_ws_norm), C.c_char_p], I32),
            "gsis_ws_load": ([P, C.POINTER(gsis_ws_norm), C.c_char_p], I32),
            "gsis_ws_targets": ([P, P], I32),
            "gsis_init_warmstart": ([P, P, C.POINTER(gsis_ws_norm), P], I32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _registered = True
    return L


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def train_opts(epochs=10, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
    return gsis_mlp_train_opts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                               int(seed))


class MLP:
    """Handle on one network in the library (weights, Adam state and work buffers live on the GPU)."""

    def __init__(self, n_in=N_IN, width=256, n_out=N_OUT, bf16=True, seed=0, device=0, stream=None):
        self.L = _lib()
        h = C.c_void_p()
        rc = self.L.gsis_mlp_create(device, n_in, width, n_out, 1 if bf16 else 0, seed, C.byref(h))
        if rc < 0:
            raise GsisError(f"gsis_mlp_create failed with code {rc}")
        self.h = h
        self.n_in, self.width, self.n_out, self.bf16 = n_in, width, n_out, bf16
        if stream is not None:
            self._check(self.L.gsis_mlp_set_stream(self.h, C.c_void_p(stream)), "gsis_mlp_set_stream")
        self.np = int(self.L.gsis_mlp_num_params(self.h))

    def _check(self, rc, what):
        if rc < 0:
            raise GsisError(f"{what} failed with code {rc}: {self.L.gsis_mlp_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.L.gsis_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shapes(self):
        """(W, b) shapes per layer in parameter-vector order."""
        ins = [self.n_in, self.width, self.width, self.width]
        outs = [self.width, self.width, self.width, self.n_out]
        return [((o, i), (o,)) for i, o in zip(ins, outs)]

    def get_params(self):
        p = np.empty(self.np, dtype=np.float32)
        self._check(self.L.gsis_mlp_get_params(self.h, _ptr(p)), "gsis_mlp_get_params")
        return p

    def set_params(self, p):
        p = _f32(p)
        assert p.size == self.np
        self._check(self.L.gsis_mlp_set_params(self.h, _ptr(p)), "gsis_mlp_set_params")

    def forward(self, x):
        x = _f32(x)
        y = np.empty((x.shape[0], self.n_out), dtype=np.float32)
        self._check(self.L.gsis_mlp_forward(self.h, x.shape[0], _ptr(x), _ptr(y)), "gsis_mlp_forward")
        return y

    def forward_noalloc(self, x_dev, y_dev, n):
        """Allocation-free inference on device memory: x_dev, y_dev are device addresses (ints) of [n][n_in] and
        [n][n_out] FP32 rows; enqueued on the handle's stream (no wait)."""
        self._check(self.L.gsis_mlp_forward_noalloc(self.h, int(n), C.c_void_p(x_dev), C.c_void_p(y_dev)),
                    "gsis_mlp_forward_noalloc")

    def loss_grad(self, x, t):
        x, t = _f32(x), _f32(t)
        g = np.empty(self.np, dtype=np.float32)
        loss = C.c_double(0)
        self._check(self.L.gsis_mlp_loss_grad(self.h, x.shape[0], _ptr(x), _ptr(t), C.byref(loss), _ptr(g)),
                    "gsis_mlp_loss_grad")
        return loss.value, g

    def adam_step(self, x, t, **kw):
        x, t = _f32(x), _f32(t)
        o = train_opts(**kw)
        loss = C.c_double(0)
        self._check(self.L.gsis_mlp_adam_step(self.h, C.byref(o), x.shape[0], _ptr(x), _ptr(t), C.byref(loss)),
                    "gsis_mlp_adam_step")
        return loss.value

    def train(self, x, t, **kw):
        x, t = _f32(x), _f32(t)
        o = train_opts(**kw)
        loss = C.c_double(0)
        self._check(self.L.gsis_mlp_train(self.h, x.shape[0], _ptr(x), _ptr(t), C.byref(o), C.byref(loss)),
                    "gsis_mlp_train")
        return loss.value


# ---------------------------------------------------------------------------------------------------------
# features and targets (cavity family)


def cavity_features(case) -> np.ndarray:
    """Per-cell features [log10 Kn, log10 tau_opt, u_lid, x, y, wall distance, lid distance]."""
    ctr = case.mesh.ctr
    x, y = ctr[:, 0], ctr[:, 1]
    lo, hi = HOLE
    d_outer = np.minimum(np.minimum(x, 1 - x), np.minimum(y, 1 - y))
    dx = np.maximum(np.maximum(lo - x, x - hi), 0.0)
    dy = np.maximum(np.maximum(lo - y, y - hi), 0.0)
    d_hole = np.hypot(dx, dy)
    ulid = [b for b in case.bcs if abs(b.get("u", (0, 0, 0))[0]) > 0]
    u_lid = ulid[0]["u"][0] if ulid else 0.0
    n = case.mesh.nc
    return np.stack([np.full(n, np.log10(case.flow.Kn_gas)), np.full(n, np.log10(case.flow.k_eff)),
                     np.full(n, u_lid), x, y, np.minimum(d_outer, d_hole), 1 - y], axis=1)


def cylinder_features(case) -> np.ndarray:
    """Per-cell features [log10 Kn, Mach, log10 tau_opt, x, y, wall distance, cos, sin of the polar angle]
    for flows past the unit cylinder."""
    ctr = case.mesh.ctr
    x, y = ctr[:, 0], ctr[:, 1]
    r = np.hypot(x, y)
    n = case.mesh.nc
    return np.stack([np.full(n, np.log10(case.flow.Kn_gas)), np.full(n, case.meta.get("Ma", 0.0)),
                     np.full(n, np.log10(case.flow.k_eff)), x, y, r - 1.0, x / r, y / r], axis=1)


FEATURES.update(cavity=(cavity_features, 7), cylinder=(cylinder_features, 8))


def field_targets(F: np.ndarray) -> np.ndarray:
    """[log rho, u_x, u_y, log T_t, log T_r, log T_v, log T_R] from the library's 2D field array."""
    return np.stack([np.log(F[:, 0]), F[:, 1], F[:, 2], np.log(F[:, 3]), np.log(F[:, 4]), np.log(F[:, 5]),
                     np.log(F[:, 6])], axis=1)


def targets_to_fields(Y: np.ndarray) -> dict:
    return dict(rho=np.exp(Y[:, 0]), u=np.ascontiguousarray(Y[:, 1:3]), Tt=np.exp(Y[:, 3]), Tr=np.exp(Y[:, 4]),
                Tv=np.exp(Y[:, 5]), TR=np.exp(Y[:, 6]))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def solver_targets(solver: Solver) -> np.ndarray:
    """[nc][D + 5] training targets of a solver's current state (log rho, u, log T_t, log T_r, log T_v,
    log T_R), computed by the library."""
    t = np.empty((solver.nc, solver.D + 5))
    rc = _lib().gsis_ws_targets(solver.h, _ptr(t))
    if rc < 0:
        raise GsisError(f"gsis_ws_targets failed with code {rc}: {solver.L.gsis_last_error(solver.h).decode()}")
    return t


class WarmStart:
    """Standardisation + network, all in the library; fit on (features, targets) of converged cases, start a
    solver from the prediction.  `family` selects the feature set ("cavity" or "cylinder")."""

    def __init__(self, width=256, bf16=True, seed=0, device=0, stream=None, family="cavity"):
        self.family = family
        self.features, n_in = FEATURES[family]
        self.net = MLP(n_in, width, N_OUT, bf16=bf16, seed=seed, device=device, stream=stream)
        self.norm = None

    def fit(self, X, Y, epochs=40, batch=4096, lr=2e-3, seed=0):
        X, Y = _f64(X), _f64(Y)
        L = self.net.L
        self.norm = gsis_ws_norm()
        rc = L.gsis_ws_fit_norm(X.shape[0], X.shape[1], _ptr(X), Y.shape[1], _ptr(Y), C.byref(self.norm))
        if rc < 0:
            raise GsisError(f"gsis_ws_fit_norm failed with code {rc}")
        o = train_opts(epochs=epochs, batch=batch, lr=lr, seed=seed)
        loss = C.c_double(0)
        self.net._check(L.gsis_ws_train(self.net.h, C.byref(self.norm), X.shape[0], _ptr(X), _ptr(Y), C.byref(o),
                                        C.byref(loss)), "gsis_ws_train")
        return loss.value

    def predict(self, X):
        """Raw (de-standardised) network outputs for raw features X."""
        X = _f64(X)
        Y = np.empty((X.shape[0], self.net.n_out))
        self.net._check(self.net.L.gsis_ws_predict(self.net.h, C.byref(self.norm), X.shape[0], _ptr(X), _ptr(Y)),
                        "gsis_ws_predict")
        return Y

    def init_solver(self, solver: Solver, case):
        """Start `solver` from the network's prediction for `case` (gsis_init_warmstart); returns the predicted
        fields (for reporting the prediction error)."""
        X = _f64(self.features(case))
        rc = self.net.L.gsis_init_warmstart(solver.h, self.net.h, C.byref(self.norm), _ptr(X))
        if rc < 0:
            raise GsisError(f"gsis_init_warmstart failed with code {rc}: {solver.L.gsis_last_error(solver.h).decode()}")
        return targets_to_fields(self.predict(X))

    def save(self, path):
        self.net._check(self.net.L.gsis_ws_save(self.net.h, C.byref(self.norm), str(path).encode()), "gsis_ws_save")

    def load(self, path):
        self.norm = gsis_ws_norm()
        self.net._check(self.net.L.gsis_ws_load(self.net.h, C.byref(self.norm), str(path).encode()), "gsis_ws_load")


def converged_fields(case, device=0, stream=None, **opts):
    """Solve a case from its uniform start; returns (fields, targets or None, iterations, seconds, converged)."""
    s = Solver(case, device=device, stream=stream, **opts)
    t0 = time.perf_counter()
    rc, rep, _ = s.solve()
    dt = time.perf_counter() - t0
    F = s.fields()
    try:
        T = solver_targets(s)
    except GsisError:
        T = None
    s.close()
    return F, T, int(rep.iters), dt, rc == 0


def training_set(cases, device=0, stream=None, family="cavity", report=None, **opts):
    """Features and targets stacked over the cases that converge (solved from their uniform start).  A case
    that does not reach the tolerance, or whose targets are not all finite, is dropped; `report` (a dict)
    receives the counts of used and dropped cases."""
    feat = FEATURES[family][0]
    X, Y = [], []
    dropped = []
    for i, c in enumerate(cases):
        F, Yc, _, _, ok = converged_fields(c, device=device, stream=stream, **opts)
        if not ok or Yc is None or not np.isfinite(Yc).all():
            dropped.append(i)
            continue
        X.append(feat(c))
        Y.append(Yc)
    if report is not None:
        report.update(used=len(X), dropped=len(dropped), dropped_cases=dropped)
    if not X:
        raise GsisError("no training case converged with finite fields")
    return np.concatenate(X), np.concatenate(Y)


def continuation_fields(case, tag, mach_steps, device=0, stream=None, stage_tol=1e-4, tol=1e-6, cont=None, **opts):
    """Solve a free-stream case by Mach continuation up to case.meta["Ma"]; `cont` holds extra arguments of
    Solver.solve_continuation.  Returns (fields, total iterations, seconds, converged)."""
    g = case.gas.gamma
    s = Solver(case, device=device, stream=stream, **opts)
    Ma = case.meta["Ma"]
    states = [(1.0, 1.0, (m * np.sqrt(g), 0.0, 0.0)) for m in list(mach_steps) + [Ma]]
    n, D = case.mesh.nc, case.mesh.dim
    u0 = np.zeros((n, D))
    u0[:, 0] = states[0][2][0]
    s.init_equilibrium(np.ones(n), u0, np.ones(n))  # uniform free stream of the first stage
    t0 = time.perf_counter()
    its, hist, ok = s.solve_continuation(tag, states, stage_tol=stage_tol, tol=tol, **(cont or {}))
    dt = time.perf_counter() - t0
    F = s.fields()
    try:
        T = solver_targets(s)
    except GsisError:
        T, ok = None, False
    s.close()
    return F, T, int(sum(its)), dt, ok


def mach_steps(Ma):
    """Intermediate free-stream Mach numbers of the continuation towards Ma (the integers from 2 below Ma)."""
    return [x for x in (2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0, 9.0) if x < Ma - 0.25]


def cylinder_case_solution(c, device=0, stream=None, tol=1e-6, first_order_fallback=True, **opts):
    """One cylinder case solved from the free stream by Mach continuation, with the first-order fallback of
    cylinder_training_set.  Returns (targets or None, record with ok, order, iterations, seconds)."""
    rec = dict(Ma=c.meta["Ma"], Kn=c.flow.Kn_gas, tau=c.flow.k_eff)
    tries = [(2, opts, None)]
    if first_order_fallback:
        tries.append((1, dict(opts, second_order=0), dict(first_order_iters=0, first_order_jump=0)))
    for order, o, cont in tries:
        try:
            F, Yc, it, dt, ok = continuation_fields(c, 1, mach_steps(c.meta["Ma"]), device=device, stream=stream,
                                                    tol=tol, cont=cont, **o)
        except GsisError as ex:
            rec.update(ok=False, order=order, error=str(ex))
            continue
        rec.update(ok=bool(ok and Yc is not None and np.isfinite(Yc).all()), order=order, iterations=it, seconds=dt)
        rec.pop("error", None)
        if rec["ok"]:
            return Yc, rec
    return None, rec


def cylinder_training_set(cases, device=0, stream=None, tol=1e-6, first_order_fallback=True, **opts):
    """Features and targets of cylinder cases solved from the free stream by Mach continuation.  A case
    whose second-order continuation fails (a NaN residual or no convergence: on coarse training meshes at
    Kn ~ 0.01-0.02 the limited second-order shock does not settle) is solved again with first-order
    reconstruction throughout, and that solution is used; cases that still fail are skipped.  Returns
    (X, Y, per-case records with the order used)."""
    X, Y, info = [], [], []
    for c in cases:
        rec = dict(Ma=c.meta["Ma"], Kn=c.flow.Kn_gas, tau=c.flow.k_eff)
        tries = [(2, opts, None)]
        if first_order_fallback:
            tries.append((1, dict(opts, second_order=0), dict(first_order_iters=0, first_order_jump=0)))
        for order, o, cont in tries:
            try:
                F, Yc, it, dt, ok = continuation_fields(c, 1, mach_steps(c.meta["Ma"]), device=device,
                                                        stream=stream, tol=tol, cont=cont, **o)
            except GsisError as ex:
                rec.update(ok=False, order=order, error=str(ex))
                continue
            rec.update(ok=ok, order=order, iterations=it, seconds=dt)
            rec.pop("error", None)
            if ok and np.isfinite(Yc).all():
                X.append(cylinder_features(c))
                Y.append(Yc)
                break
        info.append(rec)
    if not X:
        raise GsisError("no training case converged")
    return np.concatenate(X), np.concatenate(Y), info
