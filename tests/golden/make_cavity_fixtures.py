"""Writes the converged-field fixtures of the full-size cavity (20,108 triangles, 32 x 32 velocities, 32
ordinates) for the nine (Kn, optical thickness) pairs Kn in {0.01, 0.1, 1} x tau in {0.1, 1, 10}: the FP64
oracle with its default options, 10 conventional iterations then GSIS to epsilon < 1e-6.  One file per
case, `cavity_conv_Kn<Kn>_tau<tau>.npz`: the converged primary fields (float32, [cell][field]: rho, u_x,
u_y, T_t, T_r, T_v, T_R, T, the first eight of the oracle's field order), the iteration count and the
residual history.  Calls only the oracle and the input generators.

    OMP_NUM_THREADS=6 python tests/golden/make_cavity_fixtures.py [Kn tau ...]
    python tests/golden/make_cavity_fixtures.py --trim    (keep the primary fields of existing files)
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle  # noqa: E402
from workloads import case_cavity  # noqa: E402

KNS = (0.01, 0.1, 1.0)
TAUS = (0.1, 1.0, 10.0)
TOL, N_PRECOND, MAX_OUTER = 1e-6, 10, 3000
N_PRIMARY = 8


def fixture_path(Kn, tau):
    return os.path.join(HERE, f"cavity_conv_Kn{Kn:g}_tau{tau:g}.npz")


def make(Kn, tau):
    case = case_cavity(Kn=Kn, tau_opt=tau)
    o = Oracle(case)
    t0 = time.time()
    n, hist = o.solve(gsis=True, n_precond=N_PRECOND, tol=TOL, max_outer=MAX_OUTER)
    F = o.fields()
    np.savez_compressed(fixture_path(Kn, tau), fields=F[:, :N_PRIMARY].astype(np.float32), iterations=np.int64(n),
                        eps=np.asarray(hist, dtype=np.float64), tol=TOL, n_precond=N_PRECOND, Kn=Kn, tau=tau,
                        nc=case.mesh.nc)
    print(f"Kn {Kn} tau {tau}: {n} iterations, eps {hist[-1]:.3e}, {time.time() - t0:.0f} s", flush=True)


def trim():
    """Rewrite fixtures that hold more than the primary fields."""
    for k in KNS:
        for t in TAUS:
            p = fixture_path(k, t)
            if os.path.exists(p):
                z = dict(np.load(p))
                if z["fields"].shape[1] > N_PRIMARY:
                    z["fields"] = z["fields"][:, :N_PRIMARY]
                    np.savez_compressed(p, **z)


if __name__ == "__main__":
    if sys.argv[1:] == ["--trim"]:
        trim()
        sys.exit(0)
    args = [float(a) for a in sys.argv[1:]]
    pairs = list(zip(args[::2], args[1::2])) if args else [(k, t) for k in KNS for t in TAUS]
    for k, t in pairs:
        if not os.path.exists(fixture_path(k, t)):
            make(k, t)
