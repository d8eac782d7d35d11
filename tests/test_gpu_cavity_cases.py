"""The full-size cavity (20,108 triangles, 32 x 32 velocities, 32 ordinates) at the nine (Kn, optical
thickness) pairs Kn in {0.01, 0.1, 1} x tau in {0.1, 1, 10}: the GPU FP32 solve to epsilon < 1e-6 against the
converged FP64 oracle fields stored by tests/golden/make_cavity_fixtures.py (same start, same options), the
primary fields (density, velocity, the four temperatures and the total one) within 1e-5 relative L2 (volume
weights; velocities against the lid speed)."""

import os

import numpy as np
import pytest

from oracle import field_names
from paper_2601_03935_amd.gsis import Solver
from workloads import case_cavity

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PAIRS = [(k, t) for k in (0.01, 0.1, 1.0) for t in (0.1, 1.0, 10.0)]


def _fixture(Kn, tau):
    return os.path.join(GOLDEN, f"cavity_conv_Kn{Kn:g}_tau{tau:g}.npz")


def field_rel_l2(Fg, Fo, vol, names, u_scale):
    assert np.isfinite(Fg).all() and np.isfinite(Fo).all(), "non-finite field"
    w = vol / vol.sum()
    out = {}
    for i, n in enumerate(names):
        num = np.sqrt((w * (Fg[:, i] - Fo[:, i]) ** 2).sum())
        den = max(np.sqrt((w * Fo[:, i] ** 2).sum()), u_scale if n[0] == "u" else 1e-2)
        out[n] = float(num / den)
    return out


@pytest.mark.parametrize("Kn,tau", PAIRS, ids=[f"Kn{k:g}-tau{t:g}" for k, t in PAIRS])
def test_converged_fp32_cavity_matches_oracle(Kn, tau):
    path = _fixture(Kn, tau)
    if not os.path.exists(path):
        pytest.skip(f"fixture {os.path.basename(path)} not generated (tests/golden/make_cavity_fixtures.py)")
    z = np.load(path)
    case = case_cavity(Kn=Kn, tau_opt=tau)
    assert case.mesh.nc == int(z["nc"])
    s = Solver(case, precision="fp32", tol=float(z["tol"]), n_precond=int(z["n_precond"]), max_outer=3000)
    rc, rep, hist = s.solve()
    F = s.fields()
    s.close()
    assert rc == 0, (rc, rep.iters)
    Fo = z["fields"].astype(np.float64)
    errs = field_rel_l2(F[:, : Fo.shape[1]], Fo, case.mesh.vol, field_names(2)[: Fo.shape[1]], 0.18)
    print(f"Kn {Kn} tau {tau}: GPU {rep.iters} iterations, oracle {int(z['iterations'])}; errors",
          sorted(errs.items(), key=lambda kv: -kv[1])[:3])
    assert abs(rep.iters - int(z["iterations"])) <= max(3, 0.02 * int(z["iterations"]))
    assert max(errs.values()) < 1e-5, errs
