"""Warm-start network on the GPU (through the C ABI) against the FP64 reference, and what it gains."""

import numpy as np
import pytest

from oracle import mlp as M
from paper_2601_03935_amd import warmstart as WS
from paper_2601_03935_amd.gsis import Solver
from workloads import case_cavity, mesh_cavity, warmstart_cavity_params

pytestmark = pytest.mark.gpu


def _data(n, n_in, n_out, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    t = np.stack([np.sin(x[:, i % n_in] + 0.3 * i) * np.cos(0.5 * x[:, (i + 1) % n_in]) for i in range(n_out)],
                 axis=1).astype(np.float32)
    return x, t


@pytest.mark.parametrize("bf16,tol", [(True, 1e-3), (False, 1e-4)], ids=["bf16", "fp32"])
def test_forward_and_gradient_match_reference(bf16, tol):
    """300 rows (ragged against the 64-row tiles), width 96 (ragged against 64-column tiles and the 32-deep
    matrix-core k slices).  BF16: the reference rounds the same operands to bfloat16; the GPU rounds its FP32
    values, which sit within FP32 accumulation error of the reference's, so an operand near a rounding
    midpoint can land on the neighbouring bfloat16 value (a 2^-8 change of one term): tolerance 1e-3."""
    net = WS.MLP(7, 96, 7, bf16=bf16, seed=5)
    shp = M.shapes(7, 96, 7)
    x, t = _data(300, 7, 7, 0)
    p = net.get_params().astype(np.float64)
    y = net.forward(x)
    y_ref = M.forward(p, shp, x, bf16=bf16)[-1]
    assert np.abs(y - y_ref).max() <= 0.2 * tol * np.abs(y_ref).max()
    L, g = net.loss_grad(x, t)
    L_ref, g_ref = M.loss_grad(p, shp, x, t, bf16=bf16)
    assert abs(L - L_ref) <= 0.1 * tol * L_ref
    Ws, bs = M.unpack(g.astype(np.float64), shp)
    Wr, br = M.unpack(g_ref, shp)
    for l in range(4):
        assert np.linalg.norm(Ws[l] - Wr[l]) <= tol * np.linalg.norm(Wr[l]), l
        assert np.linalg.norm(bs[l] - br[l]) <= tol * np.linalg.norm(br[l]), l
    net.close()


def test_bf16_weights_are_used():
    """The BF16 path rounds the weights: its outputs differ from the FP32-weight path by the rounding."""
    x, _ = _data(64, 7, 7, 1)
    a, b = WS.MLP(7, 64, 7, bf16=True, seed=3), WS.MLP(7, 64, 7, bf16=False, seed=3)
    ya, yb = a.forward(x), b.forward(x)
    rel = np.abs(ya - yb).max() / np.abs(yb).max()
    assert 1e-4 < rel < 5e-2
    a.close()
    b.close()


def test_adam_step_matches_reference():
    net = WS.MLP(7, 64, 7, bf16=True, seed=9)
    shp = M.shapes(7, 64, 7)
    x, t = _data(200, 7, 7, 2)
    p0 = net.get_params().astype(np.float64)
    _, g_ref = M.loss_grad(p0, shp, x, t, bf16=True)
    net.adam_step(x, t, lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    p1_ref, _, _ = M.adam_step(p0, np.zeros_like(p0), np.zeros_like(p0), 1, g_ref, lr=1e-3)
    # the first step moves each parameter by about lr * sign(g): compare where the gradient is not tiny
    big = np.abs(g_ref) > 1e-3 * np.abs(g_ref).max()
    assert big.sum() > 0.5 * big.size
    assert np.abs(p1 - p1_ref)[big].max() <= 2e-6
    net.close()


def test_training_reduces_loss():
    net = WS.MLP(7, 128, 7, bf16=True, seed=1)
    x, t = _data(4000, 7, 7, 3)
    L0, _ = net.loss_grad(x, t)
    Lf = net.train(x, t, epochs=30, batch=500, lr=2e-3, seed=4)
    L1, _ = net.loss_grad(x, t)
    assert L1 < 0.1 * L0 and Lf < 0.2 * L0
    net.close()


def test_warm_start_saves_iterations():
    """Trained on converged coarse cavities, the network starts unseen cases closer to their solution:
    fewer GSIS iterations to 1e-6, and the converged fields are those of the plain solve."""
    mesh = mesh_cavity(h=0.06)
    kw = dict(nvx=12, n_theta=2, n_phi=4)
    P = warmstart_cavity_params(14, seed=7)
    cases = [case_cavity(Kn=k, tau_opt=tau, u_lid=u, mesh=mesh, **kw) for k, tau, u in P]
    train, test = cases[:11], cases[11:]
    X, Y = WS.training_set(train, tol=1e-6, max_outer=800)
    ws = WS.WarmStart(width=128, seed=0)
    ws.fit(X, Y, epochs=150, batch=1024, lr=3e-3)
    plain_it, warm_it = [], []
    for c in test:
        F0, _, it0, _, ok0 = WS.converged_fields(c, tol=1e-6, max_outer=800)
        s = Solver(c, tol=1e-6, max_outer=800)
        pred = ws.init_solver(s, c)
        rc, rep, _ = s.solve()
        F1 = s.fields()
        s.close()
        assert ok0 and rc == 0
        plain_it.append(it0)
        warm_it.append(int(rep.iters))
        # prediction error against the converged plain solve
        T_err = np.linalg.norm(pred["Tt"] - F0[:, 3]) / np.linalg.norm(F0[:, 3])
        assert T_err < 0.05, T_err
        # same fixed point
        for i in (0, 3, 7):
            assert np.linalg.norm(F1[:, i] - F0[:, i]) <= 1e-4 * np.linalg.norm(F0[:, i])
    print("plain", plain_it, "warm", warm_it)
    assert np.mean(warm_it) < np.mean(plain_it)


def test_warm_start_replaces_mach_continuation():
    """Hypersonic cylinders (Mach 3-5, Kn 0.01-0.1, optical thickness 0.3-3, 6,144 triangles, 32 x 32
    velocities): solved from the free stream they need a Mach continuation; started from the network's
    prediction they converge directly at their Mach number, in fewer iterations, to the same fields."""
    from paper_2601_03935_amd.warmstart import continuation_fields, cylinder_training_set, mach_steps
    from workloads import case_cylinder, mesh_annulus, warmstart_cylinder_params

    mesh = mesh_annulus(n_theta=96, n_r=32)
    kw = dict(nvx=32, xmax=12.0, sigma_R=0.1, n_theta=2, n_phi=4)
    P = warmstart_cylinder_params(12, seed=3)
    train = [case_cylinder(mesh=mesh, Ma=m, Kn=k, tau_opt=t, **kw) for m, k, t in P]
    X, Y, info = cylinder_training_set(train)
    # every case converges: second order, or first order where the coarse-mesh shock does not settle
    assert sum(r["ok"] for r in info) == len(train), info
    ws = WS.WarmStart(width=256, seed=0, family="cylinder")
    ws.fit(X, Y, epochs=200, batch=2048, lr=2e-3)
    tests = [case_cylinder(mesh=mesh, Ma=4.17, Kn=0.062, tau_opt=1.72, **kw),
             case_cylinder(mesh=mesh, Ma=4.48, Kn=0.037, tau_opt=2.27, **kw)]
    for c in tests:
        F0, _, it0, _, ok0 = continuation_fields(c, 1, mach_steps(c.meta["Ma"]), tol=1e-6)
        s = Solver(c, tol=1e-6, max_outer=800, n_precond=10, first_order_iters=20)
        pred = ws.init_solver(s, c)
        rc, rep, _ = s.solve()
        F1 = s.fields()
        s.close()
        print("Ma %.2f: continuation %d iterations, warm start %d" % (c.meta["Ma"], it0, rep.iters))
        assert ok0 and rc == 0
        assert rep.iters < it0
        assert np.linalg.norm(pred["Tt"] - F0[:, 3]) < 0.1 * np.linalg.norm(F0[:, 3])
        for i in (0, 3, 7):
            assert np.linalg.norm(F1[:, i] - F0[:, i]) <= 1e-4 * np.linalg.norm(F0[:, i])


@pytest.mark.parametrize("bf16,tol", [(True, 2e-3), (False, 1e-4)], ids=["bf16", "fp32"])
def test_gradient_elementwise_at_production_width(bf16, tol):
    """Width 256 (the production network): every output and every element of every layer's weight and bias
    gradient against the FP64 reference, relative to the largest magnitude of that layer (BF16: operands
    on a rounding midpoint may round the other way on one side, a 2^-8 change of one term)."""
    net = WS.MLP(8, 256, 7, bf16=bf16, seed=11)
    shp = M.shapes(8, 256, 7)
    x, t = _data(333, 8, 7, 5)
    p = net.get_params().astype(np.float64)
    y = net.forward(x)
    y_ref = M.forward(p, shp, x, bf16=bf16)[-1]
    assert np.abs(y - y_ref).max() <= 0.5 * tol * np.abs(y_ref).max()
    _, g = net.loss_grad(x, t)
    _, g_ref = M.loss_grad(p, shp, x, t, bf16=bf16)
    Ws, bs = M.unpack(g.astype(np.float64), shp)
    Wr, br = M.unpack(g_ref, shp)
    for l in range(4):
        assert np.abs(Ws[l] - Wr[l]).max() <= tol * np.abs(Wr[l]).max(), l
        assert np.abs(bs[l] - br[l]).max() <= tol * np.abs(br[l]).max(), l
    net.close()


def test_library_standardisation_prediction_and_file_round_trip(tmp_path):
    """gsis_ws_fit_norm gives the column means and spreads; gsis_ws_predict equals the de-standardised
    forward pass of the standardised rows; a network saved with gsis_ws_save and loaded into a fresh handle
    predicts the same values."""
    rng = np.random.default_rng(4)
    X = rng.normal(size=(500, 7)) * np.arange(1, 8) + np.arange(7)
    Y = rng.normal(size=(500, 7)) * 0.3 + 2.0
    ws = WS.WarmStart(width=64, seed=2)
    ws.fit(X, Y, epochs=2, batch=128, lr=1e-3)
    nm = ws.norm
    np.testing.assert_allclose(np.array(nm.x_mean[:7]), X.mean(0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.array(nm.x_scale[:7]), X.std(0) + 1e-12, rtol=1e-12)
    np.testing.assert_allclose(np.array(nm.y_scale[:7]), Y.std(0) + 1e-12, rtol=1e-12)
    P = ws.predict(X[:50])
    xm, xs = np.array(nm.x_mean[:7]), np.array(nm.x_scale[:7])
    ym, ys = np.array(nm.y_mean[:7]), np.array(nm.y_scale[:7])
    ref = ws.net.forward(((X[:50] - xm) / xs).astype(np.float32)).astype(np.float64) * ys + ym
    assert np.abs(P - ref).max() <= 1e-5 * np.abs(ref).max()
    path = tmp_path / "net.bin"
    ws.save(path)
    ws2 = WS.WarmStart(width=64, seed=99)
    ws2.load(path)
    assert np.array_equal(ws2.predict(X[:50]), P)
