"""Linear Fourier analysis of the conventional iteration (CIS) and of GSIS for the radiative kinetic model.

TEST INFRASTRUCTURE ONLY (used by the tests).  Builds the 17x17 iteration matrix C(theta) of the
CIS error propagation (Sec. 4.2, Eqs. error_function_propagation, error_function_M_phi,
eigenfunction_cis) for a wave vector along x and returns its spectral radius.

The error of each distribution obeys [1 + sqrt(2/pi) Kn_gas i theta.xi] y_l = f_l^eq {...}(alpha)
and [1 + Kn_photon i theta.Omega] y_R = (4 sigma_R / pi) alpha_Tv; the new macroscopic error is
the moment sum_l int phi_l y_l dxi + int phi_R y_R dOmega.  Velocity integrals use a Gauss-Hermite
product rule (fine along x, where the resolvent factor lives); angular integrals Gauss-Legendre in
mu = Omega_x with the azimuth integrated exactly.
"""

from __future__ import annotations

import numpy as np

NAMES = ["rho", "ux", "uy", "uz", "Tt", "Tr", "Tv", "eR", "qtx", "qty", "qtz", "qrx", "qry", "qrz", "qvx", "qvy", "qvz"]


def mason_A(d_r, d_v, Z_r, Z_v, Sc):
    """Heat-flux relaxation matrix in the Mason approximation (Sec. 2.1)."""
    return np.array([
        [2 / 3 + 5 / 6 * (d_r / ((3 + d_r) * Z_r) + d_v / ((3 + d_v) * Z_v)), -5 / (2 * (3 + d_r) * Z_r),
         -5 / (2 * (3 + d_v) * Z_v)],
        [-d_r / ((3 + d_r) * Z_r), Sc + 3 / (2 * (3 + d_r) * Z_r), 0.0],
        [-d_v / ((3 + d_v) * Z_v), 0.0, Sc + 3 / (2 * (3 + d_v) * Z_v)],
    ])


def _grids(nx=160, nt=6, nmu=64):
    x, W = np.polynomial.hermite.hermgauss(nx)
    xs, ws = np.sqrt(2) * x, np.sqrt(2) * W * np.exp(x * x)
    y, Wy = np.polynomial.hermite.hermgauss(nt)
    ys, wys = np.sqrt(2) * y, np.sqrt(2) * Wy * np.exp(y * y)
    X, Y, Z = np.meshgrid(xs, ys, ys, indexing="ij")
    WX, WY, WZ = np.meshgrid(ws, wys, wys, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    w = (WX * WY * WZ).ravel()
    mu, wm = np.polynomial.legendre.leggauss(nmu)
    return xi, w, mu, 2 * np.pi * wm


def product_grids(x, wx, mu, wmu, nt=6):
    """Velocity grid for the error integrals built from a 1D rule (x, wx) along the wave vector and exact
    Gauss-Hermite rules across it, with the ordinate rule (mu, wmu): the grids of a planar (reduced 1D)
    discrete-velocity run, whose transverse velocity integrals are exact."""
    y, Wy = np.polynomial.hermite.hermgauss(nt)
    ys, wys = np.sqrt(2) * y, np.sqrt(2) * Wy * np.exp(y * y)
    X, Y, Z = np.meshgrid(np.asarray(x, float), ys, ys, indexing="ij")
    WX, WY, WZ = np.meshgrid(np.asarray(wx, float), wys, wys, indexing="ij")
    return (np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1), (WX * WY * WZ).ravel(), np.asarray(mu, float),
            np.asarray(wmu, float))


def upwind_symbol(theta, h):
    """Fourier symbol of the first-order upwind difference for advection with speed v on a uniform grid of
    spacing h: for a mode exp(i theta x), v (1 - exp(-i theta h)) / h when v > 0 and v (exp(i theta h) - 1) / h
    when v < 0 (the continuous symbol is i theta v)."""
    def s(v):
        v = np.asarray(v, float)
        return np.where(v > 0, v * (1 - np.exp(-1j * theta * h)) / h, v * (np.exp(1j * theta * h) - 1) / h)
    return s


def _setup(theta, Kn_gas, Kn_photon, sigma_R, d_r, d_v, Z_r, Z_v, Sc, grids, symbol):
    xi, w, mu, wmu = grids if grids is not None else _grids()
    A = mason_A(d_r, d_v, Z_r, Z_v, Sc)
    x2 = (xi ** 2).sum(axis=1)
    sym = symbol if symbol is not None else (lambda v: 1j * theta * np.asarray(v, float))
    nv = xi.shape[0]
    # moment vectors phi_l (Eq. error_function_M_phi), shape [nv, 17]
    phi0 = np.zeros((nv, 17))
    phi0[:, 0] = 1
    phi0[:, 1:4] = xi
    phi0[:, 4] = x2 / 3 - 1
    phi0[:, 5] = -1
    phi0[:, 6] = -1
    phi0[:, 8:11] = (0.5 * x2 - 2.5)[:, None] * xi
    phi0[:, 11:14] = -d_r / 2 * xi
    phi0[:, 14:17] = -d_v / 2 * xi
    phi1 = np.zeros((nv, 17))
    phi1[:, 5] = 2 / d_r
    phi1[:, 11:14] = xi
    phi2 = np.zeros((nv, 17))
    phi2[:, 6] = 2 / d_v
    phi2[:, 14:17] = xi
    return dict(xi=xi, w=w, mu=mu, wmu=wmu, A=A, x2=x2, f0=(2 * np.pi) ** -1.5 * np.exp(-0.5 * x2),
                den=1 + np.sqrt(2 / np.pi) * Kn_gas * sym(xi[:, 0]), denR=1 + Kn_photon * sym(mu),
                phi0=phi0, phi1=phi1, phi2=phi2)


def _kinetic_errors(a, S, Kn_gas, Kn_photon, sigma_R, d_r, d_v, Z_r, Z_v):
    """Error of the three reduced distributions and of the intensity after one kinetic step (the transport
    inverted exactly, the reference distributions and the emission from the macroscopic error a)."""
    xi, A, x2, f0 = S["xi"], S["A"], S["x2"], S["f0"]
    ar = d_r / ((3 + d_r) * Z_r)
    av = d_v / ((3 + d_v) * Z_v)
    Pt = 0.5 * x2 - 1.5
    Pq = (2 / 15) * (0.5 * x2 - 2.5)
    qt, qr, qv = a[8:11], a[11:14], a[14:17]
    common = (a[0] + xi @ a[1:4] + a[4] * (1 - ar - av) * Pt + (ar * a[5] + av * a[6]) * Pt
              + Pq * (xi @ ((3 - 3 * A[0, 0]) * qt - 3 * A[0, 1] * qr - 3 * A[0, 2] * qv)))
    r0 = f0 * common
    r1 = (d_r / 2) * f0 * (common + 3 / ((3 + d_r) * Z_r) * a[4] + (1 - 3 / ((3 + d_r) * Z_r)) * a[5]
                           + (2 / d_r) * (xi @ (-A[1, 0] * qt + (1 - A[1, 1]) * qr - A[1, 2] * qv)))
    r2 = (d_v / 2) * f0 * (common + 3 / ((3 + d_v) * Z_v) * a[4] + (1 - 3 / ((3 + d_v) * Z_v)) * a[6]
                           + (2 / d_v) * (xi @ (-A[2, 0] * qt - A[2, 1] * qr + (1 - A[2, 2]) * qv)))
    r2 = r2 - np.sqrt(2 / np.pi) * Kn_gas / Kn_photon * f0 * (16 * sigma_R * a[6] - a[7])
    den = S["den"]
    return r0 / den, r1 / den, r2 / den, (4 * sigma_R / np.pi) * a[6] / S["denR"]


def cis_matrix(theta, Kn_gas, Kn_photon, sigma_R, d_r=2.0, d_v=1.0, Z_r=2.67, Z_v=26.7, Sc=0.8, grids=None,
               symbol=None):
    """C(theta) for a wave number theta along x.  `symbol(v)` replaces the transport symbol i theta v (e.g. the
    upwind_symbol of a discrete scheme)."""
    S = _setup(theta, Kn_gas, Kn_photon, sigma_R, d_r, d_v, Z_r, Z_v, Sc, grids, symbol)
    w, phi0, phi1, phi2 = S["w"], S["phi0"], S["phi1"], S["phi2"]
    C = np.zeros((17, 17), dtype=complex)
    for j in range(17):
        a = np.zeros(17)
        a[j] = 1.0
        y0, y1, y2, yR = _kinetic_errors(a, S, Kn_gas, Kn_photon, sigma_R, d_r, d_v, Z_r, Z_v)
        col = (w[:, None] * (phi0 * y0[:, None] + phi1 * y1[:, None] + phi2 * y2[:, None])).sum(axis=0)
        col[7] += (S["wmu"] * yR).sum()
        C[:, j] = col
    return C


def gsis_matrix(theta, Kn_gas, Kn_photon, sigma_R, d_r=2.0, d_v=1.0, Z_r=2.67, Z_v=26.7, Sc=0.8, grids=None):
    """Error propagation matrix L^-1 R of GSIS for a wave number theta along x (Sec. 4.3), derived here from the
    linearised steady synthetic equations (mass, momentum, total energy, e_r, e_v, e_R) closed by the
    constitutive relations with high-order terms: sigma^{k+1} = sigma_kin(h^{k+1/2}) - mu S(u^{k+1})
    + mu S(u^{k+1/2}) with S(u) = grad u + grad u^T - (2/3) div u I and mu = sqrt(2/pi) Kn_gas;
    q_l^{k+1} = q_l,kin + sum_m kappa_lm grad(T_m^{k+1/2} - T_m^{k+1}) with kappa = (mu / 2) A^-1 diag(5, d_r,
    d_v); q_R^{k+1} = q_R,kin + kappa_R grad(e_R^{k+1/2} - e_R^{k+1}) with kappa_R = Kn_photon / 3.  The
    kinetic half step is the conventional iteration's.  Unknowns in the order of NAMES; linearisation about
    rho = T = 1 at rest (e_R = 4 sigma_R)."""
    S = _setup(theta, Kn_gas, Kn_photon, sigma_R, d_r, d_v, Z_r, Z_v, Sc, grids, None)
    xi, w, phi0, phi1, phi2 = S["xi"], S["w"], S["phi0"], S["phi1"], S["phi2"]
    mu_v = np.sqrt(2 / np.pi) * Kn_gas
    kap = 0.5 * mu_v * np.linalg.inv(S["A"]) @ np.diag([5.0, d_r, d_v])
    kR = Kn_photon / 3.0
    k = 1.0 / Kn_photon
    cr = np.sqrt(np.pi / 2) / Kn_gas * 3 * d_r / (2 * (3 + d_r) * Z_r)
    cv = np.sqrt(np.pi / 2) / Kn_gas * 3 * d_v / (2 * (3 + d_v) * Z_v)
    it = 1j * theta
    iT = [4, 5, 6]  # T_t, T_r, T_v
    qx = [8, 11, 14]  # x components of q_t, q_r, q_v
    # L: the synthetic equations acting on the new macroscopic error
    L = np.zeros((17, 17), dtype=complex)
    L[0, 1] = it  # mass: div u = 0
    L[1, 0] = L[1, 4] = it  # x momentum: grad(rho + T_t) + div sigma
    L[1, 1] = mu_v * (4.0 / 3.0) * theta ** 2
    L[2, 2] = L[3, 3] = mu_v * theta ** 2  # transverse momentum (shear)
    for c in qx:  # total energy: div (q_t + q_r + q_v + q_R)
        L[4, c] = it
    L[4, 7] = kR * theta ** 2
    L[5, 11], L[5, 5], L[5, 4] = it, cr, -cr  # e_r: div q_r = c_r (T_t - T_r)
    L[6, 14], L[6, 6], L[6, 4] = it, cv + k * 16 * sigma_R, -cv  # e_v, with k (16 sigma_R T_v - e_R)
    L[6, 7] = -k
    L[7, 7], L[7, 6] = kR * theta ** 2 + k, -k * 16 * sigma_R  # e_R
    for li, base in enumerate((8, 11, 14)):  # q_l = q_l,kin + i theta sum_m kappa_lm (T_m^{1/2} - T_m)
        for a in range(3):
            L[base + a, base + a] = 1.0
        for m, tm in enumerate(iT):
            L[base, tm] = it * kap[li, m]
    R = np.zeros((17, 17), dtype=complex)
    for j in range(17):
        a = np.zeros(17)
        a[j] = 1.0
        y0, y1, y2, yR = _kinetic_errors(a, S, Kn_gas, Kn_photon, sigma_R, d_r, d_v, Z_r, Z_v)
        h = (w[:, None] * (phi0 * y0[:, None] + phi1 * y1[:, None] + phi2 * y2[:, None])).sum(axis=0)
        eR_h = (S["wmu"] * yR).sum()
        qR_h = (S["wmu"] * S["mu"] * yR).sum()
        x = xi[:, 0]
        sxx = (w * (x * x - S["x2"] / 3) * y0).sum()
        sxy = (w * x * xi[:, 1] * y0).sum()
        sxz = (w * x * xi[:, 2] * y0).sum()
        rhs = np.zeros(17, dtype=complex)
        rhs[1] = -it * sxx + mu_v * (4.0 / 3.0) * theta ** 2 * h[1]
        rhs[2] = -it * sxy + mu_v * theta ** 2 * h[2]
        rhs[3] = -it * sxz + mu_v * theta ** 2 * h[3]
        rhs[4] = -it * qR_h + kR * theta ** 2 * eR_h
        rhs[7] = -it * qR_h + kR * theta ** 2 * eR_h
        for li, base in enumerate((8, 11, 14)):
            rhs[base:base + 3] = h[base:base + 3]
            rhs[base] += it * sum(kap[li, m] * h[tm] for m, tm in enumerate(iT))
        R[:, j] = rhs
    return np.linalg.solve(L, R)


# the longitudinal moments of a wave along x (density, u_x, T_t, T_r, T_v, e_R, q_tx, q_rx, q_vx): the block of
# C(theta) that a planar (1D) run carries; the transverse moments decouple from it
LONGITUDINAL = [NAMES.index(n) for n in ("rho", "ux", "Tt", "Tr", "Tv", "eR", "qtx", "qrx", "qvx")]


def spectral_radius(M):
    return float(np.abs(np.linalg.eigvals(M)).max())


def gsis_emax(Kn_theta, ratio, sigma_R, Kn_gas=None, **gas):
    """Spectral radius of GSIS for Kn_gas * theta = Kn_theta and Kn_gas / Kn_photon = ratio."""
    Kn_gas = 1.0 if Kn_gas is None else Kn_gas
    theta = Kn_theta / Kn_gas
    return spectral_radius(gsis_matrix(theta, Kn_gas, Kn_gas / ratio, sigma_R, **gas))


def cis_emax(Kn_theta, ratio, sigma_R, Kn_gas=None, **gas):
    """Spectral radius of CIS for Kn_gas * theta = Kn_theta and Kn_gas / Kn_photon = ratio."""
    Kn_gas = 1.0 if Kn_gas is None else Kn_gas
    theta = Kn_theta / Kn_gas
    return spectral_radius(cis_matrix(theta, Kn_gas, Kn_gas / ratio, sigma_R, **gas))
