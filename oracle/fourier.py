"""Linear Fourier analysis of the conventional iteration (CIS) for the radiative kinetic model.

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


def cis_matrix(theta, Kn_gas, Kn_photon, sigma_R, d_r=2.0, d_v=1.0, Z_r=2.67, Z_v=26.7, Sc=0.8, grids=None,
               symbol=None):
    """C(theta) for a wave number theta along x.  `symbol(v)` replaces the transport symbol i theta v (e.g. the
    upwind_symbol of a discrete scheme)."""
    xi, w, mu, wmu = grids if grids is not None else _grids()
    A = mason_A(d_r, d_v, Z_r, Z_v, Sc)
    x2 = (xi ** 2).sum(axis=1)
    f0 = (2 * np.pi) ** -1.5 * np.exp(-0.5 * x2)
    sym = symbol if symbol is not None else (lambda v: 1j * theta * np.asarray(v, float))
    den = 1 + np.sqrt(2 / np.pi) * Kn_gas * sym(xi[:, 0])
    denR = 1 + Kn_photon * sym(mu)
    ar = d_r / ((3 + d_r) * Z_r)
    av = d_v / ((3 + d_v) * Z_v)
    Pt = 0.5 * x2 - 1.5
    Pq = (2 / 15) * (0.5 * x2 - 2.5)
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
    C = np.zeros((17, 17), dtype=complex)
    for j in range(17):
        a = np.zeros(17)
        a[j] = 1.0
        qt, qr, qv = a[8:11], a[11:14], a[14:17]
        common = (a[0] + xi @ a[1:4] + a[4] * (1 - ar - av) * Pt + (ar * a[5] + av * a[6]) * Pt
                  + Pq * (xi @ ((3 - 3 * A[0, 0]) * qt - 3 * A[0, 1] * qr - 3 * A[0, 2] * qv)))
        r0 = f0 * common
        r1 = (d_r / 2) * f0 * (common + 3 / ((3 + d_r) * Z_r) * a[4] + (1 - 3 / ((3 + d_r) * Z_r)) * a[5]
                               + (2 / d_r) * (xi @ (-A[1, 0] * qt + (1 - A[1, 1]) * qr - A[1, 2] * qv)))
        r2 = (d_v / 2) * f0 * (common + 3 / ((3 + d_v) * Z_v) * a[4] + (1 - 3 / ((3 + d_v) * Z_v)) * a[6]
                               + (2 / d_v) * (xi @ (-A[2, 0] * qt - A[2, 1] * qr + (1 - A[2, 2]) * qv)))
        r2 = r2 - np.sqrt(2 / np.pi) * Kn_gas / Kn_photon * f0 * (16 * sigma_R * a[6] - a[7])
        y0, y1, y2 = r0 / den, r1 / den, r2 / den
        yR = (4 * sigma_R / np.pi) * a[6] / denR
        col = (w[:, None] * (phi0 * y0[:, None] + phi1 * y1[:, None] + phi2 * y2[:, None])).sum(axis=0)
        col[7] += (wmu * yR).sum()
        C[:, j] = col
    return C


# the longitudinal moments of a wave along x (density, u_x, T_t, T_r, T_v, e_R, q_tx, q_rx, q_vx): the block of
# C(theta) that a planar (1D) run carries; the transverse moments decouple from it
LONGITUDINAL = [NAMES.index(n) for n in ("rho", "ux", "Tt", "Tr", "Tv", "eR", "qtx", "qrx", "qvx")]


def spectral_radius(M):
    return float(np.abs(np.linalg.eigvals(M)).max())


def cis_emax(Kn_theta, ratio, sigma_R, Kn_gas=None, **gas):
    """Spectral radius of CIS for Kn_gas * theta = Kn_theta and Kn_gas / Kn_photon = ratio."""
    Kn_gas = 1.0 if Kn_gas is None else Kn_gas
    theta = Kn_theta / Kn_gas
    return spectral_radius(cis_matrix(theta, Kn_gas, Kn_gas / ratio, sigma_R, **gas))
