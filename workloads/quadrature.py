"""Velocity-space and angular quadratures (nodes and weights only).

Velocity grids are product grids in ``dimv`` dimensions with weights such
that ``sum_k w_k g(xi_k)`` approximates ``int g(xi) dxi``.  Ordinate sets
carry unit directions ``omega[no, 3]`` and weights summing to 4*pi.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class VelocityGrid:
    dimv: int
    xi: np.ndarray  # [nv, dimv]
    w: np.ndarray  # [nv]
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.w.shape[0])


@dataclass
class Ordinates:
    omega: np.ndarray  # [no, 3]
    w: np.ndarray  # [no]
    name: str = ""

    @property
    def no(self) -> int:
        return int(self.w.shape[0])


def _gh_1d(n: int):
    """Gauss-Hermite rule for int g(x) dx with nodes scaled to the weight exp(-x^2/2)."""
    x, W = np.polynomial.hermite.hermgauss(n)
    xi = np.sqrt(2.0) * x
    w = np.sqrt(2.0) * W * np.exp(x * x)
    return xi, w


def _product(nodes_1d, weights_1d, dimv):
    if dimv == 1:
        return nodes_1d[0][:, None].copy(), weights_1d[0].copy()
    grids = np.meshgrid(*nodes_1d, indexing="ij")
    wg = np.meshgrid(*weights_1d, indexing="ij")
    xi = np.stack([g.ravel() for g in grids], axis=1)
    w = np.prod(np.stack([g.ravel() for g in wg], axis=1), axis=1)
    return xi, w


def gauss_hermite_grid(n: int, dimv: int) -> VelocityGrid:
    """n^dimv Gauss-Hermite product grid; exact for exp(-|xi|^2/2) times polynomials of degree <= 2n-1 per axis."""
    x, w = _gh_1d(n)
    xi, ww = _product([x] * dimv, [w] * dimv, dimv)
    return VelocityGrid(dimv, np.ascontiguousarray(xi), np.ascontiguousarray(ww), f"GH{n}^{dimv}")


def _simpson_mapped(n: int, xmax: float, a: float):
    """Composite Simpson on s in [-1, 1] (n odd points), mapped xi = xmax (a s + (1-a) s^3)."""
    assert n % 2 == 1, "composite Simpson needs an odd number of points"
    s = np.linspace(-1.0, 1.0, n)
    hs = 2.0 / (n - 1)
    ws = np.ones(n)
    ws[1:-1:2] = 4.0
    ws[2:-1:2] = 2.0
    ws *= hs / 3.0
    xi = xmax * (a * s + (1 - a) * s ** 3)
    jac = xmax * (a + 3 * (1 - a) * s ** 2)
    return xi, ws * jac


def _trapezoid_mapped(n: int, xmax: float, a: float):
    """Composite trapezoid (two-point closed Newton-Cotes) on s in [-1, 1], mapped as above."""
    s = np.linspace(-1.0, 1.0, n)
    ws = np.full(n, 2.0 / (n - 1))
    ws[0] *= 0.5
    ws[-1] *= 0.5
    xi = xmax * (a * s + (1 - a) * s ** 3)
    jac = xmax * (a + 3 * (1 - a) * s ** 2)
    return xi, ws * jac


def newton_cotes_grid(n: int, dimv: int, xmax: float, a: float = 0.3) -> VelocityGrid:
    """Nonuniform product grid: composite Newton-Cotes on a cubic map that clusters nodes near 0.

    Odd ``n`` uses composite Simpson, even ``n`` the composite trapezoid rule
    (spectrally accurate here because the integrands decay to zero at both ends).
    """
    if n % 2 == 1:
        x, w = _simpson_mapped(n, xmax, a)
    else:
        x, w = _trapezoid_mapped(n, xmax, a)
    xi, ww = _product([x] * dimv, [w] * dimv, dimv)
    return VelocityGrid(dimv, np.ascontiguousarray(xi), np.ascontiguousarray(ww), f"NC{n}^{dimv}_x{xmax}")


def uniform_box_grid(n: int, ranges) -> VelocityGrid:
    """n points per axis, uniform on each axis's [lo, hi] with trapezoid weights (spectrally accurate for a
    Maxwellian whose thermal speed is comparable to or above the spacing and whose tails fall inside the
    box).  ``ranges`` gives (lo, hi) per axis; a box shifted along the free stream resolves both the cold
    free stream and the hot gas at rest behind a shock with the same node count."""
    xs, ws = [], []
    for lo, hi in ranges:
        x = np.linspace(lo, hi, n)
        w = np.full(n, (hi - lo) / (n - 1))
        w[0] *= 0.5
        w[-1] *= 0.5
        xs.append(x)
        ws.append(w)
    dimv = len(ranges)
    xi, ww = _product(xs, ws, dimv)
    return VelocityGrid(dimv, np.ascontiguousarray(xi), np.ascontiguousarray(ww), f"U{n}^{dimv}")


def spherical_grid(n_r: int, n_theta: int, n_phi: int, radius: float, center=(0.0, 0.0, 0.0)) -> VelocityGrid:
    """Unstructured 3D velocity set in a ball of the given radius (the paper's capsule uses an unstructured
    spherical velocity grid, Sec. 7.4): Gauss-Legendre nodes in |xi - center| on [0, radius] (weight r^2 dr),
    Gauss-Legendre in cos(theta), uniform azimuths; n_r n_theta n_phi points, not a tensor product in
    Cartesian components.  Exact for polynomials of degree < 2 n_r - 2 in r times degree < 2 n_theta in
    cos(theta) and < n_phi in the azimuth, so a Maxwellian well inside the ball is integrated to near
    round-off."""
    xr, wr = np.polynomial.legendre.leggauss(n_r)
    r = 0.5 * radius * (xr + 1)
    wr = 0.5 * radius * wr * r * r
    mu, wmu = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    R, MU, PH = np.meshgrid(r, mu, phi, indexing="ij")
    W = wr[:, None, None] * wmu[None, :, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, None, :]
    st = np.sqrt(1 - MU * MU)
    xi = np.stack([R * MU, R * st * np.cos(PH), R * st * np.sin(PH)], axis=-1).reshape(-1, 3)
    xi = xi + np.asarray(center, dtype=np.float64)[None, :]
    return VelocityGrid(3, np.ascontiguousarray(xi), np.ascontiguousarray(W.reshape(-1)),
                        f"S{n_r}x{n_theta}x{n_phi}_r{radius}")


def ordinates_slab(n: int) -> Ordinates:
    """Plane-parallel set: Gauss-Legendre in mu = cos(theta), azimuth integrated (weight 2 pi w)."""
    mu, w = np.polynomial.legendre.leggauss(n)
    om = np.stack([mu, np.sqrt(1 - mu * mu), np.zeros_like(mu)], axis=1)
    return Ordinates(np.ascontiguousarray(om), np.ascontiguousarray(2 * np.pi * w), f"GL{n}")


def ordinates_hemisphere(n_theta: int, n_phi: int) -> Ordinates:
    """2D set with mirror symmetry in z: Gauss-Legendre in cos(theta) on [0, 1] times uniform azimuth.

    Weights count both hemispheres (sum = 4 pi).
    """
    mu, wm = np.polynomial.legendre.leggauss(n_theta)
    mu = 0.5 * (mu + 1.0)
    wm = 0.5 * wm
    phi = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    WM, _ = np.meshgrid(wm, phi, indexing="ij")
    st = np.sqrt(1 - M ** 2)
    om = np.stack([(st * np.cos(P)).ravel(), (st * np.sin(P)).ravel(), M.ravel()], axis=1)
    w = 2.0 * (WM * (2 * np.pi / n_phi)).ravel()
    return Ordinates(np.ascontiguousarray(om), np.ascontiguousarray(w), f"H{n_theta}x{n_phi}")


def ordinates_sphere(n_theta: int, n_phi: int) -> Ordinates:
    """Full-sphere set: Gauss-Legendre in cos(theta) on [-1, 1] times uniform azimuth (sum = 4 pi)."""
    mu, wm = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    WM, _ = np.meshgrid(wm, phi, indexing="ij")
    st = np.sqrt(1 - M ** 2)
    om = np.stack([(st * np.cos(P)).ravel(), (st * np.sin(P)).ravel(), M.ravel()], axis=1)
    w = (WM * (2 * np.pi / n_phi)).ravel()
    return Ordinates(np.ascontiguousarray(om), np.ascontiguousarray(w), f"S{n_theta}x{n_phi}")
