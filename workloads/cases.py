"""Case definitions: gas and flow parameters, boundary tags and initial fields.

Each builder returns a :class:`Case` holding only inputs.  Parameter values
follow the paper's test section where it gives them (gas constants,
collision numbers, viscosity index) and the synthetic workload recipes
otherwise; every random draw is seeded.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import Mesh, mesh_1d, mesh_cavity, mesh_annulus, mesh_capsule
from .quadrature import (
    VelocityGrid,
    Ordinates,
    gauss_hermite_grid,
    newton_cotes_grid,
    ordinates_slab,
    ordinates_hemisphere,
    ordinates_sphere,
    uniform_box_grid,
)

BC_WALL = 0  # diffuse, fully accommodating wall; black for radiation
BC_FARFIELD = 1  # prescribed equilibrium state on incoming characteristics


@dataclass
class Gas:
    d_r: float = 2.0
    d_v: float = 1.16
    Z_r: float = 2.67
    Z_v: float = 26.7
    omega: float = 0.74
    Sc: float = 0.8
    sigma_R: float = 0.01
    # characteristic vibrational temperature (units of the reference temperature): d_v(T) = 2 (Tv_ref / T) /
    # (exp(Tv_ref / T) - 1) (Sec. 2.1); 0 keeps the constant d_v above
    Tv_ref: float = 0.0

    @property
    def gamma(self) -> float:
        return (5 + self.d_r + self.d_v) / (3 + self.d_r + self.d_v)


@dataclass
class Flow:
    Kn_gas: float = 0.1
    k_eff: float = 1.0  # = 1 / Kn_photon (optical thickness per reference length); 0 = no absorption
    rho_inf: float = 1.0
    T_inf: float = 1.0
    u_inf: tuple = (0.0, 0.0, 0.0)


@dataclass
class Case:
    name: str
    mesh: Mesh
    vgrid: VelocityGrid
    ords: Ordinates
    gas: Gas
    flow: Flow
    bcs: list  # list of dict(kind, rho, T, u=(ux, uy, uz))
    init_rho: np.ndarray
    init_u: np.ndarray  # [nc, dim]
    init_T: np.ndarray
    meta: dict = field(default_factory=dict)

    def bc_arrays(self):
        kind = np.array([b["kind"] for b in self.bcs], dtype=np.int32)
        rho = np.array([b.get("rho", 1.0) for b in self.bcs], dtype=np.float64)
        T = np.array([b["T"] for b in self.bcs], dtype=np.float64)
        u = np.array([list(b.get("u", (0.0, 0.0, 0.0))) for b in self.bcs], dtype=np.float64)
        return kind, rho, T, u


def _uniform_init(mesh: Mesh, rho: float, u, T: float):
    nc, dim = mesh.nc, mesh.dim
    return (np.full(nc, rho), np.tile(np.asarray(u[:dim], dtype=np.float64), (nc, 1)), np.full(nc, T))


def case_fourier_1d(n: int = 64, nv: int = 48, no: int = 16, Kn: float = 0.1, tau_opt: float = 1.0,
                    Z_r: float = 5.0, Z_v: float = 50.0, sigma_R: float = 0.01, T_left: float = 1.0,
                    T_right: float = 2.0, T0: float = 1.5) -> Case:
    """Planar radiative Fourier flow between diffuse black walls at rest."""
    mesh = mesh_1d(n, 0.0, 1.0, 0, 1)
    gas = Gas(Z_r=Z_r, Z_v=Z_v, sigma_R=sigma_R)
    flow = Flow(Kn_gas=Kn, k_eff=tau_opt, rho_inf=1.0, T_inf=T0)
    bcs = [dict(kind=BC_WALL, T=T_left), dict(kind=BC_WALL, T=T_right)]
    r, u, T = _uniform_init(mesh, 1.0, (0.0, 0.0, 0.0), T0)
    return Case(f"fourier1d_n{n}_Kn{Kn}_tau{tau_opt}", mesh, gauss_hermite_grid(nv, 1), ordinates_slab(no),
                gas, flow, bcs, r, u, T)


def case_cavity(Kn: float = 0.1, tau_opt: float = 1.0, h: float = 0.0095, nvx: int = 32, n_theta: int = 4,
                n_phi: int = 8, sigma_R: float = 0.005, u_lid: float = 0.18, T_lid: float = 3.0,
                seed: int = 0, mesh: Mesh | None = None) -> Case:
    """Lid-driven, heated cavity with a concentric square obstacle, unstructured triangles."""
    mesh = mesh if mesh is not None else mesh_cavity(h=h, seed=seed)
    gas = Gas(sigma_R=sigma_R)
    flow = Flow(Kn_gas=Kn, k_eff=tau_opt, rho_inf=1.0, T_inf=1.0)
    bcs = [dict(kind=BC_WALL, T=1.0), dict(kind=BC_WALL, T=T_lid, u=(u_lid, 0.0, 0.0))]
    r, u, T = _uniform_init(mesh, 1.0, (0.0, 0.0, 0.0), 1.0)
    return Case(f"cavity_nc{mesh.nc}_Kn{Kn}_tau{tau_opt}", mesh, gauss_hermite_grid(nvx, 2),
                ordinates_hemisphere(n_theta, n_phi), gas, flow, bcs, r, u, T)


def case_cylinder(Kn: float = 0.01, tau_opt: float = 1.0, Ma: float = 5.0, nvx: int = 64, xmax: float = 12.0,
                  n_theta: int = 4, n_phi: int = 16, sigma_R: float = 0.1, T_w: float = 2.0,
                  n_theta_mesh: int = 256, n_r_mesh: int = 80, seed: int = 1, mesh: Mesh | None = None) -> Case:
    """Hypersonic flow past a cylinder of radius 1 in an annulus of outer radius 6."""
    mesh = mesh if mesh is not None else mesh_annulus(n_theta=n_theta_mesh, n_r=n_r_mesh, seed=seed)
    gas = Gas(sigma_R=sigma_R)
    u_inf = Ma * np.sqrt(gas.gamma * 1.0)
    flow = Flow(Kn_gas=Kn, k_eff=tau_opt, rho_inf=1.0, T_inf=1.0, u_inf=(u_inf, 0.0, 0.0))
    bcs = [dict(kind=BC_WALL, T=T_w), dict(kind=BC_FARFIELD, rho=1.0, T=1.0, u=(u_inf, 0.0, 0.0))]
    r, u, T = _uniform_init(mesh, 1.0, (u_inf, 0.0, 0.0), 1.0)
    return Case(f"cylinder_nc{mesh.nc}_Ma{Ma}_Kn{Kn}_tau{tau_opt}", mesh, newton_cotes_grid(nvx, 2, xmax),
                ordinates_hemisphere(n_theta, n_phi), gas, flow, bcs, r, u, T, meta=dict(Ma=Ma))


def case_capsule(Kn: float = 0.01, tau_opt: float = 1.0, Ma: float = 10.0, nvx: int = 24, xmax: float = 20.0,
                 n_theta: int = 8, n_phi: int = 12, sigma_R: float = 0.045, T_w: float = 2.0,
                 mesh_kw: dict | None = None, vgrid: str = "nc") -> Case:
    """Hypersonic flow past a blunt capsule (spherical cap + 33 degree cone), tetrahedra, full 3D velocities.
    vgrid "nc": Newton-Cotes grid on [-xmax, xmax]^3 clustered at 0; "box": uniform nvx^3 grid on
    [-15, u_inf + 9] x [-15, 15]^2, which resolves the T = 1 free stream (spacing ~1.5 at Ma 10) and hot gas at
    rest (stagnation temperature ~17 at Ma 10, thermal speed ~4)."""
    mesh = mesh_capsule(**(mesh_kw or {}))
    gas = Gas(sigma_R=sigma_R)
    u_inf = Ma * np.sqrt(gas.gamma * 1.0)
    if vgrid == "box":
        vg = uniform_box_grid(nvx, [(-15.0, u_inf + 9.0), (-15.0, 15.0), (-15.0, 15.0)])
    else:
        vg = newton_cotes_grid(nvx, 3, xmax)
    flow = Flow(Kn_gas=Kn, k_eff=tau_opt, rho_inf=1.0, T_inf=1.0, u_inf=(u_inf, 0.0, 0.0))
    bcs = [dict(kind=BC_WALL, T=T_w), dict(kind=BC_FARFIELD, rho=1.0, T=1.0, u=(u_inf, 0.0, 0.0))]
    r, u, T = _uniform_init(mesh, 1.0, (u_inf, 0.0, 0.0), 1.0)
    return Case(f"capsule_nc{mesh.nc}_Ma{Ma}_Kn{Kn}", mesh, vg, ordinates_sphere(n_theta, n_phi), gas, flow, bcs, r,
                u, T, meta=dict(Ma=Ma))


def rankine_hugoniot(Ma: float, gamma: float):
    """Downstream (rho_d, u_d, T_d) of a normal shock with upstream rho = 1, T = 1, u = sqrt(gamma) Ma,
    for a gas of constant specific-heat ratio gamma (the jump relations stated with the normal-shock case
    of Sec. 4.1)."""
    u_u = np.sqrt(gamma) * Ma
    rho_d = (gamma + 1) * Ma ** 2 / (2 + (gamma - 1) * Ma ** 2)
    T_d = (2 + (gamma - 1) * Ma ** 2) * (2 * gamma * Ma ** 2 - (gamma - 1)) / ((gamma + 1) ** 2 * Ma ** 2)
    return rho_d, u_u / rho_d, T_d


def case_normal_shock(Ma: float = 5.0, Z_r: float = 2.6, Z_v: float = 26.0, x0: float = -60.0, x1: float = 140.0,
                      dx: float = 0.25, nv: int = 64, xmax: float = 15.0, no: int = 48, Kn_photon: float = 10.0,
                      sigma_R: float = 0.01) -> Case:
    """Planar normal shock (Sec. 4.1): Kn_gas = 5 pi / 16 (reference length from the upstream mean free
    path), upstream rho = 1, T = 1, u = sqrt(gamma) Ma and the Rankine-Hugoniot downstream state as fixed
    far-field equilibria at the two ends, initial discontinuity at x = 0 with both sides at equilibrium
    (I = sigma_R T^4 / pi).  Uniform mesh of spacing dx on [x0, x1]; uniform 1D velocity grid on
    [-xmax, xmax] (the reduced model is exact for a planar flow, so only the xi_x points of the paper's
    reduced 2D grid are needed); Gauss-Legendre ordinates in mu = cos(theta)."""
    n = int(round((x1 - x0) / dx))
    mesh = mesh_1d(n, x0, x1, 0, 1)
    gas = Gas(Z_r=Z_r, Z_v=Z_v, sigma_R=sigma_R)
    g = gas.gamma
    u_u = np.sqrt(g) * Ma
    rho_d, u_d, T_d = rankine_hugoniot(Ma, g)
    flow = Flow(Kn_gas=5 * np.pi / 16, k_eff=1.0 / Kn_photon, rho_inf=1.0, T_inf=1.0, u_inf=(u_u, 0.0, 0.0))
    bcs = [dict(kind=BC_FARFIELD, rho=1.0, T=1.0, u=(u_u, 0.0, 0.0)),
           dict(kind=BC_FARFIELD, rho=rho_d, T=T_d, u=(u_d, 0.0, 0.0))]
    x = mesh.ctr[:, 0]
    up = x <= 0.0
    r = np.where(up, 1.0, rho_d)
    u = np.where(up, u_u, u_d)[:, None]
    T = np.where(up, 1.0, T_d)
    return Case(f"shock_Ma{Ma}_Z{Z_r}_{Z_v}_n{n}", mesh, newton_cotes_grid(nv, 1, xmax, a=1.0), ordinates_slab(no),
                gas, flow, bcs, r, u, T, meta=dict(Ma=Ma, rho_d=rho_d, u_d=u_d, T_d=T_d))


def warmstart_case_params(n: int = 256, seed: int = 2):
    """Seeded (Ma, Kn, optical thickness) draws for the warm-start data set."""
    rng = np.random.default_rng(seed)
    Ma = rng.uniform(3.0, 10.0, n)
    Kn = 10 ** rng.uniform(-3.0, 0.0, n)
    tau = 10 ** rng.uniform(-2.0, 2.0, n)
    return np.stack([Ma, Kn, tau], axis=1)


def warmstart_cavity_params(n: int = 32, seed: int = 2):
    """Seeded (Kn, optical thickness, lid speed) draws for warm-start training sets on the cavity family:
    Kn log-uniform in [0.03, 0.3], optical thickness log-uniform in [0.3, 3], lid speed uniform in
    [0.1, 0.3]."""
    rng = np.random.default_rng(seed)
    Kn = 10 ** rng.uniform(np.log10(0.03), np.log10(0.3), n)
    tau = 10 ** rng.uniform(np.log10(0.3), np.log10(3.0), n)
    ulid = rng.uniform(0.1, 0.3, n)
    return np.stack([Kn, tau, ulid], axis=1)


def warmstart_c5_params(n: int = 256, seed: int = 2, log10_Kn=(-2.0, 0.0), log10_tau=(-1.0, 1.0)):
    """Seeded (Mach, Kn, optical thickness) draws of the warm-start data set of hypersonic cylinders: Mach
    uniform in [3, 10], Kn and optical thickness log-uniform in the given decades (default Kn in [1e-2, 1],
    optical thickness in [0.1, 10]; the wider [1e-3, 1] x [1e-2, 1e2] puts most draws where the Mach
    continuation from the free stream does not reach a steady state on this mesh)."""
    rng = np.random.default_rng(seed)
    Ma = rng.uniform(3.0, 10.0, n)
    Kn = 10 ** rng.uniform(log10_Kn[0], log10_Kn[1], n)
    tau = 10 ** rng.uniform(log10_tau[0], log10_tau[1], n)
    return np.stack([Ma, Kn, tau], axis=1)


def case_c5_cylinder(Ma: float, Kn: float, tau: float, mesh: Mesh | None = None) -> Case:
    """One cylinder of the warm-start data set: the annulus at 180 x 56 points (20,160 triangles), 64 x 64
    Newton-Cotes velocities up to |xi| = 18 (the Mach 10 free stream at u = 11.5 with room for its thermal
    spread), 64 ordinates, sigma_R = 0.1."""
    mesh = mesh if mesh is not None else mesh_annulus(n_theta=180, n_r=56, seed=1)
    return case_cylinder(mesh=mesh, Ma=Ma, Kn=Kn, tau_opt=tau, nvx=64, xmax=18.0, n_theta=4, n_phi=16,
                         sigma_R=0.1)


def warmstart_cylinder_params(n: int = 16, seed: int = 3):
    """Seeded (Mach, Kn, optical thickness) draws for warm-start training sets on the cylinder family:
    Mach uniform in [3, 5], Kn log-uniform in [0.01, 0.1], optical thickness log-uniform in [0.3, 3]."""
    rng = np.random.default_rng(seed)
    Ma = rng.uniform(3.0, 5.0, n)
    Kn = 10 ** rng.uniform(np.log10(0.01), np.log10(0.1), n)
    tau = 10 ** rng.uniform(np.log10(0.3), np.log10(3.0), n)
    return np.stack([Ma, Kn, tau], axis=1)


def case_patch(case: Case, seeds, rings: int):
    """The case restricted to the cells within `rings` face-neighbour steps of the seed cells (mesh_patch):
    same grids, gas, flow and boundary tags, plus one far-field condition at the free-stream state on the
    faces that cut the patch from the rest of the mesh.  Returns (patch case, kept cell indices, the seeds'
    patch indices).  A stage whose result at a cell depends only on cells within r steps agrees on the two
    meshes at every seed when rings >= r (the cut faces only reach cells within r steps of them)."""
    from .mesh import mesh_patch

    pm, cells, seeds_local = mesh_patch(case.mesh, seeds, rings)
    fl = case.flow
    bcs = list(case.bcs) + [dict(kind=BC_FARFIELD, rho=fl.rho_inf, T=fl.T_inf, u=tuple(fl.u_inf))]
    out = Case(f"{case.name}_patch{pm.nc}", pm, case.vgrid, case.ords, case.gas, case.flow, bcs,
               case.init_rho[cells].copy(), case.init_u[cells].copy(), case.init_T[cells].copy(), dict(case.meta))
    return out, cells, seeds_local
