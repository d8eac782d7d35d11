"""Seeded synthetic inputs shared by the HIP path and the oracle.

This package only builds inputs: meshes (geometry and boundary tags),
velocity and ordinate quadratures, and case parameter sets.  It holds none
of the kinetic or macroscopic arithmetic of the method; both the product
path and the oracle receive what it builds as plain arrays.
"""

from .mesh import Mesh, mesh_1d, mesh_cavity, mesh_cavity_mirror, mesh_annulus, mesh_periodic_1d, mesh_capsule, mesh_patch  # noqa: F401
from .quadrature import (  # noqa: F401
    VelocityGrid,
    Ordinates,
    gauss_hermite_grid,
    newton_cotes_grid,
    ordinates_slab,
    ordinates_hemisphere,
    ordinates_sphere,
    uniform_box_grid,
    spherical_grid,
)
from .cases import (  # noqa: F401
    Gas,
    Flow,
    Case,
    BC_WALL,
    BC_FARFIELD,
    case_fourier_1d,
    case_cavity,
    case_cylinder,
    case_capsule,
    case_normal_shock,
    rankine_hugoniot,
    warmstart_case_params,
    warmstart_cavity_params,
    warmstart_cylinder_params,
    warmstart_c5_params,
    case_c5_cylinder,
    case_patch,
)
