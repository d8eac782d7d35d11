"""Input generators (no GPU): cell orderings, the warm-start data-set draws."""

import numpy as np

from workloads import warmstart_c5_params
from workloads.mesh import _hilbert_order, _morton_order, mesh_capsule


def test_hilbert_order_visits_lattice_neighbours():
    """On an 8^3 integer lattice the Hilbert order steps to an adjacent point every time (the Z order jumps)."""
    g = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    g = g.astype(float)
    p = _hilbert_order(g, bits=3)
    assert sorted(p.tolist()) == list(range(512))
    assert (np.abs(np.diff(g[p], axis=0)).sum(axis=1) == 1).all()
    assert np.abs(np.diff(g[_morton_order(g)], axis=0)).sum(axis=1).max() > 1


def test_capsule_orders_describe_the_same_mesh():
    """Morton and Hilbert numberings of the capsule are permutations of the same cells."""
    a = mesh_capsule(n_s=4, n_phi=6, n_r=3)
    b = mesh_capsule(n_s=4, n_phi=6, n_r=3, cell_order="hilbert")
    assert a.nc == b.nc and a.nf == b.nf
    assert np.allclose(np.sort(a.vol), np.sort(b.vol))
    assert np.allclose(a.vol.sum(), b.vol.sum())


def test_c5_draws_cover_the_stated_ranges():
    P = warmstart_c5_params(256, seed=2)
    assert P.shape == (256, 3)
    assert P[:, 0].min() >= 3 and P[:, 0].max() <= 10
    assert P[:, 1].min() >= 1e-2 and P[:, 1].max() <= 1
    assert P[:, 2].min() >= 0.1 and P[:, 2].max() <= 10
    assert np.array_equal(P, warmstart_c5_params(256, seed=2))
