"""Seeded unstructured meshes (geometry and boundary tags only).

A mesh is a face-based finite-volume description:

* ``vol[nc]``, ``ctr[nc, dim]``: cell volumes (lengths in 1D, areas in 2D) and centroids;
* ``face_cells[nf, 2]``: the two cells of each face.  The first entry is always
  a cell; the second is a cell or, for a boundary face, ``-(1 + bc_id)``;
* ``face_n[nf, dim]``: unit normal pointing from ``face_cells[:, 0]`` to the other side;
* ``face_area[nf]``, ``face_ctr[nf, dim]``.

Cells are emitted in Morton (Z-curve) order of their centroids so that cells
that are close in space are close in memory.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    dim: int
    vol: np.ndarray
    ctr: np.ndarray
    face_cells: np.ndarray
    face_n: np.ndarray
    face_area: np.ndarray
    face_ctr: np.ndarray
    name: str = ""
    period: float = 0.0  # > 0: periodic along x with this length (mesh_periodic_1d)

    @property
    def nc(self) -> int:
        return int(self.vol.shape[0])

    @property
    def nf(self) -> int:
        return int(self.face_area.shape[0])

    def boundary_faces(self) -> np.ndarray:
        return np.nonzero(self.face_cells[:, 1] < 0)[0]

    def check(self) -> None:
        """Geometric sanity: closed cells (sum of n*S over each cell's faces vanishes)."""
        acc = np.zeros((self.nc, self.dim))
        L = self.face_cells[:, 0]
        R = self.face_cells[:, 1]
        nS = self.face_n * self.face_area[:, None]
        np.add.at(acc, L, nS)
        inner = R >= 0
        np.add.at(acc, R[inner], -nS[inner])
        scale = self.face_area.max()
        assert np.abs(acc).max() < 1e-9 * scale, np.abs(acc).max()
        assert (self.vol > 0).all()
        assert np.allclose(np.linalg.norm(self.face_n, axis=1), 1.0)


def _morton_order(ctr: np.ndarray) -> np.ndarray:
    """Permutation that sorts points along a Z-order curve (21 bits per axis)."""
    dim = ctr.shape[1]
    lo = ctr.min(axis=0)
    span = np.maximum(ctr.max(axis=0) - lo, 1e-300)
    q = np.floor((ctr - lo) / span * ((1 << 20) - 1)).astype(np.uint64)
    code = np.zeros(ctr.shape[0], dtype=np.uint64)
    for bit in range(21):
        for a in range(dim):
            code |= ((q[:, a] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(bit * dim + a)
    return np.argsort(code, kind="stable")


def _hilbert_order(ctr: np.ndarray, bits: int = 16) -> np.ndarray:
    """Permutation that sorts points along a Hilbert curve (Skilling's transpose form of the Hilbert index,
    `bits` bits per axis): unlike the Z-order curve, consecutive points of the curve are always adjacent."""
    dim = ctr.shape[1]
    lo = ctr.min(axis=0)
    span = np.maximum(ctr.max(axis=0) - lo, 1e-300)
    X = [np.floor((ctr[:, a] - lo[a]) / span[a] * ((1 << bits) - 1)).astype(np.uint64) for a in range(dim)]
    M = np.uint64(1 << (bits - 1))
    Q = M
    while Q > 1:  # inverse undo of the excess work
        P = Q - np.uint64(1)
        for i in range(dim):
            hit = (X[i] & Q) != 0
            X[0] = np.where(hit, X[0] ^ P, X[0])
            t = np.where(hit, np.uint64(0), (X[0] ^ X[i]) & P)
            X[0] ^= t
            X[i] ^= t
        Q >>= np.uint64(1)
    for i in range(1, dim):  # Gray encode
        X[i] ^= X[i - 1]
    t = np.zeros_like(X[0])
    Q = M
    while Q > 1:
        t = np.where((X[dim - 1] & Q) != 0, t ^ (Q - np.uint64(1)), t)
        Q >>= np.uint64(1)
    for i in range(dim):
        X[i] ^= t
    key = np.zeros(ctr.shape[0], dtype=np.uint64)
    for b in range(bits - 1, -1, -1):
        for i in range(dim):
            key = (key << np.uint64(1)) | ((X[i] >> np.uint64(b)) & np.uint64(1))
    return np.argsort(key, kind="stable")


def _renumber(dim, vol, ctr, face_cells, face_n, face_area, face_ctr, name, order="morton"):
    perm = _hilbert_order(ctr) if order == "hilbert" else _morton_order(ctr)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    fc = face_cells.copy()
    fc[:, 0] = inv[face_cells[:, 0]]
    inner = face_cells[:, 1] >= 0
    fc[inner, 1] = inv[face_cells[inner, 1]]
    # faces sorted by their first cell, for locality as well
    fperm = np.lexsort((np.where(fc[:, 1] >= 0, fc[:, 1], 1 << 40), fc[:, 0]))
    m = Mesh(
        dim,
        np.ascontiguousarray(vol[perm], dtype=np.float64),
        np.ascontiguousarray(ctr[perm], dtype=np.float64),
        np.ascontiguousarray(fc[fperm], dtype=np.int64),
        np.ascontiguousarray(face_n[fperm], dtype=np.float64),
        np.ascontiguousarray(face_area[fperm], dtype=np.float64),
        np.ascontiguousarray(face_ctr[fperm], dtype=np.float64),
        name,
    )
    m.check()
    return m


def mesh_1d(n: int, x0: float = 0.0, x1: float = 1.0, bc_left: int = 0, bc_right: int = 1) -> Mesh:
    """Uniform 1D mesh of ``n`` cells on [x0, x1] with boundary tags at both ends."""
    xs = np.linspace(x0, x1, n + 1)
    vol = np.diff(xs)
    ctr = (0.5 * (xs[1:] + xs[:-1]))[:, None]
    fc = np.zeros((n + 1, 2), dtype=np.int64)
    fn = np.ones((n + 1, 1))
    fc[0] = (0, -(1 + bc_left))
    fn[0, 0] = -1.0
    for i in range(1, n):
        fc[i] = (i - 1, i)
    fc[n] = (n - 1, -(1 + bc_right))
    fa = np.ones(n + 1)
    fctr = xs[:, None].copy()
    m = Mesh(1, vol, ctr, fc, fn, fa, fctr, f"line{n}")
    m.check()
    return m


def _tri_mesh_from_points(pts: np.ndarray, keep_tri, classify_edge, name: str) -> Mesh:
    from scipy.spatial import Delaunay

    return _tri_mesh_from_simplices(pts, Delaunay(pts).simplices, keep_tri, classify_edge, name)


def _tri_mesh_from_simplices(pts: np.ndarray, simp: np.ndarray, keep_tri, classify_edge, name: str) -> Mesh:
    cen = pts[simp].mean(axis=1)
    keep = keep_tri(cen)
    simp = simp[keep]
    a, b, c = pts[simp[:, 0]], pts[simp[:, 1]], pts[simp[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    good = np.abs(area2) > 1e-14
    simp = simp[good]
    area2 = area2[good]
    nc = simp.shape[0]
    vol = 0.5 * np.abs(area2)
    ctr = pts[simp].mean(axis=1)
    # edges
    e = np.concatenate([simp[:, [0, 1]], simp[:, [1, 2]], simp[:, [2, 0]]], axis=0)
    owner = np.concatenate([np.arange(nc)] * 3)
    key = np.sort(e, axis=1)
    order = np.lexsort((key[:, 1], key[:, 0]))
    key = key[order]
    owner = owner[order]
    same = np.all(key[1:] == key[:-1], axis=1)
    faces = []
    i = 0
    ne = key.shape[0]
    while i < ne:
        if i + 1 < ne and same[i]:
            faces.append((key[i, 0], key[i, 1], owner[i], owner[i + 1]))
            i += 2
        else:
            faces.append((key[i, 0], key[i, 1], owner[i], -1))
            i += 1
    faces = np.array(faces, dtype=np.int64)
    p0 = pts[faces[:, 0]]
    p1 = pts[faces[:, 1]]
    t = p1 - p0
    length = np.linalg.norm(t, axis=1)
    n = np.stack([t[:, 1], -t[:, 0]], axis=1) / length[:, None]
    fctr = 0.5 * (p0 + p1)
    L = faces[:, 2]
    flip = np.einsum("ij,ij->i", fctr - ctr[L], n) < 0
    n[flip] *= -1.0
    R = faces[:, 3].copy()
    bnd = R < 0
    R[bnd] = -(1 + classify_edge(fctr[bnd]))
    fc = np.stack([L, R], axis=1)
    return _renumber(2, vol, ctr, fc, n, length, fctr, name)


def mesh_cavity(h: float = 0.0095, jitter: float = 0.3, seed: int = 0, hole=(0.35, 0.65)) -> Mesh:
    """Unit square with a concentric square hole, triangulated from jittered points.

    Boundary tags: 0 = stationary walls (outer bottom/left/right and the hole),
    1 = the lid at y = 1.
    """
    rng = np.random.default_rng(seed)
    lo, hi = hole
    n = int(round(1.0 / h))
    g = (np.arange(1, n) / n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    P = P + (rng.random(P.shape) - 0.5) * 2 * jitter * h
    margin = 0.5 * h
    inside_outer = (P > margin).all(axis=1) & (P < 1 - margin).all(axis=1)
    near_hole = (P > lo - margin).all(axis=1) & (P < hi + margin).all(axis=1)
    P = P[inside_outer & ~near_hole]
    B = []
    for s in np.linspace(0, 1, n + 1):
        B += [(s, 0.0), (s, 1.0), (0.0, s), (1.0, s)]
    nh = max(2, int(round((hi - lo) / h)))
    for s in np.linspace(lo, hi, nh + 1):
        B += [(s, lo), (s, hi), (lo, s), (hi, s)]
    B = np.unique(np.round(np.array(B), 12), axis=0)
    pts = np.concatenate([P, B], axis=0)

    def keep(cen):
        return ~((cen > lo).all(axis=1) & (cen < hi).all(axis=1))

    def classify(fc):
        return np.where(np.abs(fc[:, 1] - 1.0) < 1e-9, 1, 0)

    return _tri_mesh_from_points(pts, keep, classify, f"cavity_h{h}")


def mesh_cavity_mirror(h: float = 0.05, jitter: float = 0.3, seed: int = 0, hole=(0.35, 0.65)) -> Mesh:
    """Cavity mesh that is exactly mirror-symmetric about x = 1/2: the left half (jittered points plus
    points on the mid-line) is triangulated and its triangles are mirrored.  Same boundary tags as
    mesh_cavity."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    lo, hi = hole
    n = int(round(1.0 / h))
    assert n % 2 == 0, "an even number of intervals puts grid lines on the mid-line"
    g = np.arange(1, n) / n
    X, Y = np.meshgrid(g[g < 0.5 - 1e-12], g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    P = P + (rng.random(P.shape) - 0.5) * 2 * jitter * h
    margin = 0.5 * h
    inside = (P[:, 0] > margin) & (P[:, 0] < 0.5 - margin) & (P[:, 1] > margin) & (P[:, 1] < 1 - margin)
    near_hole = (P > lo - margin).all(axis=1) & (P[:, 1] < hi + margin)
    P = P[inside & ~near_hole]
    B = []
    for s_ in np.linspace(0, 1, n + 1):
        B += [(0.0, s_)]
        if s_ <= 0.5 + 1e-12:
            B += [(s_, 0.0), (s_, 1.0)]
        if s_ <= lo + 1e-12 or s_ >= hi - 1e-12:
            B += [(0.5, s_)]
    nh = max(2, int(round((hi - lo) / h)))
    for s_ in np.linspace(lo, hi, nh + 1):
        B += [(lo, s_)]
        if s_ <= 0.5 + 1e-12:
            B += [(s_, lo), (s_, hi)]
    B += [(0.5, lo), (0.5, hi)]
    B = np.unique(np.round(np.array(B), 12), axis=0)
    left = np.concatenate([P, B], axis=0)
    simp = Delaunay(left).simplices
    mid = np.abs(left[:, 0] - 0.5) < 1e-12
    # mirrored copies of the points off the mid-line
    idx_m = np.full(left.shape[0], -1)
    off = np.nonzero(~mid)[0]
    idx_m[off] = left.shape[0] + np.arange(off.size)
    idx_m[mid] = np.nonzero(mid)[0]
    right = left[off].copy()
    right[:, 0] = 1.0 - right[:, 0]
    pts = np.concatenate([left, right], axis=0)
    simp = np.concatenate([simp, idx_m[simp][:, ::-1]], axis=0)

    def keep(cen):
        return ~((cen > lo).all(axis=1) & (cen < hi).all(axis=1))

    def classify(fc):
        return np.where(np.abs(fc[:, 1] - 1.0) < 1e-9, 1, 0)

    return _tri_mesh_from_simplices(pts, simp, keep, classify, f"cavity_mirror_h{h}")


def mesh_annulus(r0: float = 1.0, r1: float = 6.0, n_theta: int = 256, n_r: int = 80, stretch: float = 1.045,
                 jitter: float = 0.15, seed: int = 1) -> Mesh:
    """Annulus r0 <= r <= r1 around a cylinder, radial spacing growing geometrically from the wall.

    Boundary tags: 0 = cylinder wall (r = r0), 1 = far field (r = r1).
    """
    rng = np.random.default_rng(seed)
    dr = np.cumprod(np.full(n_r, stretch))
    r = r0 + np.concatenate([[0.0], np.cumsum(dr)]) * (r1 - r0) / dr.sum()
    pts = []
    for k, rk in enumerate(r):
        th = np.arange(n_theta) * 2 * np.pi / n_theta
        if 0 < k < len(r) - 1:
            th = th + (rng.random(n_theta) - 0.5) * 2 * jitter * 2 * np.pi / n_theta + (k % 2) * np.pi / n_theta
        pts.append(np.stack([rk * np.cos(th), rk * np.sin(th)], axis=1))
    pts = np.concatenate(pts, axis=0)

    def keep(cen):
        return np.linalg.norm(cen, axis=1) > r0 * np.cos(np.pi / n_theta) * 1.0

    def classify(fc):
        rr = np.linalg.norm(fc, axis=1)
        return np.where(rr < 0.5 * (r0 + r1), 0, 1)

    return _tri_mesh_from_points(pts, keep, classify, f"annulus_{n_theta}x{n_r}")


def mesh_periodic_1d(n: int, length: float = 1.0) -> Mesh:
    """Uniform periodic 1D mesh of ``n`` cells on [0, length): face i (at x = i h) joins cell i - 1 (mod n) to
    cell i, unit normal +x; no boundary faces.  The geometry across the face at x = 0 is only meaningful to a
    solver that takes coordinate differences modulo ``length`` (``Mesh.period``)."""
    h = length / n
    xs = np.arange(n + 1) * h
    vol = np.full(n, h)
    ctr = (0.5 * (xs[1:] + xs[:-1]))[:, None]
    fc = np.array([((i - 1) % n, i) for i in range(n)], dtype=np.int64)
    fn = np.ones((n, 1))
    fa = np.ones(n)
    fctr = xs[:n, None].copy()
    m = Mesh(1, vol, ctr, fc, fn, fa, fctr, f"periodic{n}", period=float(length))
    m.check()
    return m


def mesh_capsule(n_s: int = 40, n_phi: int = 24, n_r: int = 24, r_nose: float = 1.0, cone_deg: float = 33.0,
                 r_out: float = 4.0, seed: int = 3, cell_order: str = "morton") -> Mesh:
    """Blunt capsule: spherical-cap forebody and conical afterbody, tetrahedral mesh.

    A body-fitted structured grid (surface coordinate s along the profile,
    azimuth phi, wall-normal index r) is split into tetrahedra (6 per hex).
    Boundary tags: 0 = capsule wall, 1 = far field.
    """
    cone = np.deg2rad(cone_deg)
    # meridian profile of the body: spherical cap from the nose to the shoulder, then the cone
    cap_angle = np.pi / 2 - cone
    s_cap = r_nose * cap_angle
    shoulder_x = r_nose * (1 - np.cos(cap_angle))
    shoulder_y = r_nose * np.sin(cap_angle)
    cone_len = 1.2 * r_nose
    total = s_cap + cone_len
    svals = np.linspace(0.0, total, n_s + 1)
    body = []
    nrm = []
    for s in svals:
        if s <= s_cap:
            a = s / r_nose
            body.append((r_nose * (1 - np.cos(a)), r_nose * np.sin(a)))
            nrm.append((-np.cos(a), np.sin(a)))
        else:
            t = s - s_cap
            body.append((shoulder_x + t * np.cos(cone), shoulder_y - t * np.sin(cone)))
            nrm.append((-np.sin(cone), np.cos(cone)))
    body = np.array(body)
    nrm = np.array(nrm)
    # outer boundary: a sphere of radius r_out centred at the nose-sphere centre
    ctr0 = np.array([r_nose, 0.0])
    outer = []
    for k in range(n_s + 1):
        ang = np.pi * k / n_s
        outer.append(ctr0 + r_out * np.array([-np.cos(ang), np.sin(ang)]))
    outer = np.array(outer)
    g = np.cumprod(np.full(n_r, 1.12))
    t = np.concatenate([[0.0], np.cumsum(g)]) / g.sum()
    # meridian grid points (k along s, j off the wall): blend body -> outer
    mer = body[:, None, :] * (1 - t[None, :, None]) + outer[:, None, :] * t[None, :, None]
    phis = np.linspace(0.0, 2 * np.pi, n_phi, endpoint=False)
    # 3D points; the axis points (y = 0 at k = 0 and k = n_s) are shared across phi
    idx = -np.ones((n_s + 1, n_r + 1, n_phi), dtype=np.int64)
    pts = []
    on_body = []
    for k in range(n_s + 1):
        for j in range(n_r + 1):
            x, y = mer[k, j]
            if abs(y) < 1e-12:
                idx[k, j, :] = len(pts)
                pts.append((x, 0.0, 0.0))
                on_body.append(j == 0)
            else:
                for p, ph in enumerate(phis):
                    idx[k, j, p] = len(pts)
                    pts.append((x, y * np.cos(ph), y * np.sin(ph)))
                    on_body.append(j == 0)
    pts = np.array(pts)
    on_body = np.array(on_body)
    tets = []
    for k in range(n_s):
        for j in range(n_r):
            for p in range(n_phi):
                q = (p + 1) % n_phi
                v = [idx[k, j, p], idx[k + 1, j, p], idx[k + 1, j, q], idx[k, j, q],
                     idx[k, j + 1, p], idx[k + 1, j + 1, p], idx[k + 1, j + 1, q], idx[k, j + 1, q]]
                # Kuhn split: six tetrahedra around the main diagonal v0-v6 (conforming on a structured grid)
                for tt in ((0, 1, 2, 6), (0, 1, 5, 6), (0, 3, 2, 6), (0, 3, 7, 6), (0, 4, 5, 6), (0, 4, 7, 6)):
                    tv = [v[a] for a in tt]
                    if len(set(tv)) == 4:
                        tets.append(tv)
    tets = np.array(tets, dtype=np.int64)
    P = pts[tets]
    vol6 = np.einsum("ij,ij->i", np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), P[:, 3] - P[:, 0])
    good = np.abs(vol6) > 1e-14
    tets = tets[good]
    vol = np.abs(vol6[good]) / 6.0
    nc = tets.shape[0]
    ctr = pts[tets].mean(axis=1)
    faces_local = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
    tri = np.concatenate([tets[:, list(fl)] for fl in faces_local], axis=0)
    owner = np.concatenate([np.arange(nc)] * 4)
    key = np.sort(tri, axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    key = key[order]
    owner = owner[order]
    tri = tri[order]
    same = np.all(key[1:] == key[:-1], axis=1)
    rows = []
    i = 0
    ne = key.shape[0]
    while i < ne:
        if i + 1 < ne and same[i]:
            rows.append((i, owner[i], owner[i + 1]))
            i += 2
        else:
            rows.append((i, owner[i], -1))
            i += 1
    rows = np.array(rows, dtype=np.int64)
    T = pts[tri[rows[:, 0]]]
    cr = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2 * area[:, None])
    fctr = T.mean(axis=1)
    L = rows[:, 1]
    flip = np.einsum("ij,ij->i", fctr - ctr[L], n) < 0
    n[flip] *= -1
    R = rows[:, 2].copy()
    bnd = R < 0
    wall = on_body[tri[rows[:, 0]]].all(axis=1)
    R[bnd] = -(1 + np.where(wall[bnd], 0, 1))
    fc = np.stack([L, R], axis=1)
    return _renumber(3, vol, ctr, fc, n, area, fctr, f"capsule_{nc}", order=cell_order)


def mesh_patch(mesh: Mesh, seeds, rings: int):
    """The cells within `rings` face-neighbour steps of the seed cells, as a mesh of its own.

    Returns (patch, cells, seeds_local): `cells` are the kept cell indices of `mesh` in increasing order
    (patch cell k is mesh cell cells[k]), `seeds_local` the seeds' patch indices.  Faces between two kept
    cells stay interior; boundary faces of kept cells keep their tags; a face between a kept and a dropped
    cell becomes a boundary face of the kept cell, oriented outward from it, with the new tag
    (largest tag of `mesh`) + 1, so every patch cell is closed."""
    fc = mesh.face_cells
    L, R = fc[:, 0], fc[:, 1]
    inner = R >= 0
    nbr = [[] for _ in range(mesh.nc)]
    for a, b in zip(L[inner], R[inner]):
        nbr[a].append(b)
        nbr[b].append(a)
    keep = np.zeros(mesh.nc, dtype=bool)
    seeds = np.asarray(seeds, dtype=np.int64)
    keep[seeds] = True
    front = list(np.unique(seeds))
    for _ in range(rings):
        nxt = []
        for c in front:
            for j in nbr[c]:
                if not keep[j]:
                    keep[j] = True
                    nxt.append(j)
        front = nxt
    cells = np.nonzero(keep)[0]
    local = np.full(mesh.nc, -1, dtype=np.int64)
    local[cells] = np.arange(len(cells))
    new_tag = int((-R[~inner] - 1).max()) + 1 if (~inner).any() else 0
    kl = keep[L]
    kr = np.where(inner, keep[np.maximum(R, 0)], False)
    sel = kl | kr
    fL, fR = L[sel], R[sel]
    n, area, fctr = mesh.face_n[sel].copy(), mesh.face_area[sel], mesh.face_ctr[sel]
    kl_s, kr_s, inner_s = kl[sel], kr[sel], inner[sel]
    out = np.empty((sel.sum(), 2), dtype=np.int64)
    both = kl_s & kr_s
    out[both, 0], out[both, 1] = local[fL[both]], local[fR[both]]
    bnd = kl_s & ~inner_s
    out[bnd, 0], out[bnd, 1] = local[fL[bnd]], fR[bnd]
    cutL = kl_s & inner_s & ~kr_s
    out[cutL, 0], out[cutL, 1] = local[fL[cutL]], -(new_tag + 1)
    cutR = kr_s & ~kl_s
    out[cutR, 0], out[cutR, 1] = local[fR[cutR]], -(new_tag + 1)
    n[cutR] = -n[cutR]
    patch = Mesh(mesh.dim, mesh.vol[cells].copy(), mesh.ctr[cells].copy(), out, n, area.copy(), fctr.copy(),
                 name=f"{mesh.name}_patch{len(cells)}")
    return patch, cells, local[seeds]
