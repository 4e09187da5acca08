"""Seeded synthetic inputs for clipped and restricted Voronoi diagrams.

This module is shared by the CPU oracle and the GPU path.  It only draws
random numbers and builds meshes; it holds none of the Voronoi method's
arithmetic (no bisectors, no clipping, no nearest-site search).

Domains follow the problem statement of the paper (Sec. 3.1): a set of
simplices.  Volumetric domains are cube grids split into six Kuhn
tetrahedra; surface domains are subdivided icosahedra.  Every generator is
seeded (NumPy PCG64) and returns float64 coordinates and int32 topology.

Face/edge numbering used by both consumers:
  * tetrahedron ``t = (q0, q1, q2, q3)`` is positively oriented
    (det(q1-q0, q2-q0, q3-q0) > 0); local face ``f`` is the face opposite
    vertex ``qf``;
  * triangle ``t = (q0, q1, q2)``; local edge ``e`` is the edge opposite
    vertex ``qe``;
  * ``adj[a, f]`` is the simplex sharing local face/edge ``f`` with simplex
    ``a``, or -1 on the domain boundary.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Domain", "kuhn_cube_grid", "icosphere", "adjacency",
    "uniform_cube_sites", "gaussian_mixture_sites", "sphere_sites",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5",
    "lattice_sites", "small_case", "kuhn_cube_subset", "l_block", "cube_with_cavity", "l_block_sites",
]


@dataclass
class Domain:
    verts: np.ndarray      # (nv, 3) float64
    simplices: np.ndarray  # (m, d+1) int32, tets (d=3) or triangles (d=2)
    adj: np.ndarray        # (m, d+1) int32, -1 = boundary
    dim: int               # 3 = tetrahedra, 2 = triangles

    @property
    def m(self) -> int:
        return int(self.simplices.shape[0])


def adjacency(simplices: np.ndarray) -> np.ndarray:
    """Neighbour across each local face (tets) or edge (triangles)."""
    simplices = np.asarray(simplices, dtype=np.int64)
    m, k = simplices.shape
    faces = []
    for f in range(k):
        cols = [c for c in range(k) if c != f]
        faces.append(np.sort(simplices[:, cols], axis=1))
    faces = np.stack(faces, axis=1).reshape(m * k, k - 1)
    owner = np.repeat(np.arange(m, dtype=np.int64), k)
    local = np.tile(np.arange(k, dtype=np.int64), m)
    order = np.lexsort(faces.T[::-1])
    fs = faces[order]
    same = np.all(fs[1:] == fs[:-1], axis=1)
    adj = -np.ones((m, k), dtype=np.int64)
    idx = np.nonzero(same)[0]
    a, b = order[idx], order[idx + 1]
    adj[owner[a], local[a]] = owner[b]
    adj[owner[b], local[b]] = owner[a]
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-manifold mesh: a face is shared by more than two simplices")
    return adj.astype(np.int32)


def _tet_volumes(verts, tets):
    q = verts[tets]
    return np.einsum("ij,ij->i", np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]),
                     q[:, 3] - q[:, 0]) / 6.0


def kuhn_cube_grid(k: int, jitter: float = 0.0, seed: int | None = None) -> Domain:
    """Unit cube split into k^3 cubes, each cut into 6 Kuhn tetrahedra.

    Every cube uses the same main diagonal (0,0,0)->(1,1,1), so the split
    is conforming.  Each tet follows one axis permutation along that
    diagonal and is reoriented to positive volume.  With ``jitter`` > 0,
    lattice vertices move by U(-jitter*h, jitter*h) per axis, except along
    axes where the vertex lies on the cube boundary, so the domain stays
    the unit cube.
    """
    n1 = k + 1
    g = np.arange(n1, dtype=np.float64) / k
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    verts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        h = 1.0 / k
        d = rng.uniform(-jitter * h, jitter * h, size=verts.shape)
        on_bnd = (verts <= 0.0) | (verts >= 1.0)
        d[on_bnd] = 0.0
        verts = verts + d

    def vid(ix, iy, iz):
        return ix + n1 * (iy + n1 * iz)

    cx, cy, cz = np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    tets = []
    for perm in itertools.permutations(range(3)):
        p = [np.stack([cx, cy, cz], axis=1)]
        cur = p[0].copy()
        for ax in perm:
            cur = cur.copy()
            cur[:, ax] += 1
            p.append(cur)
        ids = np.stack([vid(q[:, 0], q[:, 1], q[:, 2]) for q in p], axis=1)
        tets.append(ids)
    tets = np.stack(tets, axis=1).reshape(-1, 4)
    vol = _tet_volumes(verts, tets)
    neg = vol < 0
    tets[neg] = tets[neg][:, [0, 1, 3, 2]]
    vol = _tet_volumes(verts, tets)
    if not np.all(vol > 0):
        raise ValueError("inverted tetrahedron; jitter too large")
    tets = tets.astype(np.int32)
    return Domain(verts=verts, simplices=tets, adj=adjacency(tets), dim=3)


def kuhn_cube_subset(k: int, keep) -> Domain:
    """The cubes (ix, iy, iz) of a k^3 Kuhn grid of the unit cube for which
    ``keep(ix, iy, iz)`` holds, each cut into the same 6 tetrahedra as in
    ``kuhn_cube_grid`` (so the mesh stays conforming), unused vertices dropped."""
    full = kuhn_cube_grid(k)
    # kuhn_cube_grid lists the 6 tets of cube (ix, iy, iz) at rows 6c .. 6c+5,
    # c = the cube's index with ix varying slowest
    order = [(ix, iy, iz) for ix in range(k) for iy in range(k) for iz in range(k)]
    rows = [6 * c + t for c, (ix, iy, iz) in enumerate(order) if keep(ix, iy, iz) for t in range(6)]
    sub = full.simplices[np.array(rows, dtype=np.int64)]
    used = np.unique(sub)
    remap = -np.ones(len(full.verts), dtype=np.int64)
    remap[used] = np.arange(len(used))
    sub = remap[sub].astype(np.int32)
    verts = full.verts[used]
    assert np.all(_tet_volumes(verts, sub) > 0)
    return Domain(verts=verts, simplices=sub, adj=adjacency(sub), dim=3)


def l_block(k: int) -> Domain:
    """Non-convex L-shaped prism: the unit cube without the quarter
    x > 1/2, y > 1/2 (all z), as a Kuhn grid of k^3 cubes (k even)."""
    assert k % 2 == 0
    return kuhn_cube_subset(k, lambda ix, iy, iz: not (ix >= k // 2 and iy >= k // 2))


def cube_with_cavity(k: int) -> Domain:
    """Unit cube with a closed cubic cavity: the cubes of the middle third
    (k divisible by 3) are removed, leaving an inner boundary surface."""
    assert k % 3 == 0
    lo, hi = k // 3, 2 * k // 3
    return kuhn_cube_subset(k, lambda ix, iy, iz: not (lo <= ix < hi and lo <= iy < hi and lo <= iz < hi))


def l_block_sites(n: int, seed: int) -> np.ndarray:
    """n uniform sites in the L-shaped prism (rejection), off the grid planes."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        p = rng.uniform(1e-6, 1 - 1e-6, size=3)
        if p[0] > 0.5 and p[1] > 0.5:
            continue
        out.append(p)
    return _jitter_inside(rng, np.array(out), 1e-7)


def icosphere(level: int) -> Domain:
    """Icosahedron subdivided ``level`` times, midpoints projected to S^2.

    Triangles are oriented with outward normals.  Level 6 gives 81,920
    triangles and 40,962 vertices.
    """
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache: dict = {}
        verts_l = list(verts)

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                p = (np.array(verts_l[a]) + np.array(verts_l[b])) / 2.0
                p /= np.linalg.norm(p)
                cache[key] = len(verts_l)
                verts_l.append(tuple(p))
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        verts = verts_l
        f = np.array(nf, dtype=np.int64)
    verts = np.array(verts, dtype=np.float64)
    q = verts[f]
    nrm = np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0])
    flip = np.einsum("ij,ij->i", nrm, q.mean(axis=1)) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    f = f.astype(np.int32)
    return Domain(verts=verts, simplices=f, adj=adjacency(f), dim=2)


def _jitter_inside(rng, pts, eps):
    """Add U(-eps, eps) per coordinate; redraw the jitter of points that leave (0,1)^3."""
    out = pts.copy()
    todo = np.arange(len(pts))
    while todo.size:
        cand = pts[todo] + rng.uniform(-eps, eps, size=(todo.size, 3))
        ok = np.all((cand > 0.0) & (cand < 1.0), axis=1)
        out[todo[ok]] = cand[ok]
        todo = todo[~ok]
    return out


def uniform_cube_sites(n: int, seed: int, jitter: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(n, 3))
    bad = ~np.all((pts > 0.0) & (pts < 1.0), axis=1)
    while np.any(bad):
        pts[bad] = rng.uniform(0.0, 1.0, size=(int(bad.sum()), 3))
        bad = ~np.all((pts > 0.0) & (pts < 1.0), axis=1)
    if jitter > 0.0:
        pts = _jitter_inside(rng, pts, jitter)
    return pts


def gaussian_mixture_sites(n_per: int, n_gauss: int, n_background: int, sigma: float,
                           centre_seed: int, sample_seed: int, jitter: float) -> np.ndarray:
    """Isotropic Gaussian clusters in the unit cube plus a uniform background.

    Centres are U(0.2, 0.8)^3.  Samples outside (0,1)^3 are redrawn
    (rejection), never clamped, so no site lies on the cube boundary.
    """
    crng = np.random.default_rng(centre_seed)
    centres = crng.uniform(0.2, 0.8, size=(n_gauss, 3))
    rng = np.random.default_rng(sample_seed)
    parts = []
    for g in range(n_gauss):
        got = np.empty((0, 3))
        while got.shape[0] < n_per:
            need = n_per - got.shape[0]
            s = centres[g] + sigma * rng.standard_normal(size=(need + need // 4 + 16, 3))
            s = s[np.all((s > 0.0) & (s < 1.0), axis=1)]
            got = np.concatenate([got, s[:need]])
        parts.append(got)
    parts.append(rng.uniform(0.0, 1.0, size=(n_background, 3)))
    pts = np.concatenate(parts)
    pts = _jitter_inside(rng, pts, jitter)
    return pts


def sphere_sites(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(size=(n, 3))
    return p / np.linalg.norm(p, axis=1, keepdims=True)


def lattice_sites(k: int, jitter: float, seed: int) -> np.ndarray:
    """Cube-centre lattice of k^3 sites with a tiny uniform jitter."""
    g = (np.arange(k) + 0.5) / k
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    rng = np.random.default_rng(seed)
    return pts + rng.uniform(-jitter, jitter, size=pts.shape)


# --- the named workloads --------------------------------------------------

def config_c1():
    """3D clipped VD, 1,000 uniform sites, unit cube as 6 tetrahedra."""
    return uniform_cube_sites(1000, seed=101), kuhn_cube_grid(1)


def config_c2():
    """3D restricted VD, 100,000 uniform sites, 20^3 cubes x 6 tets."""
    return uniform_cube_sites(100_000, seed=102, jitter=1e-7), kuhn_cube_grid(20)


def config_c3():
    """1,000,000 sites: 8 Gaussians (sigma 0.05) + 10% background; 50^3 x 6 tets."""
    sites = gaussian_mixture_sites(112_500, 8, 100_000, 0.05, centre_seed=103,
                                   sample_seed=104, jitter=1e-7)
    return sites, kuhn_cube_grid(50)


def config_c4(num: int = 256, master_seed: int = 105):
    """Independent diagrams: log-uniform site counts in [1e3, 6.4e4], jittered k^3 grids."""
    rng = np.random.default_rng(master_seed)
    out = []
    for b in range(num):
        nb = int(round(np.exp(rng.uniform(np.log(1e3), np.log(6.4e4)))))
        kb = int(rng.integers(8, 25))
        s_seed, d_seed = (int(x) for x in rng.integers(0, 2**31 - 1, size=2))
        out.append((uniform_cube_sites(nb, seed=s_seed, jitter=1e-7),
                    kuhn_cube_grid(kb, jitter=0.1, seed=d_seed)))
    return out


def config_c5():
    """200,000 sites uniform on S^2; icosphere level 6 (81,920 triangles)."""
    return sphere_sites(200_000, seed=106), icosphere(6)


def planar_l_polygon(k: int) -> Domain:
    """L-shaped polygon in the plane z = 0: the unit square without its upper
    right quarter, on a k x k grid of squares (k even), each split into two
    counter-clockwise triangles.  A 2D clipped Voronoi diagram of sites in the
    plane is the restricted diagram of this flat mesh."""
    assert k % 2 == 0
    used = {}
    verts, tris = [], []

    def vid(x, y):
        if (x, y) not in used:
            used[(x, y)] = len(verts)
            verts.append((x / k, y / k, 0.0))
        return used[(x, y)]
    for y in range(k):
        for x in range(k):
            if x >= k // 2 and y >= k // 2:
                continue
            a, b, c, d = vid(x, y), vid(x + 1, y), vid(x + 1, y + 1), vid(x, y + 1)
            tris += [[a, b, c], [a, c, d]]
    tris = np.array(tris, dtype=np.int32)
    return Domain(verts=np.array(verts, dtype=np.float64), simplices=tris, adj=adjacency(tris), dim=2)


def planar_l_sites(n: int, seed: int) -> np.ndarray:
    """n uniform sites in the L-shaped polygon (rejection), jittered off the grid lines."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        p = rng.uniform(1e-6, 1 - 1e-6, size=2)
        if p[0] >= 0.5 and p[1] >= 0.5:
            continue
        out.append(p)
    p2 = np.array(out)
    return np.c_[p2, np.zeros(n)]


def small_case(n: int, k: int, seed: int, jitter_domain: float = 0.0):
    """Small 3D case used by tests: n uniform sites in a k^3-cube Kuhn grid."""
    return (uniform_cube_sites(n, seed=seed, jitter=1e-7),
            kuhn_cube_grid(k, jitter=jitter_domain, seed=seed + 7))
