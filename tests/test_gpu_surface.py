"""GPU parity of the restricted (surface) Voronoi path against the CPU oracle.

Triangle meshes in R^3 cut by 3D bisectors (Alg. 4 propagation inside each
triangle).  Same bar as the 3D path: bit-exact combinatorics, moments within
1e-9 relative.
"""
import numpy as np
import pytest

import vdgen
from gpu_util import (assert_neighbour_symmetry, assert_parity, assert_sampled_parity, gpu_neighbors, log, run_gpu,
                      sampled_result)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _area(dom):
    q = dom.verts[dom.simplices]
    return 0.5 * np.linalg.norm(np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), axis=1)


def _surface_case(oracle_mod, sites, dom, brute=True, **opts):
    log(f"surface case n={len(sites)} m={dom.m} opts={opts}")
    area = float(_area(dom).sum())
    gpu = run_gpu(sites, dom, bbox=(-1.01, -1.01, -1.01, 1.01, 1.01, 1.01), surface_area=area, **opts)
    ref = oracle_mod.compute(sites, dom, brute=brute)
    mom = oracle_mod.site_moments(ref, sites)
    assert_parity(gpu, ref, mom, len(sites))
    assert abs(gpu["mass"].sum() - area) <= 1e-12 * area
    return gpu


@pytest.mark.parametrize("n,level,seed", [(40, 2, 3), (500, 3, 4), (3000, 4, 5)])
def test_sphere_parity(oracle_mod, n, level, seed):
    s = vdgen.sphere_sites(n, seed=seed)
    _surface_case(oracle_mod, s, vdgen.icosphere(level), brute=(n <= 500))


@pytest.mark.parametrize("straddle,improved", [(0, 0), (1, 1)])
def test_sphere_search_variants(oracle_mod, straddle, improved):
    s = vdgen.sphere_sites(800, seed=8)
    _surface_case(oracle_mod, s, vdgen.icosphere(3), brute=False, use_straddle_edges=straddle,
                  improved_search=improved)


def test_planar_l_polygon(oracle_mod):
    """A 2D clipped Voronoi diagram on a non-convex polygon (an L of 0.75 area,
    6 x 6 squares of 2 triangles minus a quarter): sites in the plane of a flat
    mesh, whose restricted cells are the 2D clipped cells."""
    dom = vdgen.planar_l_polygon(6)
    s = vdgen.planar_l_sites(500, seed=31)
    gpu = _surface_case(oracle_mod, s, dom, brute=True)
    assert abs(gpu["mass"].sum() - 0.75) < 1e-12


def test_tiny_triangles_far_from_their_sites(oracle_mod):
    """The flat L-polygon mesh with its first grid line moved to 2^-30: a corner
    square of two triangles of area eps^2/2 about 0.5 from the five sites.
    Both pieces are emitted with their exact area; a fan with its apex at the
    site's foot point carries ~1e-17 of rounding here, 40x the area."""
    eps = 2.0 ** -30
    base = vdgen.planar_l_polygon(4)
    v = base.verts.copy()
    v[:, :2][v[:, :2] == 0.25] = eps
    dom = vdgen.Domain(verts=v, simplices=base.simplices, adj=base.adj, dim=2)
    rng = np.random.default_rng(5)
    s = np.zeros((5, 3))
    s[:, 0] = 0.3 + 0.15 * rng.random(5)
    s[:, 1] = 0.3 + 0.15 * rng.random(5)
    area = float(_area(dom).sum())
    gpu = run_gpu(s, dom, bbox=(-1.01, -1.01, -1.01, 1.01, 1.01, 1.01), surface_area=area)
    ref = oracle_mod.compute(s, dom, brute=True)
    # the thin strips beside the corner square end in tips of angle ~eps/0.25,
    # so a vertex on two of their edges is fixed only to ~1e-16 * 0.5 / 3.7e-9
    # = 1.5e-8 by either side's arithmetic; checked with ~70x room
    assert_parity(gpu, ref, oracle_mod.site_moments(ref, s), len(s), xyz_tol=1e-6)
    assert abs(gpu["mass"].sum() - area) <= 1e-12 * area
    got = gpu["res"]["piece_mass"][gpu["res"]["piece_simplex"] < 2]
    assert len(got) == 2 and np.allclose(got, eps ** 2 / 2, rtol=1e-9, atol=0)


def test_sites_off_the_surface(oracle_mod):
    """Sites at radius 0.8..1.2 around the sphere mesh (not on it)."""
    rng = np.random.default_rng(21)
    s = vdgen.sphere_sites(600, seed=22) * rng.uniform(0.8, 1.2, size=(600, 1))
    _surface_case(oracle_mod, s, vdgen.icosphere(3), brute=False)


def test_c5_full_size_sampled(oracle_mod):
    """C5 at its full size: 200,000 sites on S^2, level-6 icosphere (81,920
    triangles).  5,000 sampled sites against the oracle piece by piece;
    per-triangle partition and neighbour symmetry for all sites."""
    import torch
    import paper_2509_07175_amd as vd
    s, dom = vdgen.config_c5()
    area = float(_area(dom).sum())
    n = len(s)
    st = torch.as_tensor(s, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    g = vd.build_grid(st, bbox=(-1.01, -1.01, -1.01, 1.01, 1.01, 1.01), surface_area=area)
    c = vd.clip_cells(g, d, vd.Options.default())
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    log(f"C5 info {c.info()}")
    mass, cent, en = m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy()
    assert abs(mass.sum() - area) <= 1e-11 * area
    view = c.view()
    psite = view["piece_site"].cpu().numpy()
    used = psite >= 0
    per = np.bincount(view["piece_simplex"].cpu().numpy()[used], weights=view["piece_mass"].cpu().numpy()[used],
                      minlength=dom.m)
    assert np.allclose(per, _area(dom), rtol=1e-10, atol=0)
    nbo, nb = view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy()
    assert_neighbour_symmetry(nbo, nb)
    rng = np.random.default_rng(2025)
    sample = np.sort(rng.choice(n, size=5000, replace=False))
    ref = oracle_mod.compute(s, dom, only_sites=sample)
    mom = oracle_mod.site_moments(ref, s)
    assert_sampled_parity(sampled_result(view, sample), mass, cent, en, nbo, nb, ref, mom, sample)


@pytest.mark.parametrize("k,n", [(2, 3000), (4, 6000)])
def test_triangles_meeting_many_cells(oracle_mod, k, n):
    """Coarse flat L meshes (6 and 24 triangles) under 3,000 and 6,000 sites:
    a triangle meets hundreds of cells, more than a wave keeps in LDS, so its
    site list continues in the grown global overflow buffer."""
    dom = vdgen.planar_l_polygon(k)
    s = vdgen.planar_l_sites(n, seed=40 + k)
    gpu = _surface_case(oracle_mod, s, dom, brute=False)
    per_tri = np.bincount(gpu["res"]["piece_simplex"], minlength=dom.m)
    log(f"cells per triangle: max {per_tri.max()}, min {per_tri.min()}")
    assert per_tri.max() > 128


def test_boundary_diagram_of_a_coarse_cube():
    """The unit cube as 6 tetrahedra (12 boundary triangles) under 5,000
    sites: each boundary triangle meets a few hundred cells, so the boundary
    diagram that seeds the clip (and Alg. 5's split) needs the grown site
    lists; results equal the plain clip's."""
    s, dom = vdgen.small_case(5000, 1, seed=44)
    plain = run_gpu(s, dom)
    seeded = run_gpu(s, dom, boundary_seeds=1)
    whole = run_gpu(s, dom, whole_interior=1)  # convex, every site inside: split by the corners
    whole_b = run_gpu(s, dom, whole_interior=1, boundary_seeds=1)  # split by the boundary diagram
    assert seeded["info"]["boundary_seeded"] == 1 and whole["info"]["boundary_seeded"] == 0
    for r in (seeded, whole, whole_b):
        assert np.all(np.abs(r["mass"] - plain["mass"]) <= 1e-12 * plain["mass"])
        assert np.array_equal(r["nbr_off"], plain["nbr_off"]) and np.array_equal(r["nbr"], plain["nbr"])
    assert np.array_equal(seeded["res"]["piece_site"], plain["res"]["piece_site"])
    assert np.array_equal(seeded["res"]["piece_mass"], plain["res"]["piece_mass"])
    ra, rb = whole["res"], whole_b["res"]
    assert np.array_equal(ra["piece_site"], rb["piece_site"]) and np.array_equal(ra["piece_simplex"], rb["piece_simplex"])


def test_site_with_more_than_96_neighbours(oracle_mod):
    """A site ringed by 120 sites in the plane of a flat L mesh: its 2D cell
    has 120 neighbours, more than the per-site list a thread keeps, so the
    neighbour list is counted and written in place.  Everything against the
    oracle."""
    rng = np.random.default_rng(47)
    c = np.array([0.25, 0.25])
    ang = np.linspace(0, 2 * np.pi, 120, endpoint=False) + rng.uniform(-1e-3, 1e-3, 120)
    rad = 0.1 + rng.uniform(-1e-4, 1e-4, 120)
    ring = np.c_[c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang)]
    bg = vdgen.planar_l_sites(400, seed=48)[:, :2]
    bg = bg[np.linalg.norm(bg - c, axis=1) > 0.16]
    p2 = np.vstack([[c + 1e-5], ring, bg])
    s = np.c_[p2, np.zeros(len(p2))]
    gpu = _surface_case(oracle_mod, s, vdgen.planar_l_polygon(16), brute=False)
    nb = gpu_neighbors(gpu, len(s))
    assert len(nb[0]) > 96
