"""Oracle pins on non-convex tetrahedral domains and sites outside the domain
(Sec. 3.1: a clipped cell is the union over simplices of T_a cap Omega_i, so
Omega_i cap M may have several components and a site need not lie in M).

The L-shaped prism has a re-entrant edge, the cube with a cavity an inner
boundary; with few sites, cells wrap around the notch or the cavity and meet
M in disconnected parts.  Pins: brute force (every bisector) equals the
pruned run bit for bit, Monte-Carlo nearest-site labelling of points drawn
uniformly in M, the per-tetrahedron partition, the sampled-site mode, and the
fact that the cases really contain cells with several components."""
import numpy as np
import pytest

import vdgen
from canon import canon_pieces, compare_canon, subset_result


def _vols(dom):
    q = dom.verts[dom.simplices]
    return np.einsum("ij,ij->i", np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), q[:, 3] - q[:, 0]) / 6


def _cases():
    rng = np.random.default_rng(71)
    lb = vdgen.l_block(4)
    s_in = vdgen.l_block_sites(8, seed=14)             # the cell of site 0 wraps the notch: two parts
    s_out = np.array([[0.93, 0.96, 0.31],              # in the missing quarter: outside M, its cell meets M
                      [1.3, 0.2, 0.52]])               # outside the cube: its cell misses M
    cav = vdgen.cube_with_cavity(6)
    c_in = vdgen.uniform_cube_sites(40, seed=73, jitter=1e-7)
    keep = ~np.all((c_in > 1 / 3) & (c_in < 2 / 3), axis=1)
    c_hole = 1 / 3 + rng.random((2, 3)) / 3             # inside the cavity: outside M
    far = np.array([[1.31, 0.42, 0.57], [-0.23, 0.61, 0.38]])  # outside the cube
    return {"l_block": (np.vstack([s_in, s_out]), lb),
            "cavity": (np.vstack([c_in[keep], c_hole, far]), cav)}


def _components(r, i):
    """Connected components of site i's pieces, adjacent through shared
    tetrahedron faces (flags -(b+1))."""
    sel = np.nonzero(r["piece_site"] == i)[0]
    simp = {int(r["piece_simplex"][p]): p for p in sel}
    seen, comps = set(), 0
    for a0 in simp:
        if a0 in seen:
            continue
        comps += 1
        stack = [a0]
        seen.add(a0)
        while stack:
            a = stack.pop()
            p = simp[a]
            for f in range(r["piece_face_off"][p], r["piece_face_off"][p + 1]):
                lab = int(r["face_label"][f])
                if -2**31 + 16 < lab < 0 and (-lab - 1) in simp and (-lab - 1) not in seen:
                    seen.add(-lab - 1)
                    stack.append(-lab - 1)
    return comps


@pytest.mark.parametrize("name", ["l_block", "cavity"])
def test_brute_equals_pruned_and_partition(oracle_mod, name):
    sites, dom = _cases()[name]
    b = oracle_mod.compute(sites, dom, brute=True)
    p = oracle_mod.compute(sites, dom, brute=False)
    assert compare_canon(canon_pieces(b), canon_pieces(p), 0.0) == (0, 0, 0.0)
    # same polytopes; the moment fan's apex (a piece's first vertex) depends on
    # the clip order, so the masses agree to rounding
    assert np.allclose(b["piece_mass"], p["piece_mass"], rtol=1e-12, atol=0)
    tv = _vols(dom)
    per = np.bincount(b["piece_simplex"], weights=b["piece_mass"], minlength=dom.m)
    assert np.allclose(per, tv, rtol=1e-12, atol=0)
    m = oracle_mod.site_moments(b, sites)
    assert abs(m["mass"].sum() - tv.sum()) <= 1e-12 * tv.sum()
    assert b["min_margin"] > 1e-9


@pytest.mark.parametrize("name", ["l_block", "cavity"])
def test_cells_with_several_components_exist(oracle_mod, name):
    """The cases exercise what propagation from the site's tetrahedron alone
    would miss: a cell meeting M in several parts, or a site outside M whose
    cell still meets it."""
    sites, dom = _cases()[name]
    r = oracle_mod.compute(sites, dom, brute=True)
    comps = [_components(r, i) for i in range(len(sites))]
    m = oracle_mod.site_moments(r, sites)
    outside_with_cell = [i for i in range(len(sites)) if m["mass"][i] > 0 and not _inside(sites[i], dom)]
    assert max(comps) >= 2 or outside_with_cell, (comps, outside_with_cell)
    if name == "l_block":
        assert max(comps) >= 2
    assert outside_with_cell


def _inside(p, dom):
    q = dom.verts[dom.simplices]
    T = np.stack([q[:, 1] - q[:, 0], q[:, 2] - q[:, 0], q[:, 3] - q[:, 0]], axis=2)
    lam = np.linalg.solve(T, (p[None, :] - q[:, 0, :])[:, :, None])[:, :, 0]
    return bool(np.any(np.all(lam >= -1e-12, axis=1) & (lam.sum(axis=1) <= 1 + 1e-12)))


@pytest.mark.parametrize("name", ["l_block", "cavity"])
def test_monte_carlo_labelling(oracle_mod, name):
    """Points uniform in M (tetrahedron by volume, uniform barycentric
    coordinates): the pair (tetrahedron, nearest site by brute force) is a
    piece, and each cell's hit fraction agrees with its mass / |M| (5 sigma)."""
    sites, dom = _cases()[name]
    r = oracle_mod.compute(sites, dom, brute=True)
    m = oracle_mod.site_moments(r, sites)
    tv = _vols(dom)
    rng = np.random.default_rng(79)
    N = 40000
    tet = rng.choice(dom.m, size=N, p=tv / tv.sum())
    e = rng.exponential(size=(N, 4))
    lam = e / e.sum(axis=1, keepdims=True)
    pts = np.einsum("nk,nkd->nd", lam, dom.verts[dom.simplices[tet]])
    nn = np.argmin(((pts[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2), axis=1)
    pairs = set(zip(r["piece_site"].tolist(), r["piece_simplex"].tolist()))
    assert all((int(a), int(b)) in pairs for a, b in zip(nn, tet))
    frac = np.bincount(nn, minlength=len(sites)) / N
    w = m["mass"] / tv.sum()
    sigma = np.sqrt(w * (1 - w) / N)
    assert np.all(np.abs(frac - w) <= 5 * sigma + 1e-12)


@pytest.mark.parametrize("name", ["l_block", "cavity"])
def test_sampled_sites_equal_the_full_run(oracle_mod, name):
    sites, dom = _cases()[name]
    full = oracle_mod.compute(sites, dom)
    sample = np.arange(0, len(sites), 3, dtype=np.int32)
    part = oracle_mod.compute(sites, dom, only_sites=sample)
    sel = np.nonzero(np.isin(full["piece_site"], sample))[0]
    assert compare_canon(canon_pieces(part), canon_pieces(subset_result(full, sel)), 0.0) == (0, 0, 0.0)
