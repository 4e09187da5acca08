"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test ties the oracle to something independent of its own code:
qhull's half-space intersection (scipy), brute-force nearest-site labelling
of random points, closed forms, and invariants of Voronoi diagrams
(Sec. 3.1 Eq. 1 and the flags of Sec. 3.2).  The adjoint is pinned by
central finite differences of the forward moments and by the closed-form
CVT gradient (Sec. 7.4, Eq. 3).
"""
import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.spatial import ConvexHull, HalfspaceIntersection

import vdgen
from canon import canon_pieces, compare_canon, subset_result

BND = -2**31


def _tet_planes(q):
    """Outward half-spaces n.x <= c of a positively oriented tet (face f opposite q_f)."""
    loops = [(1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1)]
    out = []
    for f, (a, b, c) in enumerate(loops):
        n = np.cross(q[b] - q[a], q[c] - q[a])
        out.append((n, n @ q[a]))
    return out


def _qhull_piece(sites, i, planes, labels):
    """T_a intersected with all H_ij via qhull; returns (volume, active labels, vertices) or None."""
    A, b, lab = [], [], []
    for (n, c), l in zip(planes, labels):
        A.append(n); b.append(c); lab.append(l)
    vi = sites[i]
    for j in range(len(sites)):
        if j == i:
            continue
        n = sites[j] - vi
        A.append(n); b.append(0.5 * (sites[j] @ sites[j] - vi @ vi)); lab.append(j)
    A = np.array(A); b = np.array(b)
    norms = np.linalg.norm(A, axis=1)
    dim = A.shape[1]
    res = linprog(np.r_[np.zeros(dim), -1.0], A_ub=np.c_[A, norms], b_ub=b,
                  bounds=[(None, None)] * dim + [(0, None)], method="highs")
    if res.status != 0 or res.x[-1] < 1e-9:
        return None
    hs = HalfspaceIntersection(np.c_[A, -b], res.x[:dim])
    pts = hs.intersections
    hull = ConvexHull(pts)
    active = sorted({lab[k] for k in hs.dual_vertices})
    return hull.volume, active, pts


def test_brute_equals_pruned_3d(oracle_mod):
    for seed, n, k in [(11, 200, 2), (12, 500, 3)]:
        sites, dom = vdgen.small_case(n, k, seed=seed)
        a = canon_pieces(oracle_mod.compute(sites, dom, brute=True))
        b = canon_pieces(oracle_mod.compute(sites, dom, brute=False))
        nkey, ncomb, md = compare_canon(a, b, 0.0)
        assert nkey == 0 and ncomb == 0 and md == 0.0


def test_brute_equals_pruned_c1(oracle_mod):
    sites, dom = vdgen.config_c1()
    a = canon_pieces(oracle_mod.compute(sites, dom, brute=True))
    b = canon_pieces(oracle_mod.compute(sites, dom, brute=False))
    assert compare_canon(a, b, 0.0) == (0, 0, 0.0)


def test_against_qhull_halfspace_intersection(oracle_mod):
    """Every piece equals qhull's intersection of the tet and all bisector half-spaces."""
    sites, dom = vdgen.small_case(14, 1, seed=3)
    r = oracle_mod.compute(sites, dom, brute=True)
    got = {(int(s), int(a)): p for p, (s, a) in enumerate(zip(r["piece_site"], r["piece_simplex"]))}
    for a in range(dom.m):
        q = dom.verts[dom.simplices[a]]
        planes = _tet_planes(q)
        labels = [(-(int(dom.adj[a, f]) + 1)) if dom.adj[a, f] >= 0 else BND + f for f in range(4)]
        for i in range(len(sites)):
            ref = _qhull_piece(sites, i, planes, labels)
            p = got.get((i, a))
            if ref is None:
                assert p is None or r["piece_mass"][p] < 1e-12
                continue
            vol, active, pts = ref
            assert p is not None, (i, a)
            assert abs(r["piece_mass"][p] - vol) <= 1e-10 * vol
            fl = sorted(r["face_label"][r["piece_face_off"][p]:r["piece_face_off"][p + 1]].tolist())
            assert fl == active
            mine = r["vert_xyz"][r["piece_vert_off"][p]:r["piece_vert_off"][p + 1]]
            # every qhull vertex is an oracle vertex and vice versa
            d = np.linalg.norm(mine[:, None, :] - pts[None, :, :], axis=2)
            assert d.min(axis=0).max() < 1e-10 and d.min(axis=1).max() < 1e-10


def test_single_site_is_whole_domain(oracle_mod):
    dom = vdgen.kuhn_cube_grid(2)
    v = np.array([[0.3, 0.6, 0.45]])
    r = oracle_mod.compute(v, dom, brute=True)
    m = oracle_mod.site_moments(r, v)
    assert abs(m["mass"][0] - 1.0) < 1e-14
    assert np.allclose(m["centroid"][0], 0.5, atol=1e-14)
    exact = sum(1.0 / 3.0 - v[0, d] + v[0, d] ** 2 for d in range(3))
    assert abs(m["energy"][0] - exact) < 1e-14
    assert len(r["piece_site"]) == dom.m


def test_tiny_piece_far_from_its_site(oracle_mod):
    """A piece whose size is far below its distance to the site: with one site
    every piece is a whole tetrahedron, so the volume of a corner tetrahedron
    with legs 2^-20 placed ~1.7 away is eps^3/6 exactly.  A fan whose apex is
    the site carries ~1e-16 of rounding here (|y|^3 * machine epsilon), 1000x
    the volume itself, which flips the sign of the volume and drops the
    piece; an apex on the piece keeps the error ~1e-9 relative."""
    cube = vdgen.kuhn_cube_grid(1)
    eps = 2.0 ** -20
    p0 = np.array([1.25, 1.5, 1.75])
    tiny = np.stack([p0, p0 + [eps, 0, 0], p0 + [0, eps, 0], p0 + [0, 0, eps]])
    nv = len(cube.verts)
    verts = np.concatenate([cube.verts, tiny])
    tets = np.concatenate([cube.simplices, np.array([[nv, nv + 1, nv + 2, nv + 3]], dtype=cube.simplices.dtype)])
    dom = vdgen.Domain(verts=verts, simplices=tets, adj=vdgen.adjacency(tets), dim=3)
    v = np.array([[0.3, 0.6, 0.45]])
    r = oracle_mod.compute(v, dom, brute=True)
    assert len(r["piece_site"]) == dom.m
    k = int(np.nonzero(r["piece_simplex"] == dom.m - 1)[0][0])
    vol = eps ** 3 / 6
    assert abs(r["piece_mass"][k] - vol) <= 1e-8 * vol
    cen = p0 + eps / 4
    assert np.allclose(r["piece_moment"][k] / r["piece_mass"][k], cen, rtol=0, atol=1e-12)
    assert abs(r["piece_energy"][k] - vol * np.sum((cen - v[0]) ** 2)) <= 1e-8 * vol


def test_tiny_triangles_far_from_their_sites(oracle_mod):
    """2D analogue of the tiny-piece pin: the flat L-polygon mesh with its first
    grid line moved to 2^-30 has a corner square of two right triangles of area
    eps^2/2, about 0.5 from every site, so each is a whole piece of one site
    with exactly that area and the centroid of its three corners."""
    eps = 2.0 ** -30
    base = vdgen.planar_l_polygon(4)
    v = base.verts.copy()
    v[:, :2][v[:, :2] == 0.25] = eps
    dom = vdgen.Domain(verts=v, simplices=base.simplices, adj=base.adj, dim=2)
    rng = np.random.default_rng(5)
    s = np.zeros((5, 3))
    s[:, 0] = 0.3 + 0.15 * rng.random(5)
    s[:, 1] = 0.3 + 0.15 * rng.random(5)
    r = oracle_mod.compute(s, dom, brute=True)
    for t in (0, 1):
        k = np.nonzero(r["piece_simplex"] == t)[0]
        assert len(k) == 1
        k = int(k[0])
        assert abs(r["piece_mass"][k] - eps ** 2 / 2) <= 1e-9 * eps ** 2 / 2
        cen = v[dom.simplices[t]].mean(axis=0)
        assert np.allclose(r["piece_moment"][k] / r["piece_mass"][k], cen, rtol=0, atol=1e-15)
        d = np.linalg.norm(s - cen, axis=1)
        assert r["piece_site"][k] == int(np.argmin(d))


def test_two_sites_split_the_cube(oracle_mod):
    dom = vdgen.kuhn_cube_grid(1)
    x1, x2 = 0.23, 0.61
    s = np.array([[x1, 0.41, 0.52], [x2, 0.41, 0.52]])
    r = oracle_mod.compute(s, dom, brute=True)
    m = oracle_mod.site_moments(r, s)
    xm = 0.5 * (x1 + x2)
    assert abs(m["mass"][0] - xm) < 1e-14 and abs(m["mass"][1] - (1 - xm)) < 1e-14
    assert np.allclose(m["centroid"][0], [xm / 2, 0.5, 0.5], atol=1e-14)
    assert np.allclose(m["centroid"][1], [(1 + xm) / 2, 0.5, 0.5], atol=1e-14)
    assert list(m["neighbors"][0]) == [1] and list(m["neighbors"][1]) == [0]


def test_bcc_lattice_truncated_octahedra(oracle_mod):
    """BCC sites: every interior cell is a truncated octahedron (a simple
    polytope, 14 faces, 24 vertices) of volume a^3/2, centred on its site, with
    second moment 3 G V^(5/3), G = 19 / (192 * 2^(1/3)) (Conway & Sloane).
    An exact lattice puts intermediate vertices exactly on later bisectors, so
    the sites carry a jitter of 1e-7 a; the closed forms then hold to O(1e-7)."""
    a = 0.2
    shift = np.array([0.0123, 0.0271, 0.0391])
    g = np.arange(-1, 7)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    corner = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * a + shift
    s = np.concatenate([corner, corner + a / 2])
    s = s[np.all((s > 0) & (s < 1), axis=1)]
    s = s + np.random.default_rng(17).uniform(-1e-7 * a, 1e-7 * a, size=s.shape)
    dom = vdgen.kuhn_cube_grid(3)
    r = oracle_mod.compute(s, dom, brute=False)
    m = oracle_mod.site_moments(r, s)
    assert abs(m["mass"].sum() - 1.0) < 1e-12
    # all 14 neighbours present (the farthest sit at distance a along an axis)
    interior = np.all((s > a + 1e-3) & (s < 1 - a - 1e-3), axis=1)
    assert interior.sum() >= 20
    V = a ** 3 / 2
    G = 19.0 / (192.0 * 2 ** (1.0 / 3.0))
    assert np.allclose(m["mass"][interior], V, rtol=2e-6)
    assert np.allclose(m["centroid"][interior], s[interior], atol=1e-6 * a)
    assert np.allclose(m["energy"][interior], 3 * G * V ** (5.0 / 3.0), rtol=4e-6)
    assert all(len(m["neighbors"][i]) == 14 for i in np.nonzero(interior)[0])


def _kuhn_locate(p, k):
    """Index of the Kuhn tet of a k^3 unit-cube grid that contains p (brute force)."""
    dom = vdgen.kuhn_cube_grid(k)
    q = dom.verts[dom.simplices]
    T = np.stack([q[:, 1] - q[:, 0], q[:, 2] - q[:, 0], q[:, 3] - q[:, 0]], axis=2)
    Tinv = np.linalg.inv(T)
    lam = np.einsum("mij,pmj->pmi", Tinv, p[:, None, :] - q[None, :, 0, :])
    inside = np.all(lam >= -1e-12, axis=2) & (lam.sum(axis=2) <= 1 + 1e-12)
    return np.argmax(inside, axis=1), inside.any(axis=1)


def test_monte_carlo_nearest_site_labelling(oracle_mod):
    """Random points: the (tet, nearest site) pair must be a piece, and each
    cell's hit fraction must agree with its mass (5-sigma binomial)."""
    k = 2
    sites, dom = vdgen.small_case(40, k, seed=21)
    r = oracle_mod.compute(sites, dom, brute=True)
    m = oracle_mod.site_moments(r, sites)
    rng = np.random.default_rng(99)
    N = 20000
    p = rng.uniform(0, 1, size=(N, 3))
    nn = np.argmin(((p[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2), axis=1)
    tet, ok = _kuhn_locate(p, k)
    assert ok.all()
    pairs = set(zip(r["piece_site"].tolist(), r["piece_simplex"].tolist()))
    assert all((int(a), int(b)) in pairs for a, b in zip(nn, tet))
    frac = np.bincount(nn, minlength=len(sites)) / N
    sigma = np.sqrt(m["mass"] * (1 - m["mass"]) / N)
    assert np.all(np.abs(frac - m["mass"]) <= 5 * sigma + 1e-12)


def test_parity_inputs_are_in_general_position(oracle_mod):
    """The inputs of the bit-exact parity tests keep every decisive sign of the
    oracle's cuts well away from zero (relative margin |signed distance| /
    (|n| (|x| + |n|)) far above the FP64 error of the predicate), so their piece
    sets and labels are unique and any correct implementation must reproduce
    them exactly."""
    cases = [vdgen.small_case(300, 3, seed=5), vdgen.small_case(777, 5, seed=7),
             vdgen.small_case(2000, 4, seed=6), vdgen.config_c1(),
             vdgen.small_case(1500, 6, seed=9, jitter_domain=0.1)]
    for sites, dom in cases:
        r = oracle_mod.compute(sites, dom, brute=False)
        assert r["min_margin"] > 1e-9, r["min_margin"]


def test_invariants(oracle_mod):
    sites, dom = vdgen.small_case(150, 3, seed=8)
    r = oracle_mod.compute(sites, dom, brute=True)
    m = oracle_mod.site_moments(r, sites)
    n = len(sites)
    # partition of the domain and of every tet
    assert abs(m["mass"].sum() - 1.0) < 1e-12
    q = dom.verts[dom.simplices]
    tv = np.einsum("ij,ij->i", np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), q[:, 3] - q[:, 0]) / 6
    per_tet = np.bincount(r["piece_simplex"], weights=r["piece_mass"], minlength=dom.m)
    assert np.allclose(per_tet, tv, rtol=1e-12, atol=0)
    # face maps
    area = {}
    for p in range(len(r["piece_site"])):
        i, a = int(r["piece_site"][p]), int(r["piece_simplex"][p])
        for f in range(r["piece_face_off"][p], r["piece_face_off"][p + 1]):
            area[(i, a, int(r["face_label"][f]))] = r["face_measure"][f]
    for (i, a, l), ar in area.items():
        if l >= 0:   # bisector face: the neighbour's piece in the same tet has the twin face
            tw = area.get((l, a, i))
            assert tw is not None and abs(tw - ar) <= 1e-10 * ar
        elif l > BND + 3:   # shared tet face: the same site's piece in tet b has the twin face
            b = -l - 1
            tw = area.get((i, b, -(a + 1)))
            assert tw is not None and abs(tw - ar) <= 1e-10 * ar
    # neighbour symmetry
    nb = [set(x.tolist()) for x in m["neighbors"]]
    for i in range(n):
        for j in nb[i]:
            assert i in nb[j]
    # vertices: equidistant to the site and its positive labels; empty sphere
    for p in range(len(r["piece_site"])):
        i = int(r["piece_site"][p])
        for v in range(r["piece_vert_off"][p], r["piece_vert_off"][p + 1]):
            x = r["vert_xyz"][v]
            di = np.linalg.norm(x - sites[i])
            for l in r["vert_label"][v]:
                if 0 <= l < n:
                    assert abs(np.linalg.norm(x - sites[l]) - di) < 1e-12
            dall = np.linalg.norm(sites - x, axis=1)
            assert dall.min() >= di - 1e-12
    # every site lies in its own cell: the tet that contains it has its piece
    tet, ok = _kuhn_locate(sites, 3)
    pairs = set(zip(r["piece_site"].tolist(), r["piece_simplex"].tolist()))
    assert all((i, int(tet[i])) in pairs for i in range(n))


def test_face_loops_are_outward(oracle_mod):
    """Face loops run counter-clockwise seen from outside: the divergence theorem
    with the loop orientation reproduces the piece volume."""
    sites, dom = vdgen.small_case(60, 2, seed=31)
    r = oracle_mod.compute(sites, dom, brute=True)
    for p in range(0, len(r["piece_site"]), 7):
        V = 0.0
        base = r["piece_vert_off"][p]
        for f in range(r["piece_face_off"][p], r["piece_face_off"][p + 1]):
            loop = r["face_vert"][r["face_vert_off"][f]:r["face_vert_off"][f + 1]]
            y = r["vert_xyz"][base + loop]
            for t in range(1, len(y) - 1):
                V += np.dot(y[0], np.cross(y[t], y[t + 1])) / 6
        assert abs(V - r["piece_mass"][p]) < 1e-12


# --- surface (restricted VD) ------------------------------------------------

def _planar_square(k):
    """Unit square in the plane z = 0 split into 2 k^2 counter-clockwise triangles."""
    g = np.arange(k + 1) / k
    Y, X = np.meshgrid(g, g, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    tris = []
    for y in range(k):
        for x in range(k):
            a = x + (k + 1) * y
            tris += [[a, a + 1, a + k + 2], [a, a + k + 2, a + k + 1]]
    tris = np.array(tris, dtype=np.int32)
    return vdgen.Domain(verts=verts, simplices=tris, adj=vdgen.adjacency(tris), dim=2)


def test_surface_planar_matches_qhull_voronoi(oracle_mod):
    """Sites in the plane of a flat mesh: restricted cells are 2D Voronoi cells;
    bounded qhull Voronoi regions inside the square have the same areas and
    centroids."""
    from scipy.spatial import Voronoi
    rng = np.random.default_rng(41)
    p2 = rng.uniform(0, 1, size=(80, 2))
    s = np.c_[p2, np.zeros(len(p2))]
    dom = _planar_square(3)
    r = oracle_mod.compute(s, dom, brute=True)
    m = oracle_mod.site_moments(r, s)
    assert abs(m["mass"].sum() - 1.0) < 1e-12
    vor = Voronoi(p2)
    checked = 0
    for i in range(len(p2)):
        reg = vor.regions[vor.point_region[i]]
        if -1 in reg or len(reg) == 0:
            continue
        poly = vor.vertices[reg]
        if not np.all((poly > 0) & (poly < 1)):
            continue
        hull = ConvexHull(poly)
        pts = poly[hull.vertices]
        x, y = pts[:, 0], pts[:, 1]
        cr = x * np.roll(y, -1) - np.roll(x, -1) * y
        A = 0.5 * cr.sum()
        cx = ((x + np.roll(x, -1)) * cr).sum() / (6 * A)
        cy = ((y + np.roll(y, -1)) * cr).sum() / (6 * A)
        assert abs(m["mass"][i] - A) <= 1e-12 * A
        assert np.allclose(m["centroid"][i], [cx, cy, 0.0], atol=1e-12)
        nb = sorted(int(b) if a == i else int(a) for a, b in vor.ridge_points if i in (a, b))
        assert list(m["neighbors"][i]) == nb
        checked += 1
    assert checked >= 20


def test_surface_brute_equals_pruned_and_partition(oracle_mod):
    dom = vdgen.icosphere(3)
    s = vdgen.sphere_sites(300, seed=5)
    a = oracle_mod.compute(s, dom, brute=True)
    b = oracle_mod.compute(s, dom, brute=False)
    assert compare_canon(canon_pieces(a), canon_pieces(b), 0.0) == (0, 0, 0.0)
    q = dom.verts[dom.simplices]
    ta = 0.5 * np.linalg.norm(np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), axis=1)
    per = np.bincount(a["piece_simplex"], weights=a["piece_mass"], minlength=dom.m)
    assert np.allclose(per, ta, rtol=1e-12)
    # twin edges have equal lengths
    length = {}
    for p in range(len(a["piece_site"])):
        i, t = int(a["piece_site"][p]), int(a["piece_simplex"][p])
        for f in range(a["piece_face_off"][p], a["piece_face_off"][p + 1]):
            length[(i, t, int(a["face_label"][f]))] = a["face_measure"][f]
    for (i, t, l), ln in length.items():
        if l >= 0:
            assert abs(length[(l, t, i)] - ln) <= 1e-10 * ln


def test_surface_against_2d_qhull(oracle_mod):
    """Each polygon equals qhull's 2D half-space intersection in the triangle's plane."""
    dom = vdgen.icosphere(1)
    s = vdgen.sphere_sites(25, seed=9)
    r = oracle_mod.compute(s, dom, brute=True)
    got = {(int(a), int(b)): p for p, (a, b) in enumerate(zip(r["piece_site"], r["piece_simplex"]))}
    for t in range(dom.m):
        q = dom.verts[dom.simplices[t]]
        e1 = (q[1] - q[0]) / np.linalg.norm(q[1] - q[0])
        N = np.cross(q[1] - q[0], q[2] - q[0]); N /= np.linalg.norm(N)
        e2 = np.cross(N, e1)
        B = np.stack([e1, e2])            # 2D coords: u = B (x - q0)
        q2 = (q - q[0]) @ B.T
        planes, labels = [], []
        for e in range(3):
            A_, B_ = q2[(e + 1) % 3], q2[(e + 2) % 3]
            d = B_ - A_
            nrm = np.array([d[1], -d[0]])
            planes.append((nrm, nrm @ A_))
            labels.append(-(int(dom.adj[t, e]) + 1) if dom.adj[t, e] >= 0 else BND + e)
        for i in range(len(s)):
            A, b, lab = [p[0] for p in planes], [p[1] for p in planes], list(labels)
            for j in range(len(s)):
                if j == i:
                    continue
                n3 = s[j] - s[i]
                c3 = 0.5 * (s[j] @ s[j] - s[i] @ s[i])
                A.append(B @ n3); b.append(c3 - n3 @ q[0]); lab.append(j)
            A = np.array(A); b = np.array(b)
            res = linprog([0, 0, -1], A_ub=np.c_[A, np.linalg.norm(A, axis=1)], b_ub=b,
                          bounds=[(None, None)] * 2 + [(0, None)], method="highs")
            p = got.get((i, t))
            if res.status != 0 or res.x[-1] < 1e-9:
                assert p is None or r["piece_mass"][p] < 1e-12
                continue
            hs = HalfspaceIntersection(np.c_[A, -b], res.x[:2])
            area = ConvexHull(hs.intersections).volume
            assert p is not None and abs(r["piece_mass"][p] - area) <= 1e-10 * area
            fl = sorted(r["face_label"][r["piece_face_off"][p]:r["piece_face_off"][p + 1]].tolist())
            assert fl == sorted({lab[k] for k in hs.dual_vertices})


# --- adjoint ---------------------------------------------------------------

def _loss(oracle_mod, s, dom, gm, gc, ge):
    r = oracle_mod.compute(s, dom, brute=True)
    m = oracle_mod.site_moments(r, s)
    return (gm * m["mass"]).sum() + (gc * m["centroid"]).sum() + (ge * m["energy"]).sum()


def _grad(oracle_mod, s, dom, gm=None, gc=None, ge=None):
    r = oracle_mod.compute(s, dom, brute=True, keep_handle=True)
    m = oracle_mod.site_moments(r, s)
    try:
        g = oracle_mod.moments_backward(r, s, dom, m["mass"], m["centroid"], gm, gc, ge)
    finally:
        oracle_mod.free(r)
    return g, m


@pytest.mark.parametrize("surface", [False, True])
def test_adjoint_closed_forms(oracle_mod, surface):
    if surface:
        dom = vdgen.icosphere(2); s = vdgen.sphere_sites(40, seed=2)
    else:
        s, dom = vdgen.small_case(40, 2, seed=2)
    n = len(s)
    # CVT energy: the boundary terms cancel, gradient = 2 m (v - c)
    g, m = _grad(oracle_mod, s, dom, ge=np.ones(n))
    ref = 2 * m["mass"][:, None] * (s - m["centroid"])
    assert np.allclose(g, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    if not surface:
        # total mass is the domain volume: zero gradient
        g, _ = _grad(oracle_mod, s, dom, gm=np.ones(n))
        assert np.abs(g).max() < 1e-13
        # total first moment b . int_M x is constant: zero gradient
        b = np.array([0.3, -1.1, 0.7])
        g, m = _grad(oracle_mod, s, dom, gm=m["centroid"] @ b, gc=m["mass"][:, None] * b[None, :])
        assert np.abs(g).max() < 1e-12


def test_adjoint_two_sites(oracle_mod):
    """Two sites split the unit cube by the plane x = xm.  Moving v_1 moves that
    plane with normal speed (x - v_1).dv/d, so dm_1/dv_1 = int_F (x - v_1)/d dA
    = ((xm - x1), (1/2 - y), (1/2 - z)) / d over the unit square F, and
    dm_1/dv_2 = -((xm - x2), (1/2 - y), (1/2 - z)) / d."""
    dom = vdgen.kuhn_cube_grid(1)
    x1, x2, y, z = 0.23, 0.61, 0.41, 0.52
    s = np.array([[x1, y, z], [x2, y, z]])
    g, _ = _grad(oracle_mod, s, dom, gm=np.array([1.0, 0.0]))
    d, xm = x2 - x1, 0.5 * (x1 + x2)
    assert np.allclose(g[0], np.array([xm - x1, 0.5 - y, 0.5 - z]) / d, atol=1e-13)
    assert np.allclose(g[1], -np.array([xm - x2, 0.5 - y, 0.5 - z]) / d, atol=1e-13)
    assert abs(g[0, 0] - 0.5) < 1e-13


@pytest.mark.parametrize("surface", [False, True])
def test_adjoint_central_differences(oracle_mod, surface):
    if surface:
        dom = vdgen.icosphere(2); s = vdgen.sphere_sites(30, seed=12)
    else:
        s, dom = vdgen.small_case(30, 2, seed=12)
    n = len(s)
    rng = np.random.default_rng(107)
    gm, gc, ge = rng.normal(size=n), rng.normal(size=(n, 3)), rng.normal(size=n)
    g, _ = _grad(oracle_mod, s, dom, gm, gc, ge)
    d = rng.normal(size=(n, 3))
    h = 1e-6
    fd = (_loss(oracle_mod, s + h * d, dom, gm, gc, ge) - _loss(oracle_mod, s - h * d, dom, gm, gc, ge)) / (2 * h)
    an = (g * d).sum()
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # per-coordinate checks on a few sites
    for i in [0, 7, 19]:
        for k in range(3):
            e = np.zeros((n, 3)); e[i, k] = 1.0
            fd = (_loss(oracle_mod, s + h * e, dom, gm, gc, ge) - _loss(oracle_mod, s - h * e, dom, gm, gc, ge)) / (2 * h)
            assert abs(fd - g[i, k]) <= 1e-6 * max(1.0, abs(g[i, k]))


# --- face measures (areas of faces, lengths of edges) -------------------------

def _face_sums(r, site):
    """Sum of face_measure over the pieces of `site`, by face label."""
    out = {}
    for p in np.nonzero(r["piece_site"] == site)[0]:
        for f in range(r["piece_face_off"][p], r["piece_face_off"][p + 1]):
            lab = int(r["face_label"][f])
            out[lab] = out.get(lab, 0.0) + float(r["face_measure"][f])
    return out


def test_face_measure_two_sites_cube(oracle_mod):
    """Two sites split the unit cube at x = xm: the bisector face is the unit
    square (area 1, whichever tetrahedra it crosses), the boundary of cell 0
    has area 1 + 4 xm (the face x = 0 and four xm x 1 strips)."""
    dom = vdgen.kuhn_cube_grid(1)
    x1, x2 = 0.23, 0.61
    s = np.array([[x1, 0.41, 0.52], [x2, 0.41, 0.52]])
    r = oracle_mod.compute(s, dom, brute=True)
    xm = 0.5 * (x1 + x2)
    f0, f1 = _face_sums(r, 0), _face_sums(r, 1)
    assert abs(f0[1] - 1.0) < 1e-14 and abs(f1[0] - 1.0) < 1e-14
    bnd0 = sum(v for k, v in f0.items() if k <= BND + 3)
    bnd1 = sum(v for k, v in f1.items() if k <= BND + 3)
    assert abs(bnd0 - (1 + 4 * xm)) < 1e-14 and abs(bnd1 - (1 + 4 * (1 - xm))) < 1e-14


def test_face_measure_single_site_is_the_tet_faces(oracle_mod):
    """One site: every piece is a whole tetrahedron and each of its faces has
    the area of the tetrahedron's face, |(b - a) x (c - a)| / 2."""
    dom = vdgen.kuhn_cube_grid(2, jitter=0.1, seed=3)
    v = np.array([[0.41, 0.37, 0.55]])
    r = oracle_mod.compute(v, dom, brute=True)
    assert len(r["piece_site"]) == dom.m
    for p in range(dom.m):
        a = int(r["piece_simplex"][p])
        q = dom.verts[dom.simplices[a]]
        for f in range(r["piece_face_off"][p], r["piece_face_off"][p + 1]):
            lab = int(r["face_label"][f])
            if lab <= BND + 3:
                k = lab - BND
            else:
                k = int(np.nonzero(dom.adj[a] == -lab - 1)[0][0])
            tri = q[[t for t in range(4) if t != k]]
            area = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
            assert abs(r["face_measure"][f] - area) <= 1e-14 * max(area, 1.0)


def test_face_measure_bcc_truncated_octahedron(oracle_mod):
    """BCC lattice (cube side a): an interior cell is a truncated octahedron with
    6 square faces of area a^2/8 (towards the neighbours at distance a) and 8
    regular hexagons of area 3 sqrt(3) a^2 / 16 (towards the neighbours at
    distance a sqrt(3)/2), summed over the tetrahedra each face crosses.  The
    1e-7 a jitter moves the areas by O(1e-7) relative."""
    a = 0.2
    shift = np.array([0.0123, 0.0271, 0.0391])
    g = np.arange(-1, 7)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    corner = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * a + shift
    s = np.concatenate([corner, corner + a / 2])
    s = s[np.all((s > 0) & (s < 1), axis=1)]
    s = s + np.random.default_rng(17).uniform(-1e-7 * a, 1e-7 * a, size=s.shape)
    dom = vdgen.kuhn_cube_grid(3)
    r = oracle_mod.compute(s, dom, brute=False)
    interior = np.nonzero(np.all((s > a + 1e-3) & (s < 1 - a - 1e-3), axis=1))[0]
    assert len(interior) >= 20
    sq, hexa = a * a / 8, 3 * np.sqrt(3) * a * a / 16
    for i in interior:
        fs = {k: v for k, v in _face_sums(r, int(i)).items() if k >= 0}
        assert len(fs) == 14
        for j, ar in fs.items():
            d = np.linalg.norm(s[j] - s[i])
            want = sq if d > 0.95 * a else hexa
            assert abs(d - (a if want == sq else a * np.sqrt(3) / 2)) < 1e-5 * a
            assert abs(ar - want) <= 2e-6 * want, (i, j, ar, want)


def test_face_measure_2d_edge_lengths(oracle_mod):
    """Flat square mesh, two sites in its plane at (x1, y), (x2, y): the bisector
    edge is the segment x = xm across the square, of length 1; the boundary of
    cell 0 has length 1 + 2 xm."""
    dom = _planar_square(3)
    x1, x2 = 0.27, 0.58
    s = np.array([[x1, 0.43, 0.0], [x2, 0.43, 0.0]])
    r = oracle_mod.compute(s, dom, brute=True)
    xm = 0.5 * (x1 + x2)
    f0 = _face_sums(r, 0)
    assert abs(f0[1] - 1.0) < 1e-14
    assert abs(sum(v for k, v in f0.items() if k <= BND + 2) - (1 + 2 * xm)) < 1e-14
    assert abs(_face_sums(r, 1)[0] - 1.0) < 1e-14


def test_sampled_sites_equal_the_full_run(oracle_mod):
    """The sampled-site mode (candidate simplices from a grid over the simplex
    boxes) returns exactly the pieces the full pruned run gives those sites, on
    the 100,000-site, 48,000-tetrahedron workload."""
    sites, dom = vdgen.config_c2()
    full = oracle_mod.compute(sites, dom, threads=0)
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(len(sites), size=3000, replace=False)).astype(np.int32)
    part = oracle_mod.compute(sites, dom, only_sites=sample, threads=0)
    sel = np.nonzero(np.isin(full["piece_site"], sample))[0]
    a = canon_pieces(part)
    b = canon_pieces(subset_result(full, sel))
    assert len(a) == len(sel) == len(b)
    assert compare_canon(a, b, 0.0) == (0, 0, 0.0)
    assert np.array_equal(part["piece_mass"], full["piece_mass"][sel])
    assert np.array_equal(part["piece_energy"], full["piece_energy"][sel])
