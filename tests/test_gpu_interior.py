"""Alg. 5's split of interior and boundary sites (vd_options.whole_interior):
the restricted diagram of the boundary surface is computed first, and a cell
that meets no boundary triangle is returned as one piece (simplex -1), not cut
by the tetrahedra.

Checks, against the oracle (which always cuts per tetrahedron, Eq. 1):
* every site the oracle gives a boundary face is cut per tetrahedron, and its
  pieces are the oracle's (bit-exact combinatorics, vertices to 1e-10);
* an interior site has exactly one piece: its mass, centroid and energy are the
  sum of the oracle's pieces (1e-9), its faces are its neighbours, and its
  vertices are exactly the oracle's vertices of that site that lie on three
  bisectors (the Voronoi vertices of the cell), each equidistant from its four
  sites;
* per-site moments and neighbour lists equal those of the default clip, at
  full size too, with density, power weights, gradients and a non-convex
  domain."""
import numpy as np
import pytest

import vdgen
from canon import canon_pieces
from gpu_util import assert_parity, log, run_gpu

pytestmark = pytest.mark.gpu

INT32_MIN = -2 ** 31


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _oracle_boundary_sites(ref):
    """Sites with a piece that has a face on the boundary of M (per-tetrahedron
    pieces in the oracle's layout)."""
    ps, fo, fl = ref["piece_site"], ref["piece_face_off"], ref["face_label"]
    on_b = np.zeros(len(ps), bool)
    for p in range(len(ps)):
        on_b[p] = bool((fl[fo[p]:fo[p + 1]] <= INT32_MIN + 3).any())
    return set(int(s) for s in np.unique(ps[on_b]))


def _check_against_oracle(gpu, ref, mom, sites, n):
    res = gpu["res"]
    whole = res["piece_simplex"] == -1
    interior = np.unique(res["piece_site"][whole]).astype(np.int64)
    # one piece per interior site
    cnt = np.bincount(res["piece_site"], minlength=n)
    assert np.all(cnt[interior] == 1)
    bsites = _oracle_boundary_sites(ref)
    assert not (set(interior.tolist()) & bsites), "a site with a boundary face was taken as interior"
    rest = np.setdiff1d(np.arange(n), interior)
    if len(rest):
        assert_parity(gpu, ref, mom, n, sites_subset=rest)
    # interior sites: moments and neighbours as the oracle's sums
    rel = 1e-9
    m_g, m_r = gpu["mass"][interior], mom["mass"][interior]
    assert np.all(np.abs(m_g - m_r) <= rel * m_r)
    c_g, c_r = gpu["centroid"][interior], mom["centroid"][interior]
    assert np.all(np.linalg.norm(c_g - c_r, axis=1) <= rel * np.linalg.norm(c_r, axis=1))
    e_g, e_r = gpu["energy"][interior], mom["energy"][interior]
    assert np.all(np.abs(e_g - e_r) <= rel * e_r)
    off, nb = gpu["nbr_off"], gpu["nbr"]
    cg = canon_pieces(res)
    rps, rvo, rvl = ref["piece_site"], ref["piece_vert_off"], ref["vert_label"]
    ref_vertex_labels = {}
    for p in range(len(rps)):
        s = int(rps[p])
        for t in rvl[rvo[p]:rvo[p + 1]].tolist():
            if min(t) >= 0:
                ref_vertex_labels.setdefault(s, set()).add(tuple(sorted(t)))
    for i in interior.tolist():
        assert list(nb[off[i]:off[i + 1]]) == list(mom["neighbors"][i]), f"neighbours of site {i}"
        faces, labs, xyz = cg[(i, -1)]
        assert list(faces) == sorted(mom["neighbors"][i]), f"faces of the whole cell {i}"
        assert set(labs) == ref_vertex_labels.get(i, set()), f"vertices of the whole cell {i}"
        # every vertex is equidistant from its site and its three flags
        d0 = np.linalg.norm(xyz - sites[i], axis=1)
        for k in range(3):
            dk = np.linalg.norm(xyz - sites[np.array([t[k] for t in labs])], axis=1)
            assert np.all(np.abs(dk - d0) <= 1e-10)
    log(f"whole_interior: {len(interior)} interior sites of {n}, {len(rest)} cut per tetrahedron")
    return interior


@pytest.mark.parametrize("n,k,seed", [(900, 4, 401), (3000, 6, 402)])
def test_whole_interior_against_the_oracle(oracle_mod, n, k, seed):
    """Cube grids whose boundary triangles meet a few cells each: the split by
    the boundary diagram."""
    sites, dom = vdgen.small_case(n, k, seed=seed)
    gpu = run_gpu(sites, dom, whole_interior=1)
    ref = oracle_mod.compute(sites, dom, brute=False)
    mom = oracle_mod.site_moments(ref, sites)
    interior = _check_against_oracle(gpu, ref, mom, sites, n)
    assert len(interior) > n // 4
    assert abs(gpu["mass"].sum() - 1.0) < 1e-12
    assert gpu["info"]["boundary_seeded"] == 1


@pytest.mark.parametrize("n,seed", [(1000, 101), (2500, 409)])
def test_whole_interior_by_corners_against_the_oracle(oracle_mod, n, seed):
    """The unit cube as 6 tetrahedra (12 boundary triangles, each meeting
    dozens of cells): a convex domain holding every site, split by the cells'
    corners without a boundary diagram (n = 1,000: the shape of the 1k-site
    cube workload)."""
    sites, dom = vdgen.small_case(n, 1, seed=seed)
    gpu = run_gpu(sites, dom, whole_interior=1)
    assert gpu["info"]["boundary_seeded"] == 0
    ref = oracle_mod.compute(sites, dom, brute=n <= 1000)
    mom = oracle_mod.site_moments(ref, sites)
    interior = _check_against_oracle(gpu, ref, mom, sites, n)
    assert len(interior) > n // 4
    assert abs(gpu["mass"].sum() - 1.0) < 1e-12


def test_whole_interior_non_convex(oracle_mod):
    import test_oracle_nonconvex as t
    sites, dom = t._cases()["l_block"]
    gpu = run_gpu(sites, dom, bbox=(-0.5, -0.5, -0.5, 1.5, 1.5, 1.5), whole_interior=1)
    ref = oracle_mod.compute(sites, dom, brute=True)
    mom = oracle_mod.site_moments(ref, sites)
    _check_against_oracle(gpu, ref, mom, sites, len(sites))


def test_whole_interior_power(oracle_mod):
    n = 900
    sites, dom = vdgen.small_case(n, 4, seed=403)
    rng = np.random.default_rng(404)
    w = rng.uniform(-1.0 / n, 1.0 / n, size=n)
    w[0] = -0.05
    w[1] = 0.02
    gpu = run_gpu(sites, dom, weights=w, whole_interior=1)
    ref = oracle_mod.compute(sites, dom, brute=False, weights=w)
    mom = oracle_mod.site_moments(ref, sites)
    res = gpu["res"]
    interior = np.unique(res["piece_site"][res["piece_simplex"] == -1]).astype(np.int64)
    rest = np.setdiff1d(np.arange(n), interior)
    assert_parity(gpu, ref, mom, n, sites_subset=rest)
    nz = mom["mass"][interior] > 0
    assert np.all(nz)
    assert np.all(np.abs(gpu["mass"][interior] - mom["mass"][interior]) <= 1e-9 * mom["mass"][interior])
    c_g, c_r = gpu["centroid"][interior], mom["centroid"][interior]
    assert np.all(np.linalg.norm(c_g - c_r, axis=1) <= 1e-9 * np.linalg.norm(c_r, axis=1))
    assert gpu["mass"][0] == 0.0 and abs(gpu["mass"].sum() - 1.0) < 1e-12
    log(f"power whole_interior: {len(interior)} interior cells of {n}")


def _same_sites(a, b, rel=1e-12):
    assert np.all(np.abs(a["mass"] - b["mass"]) <= rel * np.maximum(b["mass"], 1e-300))
    assert np.all(np.linalg.norm(a["centroid"] - b["centroid"], axis=1) <=
                  rel * np.linalg.norm(b["centroid"], axis=1) + 1e-300)
    assert np.all(np.abs(a["energy"] - b["energy"]) <= rel * np.maximum(b["energy"], 1e-300))
    assert np.array_equal(a["nbr_off"], b["nbr_off"]) and np.array_equal(a["nbr"], b["nbr"])


def test_whole_interior_equals_default_c2():
    """100,000 uniform sites, 48,000 tetrahedra: the same per-site moments
    (1e-12) and neighbour lists as the default clip; the pieces of the sites
    cut per tetrahedron are the default's, bit for bit."""
    sites, dom = vdgen.config_c2()
    a = run_gpu(sites, dom, whole_interior=1)
    b = run_gpu(sites, dom)
    _same_sites(a, b)
    ra, rb = a["res"], b["res"]
    cut = np.setdiff1d(np.arange(len(sites)), ra["piece_site"][ra["piece_simplex"] == -1])
    sel_a = np.isin(ra["piece_site"], cut)
    sel_b = np.isin(rb["piece_site"], cut)
    assert np.array_equal(ra["piece_site"][sel_a], rb["piece_site"][sel_b])
    assert np.array_equal(ra["piece_simplex"][sel_a], rb["piece_simplex"][sel_b])
    assert np.array_equal(ra["piece_mass"][sel_a], rb["piece_mass"][sel_b])
    log(f"C2 whole_interior: {len(sites) - len(cut)} whole cells, {len(cut)} cut; "
        f"pieces {a['info']['n_pieces']} against {b['info']['n_pieces']}")


def test_whole_interior_density_and_gradient():
    """With a quadratic density and want_grad: moments and the adjoint of a
    random loss equal the default clip's."""
    import torch
    rho = [1.0, 0.5, -0.3, 0.2, 0.4, 0.1, -0.2, 0.3, 0.05, 0.6]
    sites, dom = vdgen.small_case(3000, 6, seed=405)
    n = len(sites)
    rng = np.random.default_rng(406)
    up = [torch.as_tensor(x, dtype=torch.float64, device="cuda")
          for x in (rng.normal(size=n), rng.normal(size=(n, 3)), rng.normal(size=n))]
    out = []
    for whole in (1, 0):
        r = run_gpu(sites, dom, whole_interior=whole, want_grad=1, density=rho)
        g = r["cells"].backward(*up)
        torch.cuda.synchronize()
        out.append((r, g.cpu().numpy()))
    _same_sites(out[0][0], out[1][0])
    ga, gb = out[0][1], out[1][1]
    assert np.abs(ga - gb).max() <= 1e-10 * np.abs(gb).max()


def test_whole_interior_c3_full_size():
    """The 1M clustered workload: per-site moments and neighbour lists equal
    the default clip's."""
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.config_c3()
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1), sites_per_cell=0.25)
    outs = []
    for whole in (1, 0):
        c = vd.clip_cells(g, d, vd.Options.default(whole_interior=whole, time_kernels=1))
        m, ce, e = c.moments()
        v = c.view()
        torch.cuda.synchronize()
        info = c.info()
        outs.append((m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy(), v["nbr_off"].cpu().numpy(),
                     v["nbr"].cpu().numpy(), info))
        log(f"C3 whole_interior={whole}: site kernel {info['carve_ms']:.2f} ms, pieces {info['n_pieces']}")
        del c
    (ma, ca, ea, oa, na, _), (mb, cb, eb, ob, nb, _) = outs
    assert np.all(np.abs(ma - mb) <= 1e-12 * mb)
    assert np.all(np.linalg.norm(ca - cb, axis=1) <= 1e-12 * np.linalg.norm(cb, axis=1))
    assert np.all(np.abs(ea - eb) <= 1e-12 * eb)
    assert np.array_equal(oa, ob) and np.array_equal(na, nb)
    assert abs(ma.sum() - 1.0) < 1e-11


def test_whole_interior_rejections():
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(300, 3, seed=407)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1))
    d = vd.Domain.from_vdgen(dom)
    for bad in ({"carve_mode": 0}, {"boundary_seeds": 0}):
        with pytest.raises(vd.VDError):
            vd.clip_cells(g, d, vd.Options.default(whole_interior=1, **bad))
    c = vd.clip_cells(g, d, vd.Options.default())
    with pytest.raises(vd.VDError):
        vd.clip_cells(g, d, vd.Options.default(whole_interior=1, no_sync=1), cells=c)
    sph = vdgen.icosphere(2)
    ss = torch.as_tensor(vdgen.sphere_sites(100, seed=408), dtype=torch.float64, device="cuda")
    gs = vd.build_grid(ss, bbox=(-1.3, -1.3, -1.3, 1.3, 1.3, 1.3), surface_area=12.0)
    with pytest.raises(vd.VDError):
        vd.clip_cells(gs, vd.Domain.from_vdgen(sph), vd.Options.default(whole_interior=1))


def test_whole_interior_cavity_at_scale():
    """30,000 sites around a cubic cavity (9,984 tetrahedra, not convex): the
    same per-site moments and neighbours as the default clip, which is checked
    against the oracle on this domain; sites next to the cavity are cut per
    tetrahedron."""
    sites = vdgen.uniform_cube_sites(40000, seed=93, jitter=1e-7)
    sites = sites[~np.all((sites > 1 / 3) & (sites < 2 / 3), axis=1)][:30000]
    dom = vdgen.cube_with_cavity(12)
    a = run_gpu(sites, dom, whole_interior=1)
    b = run_gpu(sites, dom)
    _same_sites(a, b)
    ra = a["res"]
    whole = set(ra["piece_site"][ra["piece_simplex"] == -1].tolist())
    # the split is exact: a cell is whole iff none of its per-tetrahedron
    # pieces in the default clip has a face on the boundary of M
    touching = _oracle_boundary_sites(b["res"])
    assert not (touching & whole)
    assert touching | whole == set(range(len(sites)))
    log(f"cavity whole_interior: {len(whole)} whole cells of {len(sites)}")
