"""GPU checks of the boundary beyond the four hot-path calls: adjacency
computed by the library, the convexity flag of a staged domain, vd_sync, the
work and margin counters of vd_cells_info, and the handling of an output
arena that overflows in a no-sync clip (bounded writes, VD_ERR_CAPACITY,
NaN gradients)."""
import numpy as np
import pytest

import vdgen
from gpu_util import log, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _tensor(x, dt):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


@pytest.mark.parametrize("name", ["cube6_jitter", "icosphere3", "l_block4", "cavity6", "planar_l8"])
def test_adjacency_computed_on_device(name):
    """Face matching on the device gives the same adjacency as the generator's
    sort-based one (Sec. 3.2 flags come from it)."""
    import torch
    import paper_2509_07175_amd as vd
    dom = {"cube6_jitter": lambda: vdgen.kuhn_cube_grid(6, jitter=0.1, seed=3),
           "icosphere3": lambda: vdgen.icosphere(3), "l_block4": lambda: vdgen.l_block(4),
           "cavity6": lambda: vdgen.cube_with_cavity(6), "planar_l8": lambda: vdgen.planar_l_polygon(8)}[name]()
    log(f"adjacency {name}: m={dom.m}")
    d = vd.Domain.from_vdgen(dom, adjacency=False)
    got = d.adjacency().cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(got, dom.adj)


def test_adjacency_computed_for_a_batch():
    import paper_2509_07175_amd as vd
    doms = [vdgen.kuhn_cube_grid(3), vdgen.l_block(4), vdgen.kuhn_cube_grid(2, jitter=0.1, seed=5)]
    vo, so = [0], [0]
    for d in doms:
        vo.append(vo[-1] + len(d.verts))
        so.append(so[-1] + d.m)
    import torch
    verts = _tensor(np.concatenate([d.verts for d in doms]), torch.float64)
    simp = _tensor(np.concatenate([d.simplices for d in doms]), torch.int32)
    D = vd.Domain.batch(verts, simp, None, vo, so, 3)
    got = D.adjacency().cpu().numpy()
    want = np.concatenate([np.where(d.adj >= 0, d.adj + so[b], -1) for b, d in enumerate(doms)])
    assert np.array_equal(got, want)
    assert D.info()["convex"] == 0  # the L-block is not convex


def test_non_manifold_mesh_is_rejected():
    """Three tetrahedra on one face: vd_domain_create refuses to compute an adjacency."""
    import torch
    import paper_2509_07175_amd as vd
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [0.2, 0.2, 0.9]], dtype=np.float64)
    tets = np.array([[0, 1, 2, 3], [0, 2, 1, 4], [0, 1, 2, 5]], dtype=np.int32)
    with pytest.raises(vd.VDError) as e:
        vd.Domain(_tensor(verts, torch.float64), _tensor(tets, torch.int32), None, 3)
    assert e.value.status == 1 and "non-manifold" in str(e.value)


def test_convexity_flag():
    import paper_2509_07175_amd as vd
    cases = {"cube": (vdgen.kuhn_cube_grid(4), 1), "jittered cube": (vdgen.kuhn_cube_grid(5, jitter=0.1, seed=2), 1),
             "L-block": (vdgen.l_block(4), 0), "cavity": (vdgen.cube_with_cavity(6), 0),
             "sphere": (vdgen.icosphere(2), -1)}
    for name, (dom, want) in cases.items():
        info = vd.Domain.from_vdgen(dom).info()
        log(f"{name}: {info}")
        assert info["convex"] == want, name
        assert info["n_simplices"] == dom.m


def test_clip_with_library_adjacency_is_identical():
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(3000, 6, seed=41, jitter_domain=0.1)
    s = _tensor(sites, torch.float64)
    out = []
    for adj in (True, False):
        d = vd.Domain.from_vdgen(dom, adjacency=adj)
        g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1))
        c = vd.clip_cells(g, d)
        m, ce, e = c.moments()
        out.append((m.cpu().numpy(), ce.cpu().numpy(), vd.pieces_as_result(c.view())))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    for k in ("piece_site", "piece_simplex", "face_label", "vert_label"):
        assert np.array_equal(out[0][2][k], out[1][2][k]), k


def test_sync_and_counters():
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(5000, 8, seed=43)
    quiet = run_gpu(sites, dom)["info"]
    assert quiet["query_rounds"] == -1 and quiet["min_margin"] == -1.0
    gpu = run_gpu(sites, dom, monitor=1)
    vd.sync()
    info = gpu["info"]
    log(f"info {info}")
    nvert = np.diff(gpu["res"]["piece_vert_off"])
    # every emitted piece is integrated on a fan of three tetrahedra per corner
    assert info["fan_simplices"] == 3 * int(nvert.sum())
    assert info["overflow_records"] == 0
    assert 0 < info["query_rounds"] <= info["nn_queries"]
    assert info["corners_created"] >= 3 * info["clips"]
    assert info["corners_classified"] > info["corners_created"]
    assert 0.0 < info["min_margin"] <= 1.0 and info["low_margin"] == 0
    assert 0 <= info["tests_wasted"] < info["nn_queries"]
    # a convex domain holding every site needs no boundary seeds
    assert info["sites_outside"] == 0 and info["boundary_seeded"] == 0


def test_surface_counters():
    sites, dom = vdgen.sphere_sites(3000, seed=44), vdgen.icosphere(3)
    gpu = run_gpu(sites, dom, bbox=(-1, -1, -1, 1, 1, 1), surface_area=4 * np.pi, monitor=1)
    info = gpu["info"]
    nvert = np.diff(gpu["res"]["piece_vert_off"])
    assert info["fan_simplices"] >= int(nvert.sum())
    assert info["overflow_records"] == 0 and info["low_margin"] == 0 and 0 < info["min_margin"] <= 1.0
    # a clip that leaves a polygon creates two corners; one that empties it, none
    assert 0 < info["corners_created"] <= 2 * info["clips"]


def test_no_sync_overflow_is_reported_and_bounded():
    """A no-sync clip cannot grow its arenas: the handle is sized on a 6-tet
    cube, then clipped without sync on a 12^3 x 6 grid (10,368 tetrahedra,
    far more pieces than the arenas hold).  Every write stays in the arenas,
    the clip reports VD_ERR_CAPACITY, the views refuse, the adjoint is NaN,
    and a synchronous clip on the same handle then grows it and is exact."""
    import torch
    import paper_2509_07175_amd as vd
    sites = vdgen.uniform_cube_sites(300, seed=45, jitter=1e-7)
    coarse, fine = vdgen.kuhn_cube_grid(1), vdgen.kuhn_cube_grid(12)
    s = _tensor(sites, torch.float64)
    g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1))
    dc, df = vd.Domain.from_vdgen(coarse), vd.Domain.from_vdgen(fine)
    c = vd.Cells()
    c.clip(g, dc, vd.Options.default(want_grad=1))
    assert c.info()["status"] == 0
    log("no-sync clip on the fine domain with the coarse sizing")
    c.clip(g, df, vd.Options.default(want_grad=1, no_sync=1))
    m, ce, e = c.moments()
    gs = c.backward(g_mass=torch.ones(len(sites), dtype=torch.float64, device="cuda"))
    vd.sync()
    info = c.info()
    log(f"overflowed no-sync info {info}")
    assert info["status"] == 4 and info["overflow_records"] > 0
    with pytest.raises(vd.VDError) as ex:
        c.view()
    assert ex.value.status == 4
    assert torch.isnan(gs).all()
    # the masses are sums formed before emission: still the fine domain's
    assert abs(float(m.sum()) - 1.0) < 1e-12
    # a synchronous clip grows the arenas and matches a fresh handle
    c.clip(g, df, vd.Options.default(want_grad=1))
    m2, _, _ = c.moments()
    ref = vd.clip_cells(g, df, vd.Options.default(want_grad=1))
    m3, _, _ = ref.moments()
    assert torch.equal(m2, m3)
    a, b = vd.pieces_as_result(c.view()), vd.pieces_as_result(ref.view())
    assert np.array_equal(a["piece_site"], b["piece_site"]) and np.array_equal(a["piece_simplex"], b["piece_simplex"])


def test_repeated_sites_are_rejected(oracle_mod):
    """Eq. 1 needs distinct sites (a copy's bisector is undefined): a 3D clip
    whose sites repeat an earlier one exactly returns VD_ERR_INVALID_ARG,
    naming the first copy, before any cell is carved; in a batch too.  A power
    diagram may hold two sites at one point with different weights (the
    lighter one has an empty cell), which matches the oracle."""
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(400, 3, seed=61)
    rep = sites.copy()
    rep[250] = rep[17]
    rep[300] = rep[17]
    with pytest.raises(vd.VDError, match="repeat an earlier site exactly \\(first: 250\\)"):
        run_gpu(rep, dom)
    so = np.array([0, 400, 800])
    both = np.vstack([sites, rep])
    d = vd.Domain.batch_from_vdgen([dom, dom])
    g = vd.build_grid_batch(_tensor(both, __import__("torch").float64), so, bboxes=[(0, 0, 0, 1, 1, 1)] * 2)
    with pytest.raises(vd.VDError, match="first: 650"):
        vd.clip_cells(g, d, vd.Options.default())
    w = np.random.default_rng(62).uniform(-1e-3, 1e-3, size=400)
    w[250] = w[17] - 0.01
    pw = sites.copy()
    pw[250] = pw[17]
    gpu = run_gpu(pw, dom, weights=w)
    ref = oracle_mod.compute(pw, dom, brute=False, weights=w)
    mom = oracle_mod.site_moments(ref, pw)
    assert gpu["mass"][250] == 0.0 and mom["mass"][250] == 0.0
    assert np.all(np.abs(gpu["mass"] - mom["mass"]) <= 1e-9 * np.maximum(mom["mass"], 1e-300))


def test_argument_errors():
    """Sites that are not finite (3D, found before any carve), no sites, an
    empty domain: VD_ERR_INVALID_ARG with a message, and the library stays
    usable afterwards."""
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(300, 3, seed=63)
    bad = sites.copy()
    bad[120, 1] = np.nan
    bad[200, 2] = np.inf
    with pytest.raises(vd.VDError, match="not finite \\(first: 120\\)"):
        run_gpu(bad, dom)
    with pytest.raises(vd.VDError, match="n < 1"):
        vd.build_grid(torch.empty((0, 3), dtype=torch.float64, device="cuda"), bbox=(0, 0, 0, 1, 1, 1))
    with pytest.raises(vd.VDError, match="empty domain"):
        vd.Domain(torch.zeros((4, 3), dtype=torch.float64, device="cuda"),
                  torch.empty((0, 4), dtype=torch.int32, device="cuda"), None, 3)
    ok = run_gpu(sites, dom)
    assert abs(ok["mass"].sum() - 1.0) < 1e-12
