"""Batches of independent diagrams (one persistent launch over all of them).

* every diagram of a batch gives exactly what a plain call on that diagram
  alone gives (same combinatorics, same moments bit for bit), with indices
  shifted by the diagram's offsets;
* one diagram of a batch against the oracle;
* the no-sync clip (graph-capturable) equals the synchronous one, and a HIP
  graph of grid build + clip + moments, replayed on changed sites with eager
  work between replays, equals eager calls every time;
* the batched workload of 256 diagrams (1,000 - 64,000 sites each, jittered
  8^3 - 24^3 cube grids) at full size: per-diagram volumes, a sample of sites
  against the oracle.
"""
import numpy as np
import pytest

import vdgen
from gpu_util import assert_parity, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small_batch(seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(5):
        n = int(rng.integers(150, 900))
        k = int(rng.integers(2, 6))
        out.append((vdgen.uniform_cube_sites(n, seed=seed * 100 + b, jitter=1e-7),
                    vdgen.kuhn_cube_grid(k, jitter=0.1, seed=seed * 100 + 50 + b)))
    return out


def _run_batch(items, **opts):
    import torch
    import paper_2509_07175_amd as vd
    so = np.concatenate([[0], np.cumsum([len(s) for s, _ in items])])
    sites = torch.as_tensor(np.concatenate([s for s, _ in items]), dtype=torch.float64, device="cuda")
    dom = vd.Domain.batch_from_vdgen([d for _, d in items])
    g = vd.build_grid_batch(sites, so, bboxes=[(0, 0, 0, 1, 1, 1)] * len(items))
    c = vd.clip_cells(g, dom, vd.Options.default(**opts))
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    view = c.view()
    return {"mass": m.cpu().numpy(), "centroid": ce.cpu().numpy(), "energy": e.cpu().numpy(),
            "res": vd.pieces_as_result(view), "nbr_off": view["nbr_off"].cpu().numpy(),
            "nbr": view["nbr"].cpu().numpy(), "site_off": so, "simp_off": dom.simp_off, "info": c.info()}


def _run_plain(sites, dom, **opts):
    from gpu_util import run_gpu
    return run_gpu(sites, dom, **opts)


def test_batch_equals_plain_per_diagram():
    items = _small_batch()
    B = _run_batch(items)
    so, mo = B["site_off"], B["simp_off"]
    res = B["res"]
    for b, (s, d) in enumerate(items):
        P = _run_plain(s, d)
        lo, hi = so[b], so[b + 1]
        assert np.array_equal(B["mass"][lo:hi], P["mass"]), f"diagram {b}: masses differ"
        assert np.array_equal(B["centroid"][lo:hi], P["centroid"])
        assert np.array_equal(B["energy"][lo:hi], P["energy"])
        # pieces of this diagram, shifted back to local indices
        sel = (res["piece_site"] >= lo) & (res["piece_site"] < hi)
        assert np.array_equal(res["piece_site"][sel] - lo, P["res"]["piece_site"])
        assert np.array_equal(res["piece_simplex"][sel] - mo[b], P["res"]["piece_simplex"])
        assert np.array_equal(res["piece_mass"][sel], P["res"]["piece_mass"])
        for i in range(len(s)):
            nb = B["nbr"][B["nbr_off"][lo + i]:B["nbr_off"][lo + i + 1]] - lo
            npl = P["nbr"][P["nbr_off"][i]:P["nbr_off"][i + 1]]
            assert np.array_equal(nb, npl), f"diagram {b} site {i}: neighbours differ"
        vol = B["mass"][lo:hi].sum()
        assert abs(vol - 1.0) < 1e-12


def test_batch_diagram_against_oracle(oracle_mod):
    items = _small_batch(seed=12)
    B = _run_batch(items)
    b = 3
    s, d = items[b]
    lo, hi = B["site_off"][b], B["site_off"][b + 1]
    ref = oracle_mod.compute(s, d, brute=True)
    mom = oracle_mod.site_moments(ref, s)
    res = B["res"]
    sel = (res["piece_site"] >= lo) & (res["piece_site"] < hi)
    # rebuild a per-diagram result in the oracle's layout (local indices)
    fo, vo = res["piece_face_off"], res["piece_vert_off"]
    idx = np.nonzero(sel)[0]
    gl = {"piece_site": res["piece_site"][idx] - lo, "piece_simplex": res["piece_simplex"][idx] - B["simp_off"][b],
          "piece_mass": res["piece_mass"][idx], "piece_moment": res["piece_moment"][idx],
          "piece_energy": res["piece_energy"][idx]}
    nf = np.diff(fo)[idx]
    nv = np.diff(vo)[idx]
    gl["piece_face_off"] = np.concatenate([[0], np.cumsum(nf)])
    gl["piece_vert_off"] = np.concatenate([[0], np.cumsum(nv)])
    fl = np.concatenate([res["face_label"][fo[p]:fo[p + 1]] for p in idx])
    vl = np.concatenate([res["vert_label"][vo[p]:vo[p + 1]] for p in idx])
    vx = np.concatenate([res["vert_xyz"][vo[p]:vo[p + 1]] for p in idx])

    def shift(lab):
        lab = lab.astype(np.int64)
        out = lab.copy()
        pos = lab >= 0
        out[pos] = lab[pos] - lo
        neg = (lab < 0) & (lab > -2**31 + 16)
        out[neg] = -((-lab[neg] - 1) - B["simp_off"][b]) - 1
        out[lab == 2**31 - 1] = 2**31 - 1
        return out
    gl["face_label"] = shift(fl)
    gl["vert_label"] = shift(vl)
    gl["vert_xyz"] = vx
    n = len(s)
    gpu = {"mass": B["mass"][lo:hi], "centroid": B["centroid"][lo:hi], "energy": B["energy"][lo:hi], "res": gl,
           "nbr_off": B["nbr_off"][lo:hi + 1] - B["nbr_off"][lo], "nbr": B["nbr"][B["nbr_off"][lo]:B["nbr_off"][hi]] - lo,
           "cell_piece_off": np.concatenate([[0], np.cumsum(np.bincount(gl["piece_site"], minlength=n))]),
           "piece_id": np.arange(len(idx)), "raw_piece_site": gl["piece_site"], "raw_piece_simplex": gl["piece_simplex"]}
    assert_parity(gpu, ref, mom, n)


def _graph_setup(items):
    import torch
    import paper_2509_07175_amd as vd
    so = np.concatenate([[0], np.cumsum([len(s) for s, _ in items])])
    host = np.concatenate([s for s, _ in items])
    sites = torch.as_tensor(host, dtype=torch.float64, device="cuda")
    dom = vd.Domain.batch_from_vdgen([d for _, d in items])
    return vd, so, host, sites, dom


def test_no_sync_clip_equals_sync():
    import torch
    items = _small_batch(seed=13)
    vd, so, host, sites, dom = _graph_setup(items)
    boxes = [(0, 0, 0, 1, 1, 1)] * len(items)
    g = vd.build_grid_batch(sites, so, bboxes=boxes)
    c = vd.clip_cells(g, dom, vd.Options.default())
    m0, c0, e0 = [t.clone() for t in c.moments()]
    info0 = c.info()
    vd.build_grid_batch(sites, so, bboxes=boxes, grid=g)
    vd.clip_cells(g, dom, vd.Options.default(no_sync=1), cells=c)
    m1, c1, e1 = c.moments()
    torch.cuda.synchronize()
    info1 = c.info()
    assert info1["status"] == 0
    assert info1["n_pieces"] == info0["n_pieces"]
    assert torch.equal(m0, m1) and torch.equal(c0, c1) and torch.equal(e0, e1)


def test_graph_replays_match_eager():
    import torch
    items = _small_batch(seed=14)
    vd, so, host, sites, dom = _graph_setup(items)
    boxes = [(0, 0, 0, 1, 1, 1)] * len(items)
    n = len(host)
    side = torch.cuda.Stream()
    mass = torch.empty(n, dtype=torch.float64, device="cuda")
    cent = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    en = torch.empty(n, dtype=torch.float64, device="cuda")
    grid, cells = vd.Grid(), vd.Cells()
    with torch.cuda.stream(side):
        vd.build_grid_batch(sites, so, bboxes=boxes, grid=grid)
        vd.clip_cells(grid, dom, vd.Options.default(), cells=cells)  # sizes the arenas
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        vd.build_grid_batch(sites, so, bboxes=boxes, grid=grid)
        vd.clip_cells(grid, dom, vd.Options.default(no_sync=1), cells=cells)
        cells.moments(mass, cent, en)
    rng = np.random.default_rng(3)
    for rep in range(3):
        # move every site a little (inside the cube) and recompute both ways
        moved = np.clip(host + rng.uniform(-1e-3, 1e-3, size=host.shape), 1e-6, 1 - 1e-6)
        sites.copy_(torch.as_tensor(moved, dtype=torch.float64))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        info = cells.info()
        assert info["status"] == 0, info
        eg = vd.build_grid_batch(sites.clone(), so, bboxes=boxes)
        ec = vd.clip_cells(eg, dom, vd.Options.default())
        em, ece, ee = ec.moments()
        torch.cuda.synchronize()
        log(f"replay {rep}: pieces {info['n_pieces']} eager {ec.info()['n_pieces']}")
        assert torch.equal(mass, em) and torch.equal(cent, ece) and torch.equal(en, ee), f"replay {rep} differs"


def test_batched_workload_full_size(oracle_mod):
    """256 diagrams, 1,000 - 64,000 sites each, jittered 8^3 - 24^3 cube grids,
    in one launch.  Every diagram: its volume, and 20 sampled sites against the
    oracle (pieces, face labels and vertex label triples bit-exact after the
    shift to diagram-local indices; vertices, masses, centroids, energies and
    neighbour lists).  Neighbour symmetry over all sites."""
    import torch
    import paper_2509_07175_amd as vd
    from gpu_util import assert_neighbour_symmetry, assert_sampled_parity, sampled_result, shift_labels
    items = vdgen.config_c4()
    so = np.concatenate([[0], np.cumsum([len(s) for s, _ in items])])
    sites = torch.as_tensor(np.concatenate([s for s, _ in items]), dtype=torch.float64, device="cuda")
    dom = vd.Domain.batch_from_vdgen([d for _, d in items])
    g = vd.build_grid_batch(sites, so, bboxes=[(0, 0, 0, 1, 1, 1)] * len(items))
    c = vd.clip_cells(g, dom, vd.Options.default())
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    info = c.info()
    log(f"batch: {len(items)} diagrams, {so[-1]} sites, info {info}")
    assert info["status"] == 0
    mass, cent, en = m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy()
    view = c.view()
    off = view["cell_piece_off"].cpu().numpy()
    nbo, nb = view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy()
    assert_neighbour_symmetry(nbo, nb)
    rng = np.random.default_rng(2026)
    npieces = 0
    for b, (s, d) in enumerate(items):
        lo = so[b]
        vol = mass[lo:so[b + 1]].sum()
        assert abs(vol - 1.0) < 1e-10, f"diagram {b}: volume {vol}"
        sample = np.sort(rng.choice(len(s), size=20, replace=False))
        ref = oracle_mod.compute(s, d, only_sites=sample)
        mom = oracle_mod.site_moments(ref, s)
        got = sampled_result(view, lo + sample, off)
        got["piece_site"] = got["piece_site"] - lo
        got["piece_simplex"] = got["piece_simplex"] - dom.simp_off[b]
        got["face_label"] = shift_labels(got["face_label"], lo, dom.simp_off[b])
        got["vert_label"] = shift_labels(got["vert_label"], lo, dom.simp_off[b])
        assert_sampled_parity(got, mass, cent, en, nbo, nb, ref, mom, sample, site_lo=lo)
        npieces += len(ref["piece_site"])
    log(f"batch: {20 * len(items)} sites, {npieces} pieces identical")


def test_batch_order_gives_identical_results():
    """The cost-sorted work order of the batch queues (most tetrahedra per site
    first, diagrams dealt by longest processing time) against grid order: the
    same pieces, moments and neighbour lists, bit for bit."""
    items = _small_batch(seed=15)
    a = _run_batch(items, batch_order=1)
    b = _run_batch(items, batch_order=0)
    assert np.array_equal(a["mass"], b["mass"]) and np.array_equal(a["centroid"], b["centroid"])
    assert np.array_equal(a["energy"], b["energy"])
    assert np.array_equal(a["nbr_off"], b["nbr_off"]) and np.array_equal(a["nbr"], b["nbr"])
    for k in ("piece_site", "piece_simplex", "piece_mass", "face_label", "vert_xyz"):
        assert np.array_equal(a["res"][k], b["res"][k]), k
