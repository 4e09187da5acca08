"""GPU parity of the 3D clipped Voronoi path against the CPU oracle.

Everything goes through the C-ABI (libvd.so) via the thin binding.  The bar:
bit-exact combinatorics (piece set = domain-simplex incidence, face labels,
vertex label triples, neighbour lists) and masses / centroids / energies
within 1e-9 relative.
"""
import numpy as np
import pytest

import vdgen
from canon import canon_pieces
from gpu_util import (assert_neighbour_symmetry, assert_parity, assert_sampled_parity, gpu_neighbors, log, run_gpu,
                      sampled_result)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _check_case(oracle_mod, sites, dom, brute=True, **opts):
    log(f"case n={len(sites)} m={dom.m} opts={opts}")
    gpu = run_gpu(sites, dom, **opts)
    ref = oracle_mod.compute(sites, dom, brute=brute)
    mom = oracle_mod.site_moments(ref, sites)
    assert_parity(gpu, ref, mom, len(sites))
    return gpu, ref, mom


def test_c1_unit_cube_1000_sites(oracle_mod):
    sites, dom = vdgen.config_c1()
    gpu, ref, mom = _check_case(oracle_mod, sites, dom)
    assert abs(gpu["mass"].sum() - 1.0) < 1e-12
    log(f"C1 info {gpu['info']}")


def test_single_site(oracle_mod):
    dom = vdgen.kuhn_cube_grid(2)
    s = np.array([[0.3, 0.6, 0.45]])
    gpu, _, _ = _check_case(oracle_mod, s, dom)
    assert abs(gpu["mass"][0] - 1.0) < 1e-14


def test_two_sites(oracle_mod):
    dom = vdgen.kuhn_cube_grid(1)
    s = np.array([[0.23, 0.41, 0.52], [0.61, 0.41, 0.52]])
    _check_case(oracle_mod, s, dom)


def test_cell_over_many_tetrahedra(oracle_mod):
    """One site in 8^3 x 6 = 3,072 tetrahedra: the cell's simplex queue goes on
    in global memory past the 256 entries a wave keeps in LDS."""
    dom = vdgen.kuhn_cube_grid(8)
    s = np.array([[0.31, 0.47, 0.59]])
    gpu, _, _ = _check_case(oracle_mod, s, dom)
    assert abs(gpu["mass"][0] - 1.0) < 1e-12
    assert len(gpu["res"]["piece_site"]) == dom.m


def test_cell_over_more_tetrahedra_than_the_first_buffer(oracle_mod):
    """One site in 9^3 x 6 = 4,374 tetrahedra: more than the per-wave simplex
    queue first holds (256 in LDS + 3,840 in global memory).  The synchronous
    clip grows the queue's buffer and runs again: every tetrahedron is one
    piece, identical to the oracle's."""
    dom = vdgen.kuhn_cube_grid(9)
    s = np.array([[0.31, 0.47, 0.59]])
    gpu, _, _ = _check_case(oracle_mod, s, dom)
    assert len(gpu["res"]["piece_site"]) == dom.m and abs(gpu["mass"][0] - 1.0) < 1e-12


def test_cell_with_more_neighbours_than_lds_holds(oracle_mod):
    """A power site with a large weight among 8,000 light ones: its cell has
    296 neighbours, more than the 96 a wave keeps in LDS plus the 160 of the
    first global overflow buffer; the clip grows the buffer and the neighbour
    list (and everything else) matches the oracle."""
    sites = vdgen.uniform_cube_sites(8000, seed=8, jitter=1e-7)
    w = np.zeros(len(sites))
    w[0] = 0.04
    sites[0] = (0.5, 0.5, 0.5)
    dom = vdgen.kuhn_cube_grid(4)
    gpu = run_gpu(sites, dom, weights=w)
    ref = oracle_mod.compute(sites, dom, weights=w)
    mom = oracle_mod.site_moments(ref, sites)
    log(f"heavy site: {len(mom['neighbors'][0])} neighbours")
    assert len(mom["neighbors"][0]) > 96 + 160
    assert_parity(gpu, ref, mom, len(sites))


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("n,k,seed", [(300, 3, 5), (2000, 4, 6), (777, 5, 7)])
def test_multi_tet_parity(oracle_mod, n, k, seed, mode):
    """Both carve modes: cell-first (1) and per-simplex carving (0)."""
    sites, dom = vdgen.small_case(n, k, seed=seed)
    _check_case(oracle_mod, sites, dom, brute=False, carve_mode=mode)


def test_jittered_domain(oracle_mod):
    sites, dom = vdgen.small_case(1500, 6, seed=9, jitter_domain=0.1)
    _check_case(oracle_mod, sites, dom, brute=False)


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("straddle,improved", [(0, 1), (1, 0), (0, 0), (1, 1)])
def test_search_variants_same_result(oracle_mod, straddle, improved, mode):
    """Alg. 1 vs Alg. 3 edges and the improved search change the path, not the result."""
    sites, dom = vdgen.small_case(800, 3, seed=13)
    _check_case(oracle_mod, sites, dom, brute=False, use_straddle_edges=straddle,
                improved_search=improved, carve_mode=mode)


@pytest.mark.parametrize("mode", [1, 0])
def test_clustered_small(oracle_mod, mode):
    s = vdgen.gaussian_mixture_sites(400, 4, 200, 0.05, centre_seed=3, sample_seed=4, jitter=1e-7)
    dom = vdgen.kuhn_cube_grid(6)
    _check_case(oracle_mod, s, dom, brute=False, carve_mode=mode)


@pytest.mark.parametrize("mode", [1, 0])
def test_c2_full_size_sampled(oracle_mod, mode):
    """C2 at its full size: 100,000 sites in 48,000 tetrahedra, both carve
    modes.  5,000 sampled sites are compared piece by piece with the oracle;
    per-tetrahedron partition and neighbour symmetry are checked for all
    sites."""
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.config_c2()
    n = len(sites)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    g = vd.build_grid(s, bbox=(0.0, 0.0, 0.0, 1.0, 1.0, 1.0))
    c = vd.clip_cells(g, d, vd.Options.default(carve_mode=mode))
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    log(f"C2 mode {mode} info {c.info()}")
    mass, cent, en = m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy()
    assert abs(mass.sum() - 1.0) < 1e-11
    view = c.view()
    psite = view["piece_site"].cpu().numpy()
    used = psite >= 0
    q = dom.verts[dom.simplices]
    tv = np.einsum("ij,ij->i", np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), q[:, 3] - q[:, 0]) / 6
    per = np.bincount(view["piece_simplex"].cpu().numpy()[used], weights=view["piece_mass"].cpu().numpy()[used],
                      minlength=dom.m)
    assert np.allclose(per, tv, rtol=1e-10, atol=0)
    nbo, nb = view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy()
    assert_neighbour_symmetry(nbo, nb)
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(n, size=5000, replace=False))
    ref = oracle_mod.compute(sites, dom, only_sites=sample)
    mom = oracle_mod.site_moments(ref, sites)
    assert_sampled_parity(sampled_result(view, sample), mass, cent, en, nbo, nb, ref, mom, sample)


@pytest.mark.parametrize("mode", [1, 0])
def test_tiny_tetrahedra_far_from_their_sites(oracle_mod, mode):
    """The 2x2x2 Kuhn grid with its middle coordinate moved to 2^-20: a corner
    cube of six tetrahedra of volume eps^3/6 (and thin slabs beside it), ~1.5
    away from the six sites.  Every such piece is emitted with its exact
    volume; a moment fan with its apex at the site rounds these volumes to
    noise of either sign and drops pieces."""
    eps = 2.0 ** -20
    base = vdgen.kuhn_cube_grid(2)
    v = base.verts.copy()
    v[v == 0.5] = eps
    dom = vdgen.Domain(verts=v, simplices=base.simplices, adj=base.adj, dim=3)
    rng = np.random.default_rng(7)
    s = 0.75 + 0.2 * rng.random((6, 3))
    gpu = run_gpu(s, dom, carve_mode=mode)
    ref = oracle_mod.compute(s, dom, brute=True)
    # the slab tetrahedra beside the corner cube have dihedral angles ~eps, so
    # a vertex on two of their planes is conditioned ~1/eps: two FP64
    # evaluations agree to ~1e-16/eps = 1e-10, checked here with 100x room
    assert_parity(gpu, ref, oracle_mod.site_moments(ref, s), len(s), xyz_tol=1e-8)
    corner = np.nonzero(ref["piece_simplex"] < 6)[0]
    assert len(corner) == 6
    assert np.allclose(ref["piece_mass"][corner], eps ** 3 / 6, rtol=1e-9, atol=0)
    got = gpu["res"]["piece_mass"][gpu["res"]["piece_simplex"] < 6]
    assert len(got) == 6 and np.allclose(got, eps ** 3 / 6, rtol=1e-9, atol=0)


@pytest.mark.parametrize("mode", [1, 0])
def test_near_degenerate_lattice(oracle_mod, mode):
    """Cube-centre lattice of 8^3 sites with a 1e-7 jitter (every lattice
    vertex is then nearly equidistant to eight sites): the near-degenerate
    case of the method.  Several encodings of the vanishing faces are correct,
    so only the moments are compared: per site with the oracle to 1e-9
    relative, and with the closed forms of the lattice (mass h^3, energy h^5/4)
    to O(jitter)."""
    k = 8
    s = vdgen.lattice_sites(k, 1e-7, seed=3)
    dom = vdgen.kuhn_cube_grid(4)
    gpu = run_gpu(s, dom, carve_mode=mode)
    ref = oracle_mod.site_moments(oracle_mod.compute(s, dom, brute=False), s)
    log(f"lattice info {gpu['info']}")
    assert abs(gpu["mass"].sum() - 1.0) < 1e-12
    assert np.all(np.abs(gpu["mass"] - ref["mass"]) <= 1e-9 * ref["mass"])
    cerr = np.linalg.norm(gpu["centroid"] - ref["centroid"], axis=1) / np.linalg.norm(ref["centroid"], axis=1)
    assert cerr.max() <= 1e-9
    assert np.all(np.abs(gpu["energy"] - ref["energy"]) <= 1e-9 * ref["energy"])
    h = 1.0 / k
    assert np.allclose(gpu["mass"], h ** 3, rtol=1e-5)
    assert np.allclose(gpu["energy"], h ** 5 / 4, rtol=1e-4)


def test_c3_full_size_sampled(oracle_mod):
    """The headline workload in the benchmark's launch configuration: 1,000,000
    clustered sites in 750,000 tetrahedra, grid at 0.25 sites per cell, default
    options.  All sites: total and per-tetrahedron volume, CSR consistency,
    neighbour symmetry.  About 12,000 sampled sites, stratified by cell size
    (cluster cores: the smallest cells; cluster edges: the middle of the
    distribution; background: the largest cells; plus a uniform draw), and
    every site with a piece below 1e-15 of its tetrahedron's volume: pieces,
    face labels and vertex label triples bit-exact, vertices, masses,
    centroids, energies and neighbour lists against the oracle."""
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.config_c3()
    n = len(sites)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    g = vd.build_grid(s, bbox=(0.0, 0.0, 0.0, 1.0, 1.0, 1.0), sites_per_cell=0.25)
    c = vd.clip_cells(g, d, vd.Options.default())
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    info = c.info()
    log(f"C3 info {info}")
    assert info["status"] == 0
    mass, cent, en = m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy()
    assert abs(mass.sum() - 1.0) < 1e-10
    view = c.view()
    psite = view["piece_site"].cpu().numpy()
    used = psite >= 0
    psimp = view["piece_simplex"].cpu().numpy()[used]
    pmass = view["piece_mass"].cpu().numpy()[used]
    q = dom.verts[dom.simplices]
    tv = np.einsum("ij,ij->i", np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), q[:, 3] - q[:, 0]) / 6
    per = np.bincount(psimp, weights=pmass, minlength=dom.m)
    assert np.allclose(per, tv, rtol=1e-10, atol=0)
    off = view["cell_piece_off"].cpu().numpy()
    assert off[0] == 0 and off[-1] == used.sum() and np.all(np.diff(off) >= 1)
    nbo, nb = view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy()
    assert_neighbour_symmetry(nbo, nb)
    rng = np.random.default_rng(3003)
    order = np.argsort(mass)
    tiny = np.unique(psite[used][pmass < 1e-15 * tv[psimp]])
    log(f"C3: {len(tiny)} sites with a piece below 1e-15 of its tetrahedron")
    sample = np.unique(np.concatenate([
        order[:3000],                                  # cluster cores
        order[n // 2 - 1500:n // 2 + 1500],            # cluster edges
        order[-3000:],                                 # background
        rng.choice(n, size=3000, replace=False),       # uniform
        tiny, [908627]]).astype(np.int64))
    log(f"C3: comparing {len(sample)} sites with the oracle")
    ref = oracle_mod.compute(sites, dom, only_sites=sample)
    mom = oracle_mod.site_moments(ref, sites)
    md = assert_sampled_parity(sampled_result(view, sample, off), mass, cent, en, nbo, nb, ref, mom, sample)
    log(f"C3: {len(sample)} sites, {len(ref['piece_site'])} pieces identical; max vertex difference {md:.2e}")


def test_c3_pieces_do_not_depend_on_the_schedule():
    """The headline workload at full size under every schedule knob (grid
    density, search edges, improved search, per-piece carve, no site cache --
    which also leaves out the clips by the neighbours the cached sites
    certify): the knobs change the order of queries and clips, never the
    result, so the set of (site, tetrahedron) pieces and every site's
    neighbour list are identical and the per-site moments agree to 1e-9
    relative."""
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.config_c3()
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    runs = [(0.25, {}), (2.0, {}), (0.25, dict(use_straddle_edges=1)), (0.25, dict(improved_search=1)),
            (0.25, dict(carve_mode=0)), (0.25, dict(site_cache=0))]
    ref = None
    for rho, kw in runs:
        log(f"C3 schedule rho={rho} {kw}")
        g = vd.build_grid(s, bbox=(0.0, 0.0, 0.0, 1.0, 1.0, 1.0), sites_per_cell=rho)
        c = vd.clip_cells(g, d, vd.Options.default(emit_polytopes=0, **kw))
        m, ce, e = c.moments()
        torch.cuda.synchronize()
        assert c.info()["status"] == 0
        v = c.view()
        ps = v["piece_site"]
        used = ps >= 0
        key = (ps[used].to(torch.int64) * dom.m + v["piece_simplex"][used].to(torch.int64)).sort().values.cpu().numpy()
        cur = (key, m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy(), v["nbr_off"].cpu().numpy(),
               v["nbr"].cpu().numpy())
        del c, g, v
        if ref is None:
            ref = cur
            continue
        assert len(cur[0]) == len(ref[0]) and np.array_equal(cur[0], ref[0]), \
            f"piece sets differ: {len(cur[0])} vs {len(ref[0])} pieces"
        assert np.all(np.abs(cur[1] - ref[1]) <= 1e-9 * ref[1])
        assert np.all(np.linalg.norm(cur[2] - ref[2], axis=1) <= 1e-9 * np.linalg.norm(ref[2], axis=1))
        assert np.all(np.abs(cur[3] - ref[3]) <= 1e-9 * ref[3])
        assert np.array_equal(cur[4], ref[4]) and np.array_equal(cur[5], ref[5]), "neighbour lists differ"
