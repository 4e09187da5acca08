"""GPU parity on non-convex tetrahedral domains and with sites outside the
domain (Alg. 5: the restricted diagram of the boundary surface seeds every
tetrahedron behind a boundary triangle that a cell meets, so parts of
Omega_i cap M that are not connected to the site's own tetrahedron are found,
and a site outside M gets the parts of its cell inside M)."""
import numpy as np
import pytest

import vdgen
from gpu_util import assert_parity, assert_sampled_parity, log, run_gpu, sampled_result

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _cases():
    import test_oracle_nonconvex as t
    return t._cases()


def _vols(dom):
    q = dom.verts[dom.simplices]
    return np.einsum("ij,ij->i", np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), q[:, 3] - q[:, 0]) / 6


BOX = (-0.5, -0.5, -0.5, 1.5, 1.5, 1.5)


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("name", ["l_block", "cavity"])
def test_small_cases_against_the_oracle(oracle_mod, name, mode):
    sites, dom = _cases()[name]
    log(f"non-convex {name} mode {mode}: n={len(sites)} m={dom.m}")
    gpu = run_gpu(sites, dom, bbox=BOX, carve_mode=mode)
    ref = oracle_mod.compute(sites, dom, brute=True)
    assert_parity(gpu, ref, oracle_mod.site_moments(ref, sites), len(sites))
    assert abs(gpu["mass"].sum() - _vols(dom).sum()) <= 1e-12


def test_outside_site_without_boundary_seeds_is_an_error():
    import paper_2509_07175_amd as vd
    sites, dom = _cases()["l_block"]
    with pytest.raises(vd.VDError) as e:
        run_gpu(sites, dom, bbox=BOX, boundary_seeds=0)
    assert e.value.status == 1 and "outside every tetrahedron" in str(e.value)


def test_sites_outside_a_convex_domain(oracle_mod):
    """A convex cube with some sites beyond its faces: those sites' cells are
    found through the boundary surface (seeding switches on by itself)."""
    rng = np.random.default_rng(91)
    inside = vdgen.uniform_cube_sites(300, seed=92, jitter=1e-7)
    out = rng.uniform(-0.3, 1.3, size=(40, 3))
    out = out[np.any((out < 0) | (out > 1), axis=1)]
    sites = np.vstack([inside, out])
    dom = vdgen.kuhn_cube_grid(4)
    for mode in (1, 0):
        gpu = run_gpu(sites, dom, bbox=BOX, carve_mode=mode)
        ref = oracle_mod.compute(sites, dom, brute=True)
        assert_parity(gpu, ref, oracle_mod.site_moments(ref, sites), len(sites))
        assert abs(gpu["mass"].sum() - 1.0) <= 1e-12
        assert np.any(gpu["mass"][300:] > 0) and np.any(gpu["mass"][300:] == 0)
        assert gpu["info"]["boundary_seeded"] == 1 and gpu["info"]["sites_outside"] == len(out)


def test_cavity_at_scale_sampled(oracle_mod):
    """30,000 sites in a 12^3-cube grid without its middle 4^3 cubes (9,984
    tetrahedra around a cubic cavity): per-tetrahedron partition for all
    sites, 2,000 sampled sites and every site next to the cavity against the
    oracle."""
    import torch
    import paper_2509_07175_amd as vd
    dom = vdgen.cube_with_cavity(12)
    s = vdgen.uniform_cube_sites(40000, seed=93, jitter=1e-7)
    s = s[~np.all((s > 1 / 3) & (s < 2 / 3), axis=1)][:30000]
    n = len(s)
    st = torch.as_tensor(s, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    assert d.info()["convex"] == 0
    g = vd.build_grid(st, bbox=(0, 0, 0, 1, 1, 1))
    c = vd.clip_cells(g, d)
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    log(f"cavity info {c.info()}")
    mass, cent, en = m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy()
    view = c.view()
    used = view["piece_site"].cpu().numpy() >= 0
    per = np.bincount(view["piece_simplex"].cpu().numpy()[used], weights=view["piece_mass"].cpu().numpy()[used],
                      minlength=dom.m)
    assert np.allclose(per, _vols(dom), rtol=1e-10, atol=0)
    rng = np.random.default_rng(94)
    near = np.nonzero(np.all((s > 1 / 3 - 0.03) & (s < 2 / 3 + 0.03), axis=1))[0]
    sample = np.unique(np.concatenate([rng.choice(n, size=2000, replace=False), near]))
    ref = oracle_mod.compute(s, dom, only_sites=sample)
    mom = oracle_mod.site_moments(ref, s)
    nbo, nb = view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy()
    assert_sampled_parity(sampled_result(view, sample), mass, cent, en, nbo, nb, ref, mom, sample)


def test_batch_with_a_non_convex_diagram():
    """A batch of a cube, the L-block case and the cavity case: every diagram
    gives what a plain call gives it.  The batch seeds all its diagrams from
    the boundary (two of them need it), so the cube's plain reference seeds
    from the boundary too (boundary_seeds = 1): the same tetrahedra visited in
    the same order, bit for bit; without the extra seeds the masses agree to
    rounding."""
    import torch
    import paper_2509_07175_amd as vd
    cases = _cases()
    items = [(vdgen.uniform_cube_sites(200, seed=95, jitter=1e-7), vdgen.kuhn_cube_grid(3)),
             cases["l_block"], cases["cavity"]]
    so = np.concatenate([[0], np.cumsum([len(s) for s, _ in items])])
    sites = torch.as_tensor(np.concatenate([s for s, _ in items]), dtype=torch.float64, device="cuda")
    dom = vd.Domain.batch_from_vdgen([d for _, d in items])
    g = vd.build_grid_batch(sites, so, bboxes=[BOX] * len(items))
    c = vd.clip_cells(g, dom)
    m, _, _ = c.moments()
    torch.cuda.synchronize()
    m = m.cpu().numpy()
    for b, (s, d) in enumerate(items):
        P = run_gpu(s, d, bbox=BOX, boundary_seeds=1)
        assert np.array_equal(m[so[b]:so[b + 1]], P["mass"]), f"diagram {b}"
        Q = run_gpu(s, d, bbox=BOX)
        assert np.allclose(m[so[b]:so[b + 1]], Q["mass"], rtol=1e-12, atol=0), f"diagram {b}"
        assert np.array_equal(P["res"]["piece_simplex"], Q["res"]["piece_simplex"])


def test_coarse_l_block_split_boundary(oracle_mod):
    """An L-shaped prism of 2^3 - 2 = 6 cubes (36 tetrahedra, 56 boundary
    triangles) under 3,000 sites and 3 sites outside it: each boundary triangle
    would meet dozens of cells, so the boundary diagram that seeds the clip runs
    on the surface with every triangle split (the split is kept in the domain
    handle).  Against the oracle (pieces bit-exact, moments to 1e-9), also with
    the interior split."""
    dom = vdgen.l_block(2)
    s = np.vstack([vdgen.l_block_sites(3000, seed=23),
                   [[0.8, 0.9, 0.4], [0.7, 0.6, 0.55], [1.2, 0.3, 0.5]]])
    ref = oracle_mod.compute(s, dom, brute=False)
    mom = oracle_mod.site_moments(ref, s)
    bbox = (-0.5, -0.5, -0.5, 1.5, 1.5, 1.5)
    gpu = run_gpu(s, dom, bbox=bbox)
    assert gpu["info"]["boundary_seeded"] == 1 and gpu["info"]["sites_outside"] == 3
    assert_parity(gpu, ref, mom, len(s))
    whole = run_gpu(s, dom, bbox=bbox, whole_interior=1)
    res = whole["res"]
    cut = np.setdiff1d(np.arange(len(s)), res["piece_site"][res["piece_simplex"] == -1])
    assert_parity(whole, ref, mom, len(s), sites_subset=cut)
    assert np.all(np.abs(whole["mass"] - mom["mass"]) <= 1e-9 * np.maximum(mom["mass"], 1e-300))
