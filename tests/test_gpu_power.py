"""Power diagrams (Sec. 7.3) on the GPU against the oracle: the sites are
lifted by their weights and the clipped / restricted cells are those of the
power distance |x - v_i|^2 - w_i.  Weights in [-|M|/n, |M|/n] as in the
paper, plus a dominated site (empty cell) and a heavy one (whose cell holds
other sites)."""
import numpy as np
import pytest

import vdgen
from gpu_util import assert_parity, assert_sampled_parity, log, run_gpu, sampled_result

pytestmark = pytest.mark.gpu
SPHERE_BOX = (-1.3, -1.3, -1.3, 1.3, 1.3, 1.3)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _weights(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    w = rng.uniform(-spread / n, spread / n, size=n)
    w[0] = -0.05
    w[1] = min(0.02, 50.0 / n)
    return w


@pytest.mark.parametrize("n,k,seed", [(120, 3, 111), (900, 4, 112)])
def test_power_3d_against_the_oracle(oracle_mod, n, k, seed):
    sites, dom = vdgen.small_case(n, k, seed=seed)
    w = _weights(n, seed)
    gpu = run_gpu(sites, dom, weights=w)
    ref = oracle_mod.compute(sites, dom, brute=n <= 200, weights=w)
    log(f"power n={n}: {len(ref['piece_site'])} pieces, info {gpu['info']}")
    assert_parity(gpu, ref, oracle_mod.site_moments(ref, sites), n)
    assert gpu["mass"][0] == 0.0 and abs(gpu["mass"].sum() - 1.0) < 1e-12


def test_equal_weights_give_the_voronoi_diagram():
    sites, dom = vdgen.small_case(800, 4, seed=113)
    a = run_gpu(sites, dom, weights=np.full(len(sites), 0.003))
    b = run_gpu(sites, dom)
    assert np.array_equal(a["res"]["piece_site"], b["res"]["piece_site"])
    assert np.array_equal(a["res"]["piece_simplex"], b["res"]["piece_simplex"])
    assert np.allclose(a["mass"], b["mass"], rtol=1e-12, atol=0)


def test_power_non_convex_domain(oracle_mod):
    import test_oracle_nonconvex as t
    sites, dom = t._cases()["l_block"]
    w = _weights(len(sites), 114, spread=0.5)
    gpu = run_gpu(sites, dom, bbox=(-0.5, -0.5, -0.5, 1.5, 1.5, 1.5), weights=w)
    ref = oracle_mod.compute(sites, dom, brute=True, weights=w)
    assert_parity(gpu, ref, oracle_mod.site_moments(ref, sites), len(sites))


def test_power_surface(oracle_mod):
    s, dom = vdgen.sphere_sites(600, seed=115), vdgen.icosphere(3)
    w = np.random.default_rng(116).uniform(-0.01, 0.01, size=len(s))
    q = dom.verts[dom.simplices]
    area = 0.5 * np.linalg.norm(np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), axis=1).sum()
    gpu = run_gpu(s, dom, bbox=SPHERE_BOX, surface_area=area, weights=w)
    ref = oracle_mod.compute(s, dom, brute=False, weights=w)
    assert_parity(gpu, ref, oracle_mod.site_moments(ref, s), len(s))


def test_power_at_scale_sampled(oracle_mod):
    """30,000 weighted sites in a 10^3-cube grid (6,000 tetrahedra): partition
    for all, 2,000 sampled sites against the oracle."""
    import torch
    import paper_2509_07175_amd as vd
    n = 30000
    sites = vdgen.uniform_cube_sites(n, seed=117, jitter=1e-7)
    dom = vdgen.kuhn_cube_grid(10)
    w = _weights(n, 118)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1), weights=torch.as_tensor(w, device="cuda"))
    c = vd.clip_cells(g, vd.Domain.from_vdgen(dom))
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    mass = m.cpu().numpy()
    assert abs(mass.sum() - 1.0) < 1e-11 and mass[0] == 0.0
    view = c.view()
    sample = np.unique(np.concatenate([[0, 1], np.random.default_rng(119).choice(n, 2000, replace=False)]))
    ref = oracle_mod.compute(sites, dom, only_sites=sample, weights=w)
    mom = oracle_mod.site_moments(ref, sites)
    nz = sample[mom["mass"][sample] > 0]
    assert_sampled_parity(sampled_result(view, nz), mass, ce.cpu().numpy(), e.cpu().numpy(),
                          view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy(), ref, mom, nz)
