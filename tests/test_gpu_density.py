"""Density-weighted moments (Sec. 7.4, Eq. 3 with a quadratic density) and
their adjoint on the GPU against the oracle (which integrates with different,
conical product, rules), and L-BFGS minimisation of the weighted CVT energy."""
import numpy as np
import pytest

import vdgen
from gpu_util import assert_sampled_parity, log, run_gpu, sampled_result

pytestmark = pytest.mark.gpu

RHO = [1.0, 0.5, -0.3, 0.2, 0.4, 0.1, -0.2, 0.3, 0.05, 0.6]
RHO_S = [1.2, 0.3, -0.2, 0.1, 0.2, 0.0, 0.1, 0.3, 0.0, 0.1]
SPHERE_BOX = (-1.3, -1.3, -1.3, 1.3, 1.3, 1.3)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _area(dom):
    q = dom.verts[dom.simplices]
    return 0.5 * np.linalg.norm(np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), axis=1).sum()


def _oracle(oracle_mod, s, dom, rho, only=None):
    r = oracle_mod.compute(s, dom, brute=only is None and len(s) <= 3000, only_sites=only, keep_handle=True)
    try:
        dr = oracle_mod.density_result(r, s, rho, dom.dim)
    finally:
        oracle_mod.free(r)
    return dr, oracle_mod.site_moments(dr, s)


def _check(gpu, dr, mom, n):
    rel = 1e-9
    m_g, m_r = gpu["mass"], mom["mass"]
    assert np.all(np.abs(m_g - m_r) <= rel * m_r), np.max(np.abs(m_g - m_r) / m_r)
    c_r = mom["centroid"]
    cerr = np.linalg.norm(gpu["centroid"] - c_r, axis=1) / np.linalg.norm(c_r, axis=1)
    assert cerr.max() <= rel, cerr.max()
    assert np.all(np.abs(gpu["energy"] - mom["energy"]) <= rel * mom["energy"])
    # per piece: the weighted mass of each (site, simplex)
    a = dict(zip(zip(gpu["res"]["piece_site"].tolist(), gpu["res"]["piece_simplex"].tolist()),
                 gpu["res"]["piece_mass"].tolist()))
    b = dict(zip(zip(dr["piece_site"].tolist(), dr["piece_simplex"].tolist()), dr["piece_mass"].tolist()))
    assert set(a) == set(b)
    scale = max(abs(v) for v in b.values())
    assert max(abs(a[k] - b[k]) for k in b) <= 1e-12 * scale


@pytest.mark.parametrize("mode", [1, 0])
def test_weighted_moments_3d(oracle_mod, mode):
    s, dom = vdgen.small_case(2000, 4, seed=87)
    gpu = run_gpu(s, dom, carve_mode=mode, density=RHO)
    dr, mom = _oracle(oracle_mod, s, dom, np.array(RHO))
    _check(gpu, dr, mom, len(s))


def test_weighted_moments_surface(oracle_mod):
    s, dom = vdgen.sphere_sites(1500, seed=88), vdgen.icosphere(3)
    gpu = run_gpu(s, dom, bbox=SPHERE_BOX, surface_area=_area(dom), density=RHO_S)
    dr, mom = _oracle(oracle_mod, s, dom, np.array(RHO_S))
    _check(gpu, dr, mom, len(s))


def test_weighted_moments_c2_sampled(oracle_mod):
    """C2 at full size with the density: 3,000 sampled sites."""
    import torch
    import paper_2509_07175_amd as vd
    s, dom = vdgen.config_c2()
    n = len(s)
    st = torch.as_tensor(s, dtype=torch.float64, device="cuda")
    g = vd.build_grid(st, bbox=(0, 0, 0, 1, 1, 1))
    c = vd.clip_cells(g, vd.Domain.from_vdgen(dom), vd.Options.default(density=RHO))
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    view = c.view()
    sample = np.sort(np.random.default_rng(89).choice(n, size=3000, replace=False))
    r = oracle_mod.compute(s, dom, only_sites=sample, keep_handle=True)
    try:
        dr = oracle_mod.density_result(r, s, np.array(RHO), 3)
    finally:
        oracle_mod.free(r)
    mom = oracle_mod.site_moments(dr, s)
    got = sampled_result(view, sample)
    assert_sampled_parity(got, m.cpu().numpy(), ce.cpu().numpy(), e.cpu().numpy(),
                          view["nbr_off"].cpu().numpy(), view["nbr"].cpu().numpy(), dr, mom, sample)
    # the pieces' weighted masses (both sorted by site, then simplex)
    assert np.allclose(got["piece_mass"], dr["piece_mass"], rtol=1e-10, atol=1e-22)


@pytest.mark.parametrize("kind", ["3d", "surface"])
def test_weighted_adjoint_against_oracle(oracle_mod, kind):
    import torch
    import paper_2509_07175_amd as vd
    if kind == "3d":
        s, dom = vdgen.small_case(400, 3, seed=90)
        bb, area, rho = (0, 0, 0, 1, 1, 1), 0.0, RHO
    else:
        s, dom = vdgen.sphere_sites(500, seed=91), vdgen.icosphere(3)
        bb, area, rho = SPHERE_BOX, _area(vdgen.icosphere(3)), RHO_S
    n = len(s)
    rng = np.random.default_rng(92)
    gm, gc, ge = rng.normal(size=n), rng.normal(size=(n, 3)), rng.normal(size=n)
    st = torch.as_tensor(s, dtype=torch.float64, device="cuda")
    g = vd.build_grid(st, bbox=bb, surface_area=area)
    c = vd.clip_cells(g, vd.Domain.from_vdgen(dom), vd.Options.default(want_grad=1, density=rho))
    mass, cent, _ = c.moments()
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()  # noqa: E731
    out = c.backward(t(gm), t(gc), t(ge)).cpu().numpy()
    cvt = c.backward(None, None, t(np.ones(n))).cpu().numpy()
    ref_cvt = 2 * mass.cpu().numpy()[:, None] * (s - cent.cpu().numpy())
    assert np.abs(cvt - ref_cvt).max() <= 1e-12 * np.abs(ref_cvt).max()
    r = oracle_mod.compute(s, dom, brute=False, keep_handle=True)
    try:
        mom = oracle_mod.site_moments(oracle_mod.density_result(r, s, np.array(rho), dom.dim), s)
        ref = oracle_mod.moments_backward(r, s, dom, mom["mass"], mom["centroid"], gm, gc, ge, rho=np.array(rho))
    finally:
        oracle_mod.free(r)
    err = np.linalg.norm(out - ref, axis=1)
    log(f"weighted adjoint {kind}: max abs err {err.max():.3e} scale {np.abs(ref).max():.3e}")
    assert err.max() <= 1e-9 * np.abs(ref).max()


def test_lbfgs_decreases_the_weighted_energy():
    import torch
    import paper_2509_07175_amd as vd
    s, dom = vdgen.small_case(3000, 4, seed=93)
    st = torch.as_tensor(s, dtype=torch.float64, device="cuda")
    x, energies = vd.cvt_lbfgs(st, vd.Domain.from_vdgen(dom), 12, options=vd.Options.default(density=RHO),
                               bbox=(0, 0, 0, 1, 1, 1))
    log(f"L-BFGS energies {energies}")
    assert all(b <= a * (1 + 1e-12) for a, b in zip(energies, energies[1:]))
    assert energies[-1] < 0.9 * energies[0]
