"""Oracle pins for the density-weighted moments of Sec. 7.4 (Eq. 3) with a
quadratic density rho(x) = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 xy + c6 xz
+ c7 y^2 + c8 yz + c9 z^2, and for the adjoint that carries rho:

* closed forms on the unit cube: one site (the whole cube) and two sites
  (the half cubes of the bisector plane), from one-dimensional integrals;
* a constant density c gives c times the unweighted moments, which the oracle
  computes by a different (closed-form) route;
* the per-domain partition equals the integral of rho over the cube;
* Monte-Carlo: the rho-weighted hit fraction of each cell agrees with its
  weighted mass (5 sigma);
* the adjoint: the weighted CVT gradient 2 m (v - c), a zero gradient of the
  total weighted mass, and central differences of a random loss."""
import numpy as np
import pytest

import vdgen

RHO = np.array([1.0, 0.5, -0.3, 0.2, 0.4, 0.1, -0.2, 0.3, 0.05, 0.6])


def _rho(x, c=RHO):
    x = np.atleast_2d(x)
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * X + c[5] * X * Y + c[6] * X * Z + c[7] * Y * Y + \
        c[8] * Y * Z + c[9] * Z * Z


def _box_moments(lo, hi, v, c=RHO):
    """Exact int over the box [lo, hi] of rho, rho x and rho |x - v|^2, by
    expanding the polynomial: int of x^a y^b z^c over the box is a product of
    one-dimensional power integrals."""
    def P(k, a):  # int_lo^hi x^a along axis k
        return (hi[k] ** (a + 1) - lo[k] ** (a + 1)) / (a + 1)

    def mono(a, b, cc):
        return P(0, a) * P(1, b) * P(2, cc)
    terms = [(c[0], (0, 0, 0)), (c[1], (1, 0, 0)), (c[2], (0, 1, 0)), (c[3], (0, 0, 1)), (c[4], (2, 0, 0)),
             (c[5], (1, 1, 0)), (c[6], (1, 0, 1)), (c[7], (0, 2, 0)), (c[8], (0, 1, 1)), (c[9], (0, 0, 2))]

    def integ(extra):  # int rho * x^extra
        return sum(w * mono(*(np.array(e) + np.array(extra))) for w, e in terms)
    m = integ((0, 0, 0))
    m1 = np.array([integ((1, 0, 0)), integ((0, 1, 0)), integ((0, 0, 1))])
    # |x - v|^2 = sum_k x_k^2 - 2 v_k x_k + v_k^2
    e = sum(integ(tuple(2 if j == k else 0 for j in range(3))) - 2 * v[k] * m1[k] + v[k] ** 2 * m for k in range(3))
    return m, m1, e


def test_single_site_closed_form(oracle_mod):
    s = np.array([[0.3, 0.6, 0.45]])
    r = oracle_mod.compute(s, vdgen.kuhn_cube_grid(2), brute=True, keep_handle=True)
    try:
        m = oracle_mod.site_moments(oracle_mod.density_result(r, s, RHO, 3), s)
    finally:
        oracle_mod.free(r)
    M, M1, E = _box_moments((0, 0, 0), (1, 1, 1), s[0])
    assert abs(m["mass"][0] - M) <= 1e-13 * M
    assert np.allclose(m["centroid"][0], M1 / M, rtol=1e-13, atol=0)
    assert abs(m["energy"][0] - E) <= 1e-13 * E


def test_two_sites_closed_form(oracle_mod):
    x1, x2 = 0.23, 0.61
    s = np.array([[x1, 0.41, 0.52], [x2, 0.41, 0.52]])
    xm = 0.5 * (x1 + x2)
    r = oracle_mod.compute(s, vdgen.kuhn_cube_grid(3), brute=True, keep_handle=True)
    try:
        m = oracle_mod.site_moments(oracle_mod.density_result(r, s, RHO, 3), s)
    finally:
        oracle_mod.free(r)
    for i, (lo, hi) in enumerate((((0, 0, 0), (xm, 1, 1)), ((xm, 0, 0), (1, 1, 1)))):
        M, M1, E = _box_moments(lo, hi, s[i])
        assert abs(m["mass"][i] - M) <= 1e-13 * M
        assert np.allclose(m["centroid"][i], M1 / M, rtol=1e-12, atol=0)
        assert abs(m["energy"][i] - E) <= 1e-12 * E


def test_constant_density_scales_the_unweighted_moments(oracle_mod):
    sites, dom = vdgen.small_case(300, 3, seed=81)
    r = oracle_mod.compute(sites, dom, keep_handle=True)
    try:
        c = np.zeros(10)
        c[0] = 2.5
        d = oracle_mod.density_result(r, sites, c, 3)
    finally:
        oracle_mod.free(r)
    assert np.allclose(d["piece_mass"], 2.5 * r["piece_mass"], rtol=1e-12, atol=1e-18)
    assert np.allclose(d["piece_moment"], 2.5 * r["piece_moment"], rtol=1e-12, atol=1e-18)
    assert np.allclose(d["piece_energy"], 2.5 * r["piece_energy"], rtol=1e-11, atol=1e-20)


def test_partition_and_monte_carlo(oracle_mod):
    sites, dom = vdgen.small_case(40, 2, seed=82)
    r = oracle_mod.compute(sites, dom, brute=True, keep_handle=True)
    try:
        m = oracle_mod.site_moments(oracle_mod.density_result(r, sites, RHO, 3), sites)
    finally:
        oracle_mod.free(r)
    M, _, _ = _box_moments((0, 0, 0), (1, 1, 1), np.zeros(3))
    assert abs(m["mass"].sum() - M) <= 1e-12 * M
    rng = np.random.default_rng(83)
    N = 200000
    p = rng.uniform(0, 1, size=(N, 3))
    w = _rho(p)
    nn = np.argmin(((p[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2), axis=1)
    est = np.bincount(nn, weights=w, minlength=len(sites)) / N
    var = np.bincount(nn, weights=w * w, minlength=len(sites)) / N - est ** 2
    assert np.all(np.abs(est - m["mass"]) <= 5 * np.sqrt(var / N) + 1e-12)


def _loss(oracle_mod, s, dom, gm, gc, ge, rho):
    r = oracle_mod.compute(s, dom, brute=False, keep_handle=True)
    try:
        m = oracle_mod.site_moments(oracle_mod.density_result(r, s, rho, dom.dim), s)
    finally:
        oracle_mod.free(r)
    return float((m["mass"] * gm).sum() + (m["centroid"] * gc).sum() + (m["energy"] * ge).sum())


def _grad(oracle_mod, s, dom, rho, gm=None, gc=None, ge=None):
    r = oracle_mod.compute(s, dom, brute=False, keep_handle=True)
    try:
        m = oracle_mod.site_moments(oracle_mod.density_result(r, s, rho, dom.dim), s)
        g = oracle_mod.moments_backward(r, s, dom, m["mass"], m["centroid"], gm, gc, ge, rho=rho)
    finally:
        oracle_mod.free(r)
    return g, m


@pytest.mark.parametrize("surface", [False, True])
def test_adjoint_with_density(oracle_mod, surface):
    if surface:
        s, dom = vdgen.sphere_sites(60, seed=84), vdgen.icosphere(2)
        rho = np.array([1.2, 0.3, -0.2, 0.1, 0.2, 0.0, 0.1, 0.3, 0.0, 0.1])
    else:
        s, dom = vdgen.small_case(50, 2, seed=85)
        rho = RHO
    n = len(s)
    # the weighted CVT energy: 2 m (v - c), face terms cancel
    g, m = _grad(oracle_mod, s, dom, rho, ge=np.ones(n))
    ref = 2 * m["mass"][:, None] * (s - m["centroid"])
    assert np.abs(g - ref).max() <= 1e-11 * np.abs(ref).max()
    if not surface:
        # the total weighted mass of a fixed domain does not depend on the sites
        g, _ = _grad(oracle_mod, s, dom, rho, gm=np.ones(n))
        assert np.abs(g).max() < 1e-12
    rng = np.random.default_rng(86)
    gm, gc, ge = rng.normal(size=n), rng.normal(size=(n, 3)), rng.normal(size=n)
    g, _ = _grad(oracle_mod, s, dom, rho, gm, gc, ge)
    d = rng.normal(size=(n, 3))
    if surface:
        d -= (d * s).sum(axis=1, keepdims=True) * s  # stay near the sphere (not needed, but keeps cells alike)
    h = 1e-6
    fd = (_loss(oracle_mod, s + h * d, dom, gm, gc, ge, rho) - _loss(oracle_mod, s - h * d, dom, gm, gc, ge, rho)) / (2 * h)
    an = float((g * d).sum())
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
