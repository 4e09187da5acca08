"""Oracle pins for power diagrams (Sec. 7.3): cells of the power distance
|x - v_i|^2 - w_i.  The paper draws weights in [-|M|/n, |M|/n]; the cases
below do the same, plus a site with a weight low enough to have an empty
cell and one whose cell does not contain it.

* two sites: the power plane sits at x* = (x1 + x2)/2 + (w1 - w2) / (2 (x2 - x1));
* equal weights give the Voronoi diagram bit for bit;
* brute force (every half-space) equals the pruned run (power security radius);
* Monte-Carlo labelling by the smallest power distance;
* the sampled-site mode equals the full run."""
import numpy as np
import pytest

import vdgen
from canon import canon_pieces, compare_canon, subset_result


def _case(n=120, k=3, seed=101):
    sites, dom = vdgen.small_case(n, k, seed=seed)
    rng = np.random.default_rng(seed + 1)
    w = rng.uniform(-1.0 / n, 1.0 / n, size=n)
    w[0] = -0.05  # far below its neighbours: an empty cell
    w[1] = 0.02   # far above: its cell swallows neighbours' sites
    return sites, dom, w


def test_two_sites_closed_form(oracle_mod):
    x1, x2, w1, w2 = 0.23, 0.61, 0.013, -0.021
    s = np.array([[x1, 0.41, 0.52], [x2, 0.41, 0.52]])
    r = oracle_mod.compute(s, vdgen.kuhn_cube_grid(3), brute=True, weights=[w1, w2])
    m = oracle_mod.site_moments(r, s)
    xs = 0.5 * (x1 + x2) + (w1 - w2) / (2 * (x2 - x1))
    assert abs(m["mass"][0] - xs) < 1e-14 and abs(m["mass"][1] - (1 - xs)) < 1e-14
    assert abs(m["centroid"][0][0] - xs / 2) < 1e-14


def test_equal_weights_are_the_voronoi_diagram(oracle_mod):
    sites, dom = vdgen.small_case(200, 3, seed=103)
    a = oracle_mod.compute(sites, dom, weights=np.full(len(sites), 0.004))
    b = oracle_mod.compute(sites, dom)
    assert compare_canon(canon_pieces(a), canon_pieces(b), 0.0) == (0, 0, 0.0)
    assert np.array_equal(a["piece_mass"], b["piece_mass"])


def test_brute_equals_pruned(oracle_mod):
    sites, dom, w = _case()
    b = oracle_mod.compute(sites, dom, brute=True, weights=w)
    p = oracle_mod.compute(sites, dom, brute=False, weights=w)
    assert compare_canon(canon_pieces(b), canon_pieces(p), 0.0) == (0, 0, 0.0)
    m = oracle_mod.site_moments(b, sites)
    assert m["mass"][0] == 0.0             # the dominated site has no cell
    assert abs(m["mass"].sum() - 1.0) < 1e-12
    assert b["min_margin"] > 1e-9


def test_monte_carlo_power_labelling(oracle_mod):
    sites, dom, w = _case(n=60, k=2, seed=105)
    r = oracle_mod.compute(sites, dom, brute=True, weights=w)
    m = oracle_mod.site_moments(r, sites)
    rng = np.random.default_rng(106)
    N = 40000
    p = rng.uniform(0, 1, size=(N, 3))
    pw = ((p[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2) - w[None, :]
    lab = np.argmin(pw, axis=1)
    frac = np.bincount(lab, minlength=len(sites)) / N
    sigma = np.sqrt(m["mass"] * (1 - m["mass"]) / N)
    assert np.all(np.abs(frac - m["mass"]) <= 5 * sigma + 1e-12)
    # some site lies outside its own (non-empty) cell
    own = np.argmin(((sites[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2) - w[None, :], axis=1)
    assert np.any((own != np.arange(len(sites))) & (m["mass"] > 0))


def test_sampled_sites_equal_the_full_run(oracle_mod):
    sites, dom, w = _case(n=400, k=4, seed=107)
    full = oracle_mod.compute(sites, dom, weights=w)
    sample = np.arange(0, len(sites), 7, dtype=np.int32)
    part = oracle_mod.compute(sites, dom, only_sites=sample, weights=w)
    sel = np.nonzero(np.isin(full["piece_site"], sample))[0]
    assert compare_canon(canon_pieces(part), canon_pieces(subset_result(full, sel)), 0.0) == (0, 0, 0.0)


def test_surface_power(oracle_mod):
    s, dom = vdgen.sphere_sites(150, seed=108), vdgen.icosphere(2)
    w = np.random.default_rng(109).uniform(-0.03, 0.03, size=len(s))
    b = oracle_mod.compute(s, dom, brute=True, weights=w)
    p = oracle_mod.compute(s, dom, brute=False, weights=w)
    assert compare_canon(canon_pieces(b), canon_pieces(p), 0.0) == (0, 0, 0.0)
