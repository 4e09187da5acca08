"""vd_cell_moments_backward_noalloc: the allocation-free adjoint against the
allocating vd_cell_moments_backward on the same handles, two calls in a row
(the second on a smaller input, so the fixed scratch array holds the first
call's weights beyond the second's sites), and the size limit."""
import numpy as np
import pytest

import vdgen
from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_07175_amd as vd
    vd.load()


def _handle(n, k, seed):
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(n, k, seed=seed)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1))
    c = vd.clip_cells(g, d, vd.Options.default(want_grad=1))
    return c, g, d, len(sites)


def test_noalloc_adjoint_equals_the_allocating_one():
    import torch
    rng = np.random.default_rng(61)
    for n, k, seed in ((4000, 6, 62), (700, 3, 63)):  # the second call is smaller
        c, g, d, n = _handle(n, k, seed)
        gm = torch.as_tensor(rng.normal(size=n), device="cuda")
        gc = torch.as_tensor(rng.normal(size=(n, 3)), device="cuda")
        ge = torch.as_tensor(rng.normal(size=n), device="cuda")
        ref = c.backward(gm, gc, ge)
        got = c.backward_noalloc(gm, gc, ge)
        torch.cuda.synchronize()
        log(f"noalloc n={n}: max |diff| {float((got - ref).abs().max()):.3e}")
        assert torch.equal(got, ref)
        # and with some upstream gradients absent (NULL)
        ref2 = c.backward(None, gc, None)
        got2 = c.backward_noalloc(None, gc, None)
        torch.cuda.synchronize()
        assert torch.equal(got2, ref2)


def test_noalloc_rejects_more_sites_than_its_array():
    import torch
    import paper_2509_07175_amd as vd
    n = vd_max = (1 << 20) + 1
    sites = vdgen.uniform_cube_sites(n, seed=64, jitter=1e-7)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(vdgen.kuhn_cube_grid(1))
    g = vd.build_grid(s, bbox=(0, 0, 0, 1, 1, 1))
    c = vd.clip_cells(g, d, vd.Options.default(want_grad=1, emit_polytopes=0))
    with pytest.raises(vd.VDError) as e:
        c.backward_noalloc(None, None, torch.ones(vd_max, dtype=torch.float64, device="cuda"))
    assert e.value.status == 4 and "fixed scratch" in str(e.value)
