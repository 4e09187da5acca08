"""Lloyd iterations (Sec. 7.4, density 1) through the library.

* three iterations on a small cube-grid case equal three iterations of the
  oracle (its centroids fed back as sites), to 1e-9 relative;
* on the 100,000-site workload the CVT energy does not increase from one
  iteration to the next (Lloyd's method decreases it monotonically), and the
  sites stay in the unit cube.
"""
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


def test_lloyd_matches_oracle_iterations(oracle_mod):
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.small_case(400, 3, seed=21)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda").contiguous()
    vd.lloyd(s, vd.Domain.from_vdgen(dom), 3, bbox=(0, 0, 0, 1, 1, 1))
    got = s.cpu().numpy()
    ref = sites.copy()
    for _ in range(3):
        mom = oracle_mod.site_moments(oracle_mod.compute(ref, dom, brute=False), ref)
        ref = np.asarray(mom["centroid"], dtype=np.float64)
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    log(f"lloyd vs oracle: max rel err {err.max():.2e}")
    assert err.max() <= 1e-9


def test_lloyd_energy_decreases():
    import torch
    import paper_2509_07175_amd as vd
    sites, dom = vdgen.config_c2()
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda").contiguous()
    _, energies = vd.lloyd(s, vd.Domain.from_vdgen(dom), 8, bbox=(0, 0, 0, 1, 1, 1), energy=True)
    log(f"CVT energy per iteration: {energies}")
    for a, b in zip(energies, energies[1:]):
        assert b <= a * (1 + 1e-12)
    assert energies[-1] < 0.9 * energies[0]
    out = s.cpu().numpy()
    assert np.all((out > 0.0) & (out < 1.0))
