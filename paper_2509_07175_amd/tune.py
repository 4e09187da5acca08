"""Autotuner for the clip: picks the schedule knobs by timing the site kernel.

The knobs are the ones that change the work of a wavefront without changing
any result: the grid density (sites per cell, which sets the candidates per
nearest-site query and the block of cells a wave keeps in LDS), the per-wave
LDS site cache (on: 128 sites, 3.7 KB of LDS per wave; off: grid queries only), the
improved search of Sec. 6.1, the choice of straddling edges (Alg. 1) over
virtual edges (Alg. 3) and, for a batch, the order in which the persistent
kernel's queues hand out the diagrams (most tetrahedra per site first, or grid
order).  Every candidate is run once synchronously with kernel
timing (hipEvents on the caller's stream); the fastest wins.  Results are
identical for every candidate, so the tuner can run on the real input.
"""
from __future__ import annotations

import itertools

DEFAULT_SPACE = {
    "sites_per_cell": (1.0, 2.0, 3.5),
    "site_cache": (1, 0),
    "improved_search": (1, 0),
    "use_straddle_edges": (0,),
}


def tune(sites, domain, site_off=None, bboxes=None, bbox=None, space: dict | None = None, repeats: int = 1,
         base_options: dict | None = None, log=None):
    """Times every combination of `space` on (sites, domain) and returns
    (best: dict of knob values, table: list of (knobs, kernel_ms)).

    site_off / bboxes: a batch (vd_build_grid_batch); else a plain grid with
    the optional bbox."""
    import torch

    from . import Cells, Grid, Options, build_grid, build_grid_batch, clip_cells
    if space is None:
        space = dict(DEFAULT_SPACE)
        if site_off is not None:
            space["batch_order"] = (1, 0)
    space = dict(space)
    keys = list(space)
    table = []
    grid, cells = Grid(), Cells()
    for combo in itertools.product(*(space[k] for k in keys)):
        knobs = dict(zip(keys, combo))
        rho = knobs.get("sites_per_cell", 2.0)
        opt_kw = dict(base_options or {})
        opt_kw.update({k: v for k, v in knobs.items() if k != "sites_per_cell"})
        opt_kw["time_kernels"] = 1
        opt_kw["no_sync"] = 0
        best_ms = None
        for _ in range(max(1, repeats)):
            if site_off is not None:
                build_grid_batch(sites, site_off, bboxes=bboxes, sites_per_cell=rho, grid=grid)
            else:
                build_grid(sites, bbox=bbox, sites_per_cell=rho, grid=grid)
            clip_cells(grid, domain, Options.default(**opt_kw), cells=cells)
            ms = cells.info()["carve_ms"]
            best_ms = ms if best_ms is None else min(best_ms, ms)
        torch.cuda.synchronize()
        table.append((knobs, best_ms))
        if log:
            log(f"tune {knobs}: {best_ms:.2f} ms")
    best = min(table, key=lambda t: t[1])[0]
    return best, table
