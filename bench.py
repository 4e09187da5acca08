"""Throughput of the clipped-Voronoi hot path on one MI355X.

One step = vd_build_grid + vd_clip_cells + vd_cell_moments on inputs resident
in HBM (sites and the staged tetrahedral domain), i.e. cells plus centroids
from device-resident inputs, excluding allocation and host transfers.
Default workload: 1,000,000 clustered sites (8 Gaussians + 10% uniform) in a
50^3-cube grid of 750,000 tetrahedra, float64.

Prints one JSON line with the metric, the carve kernel's roofline figures
(measured with hipEvents on the stream the kernel runs on) and the CPU
oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector
HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E
# algorithmic FP64 work per unit; every unit is counted on the device (vd_cells_info)
FLOPS_PER_CANDIDATE = 8          # |q - s|^2 of one candidate site: 3 sub, 1 mul, 2 fma
FLOPS_PER_CLASSIFIED = 6         # n.y - c of one corner against a clipping plane: 1 mul, 2 fma, 1 sub
FLOPS_PER_NEW_CORNER = 51        # Cramer solve of three planes: 3 cross products (27), det (5),
                                 # reciprocal (1), 3 coordinates (18)
FLOPS_PER_FAN_TET = 78           # one moment-fan tetrahedron: plane foot (15), det (14), volume (1),
                                 # corner sums (12), volume / first moment (10), energy (26)
# algorithmic HBM bytes, per counted unit
BYTES_PER_SITE = 110 + 48        # inputs (site, sorted copy, perm, grid, simplices share) + per-site outputs
BYTES_PER_PIECE = 72             # piece record
BYTES_PER_FACE = 4               # face label
BYTES_PER_VERT = 36              # vertex coordinates + 3 labels
BYTES_PER_NBR = 8                # neighbour (arena + CSR)
KERNEL_FILES = ("clip3d.hip", "vd_common.h", "vd_arena.h", "vd_internal.h")


def recorded_traffic():
    """HBM bytes per site_kernel launch from the committed counter profile, if
    the kernel sources are still the profiled ones (else None)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        with open(os.path.join(ROOT, "paper_2509_07175_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    path = os.path.join(ROOT, "profiles", "site_kernel_c3_counters.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(rec["traffic_bytes_per_launch"])


def workload(name):
    import vdgen
    if name == "c1":
        s, d = vdgen.config_c1()
        return s, d, "C1: 1,000 uniform sites, unit cube as 6 tetrahedra", 2.0
    if name == "c2":
        s, d = vdgen.config_c2()
        return s, d, "C2: 100,000 uniform sites, 20^3 cubes x 6 = 48,000 tetrahedra", 2.0
    if name == "cube5m":
        # the shape of the paper's own GPU headline run (white noise in a cube); context only
        s = vdgen.uniform_cube_sites(5_000_000, seed=108, jitter=1e-7)
        return s, vdgen.kuhn_cube_grid(1), "5,000,000 uniform sites, unit cube as 6 tetrahedra", 2.0
    s, d = vdgen.config_c3()
    return (s, d, "C3: 1,000,000 clustered sites (8 Gaussians sigma 0.05 + 10% uniform), "
                  "50^3 cubes x 6 = 750,000 tetrahedra", 0.25)


def _host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)


def cpu_baseline(sites, dom, target_s=15.0):
    """The oracle (plain CPU definition, pruned mode, -O3 -march=native build)
    on a bounded sample of sites: for each sampled site, the simplices its cell
    can meet come from a grid of simplex bounding boxes (a 1-Lipschitz bound on
    the nearest-site distance), and each piece is cut by the bisectors of the
    sites within the security radius."""
    import numpy as np
    import oracle
    oracle.build(force=True, native=True)
    threads = _host_threads()
    rng = np.random.default_rng(5)
    k = 256
    elapsed = 0.0
    while True:
        sample = np.sort(rng.choice(len(sites), size=k, replace=False)).astype(np.int32)
        t0 = time.perf_counter()
        oracle.compute(sites, dom, only_sites=sample, threads=threads, native=True)
        elapsed = time.perf_counter() - t0
        if elapsed >= target_s / 4 or k >= len(sites):
            break
        k = min(len(sites), int(k * max(2.0, min(8.0, (target_s / 2) / max(elapsed, 1e-3)))))
    return {"value": k / elapsed, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} sites drawn uniformly from the workload, all their pieces (candidate simplices "
                      f"from a simplex-box grid, bisectors within the security radius), -O3 -march=native, "
                      f"{elapsed:.2f} s wall on {threads} threads"}


def cpu_block_baseline(sites, log, k=50, lo=20, hi=30):
    """The oracle's full run (every simplex of the domain, pruned mode) on a
    spatial sub-block of the workload: the tetrahedra of the cubes
    [lo, hi)^3 of the k^3 grid, with all sites; cells/s counts the sites that
    have a piece there."""
    import numpy as np
    import oracle
    import vdgen
    oracle.build(force=False, native=True)
    threads = _host_threads()
    block = vdgen.kuhn_cube_subset(k, lambda x, y, z: lo <= x < hi and lo <= y < hi and lo <= z < hi)
    t0 = time.perf_counter()
    r = oracle.compute(sites, block, threads=threads, native=True)
    el = time.perf_counter() - t0
    cells = len(np.unique(r["piece_site"]))
    log(f"oracle full run on a {hi - lo}^3-cube block ({block.m} tetrahedra): {cells} cells in {el:.2f} s")
    return {"value": cells / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"full pruned run over the {block.m} tetrahedra of cubes [{lo},{hi})^3 of the {k}^3 grid "
                      f"({cells} cells meet them), {el:.2f} s wall"}


def cpu_single_thread(log):
    """The oracle on one host thread: the 1,000-site cube in full (brute force,
    every bisector, and pruned) and 2,000 sampled sites of the 100,000-site
    workload (pruned)."""
    import numpy as np
    import oracle
    import vdgen
    oracle.build(force=False)
    out = {}
    s1, d1 = vdgen.config_c1()
    for mode, brute in (("c1_brute", True), ("c1_pruned", False)):
        t0 = time.perf_counter()
        oracle.compute(s1, d1, brute=brute, threads=1)
        out[mode + "_cells_per_s"] = len(s1) / (time.perf_counter() - t0)
    s2, d2 = vdgen.config_c2()
    sample = np.sort(np.random.default_rng(6).choice(len(s2), size=2000, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    oracle.compute(s2, d2, only_sites=sample, threads=1)
    out["c2_sample_cells_per_s"] = len(sample) / (time.perf_counter() - t0)
    out["cores"] = 1
    log(f"oracle on one thread: {out}")
    return out


def bench_batched(steps, warmup, log):
    """256 independent diagrams: sequential plain calls vs one autotuned batch
    (grid build + clip + moments) captured in a HIP graph and replayed."""
    import numpy as np
    import torch

    import paper_2509_07175_amd as vd
    import vdgen
    from paper_2509_07175_amd import tune as vdtune
    items = vdgen.config_c4()
    B = len(items)
    so = np.concatenate([[0], np.cumsum([len(s) for s, _ in items])])
    n = int(so[-1])
    boxes = [(0.0, 0.0, 0.0, 1.0, 1.0, 1.0)] * B
    log(f"batched: {B} diagrams, {n} sites, {sum(len(d.simplices) for _, d in items)} tetrahedra")
    # --- sequential plain calls (one vd_build_grid + vd_clip_cells + vd_cell_moments per diagram)
    plain = []
    for s, d in items:
        t = torch.as_tensor(s, dtype=torch.float64, device="cuda")
        plain.append((t, vd.Domain.from_vdgen(d), vd.Grid(), vd.Cells(),
                      torch.empty(len(s), dtype=torch.float64, device="cuda"),
                      torch.empty((len(s), 3), dtype=torch.float64, device="cuda"),
                      torch.empty(len(s), dtype=torch.float64, device="cuda")))
    popt = vd.Options.default()

    def plain_pass():
        for t, dom, g, c, m, ce, e in plain:
            vd.build_grid(t, bbox=boxes[0], grid=g)
            vd.clip_cells(g, dom, popt, cells=c)
            c.moments(m, ce, e)

    for _ in range(max(1, warmup)):
        plain_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_pass()
    torch.cuda.synchronize()
    plain_ms = 1e3 * (time.perf_counter() - t0) / steps
    log(f"batched: sequential plain calls {plain_ms:.1f} ms per pass")
    # --- the batch: autotune, then capture and replay
    sites = torch.as_tensor(np.concatenate([s for s, _ in items]), dtype=torch.float64, device="cuda")
    dom = vd.Domain.batch_from_vdgen([d for _, d in items])
    best, table = vdtune.tune(sites, dom, site_off=so, bboxes=boxes, log=log)
    best = dict(best)
    rho = best.pop("sites_per_cell")
    side = torch.cuda.Stream()
    grid, cells = vd.Grid(), vd.Cells()
    mass = torch.empty(n, dtype=torch.float64, device="cuda")
    cent = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    en = torch.empty(n, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(side):
        vd.build_grid_batch(sites, so, bboxes=boxes, sites_per_cell=rho, grid=grid)
        vd.clip_cells(grid, dom, vd.Options.default(time_kernels=1, **best), cells=cells)
        kernel_ms = cells.info()["carve_ms"]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        vd.build_grid_batch(sites, so, bboxes=boxes, sites_per_cell=rho, grid=grid)
        vd.clip_cells(grid, dom, vd.Options.default(no_sync=1, **best), cells=cells)
        cells.moments(mass, cent, en)
    for _ in range(max(1, warmup)):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    batch_ms = 1e3 * (time.perf_counter() - t0) / steps
    info = cells.info()
    if info["status"] != 0:
        raise RuntimeError(f"batched replay failed: {info}")
    vols = [float(mass[so[b]:so[b + 1]].sum().item()) for b in range(B)]
    log(f"batched: graph replay {batch_ms:.1f} ms, site kernel {kernel_ms:.1f} ms")
    return {"workload": f"{B} diagrams, {n} sites (1,000-64,000 each, log-uniform), jittered 8^3-24^3 "
                        f"cube grids x 6 tetrahedra", "sites": n, "diagrams": B,
            "plain_sequential_ms": plain_ms, "plain_sequential_cells_per_s": n / (plain_ms * 1e-3),
            "batched_graph_ms": batch_ms, "batched_cells_per_s": n / (batch_ms * 1e-3),
            "speedup_vs_plain": plain_ms / batch_ms, "site_kernel_ms": kernel_ms,
            "pieces": info["n_pieces"], "pieces_per_site": info["n_pieces"] / n,
            "site_kernel_pieces_per_s": info["n_pieces"] / (kernel_ms * 1e-3),
            "tuned": dict(best, sites_per_cell=rho), "tuning": [[k, ms] for k, ms in table],
            "max_volume_error": max(abs(v - 1.0) for v in vols)}


def bench_backward(sites_t, dom_h, rho, steps, warmup, log):
    """Forward with face moments + vd_cell_moments_backward (CVT energy and a
    random linear loss on mass and centroid) vs the plain forward."""
    import torch

    import paper_2509_07175_amd as vd
    n = sites_t.shape[0]
    bbox = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    grid, cells = vd.Grid(), vd.Cells()
    mass = torch.empty(n, dtype=torch.float64, device="cuda")
    cent = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    en = torch.empty(n, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(9)
    gm = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
    gc = torch.randn((n, 3), dtype=torch.float64, device="cuda", generator=gen)
    ge = torch.ones(n, dtype=torch.float64, device="cuda")
    gs = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    opt = vd.Options.default(want_grad=1, time_kernels=1)

    def step():
        vd.build_grid(sites_t, bbox=bbox, sites_per_cell=rho, grid=grid)
        vd.clip_cells(grid, dom_h, opt, cells=cells)
        cells.moments(mass, cent, en)
        cells.backward(gm, gc, ge, out=gs)

    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    # adjoint alone
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        cells.backward(gm, gc, ge, out=gs)
    ev1.record()
    torch.cuda.synchronize()
    adj_ms = ev0.elapsed_time(ev1) / steps
    # the CVT part of the gradient is 2 m (v - c): check it on this run
    ref = 2 * mass[:, None] * (sites_t - cent)
    cells.backward(None, None, ge, out=gs)
    torch.cuda.synchronize()
    err = float((gs - ref).abs().max().item() / ref.abs().max().item())
    log(f"backward: forward+grad+adjoint {ms:.1f} ms per step, adjoint {adj_ms:.2f} ms, CVT check {err:.1e}")
    return {"forward_with_face_moments_plus_adjoint_ms": ms, "cells_per_s": n / (ms * 1e-3),
            "adjoint_kernel_ms": adj_ms, "adjoint_cells_per_s": n / (adj_ms * 1e-3),
            "site_kernel_ms_with_face_moments": cells.info()["carve_ms"], "cvt_gradient_rel_err": err}


def bench_surface(steps, warmup, log):
    """Restricted VD on the sphere (200,000 sites, 81,920-triangle icosphere):
    plain forward, forward with face moments + adjoint, adjoint alone."""
    import numpy as np
    import torch

    import paper_2509_07175_amd as vd
    import vdgen
    sites, dom = vdgen.config_c5()
    n = len(sites)
    q = dom.verts[dom.simplices]
    area = float(0.5 * np.linalg.norm(np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), axis=1).sum())
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    bbox = (-1.01, -1.01, -1.01, 1.01, 1.01, 1.01)
    grid, cells = vd.Grid(), vd.Cells()
    mass = torch.empty(n, dtype=torch.float64, device="cuda")
    cent = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    en = torch.empty(n, dtype=torch.float64, device="cuda")
    ge = torch.ones(n, dtype=torch.float64, device="cuda")
    gs = torch.empty((n, 3), dtype=torch.float64, device="cuda")

    def timed(fn):
        for _ in range(max(1, warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps

    plain_opt = vd.Options.default()
    grad_opt = vd.Options.default(want_grad=1)

    def fwd():
        vd.build_grid(s, bbox=bbox, surface_area=area, grid=grid)
        vd.clip_cells(grid, d, plain_opt, cells=cells)
        cells.moments(mass, cent, en)

    def fwd_bwd():
        vd.build_grid(s, bbox=bbox, surface_area=area, grid=grid)
        vd.clip_cells(grid, d, grad_opt, cells=cells)
        cells.moments(mass, cent, en)
        cells.backward(None, None, ge, out=gs)

    f_ms = timed(fwd)
    fb_ms = timed(fwd_bwd)
    b_ms = timed(lambda: cells.backward(None, None, ge, out=gs))
    ref = 2 * mass[:, None] * (s - cent)
    err = float((gs - ref).abs().max().item() / ref.abs().max().item())
    log(f"surface: forward {f_ms:.1f} ms, forward+adjoint {fb_ms:.1f} ms, adjoint {b_ms:.2f} ms, CVT check {err:.1e}")
    return {"workload": f"{n} sites on the unit sphere, icosphere of {dom.m} triangles",
            "forward_ms": f_ms, "forward_cells_per_s": n / (f_ms * 1e-3),
            "forward_plus_adjoint_ms": fb_ms, "forward_plus_adjoint_cells_per_s": n / (fb_ms * 1e-3),
            "adjoint_ms": b_ms, "adjoint_cells_per_s": n / (b_ms * 1e-3),
            "forward_plus_adjoint_vs_forward": f_ms / fb_ms, "cvt_gradient_rel_err": err}


def bench_cvt(log, iterations=10):
    """CVT on the 100,000-site workload with a quadratic density (Eq. 3):
    L-BFGS on the library's moments and adjoint, and Lloyd (sites <- weighted
    centroids) from the same start; energies per iteration and time."""
    import torch
    import paper_2509_07175_amd as vd
    import vdgen
    sites, dom = vdgen.config_c2()
    d = vd.Domain.from_vdgen(dom)
    rho = [1.0, 0.5, -0.3, 0.2, 0.4, 0.1, -0.2, 0.3, 0.05, 0.6]
    opt = vd.Options.default(density=rho)
    s = torch.as_tensor(sites, dtype=torch.float64, device="cuda").contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, e_lbfgs = vd.cvt_lbfgs(s, d, iterations, options=opt, bbox=(0, 0, 0, 1, 1, 1))
    torch.cuda.synchronize()
    t_lbfgs = time.perf_counter() - t0
    ls = s.clone()
    t0 = time.perf_counter()
    _, e_lloyd = vd.lloyd(ls, d, iterations, options=opt, bbox=(0, 0, 0, 1, 1, 1), energy=True)
    torch.cuda.synchronize()
    t_lloyd = time.perf_counter() - t0
    mono = all(b <= a * (1 + 1e-12) for a, b in zip(e_lbfgs, e_lbfgs[1:]))
    log(f"cvt: L-BFGS energy {e_lbfgs[0]:.6e} -> {e_lbfgs[-1]:.6e} in {t_lbfgs:.2f} s (monotone {mono}); "
        f"Lloyd -> {e_lloyd[-1]:.6e} in {t_lloyd:.2f} s")
    return {"workload": "100,000 uniform sites, 48,000 tetrahedra, density rho(x) quadratic " + str(rho),
            "iterations": iterations, "lbfgs_energies": e_lbfgs, "lbfgs_monotone": mono, "lbfgs_s": t_lbfgs,
            "lloyd_energies": e_lloyd, "lloyd_s": t_lloyd}


def measured_peaks(log):
    """Measured ceilings on this GPU: FP64 FMA rate (a HIP probe of eight
    independent v_fma_f64 chains per lane) and device-to-device copy rate
    (1 GiB read + 1 GiB written).  None where the probe is unavailable."""
    import ctypes
    import torch
    out = {"fp64_fma_tflops": None, "copy_gbs": None}
    src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = 5 * 2 * 2 ** 30 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    lib_path = os.path.join(ROOT, "paper_2509_07175_amd", "libvd_probe.so")
    if os.path.exists(lib_path):
        lib = ctypes.CDLL(lib_path)
        lib.vd_probe_fma_f64.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
        blocks, iters = 8192, 20000
        buf = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
        ms, fl = ctypes.c_float(0.0), ctypes.c_double(0.0)
        if lib.vd_probe_fma_f64(blocks, iters, ctypes.c_void_p(buf.data_ptr()), ctypes.byref(ms), ctypes.byref(fl)) == 0:
            out["fp64_fma_tflops"] = fl.value / (ms.value * 1e-3) / 1e12
    log(f"measured peaks: FP64 FMA {out['fp64_fma_tflops']} TFLOP/s, copy {out['copy_gbs']:.0f} GB/s")
    return out


def bench_plain_other(log):
    """Plain build_grid + clip + moments on the small cube workloads."""
    import torch
    import paper_2509_07175_amd as vd
    res = {}
    for name in ("c1", "c2"):
        sites, dom, desc, rho = workload(name)
        n = len(sites)
        s = torch.as_tensor(sites, dtype=torch.float64, device="cuda")
        d = vd.Domain.from_vdgen(dom)
        grid, cells = vd.Grid(), vd.Cells()
        mass = torch.empty(n, dtype=torch.float64, device="cuda")
        cent = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        en = torch.empty(n, dtype=torch.float64, device="cuda")
        opt = vd.Options.default()

        def step():
            vd.build_grid(s, bbox=(0.0, 0.0, 0.0, 1.0, 1.0, 1.0), sites_per_cell=rho, grid=grid)
            vd.clip_cells(grid, d, opt, cells=cells)
            cells.moments(mass, cent, en)

        for _ in range(3):
            step()
        torch.cuda.synchronize()
        times = []
        for _ in range(20):
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        med = float(sorted(times)[len(times) // 2])
        res[name] = {"workload": desc, "median_ms": 1e3 * med, "cells_per_s": n / med}
        log(f"{name}: {1e3 * med:.2f} ms median, {n / med:.3g} cells/s")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "cube5m"])
    ap.add_argument("--rho", type=float, default=None, help="grid sites per cell")
    ap.add_argument("--no-emit", action="store_true", help="skip writing per-piece polytopes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--carve-mode", type=int, default=1, choices=[0, 1])
    ap.add_argument("--improved", type=int, default=0, choices=[0, 1])
    ap.add_argument("--straddle", type=int, default=0, choices=[0, 1])
    ap.add_argument("--site-cache", type=int, default=1, choices=[0, 1])
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-diagrams comparison")
    ap.add_argument("--no-variants", action="store_true", help="skip timing the other search variants")
    ap.add_argument("--no-backward", action="store_true", help="skip the adjoint throughput")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured FMA / copy peaks")
    ap.add_argument("--no-small", action="store_true", help="skip the 1k- and 100k-site cube workloads")
    ap.add_argument("--lloyd-whole-interior", action="store_true",
                    help="Lloyd iterations with Alg. 5's interior split (same moments, interior cells not cut)")
    ap.add_argument("--lloyd", type=int, default=0,
                    help="also time this many Lloyd iterations (sites <- centroids) on the workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark measures exactly one GPU (asked for {args.gpus}); a multi-GPU run "
              "would give each GPU a range of grid-ordered sites with the sites, grid and domain replicated",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        # a kernel of known traffic: 2^30 bytes read and 2^30 bytes written per launch
        src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 2 ** 30, "launches": 5}), flush=True)
        return

    import paper_2509_07175_amd as vd

    vd.load()
    sites, dom, desc, rho_default = workload(args.workload)
    rho = args.rho if args.rho is not None else rho_default
    n = len(sites)
    dev = torch.device("cuda:0")
    s = torch.as_tensor(sites, dtype=torch.float64, device=dev).contiguous()
    d = vd.Domain.from_vdgen(dom)
    opts = vd.Options.default(time_kernels=1, emit_polytopes=0 if args.no_emit else 1,
                              carve_mode=args.carve_mode, improved_search=args.improved,
                              use_straddle_edges=args.straddle, site_cache=args.site_cache)
    grid, cells = vd.Grid(), vd.Cells()
    mass = torch.empty(n, dtype=torch.float64, device=dev)
    cent = torch.empty((n, 3), dtype=torch.float64, device=dev)
    en = torch.empty(n, dtype=torch.float64, device=dev)
    bbox = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    torch.cuda.synchronize()
    free_before, _ = torch.cuda.mem_get_info()  # the library's grid and output arenas come after

    def step():
        vd.build_grid(s, bbox=bbox, sites_per_cell=rho, grid=grid)
        vd.clip_cells(grid, d, opts, cells=cells)
        cells.moments(mass, cent, en)

    print(f"bench: {desc}; inputs on the device, warming up", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        print(f"bench: warmup {w} {1e3 * (time.perf_counter() - t1):.1f} ms", file=sys.stderr, flush=True)
    kern, step_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        step()
        inf = cells.info()  # waits for the step (the piece counts it reports come from the device)
        step_ms.append(1e3 * (time.perf_counter() - ts))
        kern.append(inf["carve_ms"])
        print(f"bench: step {len(kern)} site kernel {inf['carve_ms']:.2f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    free_after, _ = torch.cuda.mem_get_info()
    info = cells.info()
    ms = 1e3 * wall / args.steps
    # the work of the same step, counted by one more clip with the kernel's
    # counters on (they cost time, so the timed steps run without them; the
    # work is the same: identical inputs give identical queries and clips)
    mopts = vd.Options.default(time_kernels=1, emit_polytopes=0 if args.no_emit else 1,
                               carve_mode=args.carve_mode, improved_search=args.improved,
                               use_straddle_edges=args.straddle, site_cache=args.site_cache, monitor=1)
    mcells = vd.Cells()
    vd.clip_cells(grid, d, mopts, cells=mcells)
    minfo = mcells.info()
    del mcells
    # the dominant kernel: the persistent per-site kernel (cell carve + pieces)
    dom_ms, dom_name = float(np.mean(kern)), "site_kernel"
    flops = (FLOPS_PER_CANDIDATE * minfo["candidates"] + FLOPS_PER_CLASSIFIED * minfo["corners_classified"] +
             FLOPS_PER_NEW_CORNER * minfo["corners_created"] + FLOPS_PER_FAN_TET * minfo["fan_simplices"])
    achieved = flops / (dom_ms * 1e-3) / 1e12
    alg_bytes = (BYTES_PER_SITE * n + BYTES_PER_PIECE * info["n_pieces"] + BYTES_PER_FACE * info["n_faces"] +
                 BYTES_PER_VERT * info["n_verts"] + BYTES_PER_NBR * info["n_nbrs"])
    traffic = recorded_traffic() if args.workload == "c3" and not args.no_emit else None
    total_mass = float(mass.sum().item())

    out = {
        "metric": "clipped Voronoi cells/s at 1M 3D sites; batched & backward vs plain on same GPU",
        "value": n / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "sites": n, "tetrahedra": int(dom.m), "grid_sites_per_cell": rho,
                   "emit_polytopes": not args.no_emit, "carve_mode": args.carve_mode,
                   "improved_search": args.improved, "straddle_edges": args.straddle,
                   "site_cache": args.site_cache},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": dom_name, "kernel_ms": dom_ms, "algorithmic_flops": flops,
                     "hbm": {"algorithmic_bytes": alg_bytes,
                             "achieved": alg_bytes / (dom_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                             "frac": alg_bytes / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                             "measured": None if traffic is None else traffic / (dom_ms * 1e-3) / 1e9}},
        "step_ms_percentiles": {"p10": float(np.percentile(step_ms, 10)), "p50": float(np.percentile(step_ms, 50)),
                                "p90": float(np.percentile(step_ms, 90))},
        "device_memory_bytes": int(free_before - free_after),
        "counters": {"pieces": info["n_pieces"], "nn_queries": info["nn_queries"], "clips": info["clips"],
                     "candidates": info["candidates"], "queries_per_cell": info["nn_queries"] / n,
                     "query_rounds_per_cell": minfo["query_rounds"] / n,
                     "tests_wasted_per_cell": minfo["tests_wasted"] / n,
                     "grid_queries": info["grid_queries"], "corners_classified": minfo["corners_classified"],
                     "corners_created": minfo["corners_created"], "fan_tetrahedra": minfo["fan_simplices"],
                     "min_predicate_margin": minfo["min_margin"], "predicates_below_1e-12": minfo["low_margin"],
                     "site_kernel_ms_with_counters": minfo["carve_ms"],
                     "mass_sum": total_mass,
                     "paper_context": "Sec. 6.2: over 20.54 M nearest-neighbour searches for 1 M uniform "
                                      "cells in a cube with the serial method (one search per point-in-cell "
                                      "test); queries_per_cell counts every test of a four-corner batch and "
                                      "every search step, query_rounds_per_cell the batches a wave waits for"},
    }
    log = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)  # noqa: E731
    # the same step with the other search variants of the paper (identical results)
    variants = {}
    for name, kw in () if args.no_variants else (("improved_search", dict(improved_search=1)),
                                                  ("straddling_edges", dict(use_straddle_edges=1))):
        vopt = vd.Options.default(time_kernels=1, emit_polytopes=0 if args.no_emit else 1, carve_mode=args.carve_mode,
                                  site_cache=args.site_cache, **kw)
        vg, vc = vd.Grid(), vd.Cells()
        best = None
        for _ in range(2):
            vd.build_grid(s, bbox=bbox, sites_per_cell=rho, grid=vg)
            vd.clip_cells(vg, d, vopt, cells=vc)
            vi = vc.info()
            best = vi["carve_ms"] if best is None else min(best, vi["carve_ms"])
        variants[name] = {"site_kernel_ms": best, "nn_queries": vi["nn_queries"], "clips": vi["clips"],
                          "n_pieces": vi["n_pieces"]}
        log(f"variant {name}: site kernel {best:.2f} ms, {vi['nn_queries'] / n:.1f} queries per cell")
        del vg, vc
    if variants:
        out["search_variants"] = variants
    if not args.no_variants:
        # Alg. 5's interior / boundary split: cells that meet no boundary
        # triangle come out whole (one piece each), the rest per tetrahedron;
        # the step includes the boundary surface's restricted diagram
        wopt = vd.Options.default(time_kernels=1, emit_polytopes=0 if args.no_emit else 1,
                                  carve_mode=1, site_cache=args.site_cache, whole_interior=1)
        wg, wc = vd.Grid(), vd.Cells()
        wm = torch.empty_like(mass)
        wce = torch.empty_like(cent)
        wen = torch.empty_like(en)

        def wstep():
            vd.build_grid(s, bbox=bbox, sites_per_cell=rho, grid=wg)
            vd.clip_cells(wg, d, wopt, cells=wc)
            wc.moments(wm, wce, wen)

        wstep()
        torch.cuda.synchronize()
        wt, wk = [], []
        for _ in range(3):
            t1 = time.perf_counter()
            wstep()
            wi = wc.info()
            wt.append(1e3 * (time.perf_counter() - t1))
            wk.append(wi["carve_ms"])
        dm = float((wm - mass).abs().max().item() / mass.abs().max().item())
        out["whole_interior"] = {"ms_per_step": float(np.median(wt)), "cells_per_s": n / (np.median(wt) * 1e-3),
                                 "site_kernel_ms": float(np.median(wk)), "n_pieces": wi["n_pieces"],
                                 "max_mass_diff_vs_per_tet": dm, "vs_plain": ms / float(np.median(wt))}
        log(f"whole_interior: {np.median(wt):.2f} ms per step, site kernel {np.median(wk):.2f} ms, "
            f"{wi['n_pieces']} pieces, mass diff {dm:.2e}")
        del wg, wc
    if args.lloyd > 0:
        ls = torch.as_tensor(sites, dtype=torch.float64, device=dev).contiguous()
        lopt = vd.Options.default(whole_interior=1 if args.lloyd_whole_interior else 0)
        vd.lloyd(ls, d, 1, options=lopt, bbox=bbox, sites_per_cell=rho)  # sizes the arenas
        ls.copy_(torch.as_tensor(sites, dtype=torch.float64))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, energies = vd.lloyd(ls, d, args.lloyd, options=lopt, bbox=bbox, sites_per_cell=rho,
                               energy=True)
        torch.cuda.synchronize()
        lt = time.perf_counter() - t0
        out["lloyd"] = {"iterations": args.lloyd, "whole_interior": bool(args.lloyd_whole_interior),
                        "s_per_iteration": lt / args.lloyd,
                        "cells_per_s": n * args.lloyd / lt, "energy_first": energies[0], "energy_last": energies[-1]}
        log(f"lloyd: {args.lloyd} iterations, {lt / args.lloyd * 1e3:.1f} ms each, energy {energies[0]:.6g} -> "
            f"{energies[-1]:.6g}")
    if not args.no_peaks:
        pk = measured_peaks(log)
        out["measured_peaks"] = pk
        if pk["fp64_fma_tflops"]:
            out["roofline"]["frac_of_measured_peak"] = achieved / pk["fp64_fma_tflops"]
        if pk["copy_gbs"]:
            out["roofline"]["hbm"]["frac_of_measured_copy"] = out["roofline"]["hbm"]["achieved"] / pk["copy_gbs"]
    if not args.no_small:
        out["plain_small"] = bench_plain_other(log)
    if not args.no_backward:
        out["backward"] = bench_backward(s, d, rho, max(1, min(args.steps, 5)), 1, log)
        out["backward"]["vs_plain_forward"] = ms / out["backward"]["forward_with_face_moments_plus_adjoint_ms"]
    if not args.no_backward:
        out["backward_surface"] = bench_surface(max(1, min(args.steps, 5)), 1, log)
    if not args.no_batched:
        out["batched"] = bench_batched(max(1, min(args.steps, 5)), 1, log)
        # per piece, against the plain step's site kernel: the batch's small
        # diagrams on fine meshes have many more pieces per cell
        out["batched"]["pieces_per_s_vs_plain_site_kernel"] = (
            out["batched"]["site_kernel_pieces_per_s"] / (info["n_pieces"] / (dom_ms * 1e-3)))
    if not args.no_small:
        out["cvt_density"] = bench_cvt(log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sites, dom)
        if args.workload == "c3":
            out["cpu_baseline_block"] = cpu_block_baseline(sites, log)
        out["cpu_single_thread"] = cpu_single_thread(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
