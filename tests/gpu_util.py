"""Helpers for the GPU parity tests: run the library, compare with the oracle."""
import sys

import numpy as np

from canon import canon_pieces


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(sites, dom, bbox=(0, 0, 0, 1, 1, 1), surface_area=0.0, weights=None, **opts):
    import torch
    import paper_2509_07175_amd as vd
    s = torch.as_tensor(np.ascontiguousarray(sites), dtype=torch.float64, device="cuda")
    d = vd.Domain.from_vdgen(dom)
    w = None if weights is None else torch.as_tensor(np.ascontiguousarray(weights), dtype=torch.float64, device="cuda")
    g = vd.build_grid(s, bbox=bbox, surface_area=surface_area, weights=w)
    c = vd.clip_cells(g, d, vd.Options.default(**opts))
    m, ce, e = c.moments()
    torch.cuda.synchronize()
    view = c.view()
    res = vd.pieces_as_result(view)
    out = {
        "mass": m.cpu().numpy(), "centroid": ce.cpu().numpy(), "energy": e.cpu().numpy(),
        "info": c.info(), "res": res,
        "nbr_off": view["nbr_off"].cpu().numpy(), "nbr": view["nbr"].cpu().numpy(),
        "cell_piece_off": view["cell_piece_off"].cpu().numpy(), "piece_id": view["piece_id"].cpu().numpy(),
        "raw_piece_site": view["piece_site"].cpu().numpy(),
        "raw_piece_simplex": view["piece_simplex"].cpu().numpy(),
        "cells": c, "grid": g, "domain": d, "sites_t": s,
    }
    return out


def ranges(starts, counts):
    """Concatenation of arange(s, s + c) over (starts, counts), vectorised."""
    starts = np.asarray(starts, dtype=np.int64)
    counts = np.asarray(counts, dtype=np.int64)
    tot = int(counts.sum())
    if tot == 0:
        return np.zeros(0, np.int64)
    first = np.repeat(np.cumsum(counts) - counts, counts)
    return np.repeat(starts, counts) + (np.arange(tot, dtype=np.int64) - first)


def sampled_result(view, sample, off=None):
    """The pieces of the sites in `sample` (caller indices), gathered on the
    device, in the oracle's layout (sorted by site, then simplex): for
    workloads whose full polytope output is too large to copy to the host."""
    import torch
    off = view["cell_piece_off"].cpu().numpy() if off is None else off
    sample = np.asarray(sample, dtype=np.int64)
    dev = view["piece_id"].device
    pos = ranges(off[sample], off[sample + 1] - off[sample])
    ids = view["piece_id"][torch.as_tensor(pos, device=dev)].cpu().numpy().astype(np.int64)
    idt = torch.as_tensor(ids, device=dev)

    def take(name):
        return view[name][idt].cpu().numpy()
    site, simp = take("piece_site"), take("piece_simplex")
    order = np.lexsort((simp, site))
    ids, site, simp = ids[order], site[order], simp[order]
    idt = torch.as_tensor(ids, device=dev)
    nface = view["piece_nface"][idt].cpu().numpy().astype(np.int64)
    nvert = view["piece_nvert"][idt].cpu().numpy().astype(np.int64)
    fst = view["piece_face_start"][idt].cpu().numpy()
    vst = view["piece_vert_start"][idt].cpu().numpy()
    ft = torch.as_tensor(ranges(fst, nface), device=dev)
    vt = torch.as_tensor(ranges(vst, nvert), device=dev)
    return {
        "piece_site": site, "piece_simplex": simp,
        "piece_mass": view["piece_mass"][idt].cpu().numpy(),
        "piece_moment": view["piece_moment"][idt].cpu().numpy(),
        "piece_energy": view["piece_energy"][idt].cpu().numpy(),
        "piece_face_off": np.concatenate([[0], np.cumsum(nface)]).astype(np.int64),
        "piece_vert_off": np.concatenate([[0], np.cumsum(nvert)]).astype(np.int64),
        "face_label": view["face_label"][ft].cpu().numpy(),
        "vert_xyz": view["vert_xyz"][vt].cpu().numpy(),
        "vert_label": view["vert_label"][vt].cpu().numpy(),
    }


def shift_labels(lab, site_lo, simp_lo):
    """Batch (global) face / vertex flags of one diagram -> its local flags:
    sites minus site_lo, -(b+1) flags with b minus simp_lo, boundary flags and
    the triangle filler INT32_MAX unchanged."""
    lab = np.asarray(lab).astype(np.int64)
    out = lab.copy()
    pos = (lab >= 0) & (lab != 2**31 - 1)
    out[pos] = lab[pos] - site_lo
    neg = (lab < 0) & (lab > -2**31 + 16)
    out[neg] = -((-lab[neg] - 1) - simp_lo) - 1
    return out


def assert_sampled_parity(res_gpu, mass, cent, en, nbr_off, nbr, ref, mom, sample, xyz_tol=1e-10, rel=1e-9,
                          site_lo=0):
    """Sampled sites of a full-size run against the oracle: piece sets, face
    labels and vertex label triples bit-exact, vertices within xyz_tol,
    masses / centroids / energies within rel, neighbour lists equal.  The GPU
    arrays are indexed site_lo + i for oracle site i (batches)."""
    sample = np.asarray(sample, dtype=np.int64)
    sset = set(sample.tolist())
    a = canon_pieces(res_gpu)
    b = {k: v for k, v in canon_pieces(ref).items() if k[0] in sset}
    missing = sorted(set(b) - set(a))[:5]
    extra = sorted(set(a) - set(b))[:5]
    assert not missing and not extra, f"piece sets differ: missing {missing} extra {extra}"
    md = 0.0
    for k in b:
        assert a[k][0] == b[k][0] and a[k][1] == b[k][1], f"combinatorics differ at {k}"
        if len(b[k][2]):
            md = max(md, float(np.abs(a[k][2] - b[k][2]).max()))
    assert md <= xyz_tol, f"vertex coordinates differ by {md}"
    g = site_lo + sample
    m_r, c_r, e_r = mom["mass"][sample], mom["centroid"][sample], mom["energy"][sample]
    nz = m_r > 0
    assert np.all(np.abs(mass[g] - m_r) <= rel * m_r), "mass"
    cerr = np.linalg.norm(cent[g] - c_r, axis=1) / np.linalg.norm(c_r, axis=1)
    assert np.all(cerr[nz] <= rel), f"centroid max rel err {cerr[nz].max()}"
    assert np.all(np.abs(en[g] - e_r)[nz] <= rel * e_r[nz]), "energy"
    for i in sample:
        got = nbr[nbr_off[site_lo + i]:nbr_off[site_lo + i + 1]] - site_lo
        assert list(got) == list(mom["neighbors"][i]), f"neighbours of site {i} differ"
    return md


def assert_neighbour_symmetry(nbr_off, nbr):
    """j is a neighbour of i iff i is a neighbour of j, over all sites."""
    n = len(nbr_off) - 1
    owner = np.repeat(np.arange(n, dtype=np.int64), np.diff(nbr_off))
    fwd = owner * n + nbr.astype(np.int64)
    bwd = nbr.astype(np.int64) * n + owner
    assert np.array_equal(np.sort(fwd), np.sort(bwd)), "neighbour relation is not symmetric"


def assert_csr(gpu, n):
    """The per-site CSR lists exactly the used piece slots, each under its own
    site, by ascending simplex."""
    off, pid, site = gpu["cell_piece_off"], gpu["piece_id"], gpu["raw_piece_site"]
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    assert np.array_equal(np.sort(pid), np.nonzero(site >= 0)[0])
    owner = np.repeat(np.arange(n), np.diff(off))
    assert np.array_equal(site[pid], owner)
    simp = gpu["res"]["piece_simplex"]  # (site, simplex) order, same as the CSR
    assert np.array_equal(gpu["raw_piece_simplex"][pid], simp)


def gpu_neighbors(out, n):
    off, nb = out["nbr_off"], out["nbr"]
    return [nb[off[i]:off[i + 1]] for i in range(n)]


def assert_parity(gpu, ref_res, ref_mom, n, sites_subset=None, xyz_tol=1e-10, rel=1e-9):
    """Bit-exact combinatorics (piece set, face labels, vertex label triples)
    and moments within `rel` relative."""
    subset = None if sites_subset is None else set(int(i) for i in sites_subset)
    a = canon_pieces(gpu["res"])
    b = canon_pieces(ref_res)
    if subset is not None:
        a = {k: v for k, v in a.items() if k[0] in subset}
        b = {k: v for k, v in b.items() if k[0] in subset}
    missing = sorted(set(b) - set(a))[:5]
    extra = sorted(set(a) - set(b))[:5]
    assert not missing and not extra, f"piece sets differ: missing {missing} extra {extra}"
    nbad = 0
    md = 0.0
    for k in b:
        if a[k][0] != b[k][0] or a[k][1] != b[k][1]:
            nbad += 1
            if nbad < 4:
                log(f"combinatorics differ at {k}: gpu faces {a[k][0]} ref {b[k][0]}")
            continue
        if len(b[k][2]):
            md = max(md, float(np.abs(a[k][2] - b[k][2]).max()))
    assert nbad == 0, f"{nbad} pieces with different combinatorics"
    assert md <= xyz_tol, f"vertex coordinates differ by {md}"
    idx = np.arange(n) if subset is None else np.array(sorted(subset))
    m_g, m_r = gpu["mass"][idx], ref_mom["mass"][idx]
    nz = m_r > 0
    assert np.all(np.abs(m_g - m_r) <= rel * np.maximum(m_r, 1e-300)), \
        f"mass max rel err {np.max(np.abs(m_g - m_r)[nz] / m_r[nz])}"
    c_g, c_r = gpu["centroid"][idx], ref_mom["centroid"][idx]
    cerr = np.linalg.norm(c_g - c_r, axis=1) / np.maximum(np.linalg.norm(c_r, axis=1), 1e-300)
    assert np.all(cerr[nz] <= rel), f"centroid max rel err {cerr[nz].max()}"
    e_g, e_r = gpu["energy"][idx], ref_mom["energy"][idx]
    assert np.all(np.abs(e_g - e_r)[nz] <= rel * e_r[nz]), \
        f"energy max rel err {np.max(np.abs(e_g - e_r)[nz] / e_r[nz])}"
    assert_csr(gpu, len(gpu["mass"]))
    nb = gpu_neighbors(gpu, len(gpu["mass"]))
    for i in idx:
        assert list(nb[i]) == list(ref_mom["neighbors"][i]), f"neighbours of site {i} differ"
