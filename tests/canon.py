"""Canonical forms of piece sets, shared by the tests (compares results only).

A piece is keyed by (site, simplex).  Its canonical form is the sorted tuple of
face labels, the sorted tuple of vertex label-triples (each triple sorted) and
the vertex coordinates in that order.  Labels identify planes uniquely within
a piece, so two results describe the same polytope combinatorics iff their
canonical forms agree.
"""
import numpy as np


def canon_pieces(r):
    out = {}
    ps, pa = r["piece_site"], r["piece_simplex"]
    fo, fl = r["piece_face_off"], r["face_label"]
    vo, vl, vx = r["piece_vert_off"], r["vert_label"], r["vert_xyz"]
    for p in range(len(ps)):
        key = (int(ps[p]), int(pa[p]))
        faces = tuple(sorted(fl[fo[p]:fo[p + 1]].tolist()))
        labs = [tuple(sorted(x)) for x in vl[vo[p]:vo[p + 1]].tolist()]
        order = sorted(range(len(labs)), key=lambda k: labs[k])
        out[key] = (faces, tuple(labs[k] for k in order), vx[vo[p]:vo[p + 1]][order])
    return out


def compare_canon(a, b, xyz_tol):
    """Returns (n_key_mismatch, n_combinatorial_mismatch, max_vertex_diff)."""
    keys_a, keys_b = set(a), set(b)
    nkey = len(keys_a ^ keys_b)
    ncomb = 0
    md = 0.0
    for k in keys_a & keys_b:
        if a[k][0] != b[k][0] or a[k][1] != b[k][1]:
            ncomb += 1
            continue
        if len(a[k][2]):
            md = max(md, float(np.abs(a[k][2] - b[k][2]).max()))
    return nkey, ncomb, md


def subset_result(r, pieces):
    """The pieces with the given indices (ascending) of a result, in the same
    layout (face and vertex arrays gathered, offsets rebuilt)."""
    pieces = np.asarray(pieces, dtype=np.int64)
    fo, vo = r["piece_face_off"], r["piece_vert_off"]
    nf = fo[pieces + 1] - fo[pieces]
    nv = vo[pieces + 1] - vo[pieces]
    fidx = np.concatenate([np.arange(fo[p], fo[p + 1]) for p in pieces]) if len(pieces) else np.zeros(0, np.int64)
    vidx = np.concatenate([np.arange(vo[p], vo[p + 1]) for p in pieces]) if len(pieces) else np.zeros(0, np.int64)
    out = {k: r[k][pieces] for k in ("piece_site", "piece_simplex", "piece_mass", "piece_moment", "piece_energy")}
    out["piece_face_off"] = np.concatenate([[0], np.cumsum(nf)]).astype(np.int64)
    out["piece_vert_off"] = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
    out["face_label"] = r["face_label"][fidx]
    out["vert_xyz"] = r["vert_xyz"][vidx]
    out["vert_label"] = r["vert_label"][vidx]
    if "face_measure" in r:
        out["face_measure"] = r["face_measure"][fidx]
    return out
