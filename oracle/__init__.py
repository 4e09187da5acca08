"""CPU oracle for clipped / restricted Voronoi diagrams (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.
It shares no code with the GPU path.  See ``vd_oracle.h`` for what the C code
computes (the plain definition of Sec. 3.1, Eq. 1, with the flags of
Sec. 3.2).

Python side: ``build()`` compiles ``vd_oracle.c`` with gcc/OpenMP,
``compute()`` runs it and returns NumPy arrays, ``site_moments()`` folds pieces
into per-site mass / centroid / energy / neighbour lists, and
``moments_backward()`` evaluates the adjoint.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vd_oracle.c")
_LIB = os.path.join(_HERE, "libvdoracle.so")
_LIB_NATIVE = os.path.join(_HERE, "libvdoracle_native.so")
_lib = None
_lib_native = None

BOUNDARY_BASE = -2**31  # domain-boundary face f carries BOUNDARY_BASE + f


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc and OpenMP.

    native=False: oracle/libvdoracle.so, -O3 for the generic x86-64 target, so
    the same binary runs (and rounds the same way) on any host; the tests use it.
    native=True: oracle/libvdoracle_native.so, -O3 -march=native, built on the
    host that runs it; only the CPU-baseline timing uses it."""
    lib = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        flags = ["-O3", "-march=native"] if native else ["-O3"]
        subprocess.run(["gcc", *flags, "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, lib)
    return lib


class _Result(C.Structure):
    _fields_ = [
        ("n_pieces", C.c_int64),
        ("piece_site", C.POINTER(C.c_int32)),
        ("piece_simplex", C.POINTER(C.c_int32)),
        ("piece_mass", C.POINTER(C.c_double)),
        ("piece_moment", C.POINTER(C.c_double)),
        ("piece_energy", C.POINTER(C.c_double)),
        ("piece_face_off", C.POINTER(C.c_int64)),
        ("face_label", C.POINTER(C.c_int32)),
        ("face_measure", C.POINTER(C.c_double)),
        ("face_vert_off", C.POINTER(C.c_int64)),
        ("face_vert", C.POINTER(C.c_int32)),
        ("n_faces", C.c_int64),
        ("n_face_verts", C.c_int64),
        ("piece_vert_off", C.POINTER(C.c_int64)),
        ("vert_xyz", C.POINTER(C.c_double)),
        ("vert_label", C.POINTER(C.c_int32)),
        ("n_verts", C.c_int64),
        ("min_margin", C.c_double),
    ]


def _load(native: bool = False):
    global _lib, _lib_native
    if (_lib_native if native else _lib) is None:
        path = _LIB_NATIVE if native else _LIB
        if not os.path.exists(path):
            build(native=native)
        lib = C.CDLL(path)
        lib.vdo_compute.restype = C.c_int
        lib.vdo_compute.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_void_p,
                                    C.c_int64, C.c_int, C.POINTER(_Result)]
        lib.vdo_compute_power.restype = C.c_int
        lib.vdo_compute_power.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                          C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_void_p,
                                          C.c_int64, C.c_int, C.POINTER(_Result)]
        lib.vdo_free_result.restype = None
        lib.vdo_free_result.argtypes = [C.POINTER(_Result)]
        lib.vdo_moments_backward.restype = C.c_int
        lib.vdo_moments_backward.argtypes = [C.POINTER(_Result)] + [C.c_void_p, C.c_int64] + \
            [C.c_void_p] * 7 + [C.c_int, C.c_void_p]
        lib.vdo_moments_backward_rho.restype = C.c_int
        lib.vdo_moments_backward_rho.argtypes = [C.POINTER(_Result)] + [C.c_void_p, C.c_int64] + \
            [C.c_void_p] * 7 + [C.c_int, C.c_void_p, C.c_void_p]
        lib.vdo_density_moments.restype = C.c_int
        lib.vdo_density_moments.argtypes = [C.POINTER(_Result), C.c_void_p, C.c_void_p, C.c_int,
                                            C.c_void_p, C.c_void_p, C.c_void_p]
        if native:
            _lib_native = lib
        else:
            _lib = lib
    return _lib_native if native else _lib


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def _to_result(r: _Result) -> dict:
    npc, nf, nv, nfv = r.n_pieces, r.n_faces, r.n_verts, r.n_face_verts
    return {
        "piece_site": _arr(r.piece_site, npc, np.int32),
        "piece_simplex": _arr(r.piece_simplex, npc, np.int32),
        "piece_mass": _arr(r.piece_mass, npc, np.float64),
        "piece_moment": _arr(r.piece_moment, 3 * npc, np.float64).reshape(npc, 3),
        "piece_energy": _arr(r.piece_energy, npc, np.float64),
        "piece_face_off": _arr(r.piece_face_off, npc + 1, np.int64),
        "face_label": _arr(r.face_label, nf, np.int32),
        "face_measure": _arr(r.face_measure, nf, np.float64),
        "face_vert_off": _arr(r.face_vert_off, nf + 1, np.int64),
        "face_vert": _arr(r.face_vert, nfv, np.int32),
        "piece_vert_off": _arr(r.piece_vert_off, npc + 1, np.int64),
        "vert_xyz": _arr(r.vert_xyz, 3 * nv, np.float64).reshape(nv, 3),
        "vert_label": _arr(r.vert_label, 3 * nv, np.int32).reshape(nv, 3),
        "min_margin": float(r.min_margin),
    }


class _Keep:
    """Keeps a ctypes result alive so moments_backward can reuse it."""


def compute(sites, domain, brute: bool = False, only_sites=None, threads: int = 0,
            keep_handle: bool = False, native: bool = False, weights=None):
    """All pieces P_{a,i} (Eq. 1) of the sites in ``domain`` (a vdgen.Domain).

    Returns a dict of NumPy arrays, pieces sorted by (site, simplex).
    native=True runs the -march=native build (timing only).  ``weights`` (n)
    gives the power diagram of Sec. 7.3 instead.
    """
    lib = _load(native)
    s = np.ascontiguousarray(sites, dtype=np.float64)
    v = np.ascontiguousarray(domain.verts, dtype=np.float64)
    t = np.ascontiguousarray(domain.simplices, dtype=np.int32)
    a = np.ascontiguousarray(domain.adj, dtype=np.int32)
    only = None
    n_only = 0
    if only_sites is not None:
        only = np.ascontiguousarray(only_sites, dtype=np.int32)
        n_only = only.size
    res = _Result()
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w is not None and w.shape != (s.shape[0],):
        raise ValueError("one weight per site")
    st = lib.vdo_compute_power(s.ctypes.data, None if w is None else w.ctypes.data, s.shape[0], v.ctypes.data,
                               v.shape[0], t.ctypes.data, a.ctypes.data, t.shape[0], int(domain.dim), int(brute),
                               only.ctypes.data if only is not None else None, n_only, int(threads),
                               C.byref(res))
    if st != 0:
        raise RuntimeError(f"oracle failed with status {st}")
    out = _to_result(res)
    if keep_handle:
        out["_handle"] = res
    else:
        lib.vdo_free_result(C.byref(res))
    return out


def free(result: dict) -> None:
    h = result.pop("_handle", None)
    if h is not None:
        _load().vdo_free_result(C.byref(h))


def site_moments(result: dict, sites) -> dict:
    """Per-site mass, centroid, energy and sorted neighbour lists.

    Pieces are summed in simplex order with Neumaier compensation.  A site
    with no piece gets mass 0, centroid = its own position, energy 0.
    """
    sites = np.asarray(sites, dtype=np.float64)
    n = sites.shape[0]
    mass = np.zeros(n)
    mom = np.zeros((n, 3))
    en = np.zeros(n)
    ps = result["piece_site"]
    # pieces are sorted by (site, simplex): sum each segment in order
    bounds = np.searchsorted(ps, np.arange(n + 1))
    pm, pmo, pe = result["piece_mass"], result["piece_moment"], result["piece_energy"]
    for i in np.nonzero(bounds[1:] > bounds[:-1])[0]:
        lo, hi = bounds[i], bounds[i + 1]
        mass[i] = _nsum(pm[lo:hi])
        en[i] = _nsum(pe[lo:hi])
        for d in range(3):
            mom[i, d] = _nsum(pmo[lo:hi, d])
    cent = sites.copy()
    nz = mass > 0
    cent[nz] = mom[nz] / mass[nz, None]
    nbrs = []
    fo, fl = result["piece_face_off"], result["face_label"]
    for i in range(n):
        lo, hi = bounds[i], bounds[i + 1]
        if hi > lo:
            labs = fl[fo[lo]:fo[hi]]
            nbrs.append(np.unique(labs[labs >= 0]).astype(np.int32))
        else:
            nbrs.append(np.zeros(0, dtype=np.int32))
    return {"mass": mass, "moment": mom, "centroid": cent, "energy": en, "neighbors": nbrs,
            "piece_bounds": bounds}


def _nsum(x) -> float:
    s = 0.0
    c = 0.0
    for v in x:
        v = float(v)
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


def density_result(result: dict, sites, coef, dim: int) -> dict:
    """A copy of ``result`` (computed with ``keep_handle=True``) whose per-piece
    mass, first moment and energy are weighted by the quadratic density
    rho(x) = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 xy + c6 xz + c7 y^2 + c8 yz
    + c9 z^2 (Eq. 3), integrated exactly on each piece's fan of simplices."""
    lib = _load()
    h = result.get("_handle")
    if h is None:
        raise ValueError("compute(..., keep_handle=True) is required")
    s = np.ascontiguousarray(sites, dtype=np.float64)
    c = np.ascontiguousarray(coef, dtype=np.float64)
    if c.shape != (10,):
        raise ValueError("10 density coefficients")
    npc = len(result["piece_site"])
    m, mo, e = np.zeros(npc), np.zeros((npc, 3)), np.zeros(npc)
    st = lib.vdo_density_moments(C.byref(h), s.ctypes.data, c.ctypes.data, int(dim), m.ctypes.data,
                                 mo.ctypes.data, e.ctypes.data)
    if st != 0:
        raise RuntimeError(f"oracle density moments failed with status {st}")
    out = {k: v for k, v in result.items() if k != "_handle"}
    out["piece_mass"], out["piece_moment"], out["piece_energy"] = m, mo, e
    return out


def moments_backward(result: dict, sites, domain, mass, centroid, g_mass=None, g_centroid=None,
                     g_energy=None, rho=None):
    """Adjoint of sum_k g_m m_k + g_c.c_k + g_E E_k w.r.t. the sites (result must
    cover all sites and be computed with ``keep_handle=True``); with ``rho`` (10
    coefficients) the moments are the density-weighted ones."""
    lib = _load()
    h = result.get("_handle")
    if h is None:
        raise ValueError("compute(..., keep_handle=True) is required for the adjoint")
    s = np.ascontiguousarray(sites, dtype=np.float64)
    n = s.shape[0]
    m_ = np.ascontiguousarray(mass, dtype=np.float64)
    c_ = np.ascontiguousarray(centroid, dtype=np.float64)

    def opt(x, shape):
        if x is None:
            return None, None
        arr = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), shape))
        return arr, arr.ctypes.data

    gm, gm_p = opt(g_mass, (n,))
    gc, gc_p = opt(g_centroid, (n, 3))
    ge, ge_p = opt(g_energy, (n,))
    v = np.ascontiguousarray(domain.verts, dtype=np.float64)
    t = np.ascontiguousarray(domain.simplices, dtype=np.int32)
    out = np.zeros((n, 3))
    rc = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    st = lib.vdo_moments_backward_rho(C.byref(h), s.ctypes.data, n, m_.ctypes.data, c_.ctypes.data,
                                      gm_p, gc_p, ge_p, v.ctypes.data, t.ctypes.data, int(domain.dim),
                                      None if rc is None else rc.ctypes.data, out.ctypes.data)
    if st != 0:
        raise RuntimeError(f"oracle adjoint failed with status {st}")
    return out
