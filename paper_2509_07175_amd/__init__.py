"""Clipped and restricted Voronoi diagrams on MI355X (gfx950).

Thin Python binding over ``libvd.so`` (C-ABI in ``include/vd.h``): argument
marshalling only.  Every step of the computation runs in the library's HIP
kernels; torch supplies device memory and the stream.  If the library is not
built, every entry point raises -- there is no CPU fallback.

    grid  = build_grid(sites)                       # vd_build_grid
    dom   = Domain(verts, simplices, adjacency, 3)  # vd_domain_create
    cells = clip_cells(grid, dom)                   # vd_clip_cells
    mass, centroid, energy = cells.moments()        # vd_cell_moments
    g_sites = cells.backward(g_mass, g_centroid, g_energy)  # vd_cell_moments_backward
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["load", "Options", "Grid", "Domain", "Cells", "build_grid", "clip_cells", "lloyd", "cvt_lbfgs",
           "VoronoiMoments", "VDError", "BOUNDARY_BASE", "sync"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvd.so")
BOUNDARY_BASE = -2**31

_lib = None
_hip = None


class VDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("sites_per_cell", C.c_double), ("improved_search", C.c_int32),
                ("use_straddle_edges", C.c_int32), ("max_search_iters", C.c_int32),
                ("emit_polytopes", C.c_int32), ("want_grad", C.c_int32), ("time_kernels", C.c_int32),
                ("carve_mode", C.c_int32), ("no_sync", C.c_int32), ("site_cache", C.c_int32),
                ("boundary_seeds", C.c_int32), ("monitor", C.c_int32), ("use_density", C.c_int32),
                ("density", C.c_double * 10), ("whole_interior", C.c_int32), ("batch_order", C.c_int32)]

    @classmethod
    def default(cls, **kw) -> "Options":
        o = cls()
        load().vd_options_default(C.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            if k == "density":
                v = list(v)
                if len(v) != 10:
                    raise ValueError("density takes 10 coefficients (quadratic in x, y, z)")
                o.density = (C.c_double * 10)(*[float(x) for x in v])
                o.use_density = 1
                continue
            setattr(o, k, v)
        return o


class _Info(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("n_pieces", C.c_int64), ("n_faces", C.c_int64),
                ("n_verts", C.c_int64), ("n_nbrs", C.c_int64), ("nn_queries", C.c_int64),
                ("clips", C.c_int64), ("candidates", C.c_int64), ("grid_queries", C.c_int64),
                ("first_bad_site", C.c_int32),
                ("failed_stages", C.c_int32), ("status", C.c_int32), ("carve_ms", C.c_double),
                ("split_ms", C.c_double), ("overflow_records", C.c_int64), ("low_margin", C.c_int64),
                ("min_margin", C.c_double), ("query_rounds", C.c_int64), ("corners_classified", C.c_int64),
                ("corners_created", C.c_int64), ("tests_wasted", C.c_int64), ("fan_simplices", C.c_int64),
                ("sites_outside", C.c_int64), ("boundary_seeded", C.c_int32), ("reserved_", C.c_int32)]


class _DomainInfo(C.Structure):
    _fields_ = [("n_simplices", C.c_int64), ("n_verts", C.c_int64), ("simplex_dim", C.c_int32),
                ("n_diagrams", C.c_int32), ("measure", C.c_double), ("convex", C.c_int32)]


class _Batch(C.Structure):
    _fields_ = [("num", C.c_int32), ("site_off", C.POINTER(C.c_int64)), ("vert_off", C.POINTER(C.c_int64)),
                ("simp_off", C.POINTER(C.c_int64))]


def _batch(site_off=None, vert_off=None, simp_off=None):
    """vd_batch from host offset arrays (kept alive on the returned struct)."""
    def arr(x):
        if x is None:
            return None, None
        a = (C.c_int64 * len(x))(*[int(v) for v in x])
        return a, C.cast(a, C.POINTER(C.c_int64))
    keep = []
    num = None
    b = _Batch()
    for name, x in (("site_off", site_off), ("vert_off", vert_off), ("simp_off", simp_off)):
        a, ptr = arr(x)
        if a is not None:
            keep.append(a)
            setattr(b, name, ptr)
            num = len(x) - 1
    b.num = num if num is not None else 0
    b._keep = keep
    return b


class _View(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("n_piece_slots", C.c_int64), ("n_face_slots", C.c_int64),
                ("n_vert_slots", C.c_int64)] + [
        (name, C.c_void_p) for name in (
            "cell_piece_off", "piece_id", "piece_site", "piece_simplex", "piece_nface", "piece_nvert",
            "piece_face_start", "piece_vert_start", "piece_mass", "piece_moment", "piece_energy",
            "face_label", "vert_xyz", "vert_label", "nbr_off", "nbr")]


def load():
    """Loads libvd.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2509_07175_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    sig = {
        "vd_options_default": (None, [C.POINTER(Options)]),
        "vd_last_error": (C.c_char_p, []),
        "vd_status_string": (C.c_char_p, [C.c_int]),
        "vd_build_grid": (C.c_int, [vp, i64, vp, d, d, vp, C.POINTER(vp)]),
        "vd_build_grid_batch": (C.c_int, [vp, C.POINTER(_Batch), vp, d, vp, C.POINTER(vp)]),
        "vd_domain_create_batch": (C.c_int, [vp, vp, vp, C.POINTER(_Batch), i32, vp, C.POINTER(vp)]),
        "vd_grid_free": (None, [vp]),
        "vd_domain_create": (C.c_int, [vp, i64, vp, vp, i64, i32, vp, C.POINTER(vp)]),
        "vd_domain_free": (None, [vp]),
        "vd_clip_cells": (C.c_int, [vp, vp, C.POINTER(Options), vp, C.POINTER(vp)]),
        "vd_cells_free": (None, [vp]),
        "vd_cells_info": (C.c_int, [vp, C.POINTER(_Info)]),
        "vd_cells_view": (C.c_int, [vp, C.POINTER(_View)]),
        "vd_cell_moments": (C.c_int, [vp, vp, vp, vp, vp]),
        "vd_cell_moments_backward": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "vd_sync": (C.c_int, [vp]),
        "vd_grid_set_weights": (C.c_int, [vp, vp, vp]),
        "vd_cell_moments_backward_noalloc": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "vd_domain_info": (C.c_int, [vp, C.POINTER(_DomainInfo)]),
        "vd_domain_adjacency": (C.c_int, [vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["vd_options_default", "vd_last_error", "vd_status_string", "vd_build_grid", "vd_grid_free",
            "vd_build_grid_batch", "vd_domain_create_batch", "vd_domain_create", "vd_domain_free", "vd_clip_cells", "vd_cells_free", "vd_cells_info",
            "vd_cells_view", "vd_cell_moments", "vd_cell_moments_backward", "vd_sync", "vd_domain_info",
            "vd_domain_adjacency", "vd_cell_moments_backward_noalloc", "vd_grid_set_weights"]


def sync(stream=None):
    """vd_sync: waits for the stream's work and reports an asynchronous device error."""
    _check(load().vd_sync(_stream_ptr(stream)))


def _check(status: int):
    if status != 0:
        lib = load()
        raise VDError(status, f"{lib.vd_status_string(status).decode()}: {lib.vd_last_error().decode()}")


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t, dtype, shape_last=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"expected shape (n, {shape_last})")
    return C.c_void_p(t.data_ptr())


def _hiplib():
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the HIP runtime torch uses)
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise ImportError("libamdhip64 not found")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _hip


def _to_torch(ptr, n, dtype):
    """Copies n elements from a library-owned device array into a new tensor."""
    import torch
    out = torch.empty(int(n), dtype=dtype, device="cuda")
    if n > 0 and ptr:
        nbytes = int(n) * out.element_size()
        torch.cuda.current_stream().synchronize()
        st = _hiplib().hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), nbytes, 3)
        if st != 0:
            raise RuntimeError(f"hipMemcpy failed ({st})")
    return out


class Grid:
    """vd_build_grid handle (uniform nearest-site grid, Sec. 6.2)."""

    def __init__(self):
        self.h = C.c_void_p()
        self.sites = None

    def build(self, sites, bbox=None, sites_per_cell=0.0, surface_area=0.0, stream=None):
        import torch
        sp = _dptr(sites, torch.float64, 3)
        bb = None
        if bbox is not None:
            bb = (C.c_double * 6)(*[float(x) for x in bbox])
        _check(load().vd_build_grid(sp, sites.shape[0], bb, float(sites_per_cell), float(surface_area),
                                    _stream_ptr(stream), C.byref(self.h)))
        self.sites = sites
        return self

    def set_weights(self, weights, stream=None):
        """vd_grid_set_weights: power-diagram weights of the sites (n float64 on
        the device, caller order), or None for the Voronoi diagram."""
        import torch
        w = None
        if weights is not None:
            if weights.shape != (self.sites.shape[0],):
                raise ValueError("one weight per site")
            w = _dptr(weights, torch.float64)
        _check(load().vd_grid_set_weights(self.h, w, _stream_ptr(stream)))
        self.weights = weights
        return self

    def __del__(self):
        if _lib is not None and self.h:
            _lib.vd_grid_free(self.h)
            self.h = C.c_void_p()


def build_grid(sites, bbox=None, sites_per_cell=0.0, surface_area=0.0, grid: Grid | None = None,
               stream=None, weights=None) -> Grid:
    """vd_build_grid (and vd_grid_set_weights when ``weights`` is given: a
    power diagram)."""
    g = grid if grid is not None else Grid()
    g.build(sites, bbox, sites_per_cell, surface_area, stream)
    if weights is not None:
        g.set_weights(weights, stream)
    return g


def build_grid_batch(sites, site_off, bboxes=None, sites_per_cell=0.0, grid: Grid | None = None,
                     stream=None) -> Grid:
    """vd_build_grid_batch: one grid per diagram over the concatenated sites
    (diagram b owns sites[site_off[b]:site_off[b+1]])."""
    import torch
    g = grid if grid is not None else Grid()
    b = _batch(site_off=site_off)
    bb = None
    if bboxes is not None:
        flat = [float(x) for box in bboxes for x in box]
        bb = (C.c_double * len(flat))(*flat)
    _check(load().vd_build_grid_batch(_dptr(sites, torch.float64, 3), C.byref(b), bb, float(sites_per_cell),
                                      _stream_ptr(stream), C.byref(g.h)))
    g.sites = sites
    g.site_off = list(site_off)
    return g


class Domain:
    """vd_domain_create handle: a simplex domain staged on the device."""

    def __init__(self, verts, simplices, adjacency, dim: int, stream=None):
        """adjacency None: computed by the library (face matching on the device)."""
        import torch
        self.h = C.c_void_p()
        self.dim = int(dim)
        self.verts = verts
        self.simplices = simplices
        self.m = simplices.shape[0]
        k = self.dim + 1
        if simplices.dim() != 2 or simplices.shape[1] != k or (adjacency is not None and adjacency.shape != simplices.shape):
            raise ValueError("simplices/adjacency must be (m, dim+1)")
        _check(load().vd_domain_create(_dptr(verts, torch.float64, 3), verts.shape[0],
                                       _dptr(simplices, torch.int32),
                                       None if adjacency is None else _dptr(adjacency, torch.int32),
                                       simplices.shape[0], self.dim, _stream_ptr(stream), C.byref(self.h)))

    def info(self) -> dict:
        i = _DomainInfo()
        _check(load().vd_domain_info(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in _DomainInfo._fields_}

    def adjacency(self, stream=None):
        """The adjacency the kernels use, (m, dim+1) int32 on the device."""
        import torch
        out = torch.empty((self.m, self.dim + 1), dtype=torch.int32, device="cuda")
        _check(load().vd_domain_adjacency(self.h, _dptr(out, torch.int32), _stream_ptr(stream)))
        return out

    @classmethod
    def batch(cls, verts, simplices, adjacency, vert_off, simp_off, dim: int, stream=None):
        """vd_domain_create_batch: concatenated domains with diagram-local indices."""
        import torch
        self = cls.__new__(cls)
        self.h = C.c_void_p()
        self.dim = int(dim)
        self.verts = verts
        self.simplices = simplices
        self.m = simplices.shape[0]
        self.vert_off = list(vert_off)
        self.simp_off = list(simp_off)
        b = _batch(vert_off=vert_off, simp_off=simp_off)
        _check(load().vd_domain_create_batch(_dptr(verts, torch.float64, 3), _dptr(simplices, torch.int32),
                                             None if adjacency is None else _dptr(adjacency, torch.int32),
                                             C.byref(b), self.dim, _stream_ptr(stream), C.byref(self.h)))
        return self

    @classmethod
    def batch_from_vdgen(cls, doms):
        """Concatenates vdgen domains (diagram-local indices kept) into one batch."""
        import numpy as np
        import torch
        vo, so = [0], [0]
        for d in doms:
            vo.append(vo[-1] + len(d.verts))
            so.append(so[-1] + len(d.simplices))
        verts = np.concatenate([d.verts for d in doms])
        simp = np.concatenate([d.simplices for d in doms]).astype(np.int32)
        adj = np.concatenate([d.adj for d in doms]).astype(np.int32)
        t = lambda x, dt: torch.as_tensor(x, dtype=dt, device="cuda").contiguous()
        return cls.batch(t(verts, torch.float64), t(simp, torch.int32), t(adj, torch.int32), vo, so, doms[0].dim)

    @classmethod
    def from_vdgen(cls, dom, adjacency: bool = True):
        """adjacency=False leaves the adjacency to the library."""
        import torch
        return cls(torch.as_tensor(dom.verts, dtype=torch.float64, device="cuda").contiguous(),
                   torch.as_tensor(dom.simplices, dtype=torch.int32, device="cuda").contiguous(),
                   torch.as_tensor(dom.adj, dtype=torch.int32, device="cuda").contiguous() if adjacency else None,
                   dom.dim)

    def __del__(self):
        if _lib is not None and self.h:
            _lib.vd_domain_free(self.h)
            self.h = C.c_void_p()


class Cells:
    """vd_clip_cells handle: pieces, neighbour lists, moments."""

    def __init__(self):
        self.h = C.c_void_p()
        self.grid = None
        self.n = 0

    def clip(self, grid: Grid, domain: Domain, options: Options | None = None, stream=None):
        opt = options if options is not None else Options.default()
        self.grid = grid
        self.domain = domain
        st = load().vd_clip_cells(grid.h, domain.h, C.byref(opt), _stream_ptr(stream), C.byref(self.h))
        _check(st)
        self.n = grid.sites.shape[0]
        return self

    def info(self) -> dict:
        i = _Info()
        _check(load().vd_cells_info(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    def moments(self, mass=None, centroid=None, energy=None, stream=None):
        import torch
        n = self.n
        mass = mass if mass is not None else torch.empty(n, dtype=torch.float64, device="cuda")
        centroid = centroid if centroid is not None else torch.empty((n, 3), dtype=torch.float64, device="cuda")
        energy = energy if energy is not None else torch.empty(n, dtype=torch.float64, device="cuda")
        _check(load().vd_cell_moments(self.h, _dptr(mass, torch.float64), _dptr(centroid, torch.float64, 3),
                                      _dptr(energy, torch.float64), _stream_ptr(stream)))
        return mass, centroid, energy

    def backward(self, g_mass=None, g_centroid=None, g_energy=None, out=None, stream=None):
        import torch
        n = self.n
        out = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device="cuda")

        def p(t, last=None):
            return None if t is None else _dptr(t, torch.float64, last)

        _check(load().vd_cell_moments_backward(self.h, p(g_mass), p(g_centroid, 3), p(g_energy),
                                               _dptr(out, torch.float64, 3), _stream_ptr(stream)))
        return out

    def backward_noalloc(self, g_mass=None, g_centroid=None, g_energy=None, out=None, stream=None):
        """vd_cell_moments_backward_noalloc: the adjoint without any allocation in
        the library (its weight table sits in a fixed device array)."""
        import torch
        n = self.n
        out = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device="cuda")

        def p(t, last=None):
            return None if t is None else _dptr(t, torch.float64, last)

        _check(load().vd_cell_moments_backward_noalloc(self.h, p(g_mass), p(g_centroid, 3), p(g_energy),
                                                       _dptr(out, torch.float64, 3), _stream_ptr(stream)))
        return out

    def view(self) -> dict:
        """Copies the library's output arrays into new torch tensors (for tests)."""
        import torch
        v = _View()
        _check(load().vd_cells_view(self.h, C.byref(v)))
        info = self.info()
        n, npc = v.n_sites, v.n_piece_slots
        out = {
            "cell_piece_off": _to_torch(v.cell_piece_off, n + 1, torch.int64),
            "nbr_off": _to_torch(v.nbr_off, n + 1, torch.int64),
            "piece_site": _to_torch(v.piece_site, npc, torch.int32),
            "piece_simplex": _to_torch(v.piece_simplex, npc, torch.int32),
            "piece_nface": _to_torch(v.piece_nface, npc, torch.int32),
            "piece_nvert": _to_torch(v.piece_nvert, npc, torch.int32),
            "piece_face_start": _to_torch(v.piece_face_start, npc, torch.int64),
            "piece_vert_start": _to_torch(v.piece_vert_start, npc, torch.int64),
            "piece_mass": _to_torch(v.piece_mass, npc, torch.float64),
            "piece_moment": _to_torch(v.piece_moment, 3 * npc, torch.float64).reshape(-1, 3),
            "piece_energy": _to_torch(v.piece_energy, npc, torch.float64),
        }
        tot_p = int(out["cell_piece_off"][-1].item()) if n > 0 else 0
        tot_n = int(out["nbr_off"][-1].item()) if n > 0 else 0
        out["piece_id"] = _to_torch(v.piece_id, tot_p, torch.int32)
        out["nbr"] = _to_torch(v.nbr, tot_n, torch.int32)
        if v.n_face_slots > 0 and v.face_label:
            out["face_label"] = _to_torch(v.face_label, v.n_face_slots, torch.int32)
            out["vert_xyz"] = _to_torch(v.vert_xyz, 3 * v.n_vert_slots, torch.float64).reshape(-1, 3)
            out["vert_label"] = _to_torch(v.vert_label, 3 * v.n_vert_slots, torch.int32).reshape(-1, 3)
        return out

    def __del__(self):
        if _lib is not None and self.h:
            _lib.vd_cells_free(self.h)
            self.h = C.c_void_p()


def clip_cells(grid: Grid, domain: Domain, options: Options | None = None, cells: Cells | None = None,
               stream=None) -> Cells:
    c = cells if cells is not None else Cells()
    return c.clip(grid, domain, options, stream)


def lloyd(sites, domain: Domain, iterations: int, options: Options | None = None, bbox=None,
          sites_per_cell: float = 0.0, surface_area: float = 0.0, energy: bool = False, stream=None):
    """Lloyd iterations towards a centroidal Voronoi tessellation with density 1
    (Sec. 7.4): every iteration builds the grid, clips the cells and moves each
    site to its cell's centroid.  The centroids are written by the moments
    kernel straight over `sites` (n x 3 float64 on the device), which is updated
    in place and returned; with energy=True, the CVT energy (Eq. 3) of every
    iteration's diagram is returned as well.

    A site must stay inside the domain, which holds for convex domains (a cell's
    centroid lies in the cell).  For a surface, centroids are not projected back
    onto it.  On a tetrahedral domain, options with whole_interior=1 give the
    same moments without cutting the interior cells by the tetrahedra."""
    import torch
    if sites.dtype != torch.float64 or not sites.is_cuda or sites.dim() != 2 or sites.shape[1] != 3:
        raise ValueError("sites must be an (n, 3) float64 CUDA tensor")
    if not sites.is_contiguous():
        raise ValueError("sites must be contiguous (it is updated in place)")
    n = sites.shape[0]
    grid, cells = Grid(), Cells()
    mass = torch.empty(n, dtype=torch.float64, device=sites.device)
    en = torch.empty(n, dtype=torch.float64, device=sites.device)
    energies = []
    for _ in range(int(iterations)):
        build_grid(sites, bbox=bbox, sites_per_cell=sites_per_cell, surface_area=surface_area, grid=grid,
                   stream=stream)
        clip_cells(grid, domain, options, cells=cells, stream=stream)
        cells.moments(mass, sites, en, stream=stream)  # the grid holds its own sorted copy of the sites
        if energy:
            energies.append(float(en.sum().item()))
    return (sites, energies) if energy else sites


def cvt_lbfgs(sites, domain: Domain, iterations: int, options: Options | None = None, bbox=None,
              sites_per_cell: float = 0.0, surface_area: float = 0.0, history: int = 10, stream=None):
    """Minimises the CVT energy of Eq. 3 (with the density of ``options``, if
    any) over the sites by L-BFGS with a strong-Wolfe line search.  Every
    evaluation is a grid build, a clip and the moments through the library,
    and the gradient is the library's adjoint of the energy (2 m_i (v_i - c_i)
    for each site); torch.optim.LBFGS only keeps the optimiser's state.
    The energy's Hessian is close to 2 m_i per site (the Lloyd step is the
    Newton step), so the optimiser runs on z = sqrt(2 M / n) v, M the total
    (weighted) mass of the first diagram: there the Hessian is close to the
    identity and the first steps are well scaled.
    Returns the final sites (a new tensor) and the energy before each
    iteration and at the end (non-increasing: the line search enforces
    sufficient decrease)."""
    import torch
    if sites.dtype != torch.float64 or not sites.is_cuda or sites.dim() != 2 or sites.shape[1] != 3:
        raise ValueError("sites must be an (n, 3) float64 CUDA tensor")
    n = sites.shape[0]
    opt = Options.default() if options is None else Options.from_buffer_copy(options)
    opt.want_grad = 1
    grid, cells = Grid(), Cells()
    mass = torch.empty(n, dtype=torch.float64, device=sites.device)
    cent = torch.empty((n, 3), dtype=torch.float64, device=sites.device)
    en = torch.empty(n, dtype=torch.float64, device=sites.device)
    ones = torch.ones(n, dtype=torch.float64, device=sites.device)
    gout = torch.empty((n, 3), dtype=torch.float64, device=sites.device)
    v = sites.detach().clone().contiguous()

    def evaluate():
        build_grid(v, bbox=bbox, sites_per_cell=sites_per_cell, surface_area=surface_area, grid=grid, stream=stream)
        clip_cells(grid, domain, opt, cells=cells, stream=stream)
        cells.moments(mass, cent, en, stream=stream)
        cells.backward(None, None, ones, out=gout, stream=stream)
        return en.sum()

    evaluate()
    sigma = float((2.0 * mass.sum() / n).sqrt().item())
    z = (v * sigma).requires_grad_(False)
    lbfgs = torch.optim.LBFGS([z], lr=1.0, max_iter=1, history_size=int(history), line_search_fn="strong_wolfe",
                              tolerance_grad=0.0, tolerance_change=0.0)
    energies = []

    def closure():
        v.copy_(z.detach() / sigma)
        e = evaluate()
        z.grad = gout / sigma
        return e

    for _ in range(int(iterations)):
        energies.append(float(lbfgs.step(closure).item()))
    v.copy_(z.detach() / sigma)
    energies.append(float(evaluate().item()))
    return v, energies


def pieces_as_result(view: dict) -> dict:
    """Host (NumPy) copy of the pieces in the oracle's layout, sorted by (site, simplex)
    (unused arena slots dropped)."""
    site = view["piece_site"].cpu().numpy()
    simp = view["piece_simplex"].cpu().numpy()
    used = np.nonzero(site >= 0)[0]
    npc = len(used)
    order = used[np.lexsort((simp[used], site[used]))]
    nface = view["piece_nface"].cpu().numpy()[order]
    nvert = view["piece_nvert"].cpu().numpy()[order]
    fst = view["piece_face_start"].cpu().numpy()[order]
    vst = view["piece_vert_start"].cpu().numpy()[order]
    res = {
        "piece_site": site[order], "piece_simplex": simp[order],
        "piece_mass": view["piece_mass"].cpu().numpy()[order],
        "piece_moment": view["piece_moment"].cpu().numpy()[order],
        "piece_energy": view["piece_energy"].cpu().numpy()[order],
        "piece_face_off": np.concatenate([[0], np.cumsum(nface)]).astype(np.int64),
        "piece_vert_off": np.concatenate([[0], np.cumsum(nvert)]).astype(np.int64),
    }
    if "face_label" in view:
        fl = view["face_label"].cpu().numpy()
        vx = view["vert_xyz"].cpu().numpy()
        vl = view["vert_label"].cpu().numpy()
        fidx = np.concatenate([np.arange(s, s + c) for s, c in zip(fst, nface)]) if npc else np.zeros(0, np.int64)
        vidx = np.concatenate([np.arange(s, s + c) for s, c in zip(vst, nvert)]) if npc else np.zeros(0, np.int64)
        res["face_label"] = fl[fidx]
        res["vert_xyz"] = vx[vidx]
        res["vert_label"] = vl[vidx]
    return res


class VoronoiMoments:
    """torch.autograd.Function: sites -> (mass, centroid, energy) of the clipped /
    restricted cells, with the hand-written adjoint as backward."""

    _fn = None

    @classmethod
    def apply(cls, sites, domain: Domain, options: Options | None = None, bbox=None, surface_area=0.0):
        import torch
        if cls._fn is None:
            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, s, dom, opt, bb, area):
                    o = opt if opt is not None else Options.default()
                    o.want_grad = 1
                    g = build_grid(s.detach().contiguous(), bbox=bb, surface_area=area)
                    c = clip_cells(g, dom, o)
                    m, ce, e = c.moments()
                    ctx.cells = c
                    ctx.grid = g
                    return m, ce, e

                @staticmethod
                def backward(ctx, gm, gc, ge):
                    def cont(t):
                        return None if t is None else t.contiguous()
                    gs = ctx.cells.backward(cont(gm), cont(gc), cont(ge))
                    return gs, None, None, None, None

            cls._fn = _F
        return cls._fn.apply(sites, domain, options, bbox, surface_area)
