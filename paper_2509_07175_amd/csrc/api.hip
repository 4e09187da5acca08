// api.hip -- the C-ABI of libvd (declared in include/vd.h).
//
// Host code only: argument checks, buffer management (grow-only, reused
// between calls), kernel launches on the caller's stream and the one
// synchronisation per vd_clip_cells that reads the output sizes.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vd_internal.h"

void vd_launch_domain_fill(vd_domain d, hipStream_t st);
void vd_launch_domain_validate(vd_domain d, int *flags, double *measure, hipStream_t st);
void vd_launch_vert_bbox(vd_domain d, double *out, hipStream_t st);
void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st);

namespace {

thread_local std::string g_err;

vd_status fail(vd_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? VD_ERR_OUT_OF_MEMORY : VD_ERR_HIP,          \
                  "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

template <typename T>
hipError_t ensure(T *&p, int64_t &cap, int64_t need) {
  if (need <= cap && p) return hipSuccess;
  if (p) {
    hipError_t e = hipFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
  }
  const int64_t n = std::max<int64_t>(need, 1);
  hipError_t e = hipMalloc((void **)&p, sizeof(T) * (size_t)n);
  if (e == hipSuccess) cap = n;
  else cap = 0;
  return e;
}

// fixed-size buffers (capacity tracked elsewhere)
template <typename T>
hipError_t ensure_fixed(T *&p, int64_t n) {
  if (p) return hipSuccess;
  return hipMalloc((void **)&p, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

__global__ void reset_counters(unsigned long long *cnt) {
  const int i = threadIdx.x;
  if (i < CNT_N) cnt[i] = (i == CNT_BAD_SITE) ? 0x7fffffffull : 0ull;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

const char *vd_last_error(void) { return g_err.c_str(); }

const char *vd_status_string(vd_status s) {
  switch (s) {
    case VD_OK: return "VD_OK";
    case VD_ERR_INVALID_ARG: return "VD_ERR_INVALID_ARG";
    case VD_ERR_OUT_OF_MEMORY: return "VD_ERR_OUT_OF_MEMORY";
    case VD_ERR_HIP: return "VD_ERR_HIP";
    case VD_ERR_CAPACITY: return "VD_ERR_CAPACITY";
    case VD_ERR_DEGENERATE: return "VD_ERR_DEGENERATE";
  }
  return "VD_ERR_UNKNOWN";
}

void vd_options_default(vd_options *opt) {
  if (!opt) return;
  opt->sites_per_cell = 3.5;
  opt->improved_search = 1;
  opt->use_straddle_edges = 1;
  opt->max_search_iters = 64;
  opt->emit_polytopes = 1;
  opt->want_grad = 0;
  opt->time_kernels = 0;
  opt->carve_mode = 1;
  opt->site_cache = 1;
}

// ---------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------
vd_status vd_build_grid(const double *sites, int64_t n, const double *bbox_host, double sites_per_cell,
                        double surface_area, void *stream, vd_grid *out) {
  if (!out) return fail(VD_ERR_INVALID_ARG, "vd_build_grid: out is NULL");
  if (!sites || n < 1) return fail(VD_ERR_INVALID_ARG, "vd_build_grid: sites NULL or n < 1");
  if (n > (int64_t)INT_MAX / 4) return fail(VD_ERR_INVALID_ARG, "vd_build_grid: n too large");
  if (bbox_host)
    for (int k = 0; k < 3; k++)
      if (!(bbox_host[3 + k] >= bbox_host[k]) || !std::isfinite(bbox_host[k]) || !std::isfinite(bbox_host[3 + k]))
        return fail(VD_ERR_INVALID_ARG, "vd_build_grid: invalid bbox");
  const double rho = sites_per_cell > 0 ? sites_per_cell : 3.5;
  int g[3];
  if (surface_area > 0 && bbox_host) {
    const double h = std::sqrt(rho * surface_area / (double)n);
    for (int k = 0; k < 3; k++) g[k] = std::max(1, (int)std::ceil((bbox_host[3 + k] - bbox_host[k]) / h));
  } else if (bbox_host) {
    double vol = 1.0;
    double ext[3];
    for (int k = 0; k < 3; k++) { ext[k] = std::max(bbox_host[3 + k] - bbox_host[k], 1e-300); vol *= ext[k]; }
    const double h = std::cbrt(vol * rho / (double)n);
    for (int k = 0; k < 3; k++) g[k] = std::max(1, (int)std::ceil(ext[k] / h));
  } else {
    const int gg = std::max(1, (int)std::ceil(std::cbrt((double)n / rho)));
    g[0] = g[1] = g[2] = gg;
  }
  // keep the cell count sane for degenerate boxes
  while ((double)g[0] * g[1] * g[2] > 16.0 * (double)n + 4096.0) {
    for (int k = 0; k < 3; k++) g[k] = std::max(1, g[k] / 2);
  }
  vd_grid G = *out;
  if (!G) G = new vd_grid_s();
  G->n = n;
  G->g[0] = g[0]; G->g[1] = g[1]; G->g[2] = g[2];
  G->ncell = (int64_t)g[0] * g[1] * g[2];
  hipStream_t st = as_stream(stream);
  vd_status s = VD_OK;
  auto fin = [&](vd_status r) {
    if (r != VD_OK && !*out) { vd_grid_free(G); }
    else *out = G;
    return r;
  };
  {
    int64_t capn = G->cap_n, capc = G->cap_cell;
    hipError_t e = hipSuccess;
    int64_t tmp;
    if (capn < n) {
      tmp = 0; if ((e = ensure(G->sx, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->sy, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->sz, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->delta, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->perm, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->rank, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->cellid, tmp, n)) != hipSuccess) goto herr;
      G->cap_n = n;
    }
    if (capc < G->ncell) {
      tmp = 0; if ((e = ensure(G->cstart, tmp, G->ncell + 1)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->ccount, tmp, G->ncell)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->fill, tmp, G->ncell)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->scan_tmp, tmp, G->ncell / 1024 + 2)) != hipSuccess) goto herr;
      G->cap_cell = G->ncell;
    }
    if ((e = ensure_fixed(G->geom, 9)) != hipSuccess) goto herr;
    if ((e = ensure_fixed(G->bbox_part, 6 * 256)) != hipSuccess) goto herr;
    goto ok;
  herr:
    s = fail(e == hipErrorOutOfMemory ? VD_ERR_OUT_OF_MEMORY : VD_ERR_HIP, "vd_build_grid: %s",
             hipGetErrorString(e));
    return fin(s);
  }
ok:
  vd_launch_grid_build(G, sites, bbox_host, st);
  {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fin(fail(VD_ERR_HIP, "vd_build_grid launch: %s", hipGetErrorString(e)));
  }
  return fin(VD_OK);
}

void vd_grid_free(vd_grid G) {
  if (!G) return;
  hipFree(G->geom); hipFree(G->bbox_part); hipFree(G->sx); hipFree(G->sy); hipFree(G->sz);
  hipFree(G->delta); hipFree(G->perm); hipFree(G->rank); hipFree(G->cellid); hipFree(G->fill);
  hipFree(G->cstart); hipFree(G->ccount); hipFree(G->scan_tmp);
  delete G;
}

// ---------------------------------------------------------------------------
// domain
// ---------------------------------------------------------------------------
vd_status vd_domain_create(const double *verts, int64_t nv, const int32_t *simplices, const int32_t *adjacency,
                           int64_t m, int32_t simplex_dim, void *stream, vd_domain *out) {
  if (!out) return fail(VD_ERR_INVALID_ARG, "vd_domain_create: out is NULL");
  if (!verts || !simplices || !adjacency || nv < 1 || m < 1)
    return fail(VD_ERR_INVALID_ARG, "vd_domain_create: NULL array or empty domain");
  if (simplex_dim != 2 && simplex_dim != 3) return fail(VD_ERR_INVALID_ARG, "vd_domain_create: simplex_dim must be 2 or 3");
  if (m > INT_MAX / 8 || nv > INT_MAX / 4) return fail(VD_ERR_INVALID_ARG, "vd_domain_create: domain too large");
  hipStream_t st = as_stream(stream);
  vd_domain D = *out ? *out : new vd_domain_s();
  auto bail = [&](vd_status r) {
    if (!*out) vd_domain_free(D);
    return r;
  };
  const int k = simplex_dim + 1;
  if (D->m != m || D->nv != nv || D->dim != simplex_dim) {
    hipFree(D->verts); hipFree(D->simp); hipFree(D->adj);
    D->verts = nullptr; D->simp = nullptr; D->adj = nullptr;
    HIP_TRY(hipMalloc((void **)&D->verts, sizeof(double) * 3 * nv));
    HIP_TRY(hipMalloc((void **)&D->simp, sizeof(int) * k * m));
    HIP_TRY(hipMalloc((void **)&D->adj, sizeof(int) * k * m));
  }
  D->m = m; D->nv = nv; D->dim = simplex_dim;
  HIP_TRY(hipMemcpyAsync(D->verts, verts, sizeof(double) * 3 * nv, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(D->simp, simplices, sizeof(int) * k * m, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(D->adj, adjacency, sizeof(int) * k * m, hipMemcpyDeviceToDevice, st));
  int *flags = nullptr;
  double *measure = nullptr, *bbox = nullptr;
  HIP_TRY(hipMalloc((void **)&flags, sizeof(int) * 2));
  HIP_TRY(hipMalloc((void **)&measure, sizeof(double) * m));
  HIP_TRY(hipMalloc((void **)&bbox, sizeof(double) * 6));
  vd_launch_fill_int(flags, 2, 0, st);
  vd_launch_domain_validate(D, flags, measure, st);
  vd_launch_vert_bbox(D, bbox, st);
  int hflags[2] = {0, 0};
  double hbox[6];
  std::vector<double> hmeas((size_t)m);
  HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hbox, bbox, sizeof hbox, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hmeas.data(), measure, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  hipFree(flags); hipFree(measure); hipFree(bbox);
  if (hflags[0]) return bail(fail(VD_ERR_INVALID_ARG, "vd_domain_create: vertex or adjacency index out of range"));
  if (hflags[1])
    return bail(fail(VD_ERR_INVALID_ARG, simplex_dim == 3 ? "vd_domain_create: a tetrahedron has non-positive volume"
                                                          : "vd_domain_create: a degenerate triangle"));
  double tot = 0;
  for (double v : hmeas) tot += v;
  D->area = tot;
  for (int a = 0; a < 6; a++) D->bbox[a] = hbox[a];
  if (simplex_dim == 3) {
    // location grid: about 2 tetrahedra per cell over the vertex bounding box
    double ext[3], vol = 1;
    for (int a = 0; a < 3; a++) { ext[a] = std::max(hbox[3 + a] - hbox[a], 1e-300); vol *= ext[a]; }
    const double h = std::cbrt(vol * 2.0 / (double)m);
    for (int a = 0; a < 3; a++) D->lg[a] = std::max(1, std::min(1024, (int)std::ceil(ext[a] / h)));
    double geom[9];
    for (int a = 0; a < 3; a++) {
      const double pad = 1e-9 * ext[a];
      geom[a] = hbox[a] - pad;
      geom[3 + a] = (ext[a] + 2 * pad) / D->lg[a];
      geom[6 + a] = 1.0 / geom[3 + a];
    }
    const int64_t ncell = (int64_t)D->lg[0] * D->lg[1] * D->lg[2];
    hipFree(D->lgeom); hipFree(D->lstart); hipFree(D->lcount); hipFree(D->lfill); hipFree(D->scan_tmp); hipFree(D->litems);
    D->lgeom = nullptr; D->lstart = D->lcount = D->lfill = D->scan_tmp = D->litems = nullptr;
    HIP_TRY(hipMalloc((void **)&D->lgeom, sizeof(double) * 9));
    HIP_TRY(hipMalloc((void **)&D->lstart, sizeof(int) * (ncell + 1)));
    HIP_TRY(hipMalloc((void **)&D->lcount, sizeof(int) * ncell));
    HIP_TRY(hipMalloc((void **)&D->lfill, sizeof(int) * ncell));
    HIP_TRY(hipMalloc((void **)&D->scan_tmp, sizeof(int) * (ncell / 1024 + 2)));
    HIP_TRY(hipMemcpyAsync(D->lgeom, geom, sizeof geom, hipMemcpyHostToDevice, st));
    vd_launch_domain_locator(D, st);
    int total = 0;
    HIP_TRY(hipMemcpyAsync(&total, D->lstart + ncell, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    D->nitems = total;
    HIP_TRY(hipMalloc((void **)&D->litems, sizeof(int) * std::max(total, 1)));
    vd_launch_domain_fill(D, st);
    HIP_TRY(hipStreamSynchronize(st));
  }
  *out = D;
  return VD_OK;
}

void vd_domain_free(vd_domain D) {
  if (!D) return;
  hipFree(D->verts); hipFree(D->simp); hipFree(D->adj); hipFree(D->lgeom); hipFree(D->lstart);
  hipFree(D->litems); hipFree(D->lcount); hipFree(D->lfill); hipFree(D->scan_tmp);
  delete D;
}

// ---------------------------------------------------------------------------
// clip
// ---------------------------------------------------------------------------
namespace {

struct Caps {
  int64_t piece, face, vert, nbr, fint;
};

hipError_t alloc_cells(vd_cells c, int64_t n, const Caps &want) {
  CellsDev &d = c->d;
  hipError_t e;
  if (c->cap_n < n) {
    int64_t t;
    t = 0; if ((e = ensure(d.mass, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.mom, t, 3 * n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.energy, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.pcount, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.ncount, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.pstart, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.nstart, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.seed, t, n)) != hipSuccess) return e;
    t = 0; if ((e = ensure(c->piece_off, t, n + 1)) != hipSuccess) return e;
    t = 0; if ((e = ensure(c->nbr_off, t, n + 1)) != hipSuccess) return e;
    t = 0; if ((e = ensure(c->scan_tmp, t, n / 1024 + 2)) != hipSuccess) return e;
    t = 0; if ((e = ensure(c->fillc, t, n)) != hipSuccess) return e;
    c->cap_n = n;
  }
  if ((e = ensure_fixed(d.cnt, CNT_N)) != hipSuccess) return e;
  if ((e = ensure_fixed(d.queue, VD_QUEUES * VD_QSTRIDE)) != hipSuccess) return e;
  int64_t cp = d.cap_piece;
  if (cp < want.piece) {
    int64_t t;
    t = 0; if ((e = ensure(d.piece_site, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_simplex, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_nface, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_nvert, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_fstart, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_vstart, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_mass, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_mom, t, 3 * want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_energy, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(c->piece_id, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_fint_start, t, want.piece)) != hipSuccess) return e;
    t = 0; if ((e = ensure(d.piece_nfint, t, want.piece)) != hipSuccess) return e;
    d.cap_piece = want.piece;
    c->cap_pid = want.piece;
  }
  if (d.cap_nbr < want.nbr) {
    int64_t t = 0;
    if ((e = ensure(d.nbr_arena, t, want.nbr)) != hipSuccess) return e;
    t = 0;
    if ((e = ensure(c->nbr, t, want.nbr)) != hipSuccess) return e;
    d.cap_nbr = want.nbr;
    c->cap_nbr_csr = want.nbr;
  }
  if (want.face > 0 && d.cap_face < want.face) {
    int64_t t = 0;
    if ((e = ensure(d.face_label, t, want.face)) != hipSuccess) return e;
    d.cap_face = want.face;
  }
  if (want.vert > 0 && d.cap_vert < want.vert) {
    int64_t t = 0;
    if ((e = ensure(d.vert_xyz, t, 3 * want.vert)) != hipSuccess) return e;
    t = 0;
    if ((e = ensure(d.vert_label, t, 3 * want.vert)) != hipSuccess) return e;
    d.cap_vert = want.vert;
  }
  if (want.fint > 0 && d.cap_fint < want.fint) {
    int64_t t = 0;
    if ((e = ensure(d.fint, t, 12 * want.fint)) != hipSuccess) return e;
    t = 0;
    if ((e = ensure(d.fint_lab, t, want.fint)) != hipSuccess) return e;
    d.cap_fint = want.fint;
  }
  return hipSuccess;
}

}  // namespace

vd_status vd_clip_cells(vd_grid g, vd_domain dom, const vd_options *opt_in, void *stream, vd_cells *out) {
  if (!out || !g || !dom) return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: NULL handle");
  vd_options opt;
  vd_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.max_search_iters < 1) opt.max_search_iters = 1;
  hipStream_t st = as_stream(stream);
  vd_cells c = *out ? *out : new vd_cells_s();
  const int64_t n = g->n;
  c->n = n;
  c->dim = dom->dim;
  c->opt = opt;
  c->grid = g;
  auto bail = [&](vd_status r) {
    if (!*out) vd_cells_free(c);
    return r;
  };
  Caps want;
  want.piece = std::max<int64_t>(std::max<int64_t>(c->d.cap_piece, 6 * n + 1024), dom->dim == 2 ? 2 * dom->m + 6 * n : 0);
  want.nbr = std::max<int64_t>(c->d.cap_nbr, 20 * n + 1024);
  // surfaces always keep the edge flags of their pieces (the per-site pass reads them)
  const bool keep_faces = opt.emit_polytopes || dom->dim == 2;
  want.face = keep_faces ? std::max<int64_t>(c->d.cap_face, 10 * want.piece) : 0;
  want.vert = keep_faces ? std::max<int64_t>(c->d.cap_vert, 16 * want.piece) : 0;
  want.fint = opt.want_grad ? std::max<int64_t>(c->d.cap_fint, 4 * want.piece) : 0;
  for (int attempt = 0; attempt < 4; attempt++) {
    hipError_t e = alloc_cells(c, n, want);
    if (e != hipSuccess)
      return bail(fail(e == hipErrorOutOfMemory ? VD_ERR_OUT_OF_MEMORY : VD_ERR_HIP, "vd_clip_cells: %s",
                       hipGetErrorString(e)));
    CellsDev &d = c->d;
    d.n = (int)n;
    d.emit = opt.emit_polytopes ? 1 : 0;
    d.want_grad = opt.want_grad ? 1 : 0;
    d.improved = opt.improved_search ? 1 : 0;
    d.straddle = opt.use_straddle_edges ? 1 : 0;
    d.max_iters = opt.max_search_iters;
    d.mode = (dom->dim == 3 && opt.carve_mode == 1) ? 1 : 0;
    d.cache = opt.site_cache ? 1 : 0;
    for (int a = 0; a < 3; a++) {
      // The box strictly contains the domain so no box plane meets a simplex.
      // The six paddings differ so that no box edge lies on a plane of
      // symmetry of the domain (e.g. the diagonal planes of cube grids split
      // into tetrahedra), where a tetrahedron plane would contain the edge.
      const double ext = std::max(dom->bbox[3 + a] - dom->bbox[a], 1e-12);
      d.box_lo[a] = dom->bbox[a] - (1.01e-3 + 0.12e-3 * a) * ext - 1e-9;
      d.box_hi[a] = dom->bbox[3 + a] + (1.07e-3 + 0.14e-3 * a) * ext + 1e-9;
    }
    // persistent 3D kernel: each wave reserves output chunks of about 1/8 of an
    // arena's share per wave, so unused chunk tails stay within 1/8 of it
    const int64_t items = dom->dim == 3 ? n : dom->m;  // sites, or triangles
    const int wg = dom->dim == 3 ? vd_sites3d_workgroups(n) : vd_surface_workgroups(dom->m);
    {
      const int64_t caps[AR_N] = {d.cap_piece, d.cap_face, d.cap_vert, d.cap_nbr, d.cap_fint};
      for (int r = 0; r < AR_N; r++)
        d.chunk[r] = std::max<int64_t>(1, std::min<int64_t>(4096, caps[r] / (8 * (int64_t)wg)));
    }
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, d.cnt);
    vd_launch_queue_init(d.queue, items, st);
    GridView G = g->view();
    DomainView D = dom->view();
    if (opt.time_kernels && !c->ev0) {
      HIP_TRY(hipEventCreate(&c->ev0));
      HIP_TRY(hipEventCreate(&c->ev1));
      HIP_TRY(hipEventCreate(&c->ev2));
    }
    if (!c->d_dev) HIP_TRY(hipMalloc((void **)&c->d_dev, sizeof(CellsDev)));
    if (std::memcmp(&c->d_shadow, &d, sizeof(CellsDev)) != 0) {
      c->d_shadow = d;
      HIP_TRY(hipMemcpyAsync(c->d_dev, &c->d_shadow, sizeof(CellsDev), hipMemcpyHostToDevice, st));
    }
    if (dom->dim == 3) vd_launch_locate_sites(G, D, d.seed, d.cnt, st);
    else vd_launch_fill_int(d.pcount, n, 0, st);
    if (opt.time_kernels) HIP_TRY(hipEventRecord(c->ev0, st));
    if (dom->dim == 3) vd_launch_sites3d(G, D, c->d_dev, wg, st);
    else vd_launch_surface(G, D, c->d_dev, wg, st);
    if (opt.time_kernels) HIP_TRY(hipEventRecord(c->ev1, st));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(c->host_cnt, d.cnt, sizeof(unsigned long long) * CNT_N, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->carve_ms = c->split_ms = -1.0;
    if (opt.time_kernels) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
      c->carve_ms = ms;
      c->split_ms = 0.0;
    }
    const unsigned long long *hc = c->host_cnt;
    bool grow = false;
    Caps need = want;
    auto up = [](int64_t used) { return used + used / 4 + 1024; };
    if ((int64_t)hc[CNT_PIECES] > d.cap_piece) { need.piece = up(hc[CNT_PIECES]); grow = true; }
    if ((int64_t)hc[CNT_NBRS] > d.cap_nbr) { need.nbr = up(hc[CNT_NBRS]); grow = true; }
    if (keep_faces && (int64_t)hc[CNT_FACES] > d.cap_face) { need.face = up(hc[CNT_FACES]); grow = true; }
    if (keep_faces && (int64_t)hc[CNT_VERTS] > d.cap_vert) { need.vert = up(hc[CNT_VERTS]); grow = true; }
    if (opt.want_grad && (int64_t)hc[CNT_FINT] > d.cap_fint) { need.fint = up(hc[CNT_FINT]); grow = true; }
    if (grow) { want = need; continue; }
    int bad = (int)(hc[CNT_BAD_SITE] & 0xffffffffull);
    c->first_bad = bad == 0x7fffffff ? -1 : bad;
    if (hc[CNT_ERR_LOC]) {
      c->status = VD_ERR_INVALID_ARG;
      *out = c;
      return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: %llu site(s) outside every tetrahedron (first: %d)",
                  (unsigned long long)hc[CNT_ERR_LOC], c->first_bad);
    }
    if (hc[CNT_ERR_CAP]) {
      c->status = VD_ERR_CAPACITY;
      *out = c;
      return fail(VD_ERR_CAPACITY,
                  "vd_clip_cells: %llu site(s) exceeded a per-wave capacity (first: %d, stages 0x%llx)",
                  (unsigned long long)hc[CNT_ERR_CAP], c->first_bad, (unsigned long long)hc[CNT_STAGES]);
    }
    if (hc[CNT_ERR_DEG]) {
      c->status = VD_ERR_DEGENERATE;
      *out = c;
      return fail(VD_ERR_DEGENERATE,
                  "vd_clip_cells: %llu site(s) hit a non-converging search (first: %d, stages 0x%llx)",
                  (unsigned long long)hc[CNT_ERR_DEG], c->first_bad, (unsigned long long)hc[CNT_STAGES]);
    }
    if (dom->dim == 2) {
      // a site's neighbours are distinct flags of its pieces' edges: the
      // edges written bound the neighbour lists' total
      int64_t t = c->cap_nbr_csr;
      HIP_TRY(ensure(c->nbr, t, std::max<int64_t>((int64_t)hc[CNT_REAL_FACES], 1)));
      c->cap_nbr_csr = t;
    }
    vd_launch_finalize(c, st);
    HIP_TRY(hipGetLastError());
    c->status = VD_OK;
    *out = c;
    return VD_OK;
  }
  return bail(fail(VD_ERR_HIP, "vd_clip_cells: output arenas kept overflowing"));
}

void vd_cells_free(vd_cells c) {
  if (!c) return;
  CellsDev &d = c->d;
  hipFree(d.cnt); hipFree(d.mass); hipFree(d.mom); hipFree(d.energy); hipFree(d.pcount); hipFree(d.ncount);
  hipFree(d.pstart); hipFree(d.nstart); hipFree(d.nbr_arena); hipFree(d.piece_site); hipFree(c->fillc);
  hipFree(d.piece_simplex); hipFree(d.piece_nface); hipFree(d.piece_nvert); hipFree(d.piece_fstart);
  hipFree(d.piece_vstart); hipFree(d.piece_mass); hipFree(d.piece_mom); hipFree(d.piece_energy);
  hipFree(d.face_label); hipFree(d.vert_xyz); hipFree(d.vert_label); hipFree(d.fint); hipFree(d.seed);
  hipFree(c->piece_off); hipFree(c->nbr_off); hipFree(c->piece_id); hipFree(c->nbr); hipFree(c->scan_tmp);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->ev2) hipEventDestroy(c->ev2);
  hipFree(c->d_dev); hipFree(d.queue);
  hipFree(d.fint_lab); hipFree(d.piece_fint_start); hipFree(d.piece_nfint); hipFree(c->wbuf);
  delete c;
}

vd_status vd_cells_info(vd_cells c, vd_cells_info_t *info) {
  if (!c || !info) return fail(VD_ERR_INVALID_ARG, "vd_cells_info: NULL");
  const unsigned long long *hc = c->host_cnt;
  info->n_sites = c->n;
  info->n_pieces = (int64_t)hc[CNT_REAL_PIECES];
  info->n_faces = (int64_t)hc[CNT_REAL_FACES];
  info->n_verts = (int64_t)hc[CNT_REAL_VERTS];
  info->n_nbrs = (int64_t)hc[CNT_REAL_NBRS];
  if (c->dim == 2 && c->n > 0 && c->status == VD_OK) {
    long long tot = 0;
    HIP_TRY(hipMemcpy(&tot, c->nbr_off + c->n, sizeof(long long), hipMemcpyDeviceToHost));
    info->n_nbrs = tot;
  }
  info->nn_queries = (int64_t)hc[CNT_QUERIES];
  info->clips = (int64_t)hc[CNT_CLIPS];
  info->candidates = (int64_t)hc[CNT_CANDS];
  info->grid_queries = (int64_t)hc[CNT_GRIDQ];
  info->first_bad_site = c->first_bad;
  info->failed_stages = (int32_t)c->host_cnt[CNT_STAGES];
  info->status = c->status;
  info->carve_ms = c->carve_ms;
  info->split_ms = c->split_ms;
  return VD_OK;
}

vd_status vd_cells_view(vd_cells c, vd_cells_view_t *v) {
  if (!c || !v) return fail(VD_ERR_INVALID_ARG, "vd_cells_view: NULL");
  const CellsDev &d = c->d;
  v->n_sites = c->n;
  v->n_piece_slots = std::min<int64_t>((int64_t)c->host_cnt[CNT_PIECES], d.cap_piece);
  v->n_face_slots = d.face_label ? std::min<int64_t>((int64_t)c->host_cnt[CNT_FACES], d.cap_face) : 0;
  v->n_vert_slots = d.vert_xyz ? std::min<int64_t>((int64_t)c->host_cnt[CNT_VERTS], d.cap_vert) : 0;
  v->cell_piece_off = (const int64_t *)c->piece_off;
  v->piece_id = c->piece_id;
  v->piece_site = d.piece_site;
  v->piece_simplex = d.piece_simplex;
  v->piece_nface = d.piece_nface;
  v->piece_nvert = d.piece_nvert;
  v->piece_face_start = (const int64_t *)d.piece_fstart;
  v->piece_vert_start = (const int64_t *)d.piece_vstart;
  v->piece_mass = d.piece_mass;
  v->piece_moment = d.piece_mom;
  v->piece_energy = d.piece_energy;
  v->face_label = d.face_label;
  v->vert_xyz = d.vert_xyz;
  v->vert_label = d.vert_label;
  v->nbr_off = (const int64_t *)c->nbr_off;
  v->nbr = c->nbr;
  return VD_OK;
}

vd_status vd_cell_moments(vd_cells c, double *mass, double *centroid, double *energy, void *stream) {
  if (!c) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments: NULL handle");
  if (!mass && !centroid && !energy) return VD_OK;
  if (c->status != VD_OK) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments: the clip failed");
  vd_launch_moments(c, c->grid->view(), mass, centroid, energy, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return VD_OK;
}

vd_status vd_cell_moments_backward(vd_cells c, const double *g_mass, const double *g_centroid,
                                   const double *g_energy, double *g_sites, void *stream) {
  if (!c || !g_sites) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward: NULL argument");
  if (!c->opt.want_grad) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward: clip ran without want_grad");
  if (c->status != VD_OK) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward: the clip failed");
  {
    int64_t t = c->cap_w;
    HIP_TRY(ensure(c->wbuf, t, 5 * c->n));
    c->cap_w = t;
  }
  vd_launch_backward(c, c->grid->view(), g_mass, g_centroid, g_energy, g_sites, c->wbuf, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return VD_OK;
}

}  // extern "C"
