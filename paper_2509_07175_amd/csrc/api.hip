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
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "vd_internal.h"

void vd_launch_domain_fill(vd_domain d, hipStream_t st);
void vd_launch_domain_offsets(vd_domain d, int *flags, hipStream_t st);
void vd_launch_domain_validate(vd_domain d, int *flags, double *measure, hipStream_t st);
void vd_launch_vert_bbox(vd_domain d, double *out, hipStream_t st);
void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st);
void vd_launch_adjacency(vd_domain d, int *count, int *start, int *fill, int *items, int *scan_tmp, int *flags,
                         hipStream_t st);
void vd_launch_convexity(vd_domain d, int *on_bnd, int *pos, int *list, int *scan_tmp, const double *bbox,
                         int *convex, hipStream_t st);
void vd_launch_boundary_scan(vd_domain d, int *flag, int *pos, int *scan_tmp, hipStream_t st);
void vd_launch_boundary_extract(vd_domain d, const int *pos, int *tri, int *btet, long long *boff, hipStream_t st);
void vd_launch_refine_triangles(vd_domain bnd, const int *btet, int s, double *ov, int *otri, int *oadj, int *obtet,
                                hipStream_t st);

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
  if (i < CNT_N)
    cnt[i] = (i == CNT_BAD_SITE) ? 0x7fffffffull
                                 : (i == CNT_MINMARGIN ? (unsigned long long)__double_as_longlong(1.0) : 0ull);
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
    case VD_ERR_NOT_READY: return "VD_ERR_NOT_READY";
  }
  return "VD_ERR_UNKNOWN";
}

vd_status vd_sync(void *stream) {
  const hipError_t e = hipStreamSynchronize(as_stream(stream));
  if (e != hipSuccess) return fail(VD_ERR_HIP, "vd_sync: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return fail(VD_ERR_HIP, "vd_sync: %s", hipGetErrorString(e2));
  return VD_OK;
}

void vd_options_default(vd_options *opt) {
  if (!opt) return;
  opt->sites_per_cell = 2.0;
  opt->improved_search = 0;
  opt->use_straddle_edges = 0;
  opt->max_search_iters = 64;
  opt->emit_polytopes = 1;
  opt->want_grad = 0;
  opt->time_kernels = 0;
  opt->carve_mode = 1;
  opt->site_cache = 1;
  opt->no_sync = 0;
  opt->boundary_seeds = -1;
  opt->monitor = 0;
  opt->use_density = 0;
  opt->whole_interior = 0;
  opt->batch_order = 1;
  for (int k = 0; k < 10; k++) opt->density[k] = k == 0 ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// copies host data to device memory only when it differs from what was sent
// last (so repeated calls with the same batch layout enqueue no copies, and
// can be captured into a graph)
template <typename T>
hipError_t upload_if_changed(T *dev, const T *host, size_t count, std::vector<T> &shadow, hipStream_t st) {
  if (shadow.size() == count && std::memcmp(shadow.data(), host, sizeof(T) * count) == 0) return hipSuccess;
  shadow.assign(host, host + count);
  return hipMemcpyAsync(dev, shadow.data(), sizeof(T) * count, hipMemcpyHostToDevice, st);
}

// device temporaries of one call, freed when it returns (on every path)
struct TmpBuffers {
  std::vector<void *> p;
  ~TmpBuffers() { for (void *q : p) hipFree(q); }
  template <typename T>
  hipError_t get(T *&out, int64_t n) {
    out = nullptr;
    const hipError_t e = hipMalloc((void **)&out, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
    if (e == hipSuccess) p.push_back(out);
    return e;
  }
};

struct GridShadow {
  std::vector<long long> site_off, cell_off;
  std::vector<int> dims;
  std::vector<double> user_box;
  std::vector<unsigned char> views;
};
std::mutex g_shadow_mu;
std::unordered_map<const void *, GridShadow> g_grid_shadow;

// cells of one diagram of n sites (box: host bounding box or NULL)
void diagram_dims(int64_t n, const double *box, double rho, double surface_area, int g[3]) {
  if (surface_area > 0 && box) {
    const double h = std::sqrt(rho * surface_area / (double)n);
    for (int k = 0; k < 3; k++) g[k] = std::max(1, (int)std::ceil((box[3 + k] - box[k]) / h));
  } else if (box) {
    double vol = 1.0;
    double ext[3];
    for (int k = 0; k < 3; k++) { ext[k] = std::max(box[3 + k] - box[k], 1e-300); vol *= ext[k]; }
    const double h = std::cbrt(vol * rho / (double)n);
    for (int k = 0; k < 3; k++) g[k] = std::max(1, (int)std::ceil(ext[k] / h));
  } else {
    const int gg = std::max(1, (int)std::ceil(std::cbrt((double)n / rho)));
    g[0] = g[1] = g[2] = gg;
  }
  // keep the cell count sane for degenerate boxes
  while ((double)g[0] * g[1] * g[2] > 16.0 * (double)n + 4096.0)
    for (int k = 0; k < 3; k++) g[k] = std::max(1, g[k] / 2);
}

vd_status build_grid_impl(const double *sites, int64_t n, int nb, const int64_t *off_host, const double *bbox_host,
                          double sites_per_cell, double surface_area, void *stream, vd_grid *out, const char *who) {
  if (!out) return fail(VD_ERR_INVALID_ARG, "%s: out is NULL", who);
  if (!sites || n < 1) return fail(VD_ERR_INVALID_ARG, "%s: sites NULL or n < 1", who);
  if (n > (int64_t)INT_MAX / 4) return fail(VD_ERR_INVALID_ARG, "%s: n too large", who);
  if (nb < 1) return fail(VD_ERR_INVALID_ARG, "%s: no diagrams", who);
  std::vector<int64_t> off(nb + 1);
  if (off_host) {
    for (int b = 0; b <= nb; b++) off[b] = off_host[b];
    if (off[0] != 0 || off[nb] != n) return fail(VD_ERR_INVALID_ARG, "%s: site offsets must run from 0 to n", who);
    for (int b = 0; b < nb; b++)
      if (off[b + 1] <= off[b]) return fail(VD_ERR_INVALID_ARG, "%s: diagram %d has no sites", who, b);
  } else {
    off[0] = 0; off[1] = n;
  }
  if (bbox_host)
    for (int b = 0; b < nb; b++)
      for (int k = 0; k < 3; k++) {
        const double lo = bbox_host[6 * b + k], hi = bbox_host[6 * b + 3 + k];
        if (!(hi >= lo) || !std::isfinite(lo) || !std::isfinite(hi))
          return fail(VD_ERR_INVALID_ARG, "%s: invalid bbox of diagram %d", who, b);
      }
  // defaults: 2 sites per cell in 3D (the per-wave site cache covers the near
  // ring, so smaller cells than the paper's 3-4 pay), 3.5 per non-empty cell on a surface
  const double rho = sites_per_cell > 0 ? sites_per_cell : (surface_area > 0 ? 3.5 : 2.0);
  std::vector<int> dims(3 * (size_t)nb);
  std::vector<int64_t> coff(nb + 1, 0);
  for (int b = 0; b < nb; b++) {
    diagram_dims(off[b + 1] - off[b], bbox_host ? bbox_host + 6 * b : nullptr, rho, surface_area, &dims[3 * b]);
    coff[b + 1] = coff[b] + (int64_t)dims[3 * b] * dims[3 * b + 1] * dims[3 * b + 2];
  }
  if (coff[nb] > (int64_t)INT_MAX / 2) return fail(VD_ERR_INVALID_ARG, "%s: too many grid cells", who);
  vd_grid G = *out;
  if (!G) G = new vd_grid_s();
  auto fin = [&](vd_status r) {
    if (r != VD_OK && !*out) vd_grid_free(G);
    else *out = G;
    return r;
  };
  G->n = n;
  G->nb = nb;
  G->site_off = off;
  G->cell_off = coff;
  G->dims = dims;
  G->g[0] = dims[0]; G->g[1] = dims[1]; G->g[2] = dims[2];
  G->ncell = coff[nb];
  hipStream_t st = as_stream(stream);
  hipError_t e = hipSuccess;
  {
    int64_t tmp;
    if (G->cap_n < n) {
      tmp = 0; if ((e = ensure(G->sx, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->sy, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->sz, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->delta, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->perm, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->rank, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->cellid, tmp, n)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->diag, tmp, n)) != hipSuccess) goto herr;
      G->cap_n = n;
    }
    if (G->cap_cell < G->ncell) {
      tmp = 0; if ((e = ensure(G->cstart, tmp, G->ncell + 1)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->ccount, tmp, G->ncell)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->fill, tmp, G->ncell)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->scan_tmp, tmp, G->ncell / 1024 + 2)) != hipSuccess) goto herr;
      G->cap_cell = G->ncell;
    }
    if (G->cap_nb < nb) {
      tmp = 0; if ((e = ensure(G->geom, tmp, 9 * (int64_t)nb)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->d_site_off, tmp, nb + 1)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->d_cell_off, tmp, nb + 1)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->d_dims, tmp, 3 * (int64_t)nb)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->d_user_box, tmp, 6 * (int64_t)nb)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->d_views, tmp, nb)) != hipSuccess) goto herr;
      tmp = 0; if ((e = ensure(G->bbox_part, tmp, 6 * (int64_t)std::max(nb, 256))) != hipSuccess) goto herr;
      G->cap_nb = nb;
    }
    G->power = false;  // weights belong to one sorting of the sites
    GridShadow *sh;
    {
      std::lock_guard<std::mutex> lk(g_shadow_mu);
      sh = &g_grid_shadow[G];
    }
    static_assert(sizeof(long long) == sizeof(int64_t), "offsets");
    if ((e = upload_if_changed(G->d_site_off, (const long long *)off.data(), off.size(), sh->site_off, st)) != hipSuccess) goto herr;
    if ((e = upload_if_changed(G->d_cell_off, (const long long *)coff.data(), coff.size(), sh->cell_off, st)) != hipSuccess) goto herr;
    if ((e = upload_if_changed(G->d_dims, dims.data(), dims.size(), sh->dims, st)) != hipSuccess) goto herr;
    if (bbox_host && (e = upload_if_changed(G->d_user_box, bbox_host, 6 * (size_t)nb, sh->user_box, st)) != hipSuccess) goto herr;
    {
      std::vector<GridView> v(nb);
      for (int b = 0; b < nb; b++) v[b] = G->view_of(b);
      std::vector<unsigned char> bytes((const unsigned char *)v.data(), (const unsigned char *)(v.data() + nb));
      if (sh->views != bytes) {
        sh->views = bytes;
        if ((e = hipMemcpyAsync(G->d_views, sh->views.data(), bytes.size(), hipMemcpyHostToDevice, st)) != hipSuccess)
          goto herr;
      }
    }
    goto ok;
  herr:
    return fin(fail(e == hipErrorOutOfMemory ? VD_ERR_OUT_OF_MEMORY : VD_ERR_HIP, "%s: %s", who, hipGetErrorString(e)));
  }
ok:
  vd_launch_grid_build(G, sites, bbox_host ? G->d_user_box : nullptr, st);
  e = hipGetLastError();
  if (e != hipSuccess) return fin(fail(VD_ERR_HIP, "%s launch: %s", who, hipGetErrorString(e)));
  return fin(VD_OK);
}

}  // namespace

extern "C" {

vd_status vd_build_grid(const double *sites, int64_t n, const double *bbox_host, double sites_per_cell,
                        double surface_area, void *stream, vd_grid *out) {
  return build_grid_impl(sites, n, 1, nullptr, bbox_host, sites_per_cell, surface_area, stream, out, "vd_build_grid");
}

vd_status vd_build_grid_batch(const double *sites, const vd_batch *batch, const double *bbox_host,
                              double sites_per_cell, void *stream, vd_grid *out) {
  if (!batch || batch->num < 1 || !batch->site_off)
    return fail(VD_ERR_INVALID_ARG, "vd_build_grid_batch: missing batch or site offsets");
  return build_grid_impl(sites, batch->site_off[batch->num], batch->num, batch->site_off, bbox_host, sites_per_cell,
                         0.0, stream, out, "vd_build_grid_batch");
}

vd_status vd_grid_set_weights(vd_grid G, const double *weights, void *stream) {
  if (!G) return fail(VD_ERR_INVALID_ARG, "vd_grid_set_weights: NULL grid");
  hipStream_t st = as_stream(stream);
  if (weights) {
    int64_t t = G->cap_w;
    HIP_TRY(ensure(G->sw, t, G->n));
    t = G->cap_w;
    HIP_TRY(ensure(G->sh, t, G->n));
    G->cap_w = t;
    HIP_TRY(ensure_fixed(G->eta, 1));
    TmpBuffers tmp;
    int *flags = nullptr;
    HIP_TRY(tmp.get(flags, 1));
    vd_launch_fill_int(flags, 1, 0, st);
    vd_launch_grid_weights(G, weights, flags, st);
    int hf = 0;
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof hf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hf) return fail(VD_ERR_INVALID_ARG, "vd_grid_set_weights: a weight is not finite");
  }
  G->power = weights != nullptr;
  std::vector<GridView> v(G->nb);
  for (int b = 0; b < G->nb; b++) v[b] = G->view_of(b);
  std::vector<unsigned char> bytes((const unsigned char *)v.data(), (const unsigned char *)(v.data() + G->nb));
  {
    std::lock_guard<std::mutex> lk(g_shadow_mu);
    GridShadow &sh = g_grid_shadow[G];
    if (sh.views != bytes) {
      sh.views = bytes;
      HIP_TRY(hipMemcpyAsync(G->d_views, sh.views.data(), bytes.size(), hipMemcpyHostToDevice, st));
    }
  }
  return VD_OK;
}

void vd_grid_free(vd_grid G) {
  if (!G) return;
  hipFree(G->sw); hipFree(G->sh); hipFree(G->eta);
  hipFree(G->geom); hipFree(G->bbox_part); hipFree(G->sx); hipFree(G->sy); hipFree(G->sz);
  hipFree(G->delta); hipFree(G->perm); hipFree(G->rank); hipFree(G->cellid); hipFree(G->fill);
  hipFree(G->cstart); hipFree(G->ccount); hipFree(G->scan_tmp);
  hipFree(G->d_site_off); hipFree(G->d_cell_off); hipFree(G->d_dims); hipFree(G->diag); hipFree(G->d_user_box);
  hipFree(G->d_views);
  {
    std::lock_guard<std::mutex> lk(g_shadow_mu);
    g_grid_shadow.erase(G);
  }
  delete G;
}

// ---------------------------------------------------------------------------
// domain
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {



vd_status domain_create_impl(const double *verts, const int32_t *simplices, const int32_t *adjacency, int nb,
                             const int64_t *vert_off_host, const int64_t *simp_off_host, int32_t simplex_dim,
                             void *stream, vd_domain *out, const char *who) {
  if (!out) return fail(VD_ERR_INVALID_ARG, "%s: out is NULL", who);
  if (nb < 1) return fail(VD_ERR_INVALID_ARG, "%s: no diagrams", who);
  const int64_t nv = vert_off_host[nb], m = simp_off_host[nb];
  if (!verts || !simplices || nv < 1 || m < 1)
    return fail(VD_ERR_INVALID_ARG, "%s: NULL array or empty domain", who);
  if (simplex_dim != 2 && simplex_dim != 3) return fail(VD_ERR_INVALID_ARG, "%s: simplex_dim must be 2 or 3", who);
  if (m > INT_MAX / 8 || nv > INT_MAX / 4) return fail(VD_ERR_INVALID_ARG, "%s: domain too large", who);
  if (vert_off_host[0] != 0 || simp_off_host[0] != 0) return fail(VD_ERR_INVALID_ARG, "%s: offsets must start at 0", who);
  for (int b = 0; b < nb; b++)
    if (vert_off_host[b + 1] <= vert_off_host[b] || simp_off_host[b + 1] <= simp_off_host[b])
      return fail(VD_ERR_INVALID_ARG, "%s: diagram %d has an empty domain", who, b);
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
  D->m = m; D->nv = nv; D->dim = simplex_dim; D->nb = nb;
  D->vert_off.assign(vert_off_host, vert_off_host + nb + 1);
  D->simp_off.assign(simp_off_host, simp_off_host + nb + 1);
  hipFree(D->d_simp_off); hipFree(D->d_vert_off); hipFree(D->d_loc_off); hipFree(D->d_lg); hipFree(D->d_views);
  D->d_simp_off = D->d_vert_off = D->d_loc_off = nullptr; D->d_lg = nullptr; D->d_views = nullptr;
  HIP_TRY(hipMalloc((void **)&D->d_simp_off, sizeof(long long) * (nb + 1)));
  HIP_TRY(hipMalloc((void **)&D->d_vert_off, sizeof(long long) * (nb + 1)));
  HIP_TRY(hipMemcpy(D->d_simp_off, D->simp_off.data(), sizeof(long long) * (nb + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->d_vert_off, D->vert_off.data(), sizeof(long long) * (nb + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpyAsync(D->verts, verts, sizeof(double) * 3 * nv, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(D->simp, simplices, sizeof(int) * k * m, hipMemcpyDeviceToDevice, st));
  if (adjacency) HIP_TRY(hipMemcpyAsync(D->adj, adjacency, sizeof(int) * k * m, hipMemcpyDeviceToDevice, st));
  else vd_launch_fill_int(D->adj, k * m, -1, st);
  // temporaries of the staging (freed below, on every path)
  TmpBuffers tmp;
  int *flags = nullptr, *convex = nullptr;
  double *measure = nullptr, *bbox = nullptr;
  HIP_TRY(tmp.get(flags, 3));
  HIP_TRY(tmp.get(measure, m));
  HIP_TRY(tmp.get(bbox, 6 * nb));
  HIP_TRY(tmp.get(convex, nb));
  vd_launch_fill_int(flags, 3, 0, st);
  vd_launch_fill_int(convex, nb, 1, st);
  vd_launch_domain_offsets(D, flags, st);
  if (!adjacency) {
    // Sec. 3.2 flags need the simplex adjacency: computed here by face matching
    int *cnt = nullptr, *start = nullptr, *fill = nullptr, *items = nullptr, *stmp = nullptr;
    HIP_TRY(tmp.get(cnt, nv));
    HIP_TRY(tmp.get(start, nv + 1));
    HIP_TRY(tmp.get(fill, nv));
    HIP_TRY(tmp.get(items, k * m));
    HIP_TRY(tmp.get(stmp, nv / 1024 + 2));
    vd_launch_adjacency(D, cnt, start, fill, items, stmp, flags + 2, st);
  }
  vd_launch_domain_validate(D, flags, measure, st);
  vd_launch_vert_bbox(D, bbox, st);
  if (simplex_dim == 3) {
    int *on_bnd = nullptr, *pos = nullptr, *list = nullptr, *stmp = nullptr;
    HIP_TRY(tmp.get(on_bnd, nv));
    HIP_TRY(tmp.get(pos, nv + 1));
    HIP_TRY(tmp.get(list, nv));
    HIP_TRY(tmp.get(stmp, nv / 1024 + 2));
    vd_launch_convexity(D, on_bnd, pos, list, stmp, bbox, convex, st);
  }
  int hflags[3] = {0, 0, 0};
  std::vector<double> hbox(6 * (size_t)nb);
  std::vector<double> hmeas((size_t)m);
  std::vector<int> hconv((size_t)nb, 1);
  HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hbox.data(), bbox, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hmeas.data(), measure, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hconv.data(), convex, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hflags[0]) return bail(fail(VD_ERR_INVALID_ARG, "%s: vertex or adjacency index out of range", who));
  if (hflags[2])
    return bail(fail(VD_ERR_INVALID_ARG, "%s: a face is shared by more than two simplices (non-manifold mesh)", who));
  if (hflags[1])
    return bail(fail(VD_ERR_INVALID_ARG, simplex_dim == 3 ? "%s: a tetrahedron has non-positive volume"
                                                          : "%s: a degenerate triangle", who));
  D->convex = hconv;
  D->all_convex = simplex_dim == 3 && std::all_of(hconv.begin(), hconv.end(), [](int c) { return c != 0; });
  double tot = 0;
  for (double v : hmeas) tot += v;
  D->area = tot;
  D->bbox = hbox;
  hipFree(D->lgeom); hipFree(D->lstart); hipFree(D->lcount); hipFree(D->lfill); hipFree(D->scan_tmp); hipFree(D->litems);
  D->lgeom = nullptr; D->lstart = D->lcount = D->lfill = D->scan_tmp = D->litems = nullptr;
  D->lg.assign(3 * (size_t)nb, 1);
  D->loc_off.assign(nb + 1, 0);
  if (simplex_dim == 3) {
    // location grid of each diagram: about 2 tetrahedra per cell over its vertex box
    std::vector<double> geom(9 * (size_t)nb);
    for (int b = 0; b < nb; b++) {
      const double *bx = &hbox[6 * b];
      const int64_t mb = simp_off_host[b + 1] - simp_off_host[b];
      double ext[3], vol = 1;
      for (int a = 0; a < 3; a++) { ext[a] = std::max(bx[3 + a] - bx[a], 1e-300); vol *= ext[a]; }
      const double h = std::cbrt(vol * 2.0 / (double)mb);
      for (int a = 0; a < 3; a++) D->lg[3 * b + a] = std::max(1, std::min(1024, (int)std::ceil(ext[a] / h)));
      for (int a = 0; a < 3; a++) {
        const double pad = 1e-9 * ext[a];
        geom[9 * b + a] = bx[a] - pad;
        geom[9 * b + 3 + a] = (ext[a] + 2 * pad) / D->lg[3 * b + a];
        geom[9 * b + 6 + a] = 1.0 / geom[9 * b + 3 + a];
      }
      D->loc_off[b + 1] = D->loc_off[b] + (int64_t)D->lg[3 * b] * D->lg[3 * b + 1] * D->lg[3 * b + 2];
    }
    const int64_t ncell = D->loc_off[nb];
    if (ncell > (int64_t)INT_MAX / 2) return bail(fail(VD_ERR_INVALID_ARG, "%s: location grid too large", who));
    D->ncell = ncell;
    HIP_TRY(hipMalloc((void **)&D->lgeom, sizeof(double) * 9 * nb));
    HIP_TRY(hipMalloc((void **)&D->d_lg, sizeof(int) * 3 * nb));
    HIP_TRY(hipMalloc((void **)&D->d_loc_off, sizeof(long long) * (nb + 1)));
    HIP_TRY(hipMalloc((void **)&D->lstart, sizeof(int) * (ncell + 1)));
    HIP_TRY(hipMalloc((void **)&D->lcount, sizeof(int) * ncell));
    HIP_TRY(hipMalloc((void **)&D->lfill, sizeof(int) * ncell));
    HIP_TRY(hipMalloc((void **)&D->scan_tmp, sizeof(int) * (ncell / 1024 + 2)));
    HIP_TRY(hipMemcpy(D->lgeom, geom.data(), sizeof(double) * 9 * nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D->d_lg, D->lg.data(), sizeof(int) * 3 * nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D->d_loc_off, D->loc_off.data(), sizeof(long long) * (nb + 1), hipMemcpyHostToDevice));
    vd_launch_domain_locator(D, st);
    int total = 0;
    HIP_TRY(hipMemcpyAsync(&total, D->lstart + ncell, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    D->nitems = total;
    HIP_TRY(hipMalloc((void **)&D->litems, sizeof(int) * std::max(total, 1)));
    vd_launch_domain_fill(D, st);
  }
  {
    std::vector<DomainView> v(nb);
    for (int b = 0; b < nb; b++) v[b] = D->view_of(b);
    HIP_TRY(hipMalloc((void **)&D->d_views, sizeof(DomainView) * nb));
    HIP_TRY(hipMemcpy(D->d_views, v.data(), sizeof(DomainView) * nb, hipMemcpyHostToDevice));
  }
  if (simplex_dim == 3) {
    // the boundary surface of M as a triangle domain (Alg. 5 seeds the cells
    // that reach M away from their site's tetrahedron through it)
    int *flag = nullptr, *pos = nullptr, *stmp = nullptr, *tri = nullptr, *adjm1 = nullptr;
    long long *boff_d = nullptr;
    HIP_TRY(tmp.get(flag, 4 * m));
    HIP_TRY(tmp.get(pos, 4 * m + 1));
    HIP_TRY(tmp.get(stmp, 4 * m / 1024 + 2));
    vd_launch_boundary_scan(D, flag, pos, stmp, st);
    int nbt = 0;
    HIP_TRY(hipMemcpyAsync(&nbt, pos + 4 * m, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nbt < 4) return bail(fail(VD_ERR_INVALID_ARG, "%s: the domain has no boundary surface", who));
    HIP_TRY(tmp.get(tri, 3 * (int64_t)nbt));
    HIP_TRY(tmp.get(adjm1, 3 * (int64_t)nbt));
    HIP_TRY(tmp.get(boff_d, nb + 1));
    hipFree(D->btet);
    D->btet = nullptr;
    HIP_TRY(hipMalloc((void **)&D->btet, sizeof(int) * nbt));
    vd_launch_fill_int(adjm1, 3 * (int64_t)nbt, -1, st);
    vd_launch_boundary_extract(D, pos, tri, D->btet, boff_d, st);
    std::vector<int64_t> boff((size_t)nb + 1);
    HIP_TRY(hipMemcpyAsync(boff.data(), boff_d, sizeof(long long) * (nb + 1), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const vd_status r = domain_create_impl(D->verts, tri, adjm1, nb, D->vert_off.data(), boff.data(), 2, stream,
                                           &D->bnd, who);
    if (r != VD_OK) return bail(r);
  }
  HIP_TRY(hipStreamSynchronize(st));
  *out = D;
  return VD_OK;
}

}  // namespace

extern "C" {

vd_status vd_domain_create(const double *verts, int64_t nv, const int32_t *simplices, const int32_t *adjacency,
                           int64_t m, int32_t simplex_dim, void *stream, vd_domain *out) {
  const int64_t voff[2] = {0, nv}, soff[2] = {0, m};
  return domain_create_impl(verts, simplices, adjacency, 1, voff, soff, simplex_dim, stream, out, "vd_domain_create");
}

vd_status vd_domain_create_batch(const double *verts, const int32_t *simplices, const int32_t *adjacency,
                                 const vd_batch *batch, int32_t simplex_dim, void *stream, vd_domain *out) {
  if (!batch || batch->num < 1 || !batch->vert_off || !batch->simp_off)
    return fail(VD_ERR_INVALID_ARG, "vd_domain_create_batch: missing batch or offsets");
  return domain_create_impl(verts, simplices, adjacency, batch->num, batch->vert_off, batch->simp_off, simplex_dim,
                            stream, out, "vd_domain_create_batch");
}

vd_status vd_domain_info(vd_domain D, vd_domain_info_t *info) {
  if (!D || !info) return fail(VD_ERR_INVALID_ARG, "vd_domain_info: NULL");
  info->n_simplices = D->m;
  info->n_verts = D->nv;
  info->simplex_dim = D->dim;
  info->n_diagrams = D->nb;
  info->measure = D->area;
  info->convex = D->dim == 3 ? (D->all_convex ? 1 : 0) : -1;
  return VD_OK;
}

vd_status vd_domain_adjacency(vd_domain D, int32_t *adjacency_out, void *stream) {
  if (!D || !adjacency_out) return fail(VD_ERR_INVALID_ARG, "vd_domain_adjacency: NULL");
  HIP_TRY(hipMemcpyAsync(adjacency_out, D->adj, sizeof(int) * (D->dim + 1) * D->m, hipMemcpyDeviceToDevice,
                         as_stream(stream)));
  return VD_OK;
}

void vd_domain_free(vd_domain D) {
  if (!D) return;
  vd_domain_free(D->bnd);
  hipFree(D->btet);
  vd_domain_free(D->bnd_ref);
  hipFree(D->btet_ref);
  hipFree(D->verts); hipFree(D->simp); hipFree(D->adj); hipFree(D->lgeom); hipFree(D->lstart);
  hipFree(D->litems); hipFree(D->lcount); hipFree(D->lfill); hipFree(D->scan_tmp);
  hipFree(D->d_simp_off); hipFree(D->d_vert_off); hipFree(D->d_loc_off); hipFree(D->d_lg); hipFree(D->d_views);
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
  if (!c->host_cnt) {
    if ((e = hipHostMalloc((void **)&c->host_cnt, sizeof(unsigned long long) * CNT_N, hipHostMallocDefault)) !=
        hipSuccess)
      return e;
    std::memset(c->host_cnt, 0, sizeof(unsigned long long) * CNT_N);
  }
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
    t = 0; if ((e = ensure(c->pid_tmp, t, want.piece)) != hipSuccess) return e;
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

// The work order of a batch: each diagram costs about (1 + its tetrahedra per
// site) per site (a cell meets more tetrahedra on a finer mesh); diagrams go to
// the VD_QUEUES queues by longest processing time (the largest total first, to
// the least loaded queue), and each queue hands out its diagrams from the
// highest cost per site down, so the sites that finish a launch are cheap.
// A diagram's sites stay contiguous (grid order), which keeps an XCD's L2 warm.
hipError_t batch_order(vd_cells c, const std::vector<int64_t> &site_off, const std::vector<int64_t> &simp_off,
                       int64_t n) {
  const int nb = (int)site_off.size() - 1;
  std::vector<double> per(nb), tot(nb);
  for (int b = 0; b < nb; b++) {
    const double ns = (double)(site_off[b + 1] - site_off[b]), ms = (double)(simp_off[b + 1] - simp_off[b]);
    per[b] = 1.0 + ms / std::max(ns, 1.0);
    tot[b] = ns * per[b];
  }
  std::vector<int> idx(nb);
  for (int b = 0; b < nb; b++) idx[b] = b;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return tot[x] > tot[y]; });
  std::vector<std::vector<int>> lists(VD_QUEUES);
  std::vector<double> load(VD_QUEUES, 0.0);
  for (int b : idx) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lists[k].push_back(b);
    load[k] += tot[b];
  }
  std::vector<int> order((size_t)n);
  c->order_qoff.assign(VD_QUEUES + 1, 0);
  int64_t pos = 0;
  for (int k = 0; k < VD_QUEUES; k++) {
    std::stable_sort(lists[k].begin(), lists[k].end(), [&](int x, int y) { return per[x] > per[y]; });
    for (int b : lists[k])
      for (int64_t p = site_off[b]; p < site_off[b + 1]; p++) order[(size_t)pos++] = (int)p;
    c->order_qoff[k + 1] = pos;
  }
  hipError_t e = ensure(c->order_buf, c->order_cap, n);
  if (e != hipSuccess) return e;
  return hipMemcpy(c->order_buf, order.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice);
}

// Status of a finished clip from its counters (arena overflow included when
// `overflow_is_error`: a no-sync clip cannot grow its arenas).
vd_status check_counts(vd_cells c, bool overflow_is_error) {
  const unsigned long long *hc = c->host_cnt;
  const CellsDev &d = c->d;
  int bad = (int)(hc[CNT_BAD_SITE] & 0xffffffffull);
  c->first_bad = bad == 0x7fffffff ? -1 : bad;
  if (hc[CNT_ERR_LOC])
    return (vd_status)(c->status = fail(VD_ERR_INVALID_ARG,
                            "vd_clip_cells: %llu site(s) outside every tetrahedron and no boundary seeds "
                            "(first: %d; boundary_seeds = 0 or a no_sync clip)",
                            (unsigned long long)hc[CNT_ERR_LOC], c->first_bad));
  if (hc[CNT_ERR_CAP])
    return (vd_status)(c->status = fail(VD_ERR_CAPACITY,
                            "vd_clip_cells: %llu site(s) exceeded a per-wave capacity (first: %d, stages 0x%llx)",
                            (unsigned long long)hc[CNT_ERR_CAP], c->first_bad, (unsigned long long)hc[CNT_STAGES]));
  if (hc[CNT_ERR_DEG])
    return (vd_status)(c->status = fail(VD_ERR_DEGENERATE,
                            "vd_clip_cells: %llu site(s) hit a non-converging search (first: %d, stages 0x%llx)",
                            (unsigned long long)hc[CNT_ERR_DEG], c->first_bad, (unsigned long long)hc[CNT_STAGES]));
  if (overflow_is_error &&
      (hc[CNT_OVERFLOW] || (int64_t)hc[CNT_PIECES] > d.cap_piece || (int64_t)hc[CNT_NBRS] > d.cap_nbr ||
       (d.face_label && (int64_t)hc[CNT_FACES] > d.cap_face) || (d.vert_xyz && (int64_t)hc[CNT_VERTS] > d.cap_vert) ||
       (d.fint && (int64_t)hc[CNT_FINT] > d.cap_fint)))
    return (vd_status)(c->status = fail(VD_ERR_CAPACITY, "vd_clip_cells: an output arena overflowed in a no-sync clip "
                                             "(run a synchronous clip on this handle to grow it)"));
  c->status = VD_OK;
  return VD_OK;
}

// The boundary surface on which a clip of n sites computes its boundary
// diagram, and the tetrahedron behind each of its triangles.  The diagram
// takes one wave per triangle, so a triangle that would meet many cells
// (about (n / |M|)^(2/3) per unit area) is split into s^2 smaller ones; the
// split surface is kept in the domain handle for later clips.
vd_status boundary_for_clip(vd_domain dom, int64_t n, void *stream, vd_domain &bd, const int *&btet) {
  bd = dom->bnd;
  btet = dom->btet;
  if (!bd || bd->m < 1 || dom->area <= 0) return VD_OK;
  const double cells_per_tri = std::pow((double)n / dom->area, 2.0 / 3.0) * bd->area / (double)bd->m;
  if (!(cells_per_tri > 32.0)) return VD_OK;
  const int s = (int)std::min(64.0, std::ceil(std::sqrt(cells_per_tri / 8.0)));
  if (!(dom->bnd_ref && dom->bnd_ref_s == s)) {
    const int64_t mr = bd->m * (int64_t)s * s;
    if (mr > INT_MAX / 8) return VD_OK;  // too fine to split: keep the coarse surface
    hipStream_t st = as_stream(stream);
    TmpBuffers tmp;
    double *ov = nullptr;
    int *otri = nullptr, *oadj = nullptr;
    HIP_TRY(tmp.get(ov, 9 * mr));
    HIP_TRY(tmp.get(otri, 3 * mr));
    HIP_TRY(tmp.get(oadj, 3 * mr));
    hipFree(dom->btet_ref);
    dom->btet_ref = nullptr;
    dom->bnd_ref_s = 0;
    HIP_TRY(hipMalloc((void **)&dom->btet_ref, sizeof(int) * mr));
    vd_launch_refine_triangles(bd, dom->btet, s, ov, otri, oadj, dom->btet_ref, st);
    HIP_TRY(hipGetLastError());
    std::vector<int64_t> so(bd->nb + 1), vo(bd->nb + 1);
    for (int b = 0; b <= bd->nb; b++) {
      so[b] = bd->simp_off[b] * (int64_t)s * s;
      vo[b] = 3 * so[b];
    }
    const vd_status r = domain_create_impl(ov, otri, oadj, bd->nb, vo.data(), so.data(), 2, stream, &dom->bnd_ref,
                                           "vd_clip_cells (split boundary)");
    if (r != VD_OK) return r;
    dom->bnd_ref_s = s;
  }
  bd = dom->bnd_ref;
  btet = dom->btet_ref;
  return VD_OK;
}

}  // namespace

vd_status vd_clip_cells(vd_grid g, vd_domain dom, const vd_options *opt_in, void *stream, vd_cells *out) {
  if (!out || !g || !dom) return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: NULL handle");
  if (g->nb != dom->nb)
    return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: the grid holds %d diagram(s), the domain %d", g->nb, dom->nb);
  if (opt_in && opt_in->no_sync) {
    vd_cells c0 = *out;
    if (!c0 || c0->n != g->n || c0->cap_n < g->n || c0->d.cap_piece <= 0 ||
        (opt_in->emit_polytopes && !c0->d.face_label) || (opt_in->want_grad && !c0->d.fint))
      return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: no_sync needs a handle sized by a synchronous clip of the "
                                      "same sites and options");
  }
  vd_options opt;
  vd_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.max_search_iters < 1) opt.max_search_iters = 1;
  if (g->power) {
    // power diagram (Sec. 7.3): lifted grid queries (no site cache, no lambda
    // steps); in 3D the cell is carved first and seeded from the boundary too,
    // since a power cell need not contain its site
    if (opt.want_grad || opt.use_density || opt.no_sync)
      return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: power diagrams take no want_grad, use_density or no_sync");
    opt.improved_search = 0;
    opt.site_cache = 0;
    if (dom->dim == 3) {
      opt.carve_mode = 1;
      opt.boundary_seeds = 1;
    }
  }
  if (opt.whole_interior) {
    // Alg. 5's interior / boundary split needs the boundary diagram and the
    // cell-first carve
    if (dom->dim != 3 || opt.carve_mode != 1 || opt.boundary_seeds == 0 || opt.no_sync)
      return fail(VD_ERR_INVALID_ARG, "vd_clip_cells: whole_interior needs a tetrahedral domain, carve_mode 1, "
                                      "boundary seeds and a synchronous clip");
  }
  hipStream_t st = as_stream(stream);
  vd_cells c = *out ? *out : new vd_cells_s();
  const int64_t n = g->n;
  c->n = n;
  c->pending = false;
  c->dim = dom->dim;
  c->opt = opt;
  c->grid = g;
  auto bail = [&](vd_status r) {
    if (!*out) vd_cells_free(c);
    return r;
  };
  Caps want;
  // a site's cell meets a few simplices when simplices and cells are alike in
  // size, many when simplices are much smaller: 8 per site plus 3 per simplex
  want.piece = std::max<int64_t>(c->d.cap_piece, 8 * n + 3 * dom->m + 1024);
  want.nbr = std::max<int64_t>(c->d.cap_nbr, 20 * n + 1024);
  // surfaces always keep the edge flags of their pieces (the per-site pass reads them)
  const bool keep_faces = opt.emit_polytopes || dom->dim == 2;
  want.face = keep_faces ? std::max<int64_t>(c->d.cap_face, 10 * want.piece) : 0;
  want.vert = keep_faces ? std::max<int64_t>(c->d.cap_vert, 16 * want.piece) : 0;
  want.fint = opt.want_grad ? std::max<int64_t>(c->d.cap_fint, 4 * want.piece) : 0;
  if (opt.no_sync) {
    // no allocation: the arenas keep the sizes of the synchronous clip before
    want.piece = c->d.cap_piece; want.nbr = c->d.cap_nbr;
    want.face = keep_faces ? c->d.cap_face : 0;
    want.vert = keep_faces ? c->d.cap_vert : 0;
    want.fint = opt.want_grad ? c->d.cap_fint : 0;
  }
  for (int attempt = 0; attempt < 8; attempt++) {
    hipError_t e = alloc_cells(c, n, want);
    if (e != hipSuccess)
      return bail(fail(e == hipErrorOutOfMemory ? VD_ERR_OUT_OF_MEMORY : VD_ERR_HIP, "vd_clip_cells: %s",
                       hipGetErrorString(e)));
    CellsDev &d = c->d;
    d.n = (int)n;
    d.emit = opt.emit_polytopes ? 1 : 0;
    d.want_grad = opt.want_grad ? 1 : 0;
    d.improved = opt.improved_search ? 1 : 0;
    if (d.improved && !g->delta_valid) vd_launch_grid_delta(g, st);
    d.straddle = opt.use_straddle_edges ? 1 : 0;
    d.max_iters = opt.max_search_iters;
    d.mode = (dom->dim == 3 && opt.carve_mode == 1) ? 1 : 0;
    d.cache = opt.site_cache ? 1 : 0;
    d.monitor = opt.monitor ? 1 : 0;
    d.density = opt.use_density ? 1 : 0;
    d.power = g->power ? 1 : 0;
    for (int k = 0; k < 10; k++) d.dens[k] = opt.use_density ? opt.density[k] : (k == 0 ? 1.0 : 0.0);
    // persistent 3D kernel: each wave reserves output chunks of about 1/8 of an
    // arena's share per wave, so unused chunk tails stay within 1/8 of it
    const int64_t items = dom->dim == 3 ? n : dom->m;  // sites, or triangles
    const int wg = dom->dim == 3 ? vd_sites3d_workgroups(n) : vd_surface_workgroups(dom->m);
    if (dom->dim == 3 &&
        (c->cap_spill < wg || d.q_spill < c->q_spill_want || d.nbs_cap < c->nb_spill_want)) {
      if (opt.no_sync) return bail(fail(VD_ERR_INVALID_ARG, "vd_clip_cells: no_sync on an unsized handle"));
      const int64_t w = std::max<int64_t>(wg, c->cap_spill);
      int64_t t = 0;
      HIP_TRY(ensure(d.tq_spill, t, w * c->q_spill_want));
      t = 0;
      HIP_TRY(ensure(d.nb_spill, t, w * c->nb_spill_want));
      t = 0;
      HIP_TRY(ensure(d.saved, t, w * VD_SAVE_DOUBLES));
      c->cap_spill = w;
      d.q_spill = c->q_spill_want;
      d.nbs_cap = c->nb_spill_want;
    }
    if (dom->dim == 2) {
      // surface: a triangle's site list beyond its LDS part (none until a
      // triangle needs it; grown on retry)
      const int64_t need = (int64_t)wg * c->sq_spill_want;
      if (need > 0 && (c->sq_spill_elems < need || d.sq_cap != c->sq_spill_want)) {
        HIP_TRY(ensure(d.sq_spill, c->sq_spill_elems, need));
      }
      d.sq_cap = need > 0 ? c->sq_spill_want : 0;
    }
    {
      const int64_t caps[AR_N] = {d.cap_piece, d.cap_face, d.cap_vert, d.cap_nbr, d.cap_fint};
      for (int r = 0; r < AR_N; r++)
        d.chunk[r] = std::max<int64_t>(1, std::min<int64_t>(4096, caps[r] / (8 * (int64_t)wg)));
    }
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, d.cnt);
    // batches: the diagrams with the most tetrahedra per site first (below)
    d.order = nullptr;
    if (dom->dim == 3 && g->nb > 1 && opt.batch_order) {
      std::vector<int64_t> key = g->site_off;
      key.insert(key.end(), dom->simp_off.begin(), dom->simp_off.end());
      if (c->order_key != key && !opt.no_sync) {
        HIP_TRY(batch_order(c, g->site_off, dom->simp_off, n));
        c->order_key = key;
      }
      if (c->order_key == key) {
        d.order = c->order_buf;
        for (int k = 0; k <= VD_QUEUES; k++) d.qoff[k] = c->order_qoff[k];
      }
    }
    vd_launch_queue_init(d.queue, items, d.order ? d.qoff : nullptr, st);
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
    if (dom->dim == 3 && attempt == 0) {
      // seeds: the tetrahedron holding each site, and (Alg. 5) the boundary
      // triangles each cell meets when the domain is not convex or a site
      // lies outside it
      HIP_TRY(ensure_fixed(c->outside, 6));
      for (int k = 0; k < 6; k += 2) {
        vd_launch_fill_int(c->outside + k, 1, 0, st);
        vd_launch_fill_int(c->outside + k + 1, 1, INT_MAX, st);
      }
      vd_launch_locate_sites(G, D, d.seed, c->outside, st);
      bool use_b = false;
      c->sites_outside = -1;
      if (!opt.no_sync) {
        int ho[6] = {0, INT_MAX, 0, INT_MAX, 0, INT_MAX};
        HIP_TRY(hipMemcpyAsync(ho, c->outside, sizeof ho, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (ho[4] > 0)
          return bail(fail(VD_ERR_INVALID_ARG, "vd_clip_cells: %d site(s) with a coordinate that is not finite "
                                               "(first: %d)", ho[4], ho[5]));
        // Eq. 1 needs distinct sites: a copy of a site has no cell of its own
        if (ho[2] > 0)
          return bail(fail(VD_ERR_INVALID_ARG, "vd_clip_cells: %d site(s) repeat an earlier site exactly (first: %d)",
                           ho[2], ho[3]));
        if (opt.boundary_seeds != 0) {
          c->sites_outside = ho[0];
          use_b = opt.boundary_seeds == 1 || !dom->all_convex || ho[0] > 0;
        }
      }
      // the interior split: by the boundary diagram, or, for a convex M that
      // holds every site, by the corners of each cell (no boundary diagram).
      // The boundary diagram takes one wave per boundary triangle, so it is
      // chosen while a triangle meets few cells (about (n / |M|)^(2/3) per
      // unit area); on coarse boundaries the corner test is far cheaper.
      if (opt.whole_interior && !use_b && dom->bnd && dom->area > 0 && dom->bnd->m > 0) {
        const double per_area = std::pow((double)n / dom->area, 2.0 / 3.0);
        const double cells_per_tri = per_area * dom->bnd->area / (double)dom->bnd->m;
        use_b = cells_per_tri <= 32.0;
      }
      d.whole = !opt.whole_interior ? 0 : (use_b ? 1 : 2);
      if (use_b) {
        if (!dom->bnd) return bail(fail(VD_ERR_INVALID_ARG, "vd_clip_cells: the domain has no boundary surface"));
        vd_domain bd = nullptr;
        const int *btet = nullptr;
        {
          const vd_status r = boundary_for_clip(dom, n, stream, bd, btet);
          if (r != VD_OK) return bail(r);
        }
        vd_options bopt;
        vd_options_default(&bopt);
        bopt.emit_polytopes = 0;
        bopt.max_search_iters = opt.max_search_iters;
        bopt.site_cache = opt.site_cache;
        const vd_status r = vd_clip_cells(g, bd, &bopt, stream, &c->bcells);
        if (r != VD_OK) return bail(r);
        d.bseed_off = c->bcells->piece_off;
        d.bseed_pid = c->bcells->piece_id;
        d.bseed_tri = c->bcells->d.piece_simplex;
        d.btet = btet;
      } else {
        d.bseed_off = nullptr;
        d.bseed_pid = d.bseed_tri = d.btet = nullptr;
      }
      c->used_bseeds = use_b;
      if (std::memcmp(&c->d_shadow, &d, sizeof(CellsDev)) != 0) {
        c->d_shadow = d;
        HIP_TRY(hipMemcpyAsync(c->d_dev, &c->d_shadow, sizeof(CellsDev), hipMemcpyHostToDevice, st));
      }
    }
    if (dom->dim == 2) vd_launch_fill_int(d.pcount, n, 0, st);
    if (opt.time_kernels) HIP_TRY(hipEventRecord(c->ev0, st));
    if (dom->dim == 3) vd_launch_sites3d(G, D, c->d_dev, wg, opt.monitor != 0, opt.use_density != 0, g->power, d.whole == 2, st);
    else vd_launch_surface(G, D, c->d_dev, wg, opt.use_density != 0, g->power, st);
    if (opt.time_kernels) HIP_TRY(hipEventRecord(c->ev1, st));
    HIP_TRY(hipGetLastError());
    if (opt.no_sync) {
      // stream-ordered only: finalize from the device counters, copy them to
      // pinned host memory, and check them in vd_cells_info
      c->pending = true;
      c->last_stream = st;
      c->carve_ms = c->split_ms = -1.0;
      vd_launch_finalize(c, st);
      HIP_TRY(hipMemcpyAsync(c->host_cnt, d.cnt, sizeof(unsigned long long) * CNT_N, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipGetLastError());
      c->status = VD_OK;
      *out = c;
      return VD_OK;
    }
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
    if (dom->dim == 3 && hc[CNT_ERR_CAP] && !hc[CNT_ERR_DEG] && !hc[CNT_ERR_LOC]) {
      // a cell that meets more tetrahedra, or has more neighbours, than the
      // per-wave overflow buffers hold: grow them (within about 4 GB each) and
      // run again; the LDS capacities of the polytope itself are fixed
      const unsigned long long stg = hc[CNT_STAGES];
      const unsigned long long growable = (1ull << VD_STAGE_SIMPLICES) | (1ull << VD_STAGE_NEIGHBOURS);
      const int64_t wmax = std::max<int64_t>(1, (int64_t)(1ll << 30) / std::max<int64_t>(c->cap_spill, 1));
      bool regrow = !(stg & ~growable);
      if (regrow && (stg & (1ull << VD_STAGE_SIMPLICES))) {
        const int64_t nw = std::min<int64_t>({(int64_t)c->q_spill_want * 4, dom->m, wmax});
        regrow = nw > c->q_spill_want;
        c->q_spill_want = (int)nw;
      }
      if (regrow && (stg & (1ull << VD_STAGE_NEIGHBOURS))) {
        const int64_t nw = std::min<int64_t>({(int64_t)c->nb_spill_want * 4, n, wmax});
        regrow = nw > c->nb_spill_want;
        c->nb_spill_want = (int)nw;
      }
      if (regrow) continue;
    }
    if (dom->dim == 2 && hc[CNT_ERR_CAP] && !hc[CNT_ERR_DEG] &&
        hc[CNT_STAGES] == (1ull << VD_STAGE_TRIANGLE_SITES)) {
      // a triangle meets more cells than its wave's site list holds: grow the
      // overflow (within about 4 GB) and run again
      const int64_t wmax = (int64_t)(1ll << 30) / std::max<int64_t>(wg, 1);
      const int64_t nw = std::min<int64_t>({std::max<int64_t>(4096, (int64_t)c->sq_spill_want * 4), n, wmax});
      if (nw > c->sq_spill_want) {
        c->sq_spill_want = (int)nw;
        continue;
      }
    }
    {
      const vd_status r = check_counts(c, false);
      if (r != VD_OK) {
        *out = c;
        return r;
      }
    }
    if (dom->dim == 2) {
      // a site's neighbours are distinct flags of its pieces' edges: the
      // edges written bound the neighbour lists' total (with room for a later
      // no-sync clip of moved sites, which cannot grow it)
      int64_t t = c->cap_nbr_csr;
      HIP_TRY(ensure(c->nbr, t, up((int64_t)hc[CNT_REAL_FACES])));
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
  hipFree(c->pid_tmp);
  hipFree(d.piece_simplex); hipFree(d.piece_nface); hipFree(d.piece_nvert); hipFree(d.piece_fstart);
  hipFree(d.piece_vstart); hipFree(d.piece_mass); hipFree(d.piece_mom); hipFree(d.piece_energy);
  hipFree(d.face_label); hipFree(d.vert_xyz); hipFree(d.vert_label); hipFree(d.fint); hipFree(d.seed);
  hipFree(c->piece_off); hipFree(c->nbr_off); hipFree(c->piece_id); hipFree(c->nbr); hipFree(c->scan_tmp);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->ev2) hipEventDestroy(c->ev2);
  hipFree(c->d_dev); hipFree(d.queue); hipFree(d.tq_spill); hipFree(d.saved);
  hipFree(c->outside);
  hipFree(d.nb_spill); hipFree(d.sq_spill); hipFree(c->order_buf);
  vd_cells_free(c->bcells);
  if (c->host_cnt) hipHostFree(c->host_cnt);
  hipFree(d.fint_lab); hipFree(d.piece_fint_start); hipFree(d.piece_nfint); hipFree(c->wbuf);
  delete c;
}

vd_status vd_cells_info(vd_cells c, vd_cells_info_t *info) {
  if (!c || !info) return fail(VD_ERR_INVALID_ARG, "vd_cells_info: NULL");
  if (c->pending) {
    // a no-sync clip (possibly replayed from a graph on another stream, which
    // the caller synchronises): its counters reach host_cnt in stream order
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    check_counts(c, true);
    c->pending = false;
  }
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
  info->overflow_records = (int64_t)hc[CNT_OVERFLOW];
  const bool mon = c->opt.monitor != 0;
  info->low_margin = mon ? (int64_t)hc[CNT_LOWMARGIN] : -1;
  {
    const unsigned long long b = hc[CNT_MINMARGIN];
    double mm;
    std::memcpy(&mm, &b, sizeof mm);
    info->min_margin = mon ? mm : -1.0;
  }
  info->query_rounds = mon ? (int64_t)hc[CNT_ROUNDS] : -1;
  info->corners_classified = mon ? (int64_t)hc[CNT_CLASSIFIED] : -1;
  info->corners_created = mon ? (int64_t)hc[CNT_NEWCORNERS] : -1;
  info->tests_wasted = mon ? (int64_t)hc[CNT_WASTED] : -1;
  info->fan_simplices = mon ? (int64_t)hc[CNT_FANTETS] : -1;
  info->sites_outside = c->sites_outside;
  info->boundary_seeded = c->used_bseeds ? 1 : 0;
  info->reserved_ = 0;
  return VD_OK;
}

vd_status vd_cells_view(vd_cells c, vd_cells_view_t *v) {
  if (!c || !v) return fail(VD_ERR_INVALID_ARG, "vd_cells_view: NULL");
  if (c->pending) {
    // the sizes of a no-sync clip are known once its counters have arrived
    const hipError_t q = hipStreamQuery(c->last_stream);
    if (q == hipErrorNotReady) return fail(VD_ERR_NOT_READY, "vd_cells_view: the no-sync clip has not finished");
    if (q != hipSuccess) return fail(VD_ERR_HIP, "vd_cells_view: %s", hipGetErrorString(q));
    check_counts(c, true);
    c->pending = false;
  }
  if (c->status != VD_OK) return fail((vd_status)c->status, "vd_cells_view: the clip failed (%s)", vd_status_string((vd_status)c->status));
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

// ---------------------------------------------------------------------------
// Allocation-free adjoint.  The adjoint's only scratch memory is the table of
// per-site weights (a_i, b_i, gE_i: 5 doubles per site), written by the first
// kernel and read by the second.  Here it lives in a fixed device array of
// VD_NOALLOC_MAX_SITES entries, one per GPU for the life of the process.  In
// host code the array's name is not a device address, so its address on each
// device is looked up once (hipGetSymbolAddress, that device current) and
// only that address is handed to the kernels.  The weights are fully
// rewritten by every call, so nothing needs clearing; calls that overlap on
// one GPU share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[5 * (int64_t)VD_NOALLOC_MAX_SITES];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {};  // per device: the address of `scratch`
}  // namespace

extern "C" {

vd_status vd_cell_moments_backward_noalloc(vd_cells c, const double *g_mass, const double *g_centroid,
                                           const double *g_energy, double *g_sites, void *stream) {
  if (!c || !g_sites) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward_noalloc: NULL argument");
  if (!c->opt.want_grad)
    return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward_noalloc: clip ran without want_grad");
  if (c->status != VD_OK) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward_noalloc: the clip failed");
  if (c->n > VD_NOALLOC_MAX_SITES)
    return fail(VD_ERR_CAPACITY, "vd_cell_moments_backward_noalloc: %lld sites exceed the fixed scratch of %d sites",
                (long long)c->n, (int)VD_NOALLOC_MAX_SITES);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(VD_ERR_INVALID_ARG, "vd_cell_moments_backward_noalloc: device %d", dev);
  double *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(VD_ERR_HIP, "vd_cell_moments_backward_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
      g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    ptr = g_scratch_ptr[dev];
  }
  vd_launch_backward(c, c->grid->view(), g_mass, g_centroid, g_energy, g_sites, ptr, as_stream(stream));
  HIP_TRY(hipGetLastError());
  return VD_OK;
}

}  // extern "C"
