// grid.hip -- uniform grid over the sites for nearest-site queries (Sec. 6.2).
//
// Counting sort in five HBM-bound launches: bounding box, per-site cell id +
// histogram, exclusive scan, scatter into cell order, and an in-cell sort by
// the caller's index so the layout is deterministic.  A sixth launch computes
// delta_i = half the distance to the nearest other site (Sec. 6.1).
//
// A batch of diagrams is sorted in one pass: diagram b has its own bounding
// box and cell block [cell_off[b], cell_off[b+1]) of the shared offsets, so
// its sites land on the sorted positions [site_off[b], site_off[b+1]).
#include "vd_internal.h"
#include "vd_scan.h"

namespace {

constexpr int kB = 256;

__global__ void __launch_bounds__(kB) bbox_partial(const double *__restrict__ s, long long n,
                                                   double *__restrict__ part) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (long long i = (long long)blockIdx.x * kB + threadIdx.x; i < n; i += (long long)gridDim.x * kB) {
    for (int k = 0; k < 3; k++) {
      const double x = s[3 * i + k];
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  }
  __shared__ double red[6][kB];
  for (int k = 0; k < 3; k++) { red[k][threadIdx.x] = lo[k]; red[3 + k][threadIdx.x] = hi[k]; }
  __syncthreads();
  for (int d = kB / 2; d > 0; d >>= 1) {
    if (threadIdx.x < (unsigned)d)
      for (int k = 0; k < 3; k++) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + d]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + d]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// bounding box of each diagram's sites: one block per diagram
__global__ void __launch_bounds__(kB) bbox_seg(const double *__restrict__ s, const long long *__restrict__ off,
                                               double *__restrict__ part) {
  const int b = blockIdx.x;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (long long i = off[b] + threadIdx.x; i < off[b + 1]; i += kB) {
    for (int k = 0; k < 3; k++) {
      const double x = s[3 * i + k];
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  }
  __shared__ double red[6][kB];
  for (int k = 0; k < 3; k++) { red[k][threadIdx.x] = lo[k]; red[3 + k][threadIdx.x] = hi[k]; }
  __syncthreads();
  for (int d = kB / 2; d > 0; d >>= 1) {
    if (threadIdx.x < (unsigned)d)
      for (int k = 0; k < 3; k++) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + d]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + d]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * b + threadIdx.x] = red[threadIdx.x][0];
}

// Geometry of diagram b (thread b): the union of its sites' box (ppd partial
// boxes) and the caller's box (user, nullable), padded so points on the upper
// faces fall inside the last cells; h = extent / cells.
__global__ void grid_geom(const double *__restrict__ part, int ppd, int nb, const double *__restrict__ user,
                          const int *__restrict__ dims, double *__restrict__ geom) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double lo[3], hi[3];
  for (int k = 0; k < 3; k++) {
    lo[k] = user ? user[6 * b + k] : 1e300;
    hi[k] = user ? user[6 * b + 3 + k] : -1e300;
  }
  for (int q = 0; q < ppd; q++)
    for (int k = 0; k < 3; k++) {
      lo[k] = fmin(lo[k], part[6 * (b * ppd + q) + k]);
      hi[k] = fmax(hi[k], part[6 * (b * ppd + q) + 3 + k]);
    }
  double ext = 0;
  for (int k = 0; k < 3; k++) ext = fmax(ext, hi[k] - lo[k]);
  if (!(ext > 0)) ext = 1.0;
  for (int k = 0; k < 3; k++) {
    double e = hi[k] - lo[k];
    if (!(e > 1e-12 * ext)) e = 1e-12 * ext;
    const double pad = 1e-9 * e;
    const double l = lo[k] - pad;
    const double h = (e + 2 * pad) / dims[3 * b + k];
    geom[9 * b + k] = l;
    geom[9 * b + 3 + k] = h;
    geom[9 * b + 6 + k] = 1.0 / h;
  }
}

// diagram of every caller index
__global__ void __launch_bounds__(kB) site_diag(long long n, const long long *__restrict__ off, int nb,
                                                int *__restrict__ diag) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i < n) diag[i] = diagram_of(off, nb, i);
}

__global__ void __launch_bounds__(kB) grid_hist(const double *__restrict__ s, long long n,
                                                const int *__restrict__ diag, const double *__restrict__ geom_all,
                                                const int *__restrict__ dims, const long long *__restrict__ cell_off,
                                                int *__restrict__ cellid, int *__restrict__ count) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int b = diag ? diag[i] : 0;
  const double *geom = geom_all + 9 * b;
  const int gx = dims[3 * b], gy = dims[3 * b + 1], gz = dims[3 * b + 2];
  const int cx = cell_coord(s[3 * i + 0], geom[0], geom[6], gx);
  const int cy = cell_coord(s[3 * i + 1], geom[1], geom[7], gy);
  const int cz = cell_coord(s[3 * i + 2], geom[2], geom[8], gz);
  const int c = (int)cell_off[b] + cx + gx * (cy + gy * cz);
  cellid[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void __launch_bounds__(kB) grid_scatter(const double *__restrict__ s, long long n,
                                                   const int *__restrict__ cellid,
                                                   const int *__restrict__ cstart, int *__restrict__ fill,
                                                   double *__restrict__ sx, double *__restrict__ sy,
                                                   double *__restrict__ sz, int *__restrict__ perm) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int c = cellid[i];
  const int p = cstart[c] + atomicAdd(&fill[c], 1);
  sx[p] = s[3 * i + 0];
  sy[p] = s[3 * i + 1];
  sz[p] = s[3 * i + 2];
  perm[p] = (int)i;
}

// Order the sites of each cell by the caller's index (insertion sort; cells
// hold a handful of sites at the target density).
__global__ void __launch_bounds__(kB) grid_sort_cells(long long ncell, const int *__restrict__ cstart,
                                                      double *__restrict__ sx, double *__restrict__ sy,
                                                      double *__restrict__ sz, int *__restrict__ perm) {
  const long long c = (long long)blockIdx.x * kB + threadIdx.x;
  if (c >= ncell) return;
  const int a = cstart[c], b = cstart[c + 1];
  for (int i = a + 1; i < b; i++) {
    const int key = perm[i];
    const double x = sx[i], y = sy[i], z = sz[i];
    int j = i - 1;
    while (j >= a && perm[j] > key) {
      perm[j + 1] = perm[j]; sx[j + 1] = sx[j]; sy[j + 1] = sy[j]; sz[j + 1] = sz[j];
      j--;
    }
    perm[j + 1] = key; sx[j + 1] = x; sy[j + 1] = y; sz[j + 1] = z;
  }
}

__global__ void __launch_bounds__(kB) grid_rank(long long n, const int *__restrict__ perm,
                                                int *__restrict__ rank) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p < n) rank[perm[p]] = (int)p;
}

__global__ void __launch_bounds__(kB) grid_delta(GridView G, double *__restrict__ delta) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p >= G.n) return;
  double d2;
  const GridView Gb = grid_of(G, p);
  const int k = nn_thread(Gb, G.sx[p], G.sy[p], G.sz[p], (int)p, d2);
  delta[p] = k >= 0 ? 0.5 * sqrt(d2) : 1e300;
}

inline unsigned blocks(long long n) { return (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1); }

// Power weights in sorted order, and eta = max w (one block, fixed reduction
// order); flags[0] is set for a weight that is not finite.
__global__ void __launch_bounds__(kB) weights_gather(long long n, const int *__restrict__ perm,
                                                     const double *__restrict__ w, double *__restrict__ sw,
                                                     int *__restrict__ flags) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p >= n) return;
  const double x = w[perm[p]];
  if (!isfinite(x)) atomicOr(&flags[0], 1);
  sw[p] = x;
}

__global__ void __launch_bounds__(kB) weights_max(long long n, const double *__restrict__ sw, double *__restrict__ eta) {
  double m = -1e300;
  for (long long p = threadIdx.x; p < n; p += kB) m = fmax(m, sw[p]);
  __shared__ double red[kB];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int d = kB / 2; d > 0; d >>= 1) {
    if (threadIdx.x < (unsigned)d) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) eta[0] = red[0];
}

// the lifted coordinate h_i = sqrt(eta - w_i) of Sec. 7.3 (eta = max w, the
// smallest admissible constant)
__global__ void __launch_bounds__(kB) weights_lift(long long n, const double *__restrict__ sw,
                                                   const double *__restrict__ eta, double *__restrict__ sh) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p < n) sh[p] = sqrt(fmax(eta[0] - sw[p], 0.0));
}

}  // namespace

void vd_launch_grid_weights(vd_grid g, const double *w, int *flags, hipStream_t st) {
  const long long n = g->n;
  hipLaunchKernelGGL(weights_gather, dim3(blocks(n)), dim3(kB), 0, st, n, (const int *)g->perm, w, g->sw, flags);
  hipLaunchKernelGGL(weights_max, dim3(1), dim3(kB), 0, st, n, (const double *)g->sw, g->eta);
  hipLaunchKernelGGL(weights_lift, dim3(blocks(n)), dim3(kB), 0, st, n, (const double *)g->sw,
                     (const double *)g->eta, g->sh);
}

void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st);

void vd_launch_grid_build(vd_grid g, const double *sites, const double *user_box, hipStream_t st) {
  const long long n = g->n;
  const int nb = g->nb;
  int ppd;
  if (nb == 1) {
    ppd = 256;
    hipLaunchKernelGGL(bbox_partial, dim3(ppd), dim3(kB), 0, st, sites, n, g->bbox_part);
  } else {
    ppd = 1;
    hipLaunchKernelGGL(bbox_seg, dim3(nb), dim3(kB), 0, st, sites, (const long long *)g->d_site_off, g->bbox_part);
    hipLaunchKernelGGL(site_diag, dim3(blocks(n)), dim3(kB), 0, st, n, (const long long *)g->d_site_off, nb, g->diag);
  }
  hipLaunchKernelGGL(grid_geom, dim3((nb + 63) / 64), dim3(64), 0, st, (const double *)g->bbox_part, ppd, nb,
                     user_box, (const int *)g->d_dims, g->geom);
  vd_launch_fill_int(g->ccount, g->ncell, 0, st);
  vd_launch_fill_int(g->fill, g->ncell, 0, st);
  hipLaunchKernelGGL(grid_hist, dim3(blocks(n)), dim3(kB), 0, st, sites, n, nb == 1 ? (const int *)nullptr : g->diag,
                     (const double *)g->geom, (const int *)g->d_dims, (const long long *)g->d_cell_off, g->cellid,
                     g->ccount);
  vdscan::exclusive_scan<int, int>(g->ccount, g->ncell, g->cstart, g->scan_tmp, st);
  hipLaunchKernelGGL(grid_scatter, dim3(blocks(n)), dim3(kB), 0, st, sites, n, (const int *)g->cellid,
                     (const int *)g->cstart, g->fill, g->sx, g->sy, g->sz, g->perm);
  hipLaunchKernelGGL(grid_sort_cells, dim3(blocks(g->ncell)), dim3(kB), 0, st, (long long)g->ncell,
                     (const int *)g->cstart, g->sx, g->sy, g->sz, g->perm);
  hipLaunchKernelGGL(grid_rank, dim3(blocks(n)), dim3(kB), 0, st, n, (const int *)g->perm, g->rank);
  g->delta_valid = false;
}

// delta_i of every site (only the improved search of Sec. 6.1 reads it)
void vd_launch_grid_delta(vd_grid g, hipStream_t st) {
  hipLaunchKernelGGL(grid_delta, dim3(blocks(g->n)), dim3(kB), 0, st, g->view(), g->delta);
  g->delta_valid = true;
}
