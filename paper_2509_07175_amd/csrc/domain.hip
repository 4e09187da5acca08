// domain.hip -- domain staging (Sec. 3.1: M = {T_a}) and site location.
//
// vd_domain_create copies the simplices, validates them (index range, positive
// tetrahedron volume) and builds a uniform point-location grid whose cells list
// every tetrahedron whose bounding box overlaps them.  Each site's seed
// tetrahedron (the one containing it) is then found by barycentric tests over
// one cell's list; the lowest containing index wins, so the result does not
// depend on atomic ordering.
#include "vd_internal.h"
#include "vd_scan.h"

namespace {

constexpr int kB = 256;

inline unsigned blocks(long long n) { return (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1); }

__global__ void __launch_bounds__(kB) fill_int(int *__restrict__ p, long long n, int v) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i < n) p[i] = v;
}

// flags[0]: bad index; flags[1]: non-positive tet volume / degenerate triangle.
// measure[]: per-simplex volume or area (summed on the host).
__global__ void __launch_bounds__(kB) validate(DomainView D, int *__restrict__ flags,
                                               double *__restrict__ measure) {
  const long long a = (long long)blockIdx.x * kB + threadIdx.x;
  if (a >= D.m) return;
  const int k = D.dim + 1;
  for (int u = 0; u < k; u++) {
    const int v = D.simp[a * k + u], b = D.adj[a * k + u];
    if (v < 0 || v >= D.nv || b < -1 || b >= D.m) { atomicOr(&flags[0], 1); measure[a] = 0; return; }
  }
  const double *p0 = &D.verts[3 * (long long)D.simp[a * k + 0]];
  const double *p1 = &D.verts[3 * (long long)D.simp[a * k + 1]];
  const double *p2 = &D.verts[3 * (long long)D.simp[a * k + 2]];
  const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
  double mval;
  if (D.dim == 3) {
    const double *p3 = &D.verts[3 * (long long)D.simp[a * k + 3]];
    const double e3[3] = {p3[0] - p0[0], p3[1] - p0[1], p3[2] - p0[2]};
    mval = (cr[0] * e3[0] + cr[1] * e3[1] + cr[2] * e3[2]) / 6.0;
  } else {
    mval = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  }
  if (!(mval > 0.0)) atomicOr(&flags[1], 1);
  measure[a] = mval;
}

__global__ void __launch_bounds__(kB) vert_bbox(const double *__restrict__ v, long long nv,
                                                double *__restrict__ out) {
  if (blockIdx.x != 0) return;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (long long i = threadIdx.x; i < nv; i += kB)
    for (int k = 0; k < 3; k++) { lo[k] = fmin(lo[k], v[3 * i + k]); hi[k] = fmax(hi[k], v[3 * i + k]); }
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
  if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ void tet_cell_range(const DomainView &D, long long a, int *c0, int *c1) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int u = 0; u < 4; u++) {
    const double *p = &D.verts[3 * (long long)D.simp[a * 4 + u]];
    for (int k = 0; k < 3; k++) { lo[k] = fmin(lo[k], p[k]); hi[k] = fmax(hi[k], p[k]); }
  }
  for (int k = 0; k < 3; k++) {
    c0[k] = cell_coord(lo[k], D.lgeom[k], D.lgeom[6 + k], D.lg[k]);
    c1[k] = cell_coord(hi[k], D.lgeom[k], D.lgeom[6 + k], D.lg[k]);
  }
}

__global__ void __launch_bounds__(kB) loc_count(DomainView D, int *__restrict__ count) {
  const long long a = (long long)blockIdx.x * kB + threadIdx.x;
  if (a >= D.m) return;
  int c0[3], c1[3];
  tet_cell_range(D, a, c0, c1);
  for (int z = c0[2]; z <= c1[2]; z++)
    for (int y = c0[1]; y <= c1[1]; y++)
      for (int x = c0[0]; x <= c1[0]; x++) atomicAdd(&count[x + D.lg[0] * (y + D.lg[1] * z)], 1);
}

__global__ void __launch_bounds__(kB) loc_fill(DomainView D, const int *__restrict__ start,
                                               int *__restrict__ fill, int *__restrict__ items) {
  const long long a = (long long)blockIdx.x * kB + threadIdx.x;
  if (a >= D.m) return;
  int c0[3], c1[3];
  tet_cell_range(D, a, c0, c1);
  for (int z = c0[2]; z <= c1[2]; z++)
    for (int y = c0[1]; y <= c1[1]; y++)
      for (int x = c0[0]; x <= c1[0]; x++) {
        const int c = x + D.lg[0] * (y + D.lg[1] * z);
        items[start[c] + atomicAdd(&fill[c], 1)] = (int)a;
      }
}

// Seed tetrahedron of each site (by sorted position): lowest index among the
// tetrahedra of its location cell whose barycentric coordinates are all
// >= -1e-12 (relative).
__global__ void __launch_bounds__(kB) locate_sites(GridView G, DomainView D, int *__restrict__ seed,
                                                   unsigned long long *__restrict__ cnt) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p >= G.n) return;
  const double q[3] = {G.sx[p], G.sy[p], G.sz[p]};
  int cc[3];
  for (int k = 0; k < 3; k++) cc[k] = cell_coord(q[k], D.lgeom[k], D.lgeom[6 + k], D.lg[k]);
  const int c = cc[0] + D.lg[0] * (cc[1] + D.lg[1] * cc[2]);
  int best = -1;
  for (int t = D.lstart[c]; t < D.lstart[c + 1]; t++) {
    const int a = D.litems[t];
    if (best >= 0 && a >= best) continue;
    const double *P[4];
    for (int u = 0; u < 4; u++) P[u] = &D.verts[3 * (long long)D.simp[(long long)a * 4 + u]];
    double vol6;
    {
      const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
      const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
      const double e3[3] = {P[3][0] - P[0][0], P[3][1] - P[0][1], P[3][2] - P[0][2]};
      vol6 = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
             e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    }
    bool in = true;
    for (int f = 0; f < 4 && in; f++) {
      // replace vertex f by q: signed volume of the sub-tetrahedron
      const double *R[4] = {P[0], P[1], P[2], P[3]};
      R[f] = q;
      const double e1[3] = {R[1][0] - R[0][0], R[1][1] - R[0][1], R[1][2] - R[0][2]};
      const double e2[3] = {R[2][0] - R[0][0], R[2][1] - R[0][1], R[2][2] - R[0][2]};
      const double e3[3] = {R[3][0] - R[0][0], R[3][1] - R[0][1], R[3][2] - R[0][2]};
      const double v = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                       e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
      if (v < -1e-12 * vol6) in = false;
    }
    if (in) best = a;
  }
  seed[p] = best;
  if (best < 0) {
    atomicAdd(&cnt[CNT_ERR_LOC], 1ull);
    atomicMin((int *)&cnt[CNT_BAD_SITE], G.perm[p]);
  }
}

}  // namespace

void vd_launch_domain_locator(vd_domain d, hipStream_t st) {
  DomainView D = d->view();
  const long long ncell = (long long)d->lg[0] * d->lg[1] * d->lg[2];
  hipLaunchKernelGGL(fill_int, dim3(blocks(ncell)), dim3(kB), 0, st, d->lcount, ncell, 0);
  hipLaunchKernelGGL(fill_int, dim3(blocks(ncell)), dim3(kB), 0, st, d->lfill, ncell, 0);
  hipLaunchKernelGGL(loc_count, dim3(blocks(d->m)), dim3(kB), 0, st, D, d->lcount);
  vdscan::exclusive_scan<int, int>(d->lcount, ncell, d->lstart, d->scan_tmp, st);
}

void vd_launch_domain_fill(vd_domain d, hipStream_t st) {
  DomainView D = d->view();
  hipLaunchKernelGGL(loc_fill, dim3(blocks(d->m)), dim3(kB), 0, st, D, (const int *)d->lstart, d->lfill,
                     d->litems);
}

void vd_launch_domain_validate(vd_domain d, int *flags, double *measure, hipStream_t st) {
  hipLaunchKernelGGL(validate, dim3(blocks(d->m)), dim3(kB), 0, st, d->view(), flags, measure);
}

void vd_launch_vert_bbox(vd_domain d, double *out, hipStream_t st) {
  hipLaunchKernelGGL(vert_bbox, dim3(1), dim3(kB), 0, st, (const double *)d->verts, (long long)d->nv, out);
}

void vd_launch_locate_sites(const GridView &G, const DomainView &D, int *seed, unsigned long long *cnt,
                            hipStream_t st) {
  hipLaunchKernelGGL(locate_sites, dim3(blocks(G.n)), dim3(kB), 0, st, G, D, seed, cnt);
}

void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_int, dim3(blocks(n)), dim3(kB), 0, st, p, n, v);
}
