// domain.hip -- domain staging (Sec. 3.1: M = {T_a}) and site location.
//
// vd_domain_create copies the simplices, validates them (index range, positive
// tetrahedron volume) and builds a uniform point-location grid whose cells list
// every tetrahedron whose bounding box overlaps them.  Each site's seed
// tetrahedron (the one containing it) is then found by barycentric tests over
// one cell's list; the lowest containing index wins, so the result does not
// depend on atomic ordering.
//
// A batch of domains is staged as one disjoint union: local vertex and simplex
// indices are shifted by the diagram's offsets, and each diagram gets its own
// bounding box and location grid (a block of the shared cell offsets).
#include "vd_internal.h"
#include "vd_scan.h"

namespace {

constexpr int kB = 256;

inline unsigned blocks(long long n) { return (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1); }

__global__ void __launch_bounds__(kB) fill_int(int *__restrict__ p, long long n, int v) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i < n) p[i] = v;
}

// Shift diagram-local indices to global ones and check their range:
// vertex indices in [0, nv_b), adjacency in [-1, m_b).  flags[0] set on error.
__global__ void __launch_bounds__(kB) offset_indices(int *__restrict__ simp, int *__restrict__ adj, long long m,
                                                     int k, int nb, const long long *__restrict__ simp_off,
                                                     const long long *__restrict__ vert_off, int *__restrict__ flags) {
  const long long a = (long long)blockIdx.x * kB + threadIdx.x;
  if (a >= m) return;
  const int b = diagram_of(simp_off, nb, a);
  const long long vo = vert_off[b], nvb = vert_off[b + 1] - vo, so = simp_off[b], mb = simp_off[b + 1] - so;
  for (int u = 0; u < k; u++) {
    const int v = simp[a * k + u], w = adj[a * k + u];
    if (v < 0 || v >= nvb || w < -1 || w >= mb) { atomicOr(&flags[0], 1); return; }
    simp[a * k + u] = (int)(v + vo);
    adj[a * k + u] = w < 0 ? -1 : (int)(w + so);
  }
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

// vertex bounding box of each diagram (one block per diagram)
__global__ void __launch_bounds__(kB) vert_bbox(const double *__restrict__ v, const long long *__restrict__ vert_off,
                                                double *__restrict__ out_all) {
  const int b = blockIdx.x;
  double *out = out_all + 6 * b;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (long long i = vert_off[b] + threadIdx.x; i < vert_off[b + 1]; i += kB)
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

// location cells of diagram b overlapped by the bounding box of tetrahedron a
__device__ __forceinline__ void tet_cell_range(const double *__restrict__ verts, const int *__restrict__ simp,
                                               long long a, const double *lgeom, const int *lg, int *c0, int *c1) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int u = 0; u < 4; u++) {
    const double *p = &verts[3 * (long long)simp[a * 4 + u]];
    for (int k = 0; k < 3; k++) { lo[k] = fmin(lo[k], p[k]); hi[k] = fmax(hi[k], p[k]); }
  }
  for (int k = 0; k < 3; k++) {
    c0[k] = cell_coord(lo[k], lgeom[k], lgeom[6 + k], lg[k]);
    c1[k] = cell_coord(hi[k], lgeom[k], lgeom[6 + k], lg[k]);
  }
}

struct LocArgs {
  const double *verts;
  const int *simp;
  long long m;
  int nb;
  const long long *simp_off, *loc_off;
  const double *lgeom;  // [9 nb]
  const int *lg;        // [3 nb]
};

__global__ void __launch_bounds__(kB) loc_count(LocArgs L, int *__restrict__ count) {
  const long long a = (long long)blockIdx.x * kB + threadIdx.x;
  if (a >= L.m) return;
  const int b = diagram_of(L.simp_off, L.nb, a);
  const int *lg = L.lg + 3 * b;
  int c0[3], c1[3];
  tet_cell_range(L.verts, L.simp, a, L.lgeom + 9 * b, lg, c0, c1);
  int *cnt = count + L.loc_off[b];
  for (int z = c0[2]; z <= c1[2]; z++)
    for (int y = c0[1]; y <= c1[1]; y++)
      for (int x = c0[0]; x <= c1[0]; x++) atomicAdd(&cnt[x + lg[0] * (y + lg[1] * z)], 1);
}

__global__ void __launch_bounds__(kB) loc_fill(LocArgs L, const int *__restrict__ start, int *__restrict__ fill,
                                               int *__restrict__ items) {
  const long long a = (long long)blockIdx.x * kB + threadIdx.x;
  if (a >= L.m) return;
  const int b = diagram_of(L.simp_off, L.nb, a);
  const int *lg = L.lg + 3 * b;
  int c0[3], c1[3];
  tet_cell_range(L.verts, L.simp, a, L.lgeom + 9 * b, lg, c0, c1);
  const long long base = L.loc_off[b];
  for (int z = c0[2]; z <= c1[2]; z++)
    for (int y = c0[1]; y <= c1[1]; y++)
      for (int x = c0[0]; x <= c1[0]; x++) {
        const long long c = base + x + lg[0] * (y + lg[1] * z);
        items[start[c] + atomicAdd(&fill[c], 1)] = (int)a;
      }
}

// Seed tetrahedron of each site (by sorted position): lowest index among the
// tetrahedra of its location cell whose barycentric coordinates are all
// >= -1e-12 (relative).
__global__ void __launch_bounds__(kB) locate_sites(GridView G, DomainView Dall, int *__restrict__ seed,
                                                   unsigned long long *__restrict__ cnt) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p >= G.n) return;
  const DomainView D = domain_of(Dall, G.nb > 1 ? diagram_of(G.site_off, G.nb, p) : 0);
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

namespace {
LocArgs loc_args(vd_domain d) {
  LocArgs L;
  L.verts = d->verts; L.simp = d->simp; L.m = d->m; L.nb = d->nb;
  L.simp_off = d->d_simp_off; L.loc_off = d->d_loc_off; L.lgeom = d->lgeom; L.lg = d->d_lg;
  return L;
}
}  // namespace

void vd_launch_domain_locator(vd_domain d, hipStream_t st) {
  const long long ncell = d->ncell;
  hipLaunchKernelGGL(fill_int, dim3(blocks(ncell)), dim3(kB), 0, st, d->lcount, ncell, 0);
  hipLaunchKernelGGL(fill_int, dim3(blocks(ncell)), dim3(kB), 0, st, d->lfill, ncell, 0);
  hipLaunchKernelGGL(loc_count, dim3(blocks(d->m)), dim3(kB), 0, st, loc_args(d), d->lcount);
  vdscan::exclusive_scan<int, int>(d->lcount, ncell, d->lstart, d->scan_tmp, st);
}

void vd_launch_domain_fill(vd_domain d, hipStream_t st) {
  hipLaunchKernelGGL(loc_fill, dim3(blocks(d->m)), dim3(kB), 0, st, loc_args(d), (const int *)d->lstart, d->lfill,
                     d->litems);
}

void vd_launch_domain_offsets(vd_domain d, int *flags, hipStream_t st) {
  hipLaunchKernelGGL(offset_indices, dim3(blocks(d->m)), dim3(kB), 0, st, d->simp, d->adj, (long long)d->m,
                     d->dim + 1, d->nb, (const long long *)d->d_simp_off, (const long long *)d->d_vert_off, flags);
}

void vd_launch_domain_validate(vd_domain d, int *flags, double *measure, hipStream_t st) {
  hipLaunchKernelGGL(validate, dim3(blocks(d->m)), dim3(kB), 0, st, d->view(), flags, measure);
}

void vd_launch_vert_bbox(vd_domain d, double *out, hipStream_t st) {
  hipLaunchKernelGGL(vert_bbox, dim3(d->nb), dim3(kB), 0, st, (const double *)d->verts,
                     (const long long *)d->d_vert_off, out);
}

void vd_launch_locate_sites(const GridView &G, const DomainView &D, int *seed, unsigned long long *cnt,
                            hipStream_t st) {
  hipLaunchKernelGGL(locate_sites, dim3(blocks(G.n)), dim3(kB), 0, st, G, D, seed, cnt);
}

void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_int, dim3(blocks(n)), dim3(kB), 0, st, p, n, v);
}
