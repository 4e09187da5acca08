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
// >= -1e-12 (relative); -1 for a site outside M (counted in outside[0]; the
// lowest such caller index in outside[1], which starts at INT_MAX).
// the tetrahedra of each location cell in ascending index order, so that a
// scan for the lowest-index tetrahedron containing a point stops at its
// first hit (insertion sort: a cell lists a few tetrahedra)
__global__ void __launch_bounds__(kB) loc_sort(const int *__restrict__ start, long long ncell, int *__restrict__ items) {
  const long long c = (long long)blockIdx.x * kB + threadIdx.x;
  if (c >= ncell) return;
  const int a = start[c], b = start[c + 1];
  for (int x = a + 1; x < b; x++) {
    const int v = items[x];
    int y = x - 1;
    while (y >= a && items[y] > v) { items[y + 1] = items[y]; y--; }
    items[y + 1] = v;
  }
}

__global__ void __launch_bounds__(kB) locate_sites(GridView G, DomainView Dall, int *__restrict__ seed,
                                                   int *__restrict__ outside) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  if (p >= G.n) return;
  const DomainView D = domain_of(Dall, G.nb > 1 ? diagram_of(G.site_off, G.nb, p) : 0);
  const double q[3] = {G.sx[p], G.sy[p], G.sz[p]};
  if (!(isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]))) {
    // outside[4] counts sites with a coordinate that is not finite, outside[5]
    // holds the lowest such caller index
    atomicAdd(&outside[4], 1);
    atomicMin(&outside[5], G.perm[p]);
    seed[p] = -1;
    return;
  }
  int cc[3];
  for (int k = 0; k < 3; k++) cc[k] = cell_coord(q[k], D.lgeom[k], D.lgeom[6 + k], D.lg[k]);
  const int c = cc[0] + D.lg[0] * (cc[1] + D.lg[1] * cc[2]);
  int best = -1;
  // the cell's tetrahedra in ascending order: the first that holds q is the lowest
  for (int t = D.lstart[c]; t < D.lstart[c + 1] && best < 0; t++) {
    const int a = D.litems[t];
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
    // outside every tetrahedron: outside[0] counts them, outside[1] the lowest caller index
    atomicAdd(&outside[0], 1);
    atomicMin(&outside[1], G.perm[p]);
  }
  // an exact copy of this site (the same point, and for a power diagram the
  // same weight) sits in the same grid cell: outside[2] counts the copies with
  // a higher caller index, outside[3] holds the lowest such index
  const GridView Gb = G.nb > 1 ? G.views[diagram_of(G.site_off, G.nb, p)] : G;
  int gc[3];
  for (int k = 0; k < 3; k++) gc[k] = cell_coord(q[k], Gb.geom[k], Gb.geom[6 + k], Gb.g[k]);
  const int gcell = gc[0] + Gb.g[0] * (gc[1] + Gb.g[1] * gc[2]);
  const int me = G.perm[p];
  for (int t = Gb.cstart[gcell]; t < Gb.cstart[gcell + 1]; t++) {
    if (t == p || G.sx[t] != q[0] || G.sy[t] != q[1] || G.sz[t] != q[2]) continue;
    if (G.sh && G.sh[t] != G.sh[p]) continue;
    if (G.perm[t] > me) {
      atomicAdd(&outside[2], 1);
      atomicMin(&outside[3], G.perm[t]);
    }
  }
}

// ---------------------------------------------------------------------------
// Adjacency from the simplices (Sec. 3.2: a face shared by T_a and T_b is
// flagged -(b+1) in T_a).  Face f of simplex a (the facet opposite vertex f) is
// bucketed by its smallest vertex index (counting sort: histogram, scan,
// scatter); a face then looks for the face with the same vertex set in its own
// bucket.  Buckets hold the faces around one vertex, so the pairwise search is
// short.  A face matched by more than one other face (a non-manifold mesh)
// sets flags[0].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void face_verts(const int *__restrict__ simp, int k, long long a, int f, int *w) {
  int c = 0;
  for (int u = 0; u < k; u++)
    if (u != f) w[c++] = simp[a * k + u];
  // sort the k-1 (2 or 3) vertex ids
  for (int i = 0; i < k - 1; i++)
    for (int j = i + 1; j < k - 1; j++)
      if (w[j] < w[i]) { const int t = w[i]; w[i] = w[j]; w[j] = t; }
}

__global__ void __launch_bounds__(kB) adj_count(const int *__restrict__ simp, long long m, int k, int *__restrict__ count) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x >= m * k) return;
  int w[3] = {0, 0, 0};
  face_verts(simp, k, x / k, (int)(x % k), w);
  atomicAdd(&count[w[0]], 1);
}

__global__ void __launch_bounds__(kB) adj_scatter(const int *__restrict__ simp, long long m, int k,
                                                  const int *__restrict__ start, int *__restrict__ fill,
                                                  int *__restrict__ items) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x >= m * k) return;
  int w[3] = {0, 0, 0};
  face_verts(simp, k, x / k, (int)(x % k), w);
  items[start[w[0]] + atomicAdd(&fill[w[0]], 1)] = (int)x;
}

__global__ void __launch_bounds__(kB) adj_match(const int *__restrict__ simp, long long m, int k,
                                                const int *__restrict__ start, const int *__restrict__ items,
                                                int *__restrict__ adj, int *__restrict__ flags) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x >= m * k) return;
  const long long a = x / k;
  int w[3] = {0, 0, 0};
  face_verts(simp, k, a, (int)(x % k), w);
  int other = -1, matches = 0;
  for (int t = start[w[0]]; t < start[w[0] + 1]; t++) {
    const int y = items[t];
    if (y == (int)x) continue;
    int z[3] = {0, 0, 0};
    face_verts(simp, k, y / k, y % k, z);
    if (z[0] == w[0] && z[1] == w[1] && (k == 3 || z[2] == w[2])) {
      matches++;
      other = y / k;
    }
  }
  if (matches > 1 || other == (int)a) atomicOr(&flags[0], 1);
  adj[x] = matches == 1 ? other : -1;
}

// ---------------------------------------------------------------------------
// Convexity of each tetrahedral domain.  M is convex iff every vertex of its
// boundary lies on the inner side of the plane of every boundary face: then M
// is contained in the intersection K of those half-spaces, and a segment from
// the interior of M to a point of K outside M would have to leave M through a
// boundary face and so leave K too.  The extreme points of M are boundary
// vertices, so testing those is enough.  One thread per boundary face tests
// its diagram's boundary vertices (relative tolerance 1e-10 of the diagram's
// extent); a violation clears convex[b].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kB) bnd_mark(const int *__restrict__ simp, const int *__restrict__ adj, long long m,
                                               int *__restrict__ on_bnd) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x >= m * 4) return;
  if (adj[x] >= 0) return;
  const long long a = x / 4;
  const int f = (int)(x % 4);
  for (int u = 0; u < 4; u++)
    if (u != f) on_bnd[simp[a * 4 + u]] = 1;
}

__global__ void __launch_bounds__(kB) bnd_collect(const int *__restrict__ on_bnd, const int *__restrict__ pos,
                                                  long long nv, int *__restrict__ list) {
  const long long v = (long long)blockIdx.x * kB + threadIdx.x;
  if (v < nv && on_bnd[v]) list[pos[v]] = (int)v;
}

__global__ void __launch_bounds__(kB) convex_check(DomainView D, const int *__restrict__ pos,
                                                   const int *__restrict__ list, const long long *__restrict__ vert_off,
                                                   const double *__restrict__ bbox, int *__restrict__ convex) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x >= (long long)D.m * 4) return;
  if (D.adj[x] >= 0) return;
  const long long a = x / 4;
  const int f = (int)(x % 4);
  const int b = D.nb > 1 ? diagram_of(D.simp_off, D.nb, a) : 0;
  if (!convex[b]) return;
  // face f opposite vertex f, oriented outward for a positively oriented tet
  const unsigned loops = (1u | 2u << 2 | 3u << 4) | (0u | 3u << 2 | 2u << 4) << 6 |
                         (0u | 1u << 2 | 3u << 4) << 12 | (0u | 2u << 2 | 1u << 4) << 18;
  const unsigned lf = loops >> (6 * f);
  const double *pA = &D.verts[3 * (long long)D.simp[a * 4 + (lf & 3)]];
  const double *pB = &D.verts[3 * (long long)D.simp[a * 4 + ((lf >> 2) & 3)]];
  const double *pC = &D.verts[3 * (long long)D.simp[a * 4 + ((lf >> 4) & 3)]];
  const double ab[3] = {pB[0] - pA[0], pB[1] - pA[1], pB[2] - pA[2]};
  const double ac[3] = {pC[0] - pA[0], pC[1] - pA[1], pC[2] - pA[2]};
  const double n[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
  const double *bx = &bbox[6 * b];
  const double ext = fmax(fmax(bx[3] - bx[0], bx[4] - bx[1]), bx[5] - bx[2]);
  const double tol = 1e-10 * ext * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int t = pos[vert_off[b]]; t < pos[vert_off[b + 1]]; t++) {
    const double *p = &D.verts[3 * (long long)list[t]];
    const double s = n[0] * (p[0] - pA[0]) + n[1] * (p[1] - pA[1]) + n[2] * (p[2] - pA[2]);
    if (s > tol) { convex[b] = 0; return; }
  }
}

// ---------------------------------------------------------------------------
// Boundary surface of a tetrahedral domain: every face without a neighbour
// becomes a triangle, oriented outward (the loop of face f of a positively
// oriented tetrahedron), with diagram-local vertex indices; btet[t] is the
// (global) tetrahedron it bounds.  pos[] is the exclusive scan of the
// boundary-face flags, so triangles keep tetrahedron order (and diagrams stay
// contiguous).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kB) bnd_flags(const int *__restrict__ adj, long long nf, int *__restrict__ flag) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x < nf) flag[x] = adj[x] < 0 ? 1 : 0;
}

__global__ void __launch_bounds__(kB) bnd_extract(const int *__restrict__ simp, const int *__restrict__ adj,
                                                  long long m, int nb, const long long *__restrict__ simp_off,
                                                  const long long *__restrict__ vert_off,
                                                  const int *__restrict__ pos, int *__restrict__ tri,
                                                  int *__restrict__ btet) {
  const long long x = (long long)blockIdx.x * kB + threadIdx.x;
  if (x >= m * 4 || adj[x] >= 0) return;
  const long long a = x / 4;
  const int f = (int)(x % 4);
  const int b = nb > 1 ? diagram_of(simp_off, nb, a) : 0;
  const int vo = (int)vert_off[b];
  const unsigned loops = (1u | 2u << 2 | 3u << 4) | (0u | 3u << 2 | 2u << 4) << 6 |
                         (0u | 1u << 2 | 3u << 4) << 12 | (0u | 2u << 2 | 1u << 4) << 18;
  const unsigned lf = loops >> (6 * f);
  const int t = pos[x];
  tri[3 * (long long)t + 0] = simp[a * 4 + (lf & 3)] - vo;
  tri[3 * (long long)t + 1] = simp[a * 4 + ((lf >> 2) & 3)] - vo;
  tri[3 * (long long)t + 2] = simp[a * 4 + ((lf >> 4) & 3)] - vo;
  btet[t] = (int)a;
}

// out[b] = pos[4 simp_off[b]]: boundary triangles before diagram b
__global__ void bnd_offsets(const int *__restrict__ pos, const long long *__restrict__ simp_off, int nb,
                            long long *__restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= nb) out[b] = pos[4 * simp_off[b]];
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
  hipLaunchKernelGGL(loc_sort, dim3(blocks(d->ncell)), dim3(kB), 0, st, (const int *)d->lstart, (long long)d->ncell,
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

void vd_launch_locate_sites(const GridView &G, const DomainView &D, int *seed, int *outside, hipStream_t st) {
  hipLaunchKernelGGL(locate_sites, dim3(blocks(G.n)), dim3(kB), 0, st, G, D, seed, outside);
}

void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_int, dim3(blocks(n)), dim3(kB), 0, st, p, n, v);
}

// adjacency of every simplex face from the (global) vertex indices; flags[0]
// is set for a non-manifold face.  Temporary buffers are the caller's.
void vd_launch_adjacency(vd_domain d, int *count, int *start, int *fill, int *items, int *scan_tmp, int *flags,
                         hipStream_t st) {
  const long long nf = d->m * (d->dim + 1);
  const int k = d->dim + 1;
  hipLaunchKernelGGL(fill_int, dim3(blocks(d->nv)), dim3(kB), 0, st, count, d->nv, 0);
  hipLaunchKernelGGL(fill_int, dim3(blocks(d->nv)), dim3(kB), 0, st, fill, d->nv, 0);
  hipLaunchKernelGGL(adj_count, dim3(blocks(nf)), dim3(kB), 0, st, (const int *)d->simp, (long long)d->m, k, count);
  vdscan::exclusive_scan<int, int>(count, d->nv, start, scan_tmp, st);
  hipLaunchKernelGGL(adj_scatter, dim3(blocks(nf)), dim3(kB), 0, st, (const int *)d->simp, (long long)d->m, k,
                     (const int *)start, fill, items);
  hipLaunchKernelGGL(adj_match, dim3(blocks(nf)), dim3(kB), 0, st, (const int *)d->simp, (long long)d->m, k,
                     (const int *)start, (const int *)items, d->adj, flags);
}

// per-diagram convexity of a tetrahedral domain (convex[b] = 1 on entry)
void vd_launch_convexity(vd_domain d, int *on_bnd, int *pos, int *list, int *scan_tmp, const double *bbox,
                         int *convex, hipStream_t st) {
  hipLaunchKernelGGL(fill_int, dim3(blocks(d->nv)), dim3(kB), 0, st, on_bnd, d->nv, 0);
  hipLaunchKernelGGL(bnd_mark, dim3(blocks(d->m * 4)), dim3(kB), 0, st, (const int *)d->simp, (const int *)d->adj,
                     (long long)d->m, on_bnd);
  vdscan::exclusive_scan<int, int>(on_bnd, d->nv, pos, scan_tmp, st);
  hipLaunchKernelGGL(bnd_collect, dim3(blocks(d->nv)), dim3(kB), 0, st, (const int *)on_bnd, (const int *)pos,
                     (long long)d->nv, list);
  hipLaunchKernelGGL(convex_check, dim3(blocks(d->m * 4)), dim3(kB), 0, st, d->view(), (const int *)pos,
                     (const int *)list, (const long long *)d->d_vert_off, bbox, convex);
}

// boundary faces of a tetrahedral domain: flags / scan into pos[4m+1], then
// the outward triangles (diagram-local vertex indices), their tetrahedra and
// the per-diagram triangle offsets boff[nb+1]
void vd_launch_boundary_scan(vd_domain d, int *flag, int *pos, int *scan_tmp, hipStream_t st) {
  const long long nf = d->m * 4;
  hipLaunchKernelGGL(bnd_flags, dim3(blocks(nf)), dim3(kB), 0, st, (const int *)d->adj, nf, flag);
  vdscan::exclusive_scan<int, int>(flag, nf, pos, scan_tmp, st);
}

// Each boundary triangle (A, B, C) split into s^2 congruent triangles of the
// same orientation: row r (0 <= r < s) holds s - r "up" triangles
// P(r,c) P(r,c+1) P(r+1,c) and then s - r - 1 "down" triangles
// P(r,c+1) P(r+1,c+1) P(r+1,c), P(r,c) = A + (c/s)(B - A) + (r/s)(C - A).
// Sub-triangle t gets its own three vertices 3t .. 3t+2, no neighbours, and
// the tetrahedron of its triangle.  Vertex indices are diagram-local, as a
// batched domain takes them (diagram b of the triangles starts at simp_off[b]).
__global__ void __launch_bounds__(kB) refine_triangles(const double *__restrict__ verts, const int *__restrict__ tri,
                                                       const int *__restrict__ btet, long long m, int nb,
                                                       const long long *__restrict__ simp_off, int s,
                                                       double *__restrict__ ov, int *__restrict__ otri,
                                                       int *__restrict__ oadj, int *__restrict__ obtet) {
  const long long t = (long long)blockIdx.x * kB + threadIdx.x;
  const long long ss = (long long)s * s;
  if (t >= m * ss) return;
  const long long a = t / ss;
  const long long t0 = nb > 1 ? simp_off[diagram_of(simp_off, nb, a)] * ss : 0;  // first sub-triangle of the diagram
  int k = (int)(t - a * ss), r = 0;
  while (k >= 2 * (s - r) - 1) { k -= 2 * (s - r) - 1; r++; }
  int pr[3], pc[3];
  if (k < s - r) {
    pr[0] = r; pc[0] = k; pr[1] = r; pc[1] = k + 1; pr[2] = r + 1; pc[2] = k;
  } else {
    const int c = k - (s - r);
    pr[0] = r; pc[0] = c + 1; pr[1] = r + 1; pc[1] = c + 1; pr[2] = r + 1; pc[2] = c;
  }
  const double *A = verts + 3 * (long long)tri[3 * a], *B = verts + 3 * (long long)tri[3 * a + 1],
               *C = verts + 3 * (long long)tri[3 * a + 2];
  for (int v = 0; v < 3; v++) {
    const double u = (double)pc[v] / s, w = (double)pr[v] / s;
    for (int x = 0; x < 3; x++) ov[9 * t + 3 * v + x] = A[x] + u * (B[x] - A[x]) + w * (C[x] - A[x]);
    otri[3 * t + v] = (int)(3 * (t - t0) + v);
    oadj[3 * t + v] = -1;
  }
  obtet[t] = btet[a];
}

void vd_launch_refine_triangles(vd_domain bnd, const int *btet, int s, double *ov, int *otri, int *oadj, int *obtet,
                                hipStream_t st) {
  hipLaunchKernelGGL(refine_triangles, dim3(blocks(bnd->m * (long long)s * s)), dim3(kB), 0, st,
                     (const double *)bnd->verts, (const int *)bnd->simp, btet, (long long)bnd->m, bnd->nb,
                     (const long long *)bnd->d_simp_off, s, ov, otri, oadj, obtet);
}

void vd_launch_boundary_extract(vd_domain d, const int *pos, int *tri, int *btet, long long *boff, hipStream_t st) {
  hipLaunchKernelGGL(bnd_extract, dim3(blocks(d->m * 4)), dim3(kB), 0, st, (const int *)d->simp,
                     (const int *)d->adj, (long long)d->m, d->nb, (const long long *)d->d_simp_off,
                     (const long long *)d->d_vert_off, pos, tri, btet);
  hipLaunchKernelGGL(bnd_offsets, dim3((d->nb + 1 + 255) / 256), dim3(256), 0, st, pos,
                     (const long long *)d->d_simp_off, d->nb, boff);
}
