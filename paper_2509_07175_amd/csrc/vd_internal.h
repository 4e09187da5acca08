// vd_internal.h -- host-side handle layouts and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/vd.h"
#include "vd_common.h"

// ---------------------------------------------------------------------------
// per-wave LDS capacities of the 3D carve (one wavefront per site)
// ---------------------------------------------------------------------------
#define VD_P_MAX 64    // planes of one intermediate polytope
#define VD_C_MAX 128   // corners (two slots per lane)
#define VD_Q_MAX 256   // tetrahedra visited for one site in LDS (4 per lane) ...
#define VD_Q_SPILL 3840  // ... and after them in a per-wave global buffer (initial size, grown on retry)
#define VD_NB_SPILL 160  // neighbours past VD_NB_MAX: per-wave global buffer (initial size, grown on retry)
#define VD_NB_MAX 96   // distinct neighbours of one site
#define VD_F_MAX 48    // planes of a saved cell (cell-first mode)
#define VD_CB_MAX 96   // corners of a saved cell
// doubles of one wave's saved cell in global memory: planes (4 doubles each),
// corners (3 doubles each), then plane flags and corner planes / neighbours
#define VD_SAVE_DOUBLES (VD_F_MAX * 4 + VD_CB_MAX * 3 + (VD_F_MAX + 2 * VD_CB_MAX + 1) / 2)

// Output arenas.  Waves reserve chunks of an arena with one atomic on its
// counter and hand out slots from the chunk, so a counter is the arena's
// high-water mark (unused chunk tails included), not the number of records.
enum { AR_PIECE = 0, AR_FACE, AR_VERT, AR_NBR, AR_FINT, AR_N };

// device counters written by the clip kernels; the first AR_N are the arena
// high-water marks (index = arena id), CNT_REAL_* the records actually written
enum {
  CNT_PIECES = AR_PIECE, CNT_FACES = AR_FACE, CNT_VERTS = AR_VERT, CNT_NBRS = AR_NBR, CNT_FINT = AR_FINT,
  CNT_QUERIES = AR_N, CNT_CLIPS, CNT_CANDS, CNT_ERR_CAP, CNT_ERR_DEG, CNT_ERR_LOC, CNT_BAD_SITE,
  CNT_REAL_PIECES, CNT_REAL_FACES, CNT_REAL_VERTS, CNT_REAL_NBRS, CNT_STAGES, CNT_GRIDQ,
  CNT_OVERFLOW,    // records dropped because an arena was full (pieces, per-piece faces / vertices /
                   // face moments, per-site neighbour lists)
  CNT_LOWMARGIN,   // corner classifications whose relative margin was below 1e-12
  CNT_MINMARGIN,   // bits of the smallest relative margin seen (a non-negative double)
  CNT_ROUNDS,      // nearest-site query rounds (a batch of up to four tests is one round)
  CNT_CLASSIFIED,  // corners classified against a clipping plane
  CNT_NEWCORNERS,  // corners created by clips (one 3x3 solve each)
  CNT_WASTED,      // tested corners that a clip removed besides the one that triggered it
  CNT_FANTETS,     // fan tetrahedra integrated for piece moments
  CNT_N
};
static_assert(CNT_N <= 64, "reset_counters clears the counters with one wave");

// persistent kernels: one work queue per XCD (8 heads, one per 128-byte line)
#define VD_QUEUES 8
#define VD_QSTRIDE 32

struct vd_grid_s {
  int64_t n = 0, cap_n = 0;
  int g[3] = {1, 1, 1};       // dims of diagram 0 (the plain grid)
  int64_t ncell = 0, cap_cell = 0;  // cells of all diagrams
  double *geom = nullptr;     // [9 nb]: lo[3], h[3], ih[3] per diagram
  double *bbox_part = nullptr;  // per-block partial boxes
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *delta = nullptr;
  bool delta_valid = false;   // delta is computed by the first clip that needs it after a build
  // power diagram (vd_grid_set_weights): weights and lifted coordinates in
  // sorted order, eta = max w; cleared by every build
  double *sw = nullptr, *sh = nullptr, *eta = nullptr;
  int64_t cap_w = 0;
  bool power = false;
  int *perm = nullptr, *rank = nullptr, *cellid = nullptr, *fill = nullptr;
  int *cstart = nullptr, *ccount = nullptr, *scan_tmp = nullptr;
  // batch of nb diagrams (nb = 1: plain)
  int nb = 1, cap_nb = 0;
  std::vector<int64_t> site_off, cell_off;  // host [nb + 1]
  std::vector<int> dims;                    // host [3 nb]
  long long *d_site_off = nullptr, *d_cell_off = nullptr;  // device [nb + 1]
  int *d_dims = nullptr, *diag = nullptr;   // [3 nb]; diagram of each caller index [n]
  double *d_user_box = nullptr;             // [6 nb]
  GridView *d_views = nullptr;              // [nb]
  std::vector<GridView> h_views;            // host copy last uploaded
  GridView view_of(int b) const {
    GridView v;
    v.n = (int)(site_off[b + 1] - site_off[b]);
    v.g[0] = dims[3 * b]; v.g[1] = dims[3 * b + 1]; v.g[2] = dims[3 * b + 2];
    v.geom = geom + 9 * b; v.sx = sx; v.sy = sy; v.sz = sz; v.cstart = cstart + cell_off[b];
    v.perm = perm; v.delta = delta;
    v.sw = power ? sw : nullptr; v.sh = power ? sh : nullptr;
    v.nb = 1; v.views = nullptr; v.site_off = nullptr;
    return v;
  }
  // the view the kernels get: all sites; views[b] for each diagram (also for
  // a plain grid, whose views[0] is itself)
  GridView view() const {
    GridView v = view_of(0);
    v.n = (int)n; v.nb = nb; v.views = d_views; v.site_off = d_site_off;
    return v;
  }
};

// Device view of a domain.  A batch of domains is one disjoint union with
// global vertex and simplex indices; views[b] holds diagram b's point-location
// grid and bounding box.
struct DomainView {
  int m, nv, dim;       // all simplices / vertices of the (batched) domain
  const double *verts;
  const int *simp, *adj;
  // point location grid over the simplices (tetrahedra only)
  int lg[3];
  const double *lgeom;  // lo[3], h[3], ih[3]
  const int *lstart, *litems;
  double box_lo[3], box_hi[3];  // padded bounding box (cell-first carve)
  int nb;
  const DomainView *views;      // [nb] (nb > 1)
  const long long *simp_off;    // [nb + 1] (nb > 1)
};

__device__ __forceinline__ DomainView domain_of(const DomainView &D, int b) { return D.nb > 1 ? D.views[b] : D; }

struct vd_domain_s {
  int64_t m = 0, nv = 0;
  int dim = 3;
  double *verts = nullptr;
  int *simp = nullptr, *adj = nullptr;
  double *lgeom = nullptr;  // [9 nb]
  int *lstart = nullptr, *litems = nullptr, *lcount = nullptr, *lfill = nullptr, *scan_tmp = nullptr;
  int64_t nitems = 0, ncell = 0;
  double area = 0.0;  // surface area (triangles) or volume (tets), all diagrams
  std::vector<int> convex;  // host [nb]: 1 if the tetrahedral domain of diagram b is convex
  bool all_convex = false;  // every diagram's tetrahedral domain is convex
  // tetrahedra: the boundary surface of M as a triangle domain (outward
  // triangles, edges all flagged as boundary) and the tetrahedron owning each
  // of its triangles; its restricted diagram seeds the cells that reach M
  // from outside the tetrahedron of their site (Alg. 5)
  vd_domain_s *bnd = nullptr;
  int *btet = nullptr;
  // the boundary surface with every triangle split into bnd_ref_s^2, for the
  // boundary diagram when a triangle would meet many cells (built by a clip
  // and kept for later clips of the same density), and its tetrahedra
  vd_domain_s *bnd_ref = nullptr;
  int *btet_ref = nullptr;
  int bnd_ref_s = 0;
  // batch of nb domains (nb = 1: plain)
  int nb = 1;
  std::vector<int64_t> vert_off, simp_off, loc_off;  // host [nb + 1]
  std::vector<int> lg;                               // host [3 nb] location grid dims
  std::vector<double> bbox;                          // host [6 nb] vertex bounding boxes
  long long *d_simp_off = nullptr, *d_vert_off = nullptr, *d_loc_off = nullptr;
  int *d_lg = nullptr;
  DomainView *d_views = nullptr;
  DomainView view_of(int b) const {
    DomainView d;
    d.m = (int)m; d.nv = (int)nv; d.dim = dim; d.verts = verts; d.simp = simp; d.adj = adj;
    d.lg[0] = lg.empty() ? 1 : lg[3 * b]; d.lg[1] = lg.empty() ? 1 : lg[3 * b + 1];
    d.lg[2] = lg.empty() ? 1 : lg[3 * b + 2];
    d.lgeom = lgeom ? lgeom + 9 * b : nullptr;
    d.lstart = lstart ? lstart + (loc_off.empty() ? 0 : loc_off[b]) : nullptr;
    d.litems = litems;
    for (int a = 0; a < 3; a++) {
      // The box strictly contains the domain so no box plane meets a simplex.
      // The six paddings differ so that no box edge lies on a plane of
      // symmetry of the domain (e.g. the diagonal planes of cube grids split
      // into tetrahedra), where a tetrahedron plane would contain the edge.
      const double lo = bbox.empty() ? 0.0 : bbox[6 * b + a], hi = bbox.empty() ? 0.0 : bbox[6 * b + 3 + a];
      const double ext = hi - lo > 1e-12 ? hi - lo : 1e-12;
      d.box_lo[a] = lo - (1.01e-3 + 0.12e-3 * a) * ext - 1e-9;
      d.box_hi[a] = hi + (1.07e-3 + 0.14e-3 * a) * ext + 1e-9;
    }
    d.nb = 1; d.views = nullptr; d.simp_off = nullptr;
    return d;
  }
  DomainView view() const {
    DomainView d = view_of(0);
    d.nb = nb; d.views = d_views; d.simp_off = d_simp_off;
    return d;
  }
};

// Output arenas of a clip (device).  Per-piece records live in arena order;
// per-site lists are reserved by atomics and compacted into CSR afterwards.
struct CellsDev {
  int n;           // sites
  int emit;        // write faces / vertices
  int want_grad;   // write face integrals
  int improved;    // Sec. 6.1 search
  int straddle;    // Alg. 1 edges when available
  int max_iters;
  int mode;        // 0 per-simplex carve, 1 cell-first
  int cache;       // LDS copy of the sites around each site for its queries
  int monitor;     // count work and track predicate margins
  int density;     // weight the moments by the quadratic density dens[] (Eq. 3)
  int power;       // power diagram: the grid's weights (Sec. 7.3)
  int whole;       // interior cells as one piece: 1 no boundary triangle met (needs bseed_off),
                   // 2 every corner in M (a convex M holding every site)
  double dens[10]; // rho(x) = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 xy + c6 xz + c7 y^2 + c8 yz + c9 z^2
  unsigned long long *cnt;  // CNT_N counters
  // per site (caller index)
  double *mass, *mom, *energy;
  int *pcount, *ncount;
  long long *pstart, *nstart;
  // arenas + capacities
  int *nbr_arena; long long cap_nbr;
  int *piece_site, *piece_simplex, *piece_nface, *piece_nvert;
  long long *piece_fstart, *piece_vstart;
  double *piece_mass, *piece_mom, *piece_energy;
  long long cap_piece;
  int *face_label; long long cap_face;
  double *vert_xyz; int *vert_label; long long cap_vert;
  // face moments for the adjoint (want_grad): one record per bisector face of a
  // piece: 12 doubles {I0[3], I1[6] (xx,xy,xz,yy,yz,zz), I2[3]} with
  // I0 = int y/d, I1 = int y y^T/d, I2 = int |y|^2 y/d (y = x - v_i, d = |v_k - v_i|,
  // divided by the in-plane sine for surface edges), and the neighbour k
  double *fint; int *fint_lab; long long cap_fint;
  long long *piece_fint_start; int *piece_nfint;
  int *seed;  // 3D: tetrahedron containing each site (sorted position order), -1 outside M
  // 3D, boundary seeds (Alg. 5): pieces of each site (caller index) on the
  // boundary surface -- CSR offsets, piece ids, their triangles -- and the
  // tetrahedron behind each boundary triangle; all NULL when not used
  const long long *bseed_off;
  const int *bseed_pid, *bseed_tri, *btet;
  long long chunk[AR_N];  // slots a wave reserves at a time in each arena
  int *queue;             // [VD_QUEUES * VD_QSTRIDE] work-queue heads
  // batches: the sorted positions in the order the queues hand them out
  // (NULL: queue k owns the k-th eighth of the sites in grid order), queue k
  // owning order[qoff[k] .. qoff[k+1])
  const int *order;
  long long qoff[VD_QUEUES + 1];
  int *tq_spill;          // [workgroups * q_spill] overflow of the per-site simplex queue
  int *nb_spill;          // [workgroups * nbs_cap] overflow of the per-site neighbour list
  int q_spill, nbs_cap;   // entries per workgroup of the two overflow buffers
  int *sq_spill;          // [workgroups * sq_cap] surface: overflow of a triangle's site list
  int sq_cap;             // entries per workgroup of sq_spill (0: none yet)
  double *saved;          // [workgroups * VD_SAVE_DOUBLES] each wave's carved cell (cell-first mode)
};

struct vd_cells_s {
  int64_t n = 0;
  int dim = 3;
  vd_options opt;
  CellsDev d{};
  unsigned long long *host_cnt = nullptr;  // [CNT_N] pinned host copy of the counters
  bool pending = false;                    // a no-sync clip whose counters are not checked yet
  hipStream_t last_stream = nullptr;
  // capacities (host copy) and allocations
  int64_t cap_n = 0;
  long long *piece_off = nullptr, *nbr_off = nullptr;  // CSR [n+1]
  int *piece_id = nullptr, *nbr = nullptr;             // CSR payloads
  int *fillc = nullptr;                                // per-site scatter counters
  int *pid_tmp = nullptr;                              // piece ids grouped by site, before the sort
  long long *scan_tmp = nullptr;
  int64_t cap_pid = 0, cap_nbr_csr = 0;
  const double *sites_sorted_x = nullptr;  // borrowed from the grid for moments
  vd_grid grid = nullptr;
  int status = 0;
  int first_bad = -1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;  // kernel timing (time_kernels)
  double carve_ms = -1.0, split_ms = -1.0;
  CellsDev *d_dev = nullptr;  // device copy of d (read by the piece kernel)
  int64_t cap_spill = 0;      // workgroups covered by d.tq_spill / d.nb_spill / d.saved
  int q_spill_want = VD_Q_SPILL, nb_spill_want = VD_NB_SPILL;  // per-workgroup sizes (grow on retry)
  int64_t sq_spill_elems = 0;  // allocated entries of d.sq_spill
  int *order_buf = nullptr;     // d.order's storage, and the batch layout it was built for
  int64_t order_cap = 0;
  std::vector<int64_t> order_key;
  std::vector<long long> order_qoff;
  int sq_spill_want = 0;       // surface: per-workgroup entries of d.sq_spill (grow on retry)
  CellsDev d_shadow{};        // host copy last sent to d_dev
  double *wbuf = nullptr;     // adjoint weights [5n]
  int64_t cap_w = 0;
  int *outside = nullptr;     // [2] sites outside every tetrahedron: count, lowest caller index
  int64_t sites_outside = -1;  // sites outside every tetrahedron (-1: not counted)
  vd_cells_s *bcells = nullptr;  // restricted diagram of the domain's boundary (boundary seeds)
  bool used_bseeds = false;      // the last clip seeded from the boundary
};

// Whether tetrahedron a (positively oriented) contains q: every sub-volume with
// q in place of one vertex is >= -1e-12 of the volume.
__device__ __forceinline__ bool tet_contains(const DomainView &D, long long a, const double *q) {
  const double *P[4];
  for (int u = 0; u < 4; u++) P[u] = &D.verts[3 * (long long)D.simp[a * 4 + u]];
  auto vol6 = [](const double *A, const double *B, const double *Cc, const double *Dd) {
    const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double e2[3] = {Cc[0] - A[0], Cc[1] - A[1], Cc[2] - A[2]};
    const double e3[3] = {Dd[0] - A[0], Dd[1] - A[1], Dd[2] - A[2]};
    return e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
           e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
  };
  const double v = vol6(P[0], P[1], P[2], P[3]);
  return vol6(q, P[1], P[2], P[3]) >= -1e-12 * v && vol6(P[0], q, P[2], P[3]) >= -1e-12 * v &&
         vol6(P[0], P[1], q, P[3]) >= -1e-12 * v && vol6(P[0], P[1], P[2], q) >= -1e-12 * v;
}

// The density of Eq. 3 at the absolute point (x, y, z).
__device__ __forceinline__ double density_at(const double *c, double x, double y, double z) {
  return c[0] + x * (c[1] + c[4] * x + c[5] * y + c[6] * z) + y * (c[2] + c[7] * y + c[8] * z) + z * (c[3] + c[9] * z);
}

// Density-weighted moments of a tetrahedron with corners V0..V3 relative to
// the site v (6 vol = det(V1 - V0, V2 - V0, V3 - V0)): mass += int rho,
// m1 += int rho y, e += int rho |y|^2 (y = x - v).  Rule of Grundmann and
// Moeller of degree 5 (15 points, barycentric (5,1,1,1)/8, (3,3,1,1)/8,
// (3,1,1,1)/6, (1,1,1,1)/4 with weights 16/315, 16/315, -27/280, 2/45 of the
// unit simplex): exact for a quadratic density, whose integrands have degree
// at most 4.
__device__ __forceinline__ void tet_density_moments(const double *c, double vx, double vy, double vz,
                                                    const double *V0, const double *V1, const double *V2,
                                                    const double *V3, double vol, double &mass, double &m0,
                                                    double &m1, double &m2, double &e) {
  double am = 0, a0 = 0, a1 = 0, a2 = 0, ae = 0;
  auto add = [&](double w, double y0, double y1, double y2) {
    const double wr = w * density_at(c, vx + y0, vy + y1, vz + y2);
    am += wr;
    a0 += wr * y0; a1 += wr * y1; a2 += wr * y2;
    ae += wr * (y0 * y0 + y1 * y1 + y2 * y2);
  };
  const double S0 = V0[0] + V1[0] + V2[0] + V3[0], S1 = V0[1] + V1[1] + V2[1] + V3[1],
               S2 = V0[2] + V1[2] + V2[2] + V3[2];
  constexpr double wA = 16.0 / 315.0, wC = -27.0 / 280.0, wD = 2.0 / 45.0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const double *Vk = k == 0 ? V0 : (k == 1 ? V1 : (k == 2 ? V2 : V3));
    add(wA, S0 * 0.125 + Vk[0] * 0.5, S1 * 0.125 + Vk[1] * 0.5, S2 * 0.125 + Vk[2] * 0.5);           // (5,1,1,1)/8
    add(wC, S0 / 6.0 + Vk[0] / 3.0, S1 / 6.0 + Vk[1] / 3.0, S2 / 6.0 + Vk[2] / 3.0);                   // (3,1,1,1)/6
  }
#pragma unroll
  for (int k = 1; k < 4; k++) {
    // the pair {0, k} and its complement: (3,3,1,1)/8
    const double *Vk = k == 1 ? V1 : (k == 2 ? V2 : V3);
    const double P0 = V0[0] + Vk[0], P1 = V0[1] + Vk[1], P2 = V0[2] + Vk[2];
    add(wA, S0 * 0.125 + P0 * 0.25, S1 * 0.125 + P1 * 0.25, S2 * 0.125 + P2 * 0.25);
    add(wA, S0 * 0.375 - P0 * 0.25, S1 * 0.375 - P1 * 0.25, S2 * 0.375 - P2 * 0.25);
  }
  add(wD, S0 * 0.25, S1 * 0.25, S2 * 0.25);
  const double sc = 6.0 * vol;
  mass += sc * am; m0 += sc * a0; m1 += sc * a1; m2 += sc * a2; e += sc * ae;
}

// Density-weighted integrals over a triangle (A0, A1, A2 relative to v,
// area `area`) of y, y y^T and |y|^2 y (the adjoint's face moments before the
// division by |v_k - v|): rule of Grundmann and Moeller of degree 5
// (barycentric (5,1,1)/7 and (3,3,1)/7 with weight 16807/80640, (3,1,1)/5
// with -3125/11520, (1,1,1)/3 with 243/3840, of the unit triangle), exact
// for a quadratic density times a cubic.
__device__ __forceinline__ void tri_density_face(const double *c, double vx, double vy, double vz, const double *A0,
                                                 const double *A1, const double *A2, double area, double *I) {
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; k++) acc[k] = 0.0;
  auto add = [&](double w, double y0, double y1, double y2) {
    const double wr = w * density_at(c, vx + y0, vy + y1, vz + y2);
    const double yy = y0 * y0 + y1 * y1 + y2 * y2;
    acc[0] += wr * y0; acc[1] += wr * y1; acc[2] += wr * y2;
    acc[3] += wr * y0 * y0; acc[4] += wr * y0 * y1; acc[5] += wr * y0 * y2;
    acc[6] += wr * y1 * y1; acc[7] += wr * y1 * y2; acc[8] += wr * y2 * y2;
    acc[9] += wr * yy * y0; acc[10] += wr * yy * y1; acc[11] += wr * yy * y2;
  };
  const double T0 = A0[0] + A1[0] + A2[0], T1 = A0[1] + A1[1] + A2[1], T2 = A0[2] + A1[2] + A2[2];
  constexpr double w0 = 16807.0 / 80640.0, w1 = -3125.0 / 11520.0, w2 = 243.0 / 3840.0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const double *Ak = k == 0 ? A0 : (k == 1 ? A1 : A2);
    add(w0, (T0 + 4.0 * Ak[0]) / 7.0, (T1 + 4.0 * Ak[1]) / 7.0, (T2 + 4.0 * Ak[2]) / 7.0);        // (5,1,1)/7
    add(w0, (3.0 * T0 - 2.0 * Ak[0]) / 7.0, (3.0 * T1 - 2.0 * Ak[1]) / 7.0, (3.0 * T2 - 2.0 * Ak[2]) / 7.0);  // (3,3,1)/7
    add(w1, (T0 + 2.0 * Ak[0]) / 5.0, (T1 + 2.0 * Ak[1]) / 5.0, (T2 + 2.0 * Ak[2]) / 5.0);        // (3,1,1)/5
  }
  add(w2, T0 / 3.0, T1 / 3.0, T2 / 3.0);
#pragma unroll
  for (int k = 0; k < 12; k++) I[k] += 2.0 * area * acc[k];
}

// Density-weighted moments of a triangle (A0, A1, A2 relative to v, area
// `area`): mass += int rho, m1 += int rho y, e += int rho |y|^2, with the same
// degree-5 rule.
__device__ __forceinline__ void tri_density_moments(const double *c, double vx, double vy, double vz,
                                                    const double *A0, const double *A1, const double *A2,
                                                    double area, double &mass, double &m0, double &m1, double &m2,
                                                    double &e) {
  double am = 0, a0 = 0, a1 = 0, a2 = 0, ae = 0;
  auto add = [&](double w, double y0, double y1, double y2) {
    const double wr = w * density_at(c, vx + y0, vy + y1, vz + y2);
    am += wr;
    a0 += wr * y0; a1 += wr * y1; a2 += wr * y2;
    ae += wr * (y0 * y0 + y1 * y1 + y2 * y2);
  };
  const double T0 = A0[0] + A1[0] + A2[0], T1 = A0[1] + A1[1] + A2[1], T2 = A0[2] + A1[2] + A2[2];
  constexpr double w0 = 16807.0 / 80640.0, w1 = -3125.0 / 11520.0, w2 = 243.0 / 3840.0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const double *Ak = k == 0 ? A0 : (k == 1 ? A1 : A2);
    add(w0, (T0 + 4.0 * Ak[0]) / 7.0, (T1 + 4.0 * Ak[1]) / 7.0, (T2 + 4.0 * Ak[2]) / 7.0);
    add(w0, (3.0 * T0 - 2.0 * Ak[0]) / 7.0, (3.0 * T1 - 2.0 * Ak[1]) / 7.0, (3.0 * T2 - 2.0 * Ak[2]) / 7.0);
    add(w1, (T0 + 2.0 * Ak[0]) / 5.0, (T1 + 2.0 * Ak[1]) / 5.0, (T2 + 2.0 * Ak[2]) / 5.0);
  }
  add(w2, T0 / 3.0, T1 / 3.0, T2 / 3.0);
  const double sc = 2.0 * area;
  mass += sc * am; m0 += sc * a0; m1 += sc * a1; m2 += sc * a2; e += sc * ae;
}

// launchers (defined in the .hip files)
void vd_launch_grid_build(vd_grid g, const double *sites, const double *user_box, hipStream_t st);
void vd_launch_grid_delta(vd_grid g, hipStream_t st);
void vd_launch_grid_weights(vd_grid g, const double *w, int *flags, hipStream_t st);
void vd_launch_domain_locator(vd_domain d, hipStream_t st);
void vd_launch_locate_sites(const GridView &G, const DomainView &D, int *seed, int *outside, hipStream_t st);
// workgroups of the persistent 3D site kernel (resident waves of the device)
int vd_sites3d_workgroups(long long n);
void vd_launch_queue_init(int *queue, long long n, const long long *qoff, hipStream_t st);
void vd_launch_sites3d(const GridView &G, const DomainView &D, const CellsDev *Cdev, int workgroups, bool monitor,
                       bool density, bool power, bool corners, hipStream_t st);
int vd_surface_workgroups(long long m);
void vd_launch_surface(const GridView &G, const DomainView &D, const CellsDev *Cdev, int workgroups, bool density,
                       bool power, hipStream_t st);
void vd_launch_site_nbrs(long long n, const long long *poff, const int *pid, const long long *noff, int *nbr,
                         long long cap, const CellsDev *Cdev, hipStream_t st);
void vd_launch_site_reduce(long long n, const long long *poff, const int *pid, const CellsDev *Cdev,
                           hipStream_t st);
void vd_launch_finalize(vd_cells c, hipStream_t st);
void vd_launch_moments(const vd_cells_s *c, const GridView &G, double *mass, double *cent,
                       double *energy, hipStream_t st);
void vd_launch_backward(const vd_cells_s *c, const GridView &G, const double *gm, const double *gc,
                        const double *ge, double *gs, double *work, hipStream_t st);
