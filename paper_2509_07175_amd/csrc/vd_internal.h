// vd_internal.h -- host-side handle layouts and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vd.h"
#include "vd_common.h"

// ---------------------------------------------------------------------------
// per-wave LDS capacities of the 3D carve (one wavefront per site)
// ---------------------------------------------------------------------------
#define VD_P_MAX 64    // planes of one intermediate polytope
#define VD_C_MAX 128   // corners (two slots per lane)
#define VD_Q_MAX 256   // tetrahedra visited for one site (4 per lane)
#define VD_NB_MAX 96   // distinct neighbours of one site
#define VD_F_MAX 48    // planes of a saved cell (cell-first mode)
#define VD_CB_MAX 96   // corners of a saved cell

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
  CNT_N
};

// persistent kernels: one work queue per XCD (8 heads, one per 128-byte line)
#define VD_QUEUES 8
#define VD_QSTRIDE 32

struct vd_grid_s {
  int64_t n = 0, cap_n = 0;
  int g[3] = {1, 1, 1};
  int64_t ncell = 0, cap_cell = 0;
  double *geom = nullptr;     // lo[3], h[3], ih[3]
  double *bbox_part = nullptr;  // per-block partial boxes
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *delta = nullptr;
  int *perm = nullptr, *rank = nullptr, *cellid = nullptr, *fill = nullptr;
  int *cstart = nullptr, *ccount = nullptr, *scan_tmp = nullptr;
  GridView view() const {
    GridView v;
    v.n = (int)n; v.g[0] = g[0]; v.g[1] = g[1]; v.g[2] = g[2];
    v.geom = geom; v.sx = sx; v.sy = sy; v.sz = sz; v.cstart = cstart; v.perm = perm; v.delta = delta;
    return v;
  }
};

struct DomainView {
  int m, nv, dim;
  const double *verts;
  const int *simp, *adj;
  // point location grid over the simplices (tetrahedra only)
  int lg[3];
  const double *lgeom;  // lo[3], h[3], ih[3]
  const int *lstart, *litems;
};

struct vd_domain_s {
  int64_t m = 0, nv = 0;
  int dim = 3;
  double *verts = nullptr;
  int *simp = nullptr, *adj = nullptr;
  int lg[3] = {1, 1, 1};
  double *lgeom = nullptr;
  int *lstart = nullptr, *litems = nullptr, *lcount = nullptr, *lfill = nullptr, *scan_tmp = nullptr;
  int64_t nitems = 0;
  double area = 0.0;  // surface area (triangles) or volume (tets)
  double bbox[6] = {0, 0, 0, 0, 0, 0};  // vertex bounding box
  DomainView view() const {
    DomainView d;
    d.m = (int)m; d.nv = (int)nv; d.dim = dim; d.verts = verts; d.simp = simp; d.adj = adj;
    d.lg[0] = lg[0]; d.lg[1] = lg[1]; d.lg[2] = lg[2];
    d.lgeom = lgeom; d.lstart = lstart; d.litems = litems;
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
  double box_lo[3], box_hi[3];  // padded domain box (cell-first)
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
  int *seed;  // 3D: tetrahedron containing each site (sorted position order)
  long long chunk[AR_N];  // slots a wave reserves at a time in each arena
  int *queue;             // [VD_QUEUES * VD_QSTRIDE] work-queue heads
};

struct vd_cells_s {
  int64_t n = 0;
  int dim = 3;
  vd_options opt;
  CellsDev d{};
  unsigned long long host_cnt[CNT_N] = {0};
  // capacities (host copy) and allocations
  int64_t cap_n = 0;
  long long *piece_off = nullptr, *nbr_off = nullptr;  // CSR [n+1]
  int *piece_id = nullptr, *nbr = nullptr;             // CSR payloads
  int *fillc = nullptr;                                // per-site scatter counters
  long long *scan_tmp = nullptr;
  int64_t cap_pid = 0, cap_nbr_csr = 0;
  const double *sites_sorted_x = nullptr;  // borrowed from the grid for moments
  vd_grid grid = nullptr;
  int status = 0;
  int first_bad = -1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;  // kernel timing (time_kernels)
  double carve_ms = -1.0, split_ms = -1.0;
  CellsDev *d_dev = nullptr;  // device copy of d (read by the piece kernel)
  CellsDev d_shadow{};        // host copy last sent to d_dev
  double *wbuf = nullptr;     // adjoint weights [5n]
  int64_t cap_w = 0;
};

// launchers (defined in the .hip files)
void vd_launch_grid_build(vd_grid g, const double *sites, const double *bbox_host, hipStream_t st);
void vd_launch_domain_locator(vd_domain d, hipStream_t st);
void vd_launch_locate_sites(const GridView &G, const DomainView &D, int *seed, unsigned long long *cnt,
                            hipStream_t st);
// workgroups of the persistent 3D site kernel (resident waves of the device)
int vd_sites3d_workgroups(long long n);
void vd_launch_queue_init(int *queue, long long n, hipStream_t st);
void vd_launch_sites3d(const GridView &G, const DomainView &D, const CellsDev *Cdev, int workgroups,
                       hipStream_t st);
int vd_surface_workgroups(long long m);
void vd_launch_surface(const GridView &G, const DomainView &D, const CellsDev *Cdev, int workgroups,
                       hipStream_t st);
void vd_launch_site_nbrs(long long n, const long long *poff, const int *pid, const long long *noff, int *nbr,
                         const CellsDev *Cdev, hipStream_t st);
void vd_launch_site_reduce(long long n, const long long *poff, const int *pid, const CellsDev *Cdev,
                           hipStream_t st);
void vd_launch_finalize(vd_cells c, hipStream_t st);
void vd_launch_moments(const vd_cells_s *c, const GridView &G, double *mass, double *cent,
                       double *energy, hipStream_t st);
void vd_launch_backward(const vd_cells_s *c, const GridView &G, const double *gm, const double *gc,
                        const double *ge, double *gs, double *work, hipStream_t st);
