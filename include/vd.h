/*
 * vd.h -- clipped and restricted Voronoi diagrams on one MI355X (gfx950).
 *
 * Method: Xiao, Cao & Chen, "Efficient Computation of Voronoi Diagrams Using
 * Point-in-Cell Tests".  Given sites V = {v_i} and a domain M = {T_a} made of
 * simplices (tetrahedra, or triangles in R^3), the library computes every
 * domain-cell intersection P_{a,i} = T_a intersected with the Voronoi cell
 * Omega_i (Sec. 3.1, Eq. 1), with the face flags of Sec. 3.2, and per site the
 * mass, centroid and CVT energy integrand (Sec. 7.4, Eq. 3, density 1).
 * Each piece is carved by point-in-cell tests (Sec. 4.1, Eq. 2) and the
 * edge-based bisector search (Sec. 4.2, improved as in Sec. 6.1) on straddling
 * or virtual edges (Alg. 1 and Alg. 3), the clip removing only the connected
 * outside component R_p (Sec. 6.3).  Nearest-site queries use a uniform grid
 * built by counting sort (Sec. 6.2).
 *
 * Conventions shared by every entry point
 *  - C linkage; only plain types cross the boundary.  Pointers named *_host
 *    are host memory; every other array pointer is DEVICE memory (HIP).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it; calls return once the work is enqueued unless
 *    stated otherwise.
 *  - Coordinates are float64, row-major (x, y, z) per point; topology is int32.
 *  - Indices are 0-based.  Face/edge labels (Sec. 3.2): a face on the bisector
 *    of v_i and v_j carries j >= 0; a face shared with simplex T_b carries
 *    -(b+1); a face on the domain boundary carries VD_BOUNDARY_BASE + f, where
 *    f is the local face (tet: opposite vertex f; triangle: opposite vertex f).
 *  - Every call returns a vd_status and never aborts.  vd_last_error() gives a
 *    thread-local message for the last failure.  Handles are not thread-safe;
 *    use one per stream.
 *  - Handles own their device memory and keep it between calls: passing an
 *    existing handle back in (*out != NULL) reuses its buffers when they are
 *    large enough, so a steady-state loop performs no allocation.
 */
#ifndef VD_H
#define VD_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VD_BOUNDARY_BASE (-2147483647 - 1)

typedef enum {
  VD_OK = 0,
  VD_ERR_INVALID_ARG = 1,   /* bad sizes, NULL pointers, a site outside the domain */
  VD_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed */
  VD_ERR_HIP = 3,           /* a HIP runtime call failed (message has details) */
  VD_ERR_CAPACITY = 4,      /* a per-wave LDS capacity was exceeded (see vd_options) */
  VD_ERR_DEGENERATE = 5,    /* a search did not converge (inputs not in general position) */
  VD_ERR_NOT_READY = 6      /* the results of enqueued work are not available yet */
} vd_status;

typedef struct vd_grid_s *vd_grid;
typedef struct vd_domain_s *vd_domain;
typedef struct vd_cells_s *vd_cells;

/* Stages of the per-site work, as bits of vd_cells_info_t.failed_stages. */
enum {
  VD_STAGE_CELL = 1,        /* carving the cell from the domain box (cell-first) */
  VD_STAGE_PIECE_CUT = 2,   /* cutting the saved cell by a tetrahedron's planes */
  VD_STAGE_PIECE_CARVE = 3, /* carving a piece from its simplex */
  VD_STAGE_NEIGHBOURS = 4,  /* more distinct neighbours than a wave holds */
  VD_STAGE_SIMPLICES = 5,   /* more simplices in one cell than a wave holds */
  VD_STAGE_TRIANGLE = 6,    /* surface: carving the pieces of a triangle */
  VD_STAGE_TRIANGLE_SITES = 7 /* surface: more sites in one triangle than a wave holds */
};

/* Tuning and behaviour knobs; vd_options_default() fills the defaults. */
typedef struct {
  double sites_per_cell;   /* unused by vd_clip_cells (the grid density is an argument
                              of vd_build_grid); kept for callers that store it here */
  int32_t improved_search; /* 1: shorten search edges by lambda*delta steps (Sec. 6.1).
                              Default 0: with the per-wave site cache a far query costs
                              about what a near one does, so the extra lambda queries
                              no longer pay (same results either way) */
  int32_t use_straddle_edges; /* 1: prefer edges with one inside end (Alg. 1);
                                 0: virtual edges from the site only (Alg. 3).
                                 Default 0: the same number of queries and a
                                 simpler edge choice (same results either way) */
  int32_t max_search_iters;   /* cap of the bisector search and of the lambda loop */
  int32_t emit_polytopes;     /* 1: write per-piece faces and vertices */
  int32_t want_grad;          /* 1: also store the face integrals the adjoint needs */
  int32_t time_kernels;       /* 1: record hipEvents around the carve kernel (see
                                 vd_cells_info_t.carve_ms) */
  int32_t carve_mode;         /* tetrahedral domains.  0: every piece T_a cap Omega_i is
                                 carved by point-in-cell tests and the bisector search.
                                 1 (default): the cell is carved once from the padded
                                 bounding box of the domain (Sec. 5.2), then each piece is
                                 T_a cut by the cell's certified bisector facets.  With the
                                 site cache, the box is first cut by the bisectors of the
                                 Delaunay neighbours that the cached sites certify (an empty
                                 sphere through v_i and the neighbour), which are faces of
                                 the cell.  Both modes give the same pieces. */
  int32_t no_sync;            /* 1: vd_clip_cells only enqueues work (no host synchronisation,
                                 no allocation), so it can be captured into a HIP graph.
                                 Needs a handle sized by an earlier synchronous clip of the
                                 same sites and options (tetrahedra or triangles); errors and
                                 arena overflow (records that did not fit the sized arenas,
                                 surface neighbour lists included) are reported by
                                 vd_cells_info, which then synchronises the stream.  Default 0. */
  int32_t site_cache;         /* 1 (default): each wave keeps the sites of a block of grid
                                 cells around its site (3D) or its triangle's centroid
                                 (surfaces) in LDS and answers a nearest-site query there
                                 when the query's ball lies inside the block (same answer as
                                 the grid query); 0: grid queries only */
  int32_t boundary_seeds;     /* tetrahedral domains.  A cell Omega_i cap M can have parts that
                                 are not connected to the tetrahedron holding v_i (a non-convex
                                 M), and a site may lie outside M.  Such parts touch the boundary
                                 of M, so, as in Alg. 5, the restricted diagram of the boundary
                                 surface is computed first and every boundary triangle a cell
                                 meets seeds the tetrahedron behind it.  -1 (default): only when
                                 needed -- the domain is not convex or a site lies outside it
                                 (one extra synchronisation to find out); 0: never (a site
                                 outside M is then VD_ERR_INVALID_ARG); 1: always.  A no_sync
                                 clip never seeds from the boundary. */
  int32_t monitor;            /* 1: count the clips' work (query rounds, corners classified and
                                 created, wasted tests, fan simplices) and track the relative
                                 margins of the corner classifications (vd_cells_info_t).
                                 Default 0: those counters cost about 6 % of the 3D kernel's time
                                 and read -1. */
  int32_t use_density;        /* 1: every moment is weighted by the density rho of Eq. 3 given in
                                 density[] (mass = integral of rho, centroid = integral of rho x
                                 over it, energy = integral of rho |x - v_i|^2; the per-piece
                                 records too), integrated exactly by degree-5 simplex rules on
                                 the moment fans; the adjoint then carries rho as well.  Pieces
                                 still exist by positive volume (area).  Default 0: rho = 1. */
  double density[10];         /* rho(x) = d0 + d1 x + d2 y + d3 z + d4 x^2 + d5 x y + d6 x z
                                 + d7 y^2 + d8 y z + d9 z^2 (absolute coordinates); it should be
                                 positive on M */
  int32_t whole_interior;     /* tetrahedral domains, carve_mode 1, synchronous clips.  1: Alg. 5's
                                 split of boundary and interior sites -- a cell that lies entirely
                                 inside M is returned as ONE piece with simplex -1: the whole
                                 cell, not cut by the tetrahedra (its moments, faces, vertices and
                                 neighbours are the cell's).  Cells that meet the boundary are cut
                                 per tetrahedron as usual.  Interior cells are those that meet no
                                 triangle of the restricted diagram of the boundary surface
                                 (computed first) and have a point in M; when M is convex, holds
                                 every site and boundary_seeds is not 1, no boundary diagram is
                                 needed: a cell is interior when all its corners lie in M.  Per-site
                                 moments and neighbour lists equal those of the default up to
                                 rounding.  Default 0: every piece is T_a cap Omega_i. */
  int32_t batch_order;        /* batches of tetrahedral domains.  1 (default): the persistent
                                 kernel's queues hand out the sites of the diagrams with the most
                                 tetrahedra per site (the most pieces per cell) first, diagrams
                                 dealt over the queues by longest processing time, so the last
                                 sites to finish are cheap ones; the order is built by a
                                 synchronous clip and kept in the handle for later (no_sync)
                                 clips of the same layout.  0: grid order.  Same results. */
} vd_options;

void vd_options_default(vd_options *opt);

const char *vd_last_error(void);
const char *vd_status_string(vd_status s);

/* Waits for all work enqueued on `stream` and reports an asynchronous device
 * error (a fault or a failed launch) as VD_ERR_HIP.  Errors of enqueued clips
 * (capacity, degeneracy, arena overflow) are reported by vd_cells_info. */
vd_status vd_sync(void *stream);

/* ---------------------------------------------------------------------
 * vd_build_grid -- uniform grid over the sites for nearest-site queries
 * (Sec. 6.2), built by counting sort: per-site cell ids and a histogram,
 * an exclusive scan into cell offsets and a scatter of the coordinates into
 * cell order (sites of one cell ordered by index).  delta_i = |N_i - v_i| / 2,
 * half the distance to its nearest other site (Sec. 6.1), is computed on the
 * grid by the first vd_clip_cells with improved_search = 1 after a build.
 *   sites      [n*3] device, caller-owned; read during the call's stream work only.
 *   n          >= 1.
 *   bbox_host  [6] host (xmin,ymin,zmin,xmax,ymax,zmax) or NULL; the grid box
 *              is the union of this box and the sites' bounding box.
 *   sites_per_cell  mean sites per grid cell (<= 0 -> 2 in 3D, 3.5 for a surface).
 *   surface_area    > 0 for sites spread over a surface of this area: the
 *              cell size then targets sites_per_cell per non-empty cell.
 *   out        *out == NULL -> a new handle; else the handle is rebuilt in place.
 * Errors: VD_ERR_INVALID_ARG (n < 1, NULL), VD_ERR_OUT_OF_MEMORY, VD_ERR_HIP.
 * --------------------------------------------------------------------- */
vd_status vd_build_grid(const double *sites, int64_t n, const double *bbox_host,
                        double sites_per_cell, double surface_area, void *stream, vd_grid *out);
void vd_grid_free(vd_grid g);

/* ---------------------------------------------------------------------
 * vd_grid_set_weights -- turns the grid's sites into weighted sites of a
 * power diagram (Sec. 7.3): the cell of v_i is the set of points x with
 * |x - v_i|^2 - w_i <= |x - v_j|^2 - w_j for all j.  The sites are lifted to
 * (v_i, sqrt(eta - w_i)) with eta = max w (the smallest admissible constant),
 * so a nearest-site query of the lifted point is the smallest power distance,
 * and vd_clip_cells computes the restricted Voronoi diagram of the lifted
 * sites on the domain.  A power cell may be empty and need not contain its
 * site.  The clips of a weighted grid use lifted grid queries (no site cache,
 * no lambda steps), carve each 3D cell from the domain box and seed it from
 * the boundary surface and from the tetrahedron holding the mean of its
 * corners; they take no want_grad, use_density or no_sync.
 *   weights [n] device, caller's site order, copied; NULL clears them.
 * Must follow every vd_build_grid of the handle (a rebuild clears them).
 * Synchronises `stream` once (validation).
 * Errors: VD_ERR_INVALID_ARG (NULL grid, a weight that is not finite),
 * VD_ERR_OUT_OF_MEMORY, VD_ERR_HIP.
 * --------------------------------------------------------------------- */
vd_status vd_grid_set_weights(vd_grid g, const double *weights, void *stream);

/* ---------------------------------------------------------------------
 * vd_domain_create -- stages a simplex domain M = {T_a} (Sec. 3.1) on the
 * device: copies verts/simplices/adjacency and, for tetrahedra, builds the
 * point-location grid that finds the simplex containing each site (the seed of
 * the per-site propagation over negative face flags, Alg. 5).
 *   verts [nv*3], simplices [m*(dim+1)]: device pointers, caller-owned,
 *   copied during the call.
 *   adjacency [m*(dim+1)] (-1 = boundary), device, or NULL: then it is
 *   computed on the device by matching the vertex sets of the simplices'
 *   faces (a face shared by more than two simplices is an error).
 *   simplex_dim 3: tetrahedra, positively oriented, local face f opposite
 *   vertex f.  simplex_dim 2: triangles in R^3, local edge f opposite vertex f.
 * Tetrahedral domains are also tested for convexity (vd_domain_info): M is
 * convex iff every boundary vertex lies inside the plane of every boundary face.
 * Synchronises `stream` once (validation result).
 * Errors: VD_ERR_INVALID_ARG (indices out of range, non-positive tet volume,
 * non-manifold faces), VD_ERR_OUT_OF_MEMORY, VD_ERR_HIP.
 * --------------------------------------------------------------------- */
vd_status vd_domain_create(const double *verts, int64_t nv, const int32_t *simplices,
                           const int32_t *adjacency, int64_t m, int32_t simplex_dim,
                           void *stream, vd_domain *out);
void vd_domain_free(vd_domain d);

typedef struct {
  int64_t n_simplices, n_verts;
  int32_t simplex_dim, n_diagrams;
  double measure;     /* total volume (tetrahedra) or area (triangles) */
  int32_t convex;     /* tetrahedra: 1 if every diagram's domain is convex, else 0;
                         triangles: -1 */
} vd_domain_info_t;

/* Host struct describing a staged domain (no device work). */
vd_status vd_domain_info(vd_domain d, vd_domain_info_t *info_host);

/* Adjacency of a staged domain as used by the kernels: [m*(dim+1)] int32 into
 * `adjacency_out` (device, caller-owned), global simplex indices for batches.
 * Enqueued on `stream`. */
vd_status vd_domain_adjacency(vd_domain d, int32_t *adjacency_out, void *stream);

/* ---------------------------------------------------------------------
 * Batches of independent diagrams (each with its own sites and its own
 * domain, uneven sizes).  Diagram b owns the sites [site_off[b], site_off[b+1]),
 * the vertices [vert_off[b], vert_off[b+1]) and the simplices
 * [simp_off[b], simp_off[b+1]) of the concatenated arrays.  A batch is handled
 * as one disjoint union: every diagram keeps its own grid and location grid,
 * nearest-site queries only see the diagram's own sites, and one persistent
 * launch covers the sites of all diagrams.  Results use the concatenated
 * numbering: site indices (neighbours, positive flags) and simplex indices
 * (piece_simplex, -(b+1) flags) are global; subtract site_off / simp_off for
 * diagram-local ones.  A plain call is the batch of one.
 * --------------------------------------------------------------------- */
typedef struct {
  int32_t num;              /* diagrams, >= 1 */
  const int64_t *site_off;  /* [num+1] host, site_off[0] = 0 */
  const int64_t *vert_off;  /* [num+1] host, vert_off[0] = 0 */
  const int64_t *simp_off;  /* [num+1] host, simp_off[0] = 0 */
} vd_batch;

/* vd_build_grid for a batch: one counting sort over all sites, each diagram
 * with its own cells (sites_per_cell per cell of its own box).
 *   sites      [site_off[num]*3] device.
 *   bbox_host  [6*num] host boxes (as in vd_build_grid) or NULL.
 * Repeated calls with the same batch layout enqueue kernels only (no host
 * copies, no allocation), so they can be captured into a HIP graph.
 * Errors as vd_build_grid, plus VD_ERR_INVALID_ARG for offsets that are not
 * increasing from 0. */
vd_status vd_build_grid_batch(const double *sites, const vd_batch *batch, const double *bbox_host,
                              double sites_per_cell, void *stream, vd_grid *out);

/* vd_domain_create for a batch: simplices and adjacency hold diagram-local
 * indices (vertex indices into the diagram's vertices, adjacency into its
 * simplices, -1 boundary); they are stored shifted to global indices.
 * Synchronises `stream`.  Errors as vd_domain_create. */
vd_status vd_domain_create_batch(const double *verts, const int32_t *simplices,
                                 const int32_t *adjacency, const vd_batch *batch,
                                 int32_t simplex_dim, void *stream, vd_domain *out);

/* ---------------------------------------------------------------------
 * vd_clip_cells -- all domain-cell intersections P_{a,i} (Sec. 3.1).
 * 3D (tetrahedra): one wavefront per site; the site's tetrahedra are visited
 * through negative face flags starting from the tetrahedron that contains the
 * site (Alg. 5, propagation part), and each piece is carved by Alg. 1/Alg. 3.
 * When the domain is not convex or a site lies outside it (see
 * vd_options.boundary_seeds), the restricted diagram of the domain's boundary
 * surface is computed first and every boundary triangle a cell meets seeds the
 * tetrahedron behind it (Alg. 5), so cells that meet M in several parts, and
 * sites outside M, get all their pieces; a site whose cell misses M gets none.
 * With vd_options.whole_interior = 1 a cell inside M is one piece (simplex -1).
 * When the boundary triangles are coarse for the number of sites, the
 * boundary diagram runs on a copy of the surface with every triangle split,
 * which the clip keeps in the domain handle: a domain handle must not be used
 * by two clips at the same time.
 * Surface (triangles): one wavefront per triangle; the triangle's sites are
 * found by propagation over positive edge flags from the site nearest to the
 * triangle's centroid (Alg. 4), each piece carved by Alg. 3.
 *   g, d    handles from vd_build_grid / vd_domain_create.
 *   opt     NULL -> defaults.
 *   out     *out == NULL -> a new handle; else reused.
 * Synchronises `stream` once to read the output sizes (and re-runs with
 * larger arenas if an output arena overflowed).
 * Errors: VD_ERR_INVALID_ARG (3D: a site with a coordinate that is not finite,
 * or that repeats an earlier one exactly --
 * the same point, and for a power diagram the same weight -- found before any
 * cell is carved, except in a no_sync clip, which assumes distinct sites; a
 * site outside every tetrahedron while the clip does not seed from the
 * boundary: boundary_seeds = 0, or no_sync;
 * whole_interior with a surface, carve_mode 0, boundary_seeds = 0 or no_sync),
 * VD_ERR_CAPACITY, VD_ERR_DEGENERATE, VD_ERR_OUT_OF_MEMORY, VD_ERR_HIP.
 * --------------------------------------------------------------------- */
vd_status vd_clip_cells(vd_grid g, vd_domain d, const vd_options *opt, void *stream,
                        vd_cells *out);
void vd_cells_free(vd_cells c);

typedef struct {
  int64_t n_sites, n_pieces, n_faces, n_verts, n_nbrs;
  int64_t nn_queries;  /* point-in-cell tests (nearest-site queries) performed */
  int64_t clips;       /* clips applied */
  int64_t candidates;  /* sites examined by the nearest-site queries */
  int64_t grid_queries; /* queries not answered by the per-wave site cache (0 for surfaces) */
  int32_t first_bad_site; /* -1, or a site whose carve hit a capacity/degeneracy */
  int32_t failed_stages;  /* bit mask of the stages that failed (VD_STAGE_*), 0 if none */
  int32_t status;         /* vd_status of the last clip */
  double carve_ms;        /* duration of the last clip's main kernel (the persistent
                             per-site kernel for tetrahedra, the per-triangle kernel for
                             surfaces), measured with hipEvents on the caller's stream
                             when time_kernels = 1 (else -1) */
  double split_ms;        /* 0 when timed (no second kernel), else -1 */
  int64_t overflow_records; /* records dropped because an output arena was full
                               (only a no_sync clip can leave them: the status is
                               then VD_ERR_CAPACITY) */
  /* the next six are counted with vd_options.monitor = 1 and read -1 otherwise */
  int64_t low_margin;     /* corner classifications against a clipping plane whose
                             relative margin |n.y - c| / (|n0 y0|+|n1 y1|+|n2 y2|+|c|)
                             was below 1e-12 (near-degenerate decisions) */
  double min_margin;      /* the smallest such relative margin (1 if none below 1e-3) */
  int64_t query_rounds;   /* nearest-site query rounds: a batch of up to four corner
                             tests or lambda steps is one round */
  int64_t corners_classified; /* corner-plane classifications made by the clips */
  int64_t corners_created;    /* corners created by the clips (one 3x3 solve each) */
  int64_t tests_wasted;   /* tested corners that a clip removed besides the one
                             whose test led to it */
  int64_t fan_simplices;  /* simplices of the moment fans (3D: tetrahedra, three per
                             piece corner; surfaces: triangles, one per vertex) */
  int64_t sites_outside;  /* 3D: sites outside every tetrahedron (-1 if not counted:
                             a no_sync clip, or boundary_seeds = 0) */
  int32_t boundary_seeded; /* 3D: 1 if the clip seeded cells from the boundary surface */
  int32_t reserved_;
} vd_cells_info_t;

/* Host struct of sizes and counters (synchronises `stream` of the last call). */
vd_status vd_cells_info(vd_cells c, vd_cells_info_t *info_host);

/* Device pointers into library memory, valid until the next vd_clip_cells on
 * the same handle or vd_cells_free.  After a no_sync clip whose work has not
 * finished yet this returns VD_ERR_NOT_READY (call vd_cells_info, which waits,
 * or retry); after a failed clip it returns that clip's status.  Sites and simplices use the caller's
 * indices.  Pieces of site i are piece_id[cell_piece_off[i] .. cell_piece_off[i+1]),
 * per piece p (an index into the piece arrays):
 *   piece_site[p], piece_simplex[p], piece_mass[p], piece_moment[3p..] (first
 *   moment, absolute coordinates), piece_energy[p],
 *   faces face_label[piece_face_start[p] + k], k < piece_nface[p],
 *   vertices vert_xyz[3(piece_vert_start[p] + k)..], vert_label[3(..)..]
 *   (the labels of the vertex's three planes, counter-clockwise seen from
 *   outside; for triangles the vertex lies on two edges and the third label
 *   is INT32_MAX), k < piece_nvert[p].
 * Pieces of one site are listed by ascending simplex index.
 * Neighbours of site i: nbr[nbr_off[i] .. nbr_off[i+1]), ascending.
 * The piece, face and vertex arrays are arenas of n_piece_slots, n_face_slots
 * and n_vert_slots records: waves fill them in chunks, so a piece slot with
 * piece_site = -1 is unused, and faces / vertices are reached only through
 * the piece offsets. */
typedef struct {
  int64_t n_sites, n_piece_slots, n_face_slots, n_vert_slots;
  const int64_t *cell_piece_off; /* [n+1] */
  const int32_t *piece_id;       /* [cell_piece_off[n]] */
  const int32_t *piece_site, *piece_simplex, *piece_nface, *piece_nvert;
  const int64_t *piece_face_start, *piece_vert_start;
  const double *piece_mass, *piece_moment, *piece_energy;
  const int32_t *face_label;
  const double *vert_xyz;
  const int32_t *vert_label;
  const int64_t *nbr_off; /* [n+1] */
  const int32_t *nbr;
} vd_cells_view_t;

vd_status vd_cells_view(vd_cells c, vd_cells_view_t *view_host);

/* ---------------------------------------------------------------------
 * vd_cell_moments -- per-site mass (volume, or area for surfaces), centroid
 * and energy E_i = integral over Omega_i cap M of |x - v_i|^2 (Eq. 3 with
 * density 1).  A site whose cell misses the domain gets mass 0, centroid
 * v_i, energy 0.  Per-site sums run over the site's pieces in a fixed order
 * (no floating-point atomics), so results are bitwise reproducible.
 *   mass [n], centroid [n*3], energy [n] (nullable): caller-owned device memory.
 * --------------------------------------------------------------------- */
vd_status vd_cell_moments(vd_cells c, double *mass, double *centroid, double *energy,
                          void *stream);

/* ---------------------------------------------------------------------
 * vd_cell_moments_backward -- adjoint of the moments at fixed combinatorics.
 * For L = sum_k g_mass[k] m_k + g_centroid[k].c_k + g_energy[k] E_k it writes
 * dL/dv_i = 2 gE_i m_i (v_i - c_i)
 *         + sum over faces F_ik of cell i of  integral over F_ik of
 *           [(a_i - a_k) + (b_i - b_k).x + (gE_i - gE_k)|x - v_i|^2] (x - v_i)/|v_k - v_i| dA
 * with a_k = g_mass[k] - g_centroid[k].c_k/m_k, b_k = g_centroid[k]/m_k: a face
 * on the bisector of v_i and v_k moves with normal speed (x - v_i).dv_i/|v_k - v_i|
 * (Reynolds transport applied to Eq. 1 and Eq. 3; the paper has no gradient).
 * For surfaces the face is a segment and the speed is divided by the sine
 * between the bisector and the triangle plane.  Requires want_grad = 1 in the
 * options of the vd_clip_cells call.  Deterministic, no atomics.
 *   g_mass [n], g_centroid [n*3], g_energy [n]: device, each nullable (zero).
 *   g_sites [n*3]: device, overwritten.
 * --------------------------------------------------------------------- */
vd_status vd_cell_moments_backward(vd_cells c, const double *g_mass, const double *g_centroid,
                                   const double *g_energy, double *g_sites, void *stream);

/* ---------------------------------------------------------------------
 * vd_cell_moments_backward_noalloc -- vd_cell_moments_backward for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, same
 * kernels and the same result; the per-site weight table the adjoint needs
 * (40 bytes per site) lives in a fixed device array of VD_NOALLOC_MAX_SITES
 * sites that each GPU holds until the process ends, instead of the handle's
 * lazily allocated buffer.  Call it with the device of the handle current.
 * Calls that overlap on one GPU share that array and race: serialise them.
 * Errors: as vd_cell_moments_backward, plus VD_ERR_CAPACITY when the handle
 * has more than VD_NOALLOC_MAX_SITES sites.
 * --------------------------------------------------------------------- */
#define VD_NOALLOC_MAX_SITES (1 << 20)
vd_status vd_cell_moments_backward_noalloc(vd_cells c, const double *g_mass, const double *g_centroid,
                                           const double *g_energy, double *g_sites, void *stream);

#ifdef __cplusplus
}
#endif
#endif
