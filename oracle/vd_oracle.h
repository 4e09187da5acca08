/*
 * vd_oracle.h -- CPU oracle for clipped / restricted Voronoi diagrams.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes is the plain definition of the paper (Sec. 3.1, Eq. 1):
 * for every domain simplex T_a and site v_i the piece
 *     P_{a,i} = T_a  intersected with  { x : |x - v_i| <= |x - v_j|, all j != i },
 * with face labels as in Sec. 3.2 (Fig. 2): a face on the bisector of v_i and
 * v_j carries label j >= 0, a face shared with simplex T_b carries -(b+1),
 * and a face on the domain boundary carries INT32_MIN + f (f = local face).
 *
 * Two modes:
 *   brute  : every site of every simplex is clipped by all n-1 bisectors in
 *            index order -- Eq. 1 written out.
 *   pruned : candidate (simplex, site) pairs are filtered with a Lipschitz
 *            bound on the nearest-site distance, and bisectors are applied in
 *            grid shells around v_i until the security radius of the related
 *            work (Sec. 2.2) proves every remaining half-space contains the
 *            piece.  Every skipped clip is provably a no-op, and vertices are
 *            always recomputed from their three defining planes, so both modes
 *            take the same sign decisions in general position.
 *
 * Status codes: 0 ok, 1 invalid argument, 2 out of memory, 3 degenerate
 * geometry (a vertex not defined by exactly three planes, or a capacity of
 * the fixed-size polytope exceeded).
 */
#ifndef VD_ORACLE_H
#define VD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Result of an oracle run.  All arrays are malloc'd by the oracle and
 * released with vdo_free_result.  Pieces are sorted by (site, simplex). */
typedef struct {
  int64_t n_pieces;
  int32_t *piece_site;     /* [n_pieces] */
  int32_t *piece_simplex;  /* [n_pieces] */
  double *piece_mass;      /* [n_pieces] volume (tets) or area (triangles) */
  double *piece_moment;    /* [n_pieces*3] first moment, absolute coords */
  double *piece_energy;    /* [n_pieces] integral of |x - v_i|^2 */
  int64_t *piece_face_off; /* [n_pieces+1] */
  int32_t *face_label;     /* [n_faces] face/edge labels of each piece */
  double *face_measure;    /* [n_faces] area (tets) or length (triangles) */
  int64_t *face_vert_off;  /* [n_faces+1] */
  int32_t *face_vert;      /* [n_face_verts] piece-local vertex indices; loops are
                              counter-clockwise seen from outside the piece */
  int64_t n_faces, n_face_verts;
  int64_t *piece_vert_off; /* [n_pieces+1] */
  double *vert_xyz;        /* [n_verts*3] absolute coords */
  int32_t *vert_label;     /* [n_verts*3] labels of the defining planes, ascending
                              (for triangles: 2 labels + the slot holds INT32_MAX) */
  int64_t n_verts;
  double min_margin;       /* smallest |signed distance| / scale seen in a cut */
} vdo_result;

/* Clipped VD (simplex_dim 3, k = 4) or restricted VD (simplex_dim 2, k = 3).
 * sites [n*3], verts [nv*3], simp [m*k], adj [m*k] (-1 = boundary).
 * only_sites: NULL -> all sites; else n_only site indices whose pieces are
 * computed (pruned mode only); their candidate simplices are found through a
 * grid over the simplices' bounding boxes with the same Lipschitz filter as
 * the full run, so each listed site gets exactly the pieces the full run
 * gives it.  threads <= 0 -> OpenMP default. */
int vdo_compute(const double *sites, int64_t n, const double *verts, int64_t nv,
                const int32_t *simp, const int32_t *adj, int64_t m, int simplex_dim,
                int brute, const int32_t *only_sites, int64_t n_only, int threads,
                vdo_result *out);

/* Power diagram (Sec. 7.3): as vdo_compute with the half-spaces
 * |x - v_i|^2 - w_i <= |x - v_j|^2 - w_j (weights [n]; NULL = Voronoi).  A
 * site's cell may be empty, and need not contain the site.  The pruned mode
 * uses the matching security radius and candidate bound. */
int vdo_compute_power(const double *sites, const double *weights, int64_t n, const double *verts, int64_t nv,
                      const int32_t *simp, const int32_t *adj, int64_t m, int simplex_dim,
                      int brute, const int32_t *only_sites, int64_t n_only, int threads,
                      vdo_result *out);

void vdo_free_result(vdo_result *r);

/* Adjoint of L = sum_k g_m[k] m_k + g_c[k].c_k + g_E[k] E_k with respect to the
 * sites, at fixed combinatorics, from a result that covers ALL sites.
 * mass/cent are the per-site masses and centroids (from the same result).
 * g_* may be NULL (treated as zero).  g_sites [n*3] is overwritten. */
int vdo_moments_backward(const vdo_result *r, const double *sites, int64_t n,
                         const double *mass, const double *cent,
                         const double *g_m, const double *g_c, const double *g_E,
                         const double *verts, const int32_t *simp, int simplex_dim,
                         double *g_sites);

/* As vdo_moments_backward, for moments weighted by the quadratic density
 * rho (10 coefficients, see vdo_density_moments; NULL = density 1): mass and
 * cent are then the weighted ones and every face integrand carries rho. */
int vdo_moments_backward_rho(const vdo_result *r, const double *sites, int64_t n,
                             const double *mass, const double *cent,
                             const double *g_m, const double *g_c, const double *g_E,
                             const double *verts, const int32_t *simp, int simplex_dim,
                             const double *rho, double *g_sites);

/* Density-weighted moments of every piece of a result (Sec. 7.4, Eq. 3 with
 * rho(x) = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 xy + c6 xz + c7 y^2 + c8 yz
 * + c9 z^2): mass = int rho, moment = int rho x (absolute coordinates),
 * energy = int rho |x - v_i|^2 over each piece, on the fan of simplices from
 * the piece's first vertex with conical (Duffy) product Gauss rules, exact
 * for these polynomial degrees.  Arrays [n_pieces], [3 n_pieces], [n_pieces]. */
int vdo_density_moments(const vdo_result *r, const double *sites, const double *coef, int simplex_dim,
                        double *mass, double *moment, double *energy);

#ifdef __cplusplus
}
#endif
#endif
