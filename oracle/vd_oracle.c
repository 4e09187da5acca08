/*
 * vd_oracle.c -- CPU oracle for clipped / restricted Voronoi diagrams.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the
 * benchmark).  Shares no code with the GPU library.
 *
 * The oracle evaluates the plain definition of a domain-cell intersection
 * (Sec. 3.1, Eq. 1): P_{a,i} = T_a cut by every half-space
 *     H_ij = { x : (x - (v_i+v_j)/2) . (v_j - v_i) <= 0 },   j != i,
 * with the face/edge flags of Sec. 3.2.  Points on a bisector count as
 * inside (Eq. 1 uses "<=").  Polytopes are kept as face loops; a vertex
 * always stores the three planes that define it and its coordinates are
 * recomputed from those planes by Cramer's rule with the planes sorted by
 * key, so a vertex never depends on the order of the clips.  All geometry is
 * in coordinates relative to the site v_i.
 *
 * Moments: volume/area, first moment and the CVT energy integrand of
 * Eq. 3 (density 1) by exact formulas on a fan of simplices.
 * Adjoint: derivative of those moments with respect to the sites at fixed
 * combinatorics (Reynolds transport: a face on the bisector of v_i and v_k
 * moves with normal speed (x - v_i).dv_i / |v_k - v_i|), integrated with
 * exact closed-form simplex monomial integrals.
 */
#include "vd_oracle.h"

#include <float.h>
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OP_MAXPL 128
#define OP_MAXV 256
#define OP_MAXFV 96
#define KEY_SUPPORT (-100)
#define LABEL_NONE INT32_MAX

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static void sub3(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}

/* ------------------------------------------------------------------ */
/* planes and polytopes                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
  double n[3]; /* outward normal (unnormalised) */
  double c;    /* inside: n . y <= c, y relative to the site */
  int key;     /* unique ordering key: bisector j -> j, simplex face f -> -1-f */
  int label;   /* face flag reported to the caller */
} opl;

typedef struct {
  int p[3];    /* plane slots, sorted by key */
  double y[3]; /* coordinates relative to the site */
} ovx;

typedef struct {
  int plane;
  int nv;
  int v[OP_MAXFV];
} ofc;

typedef struct {
  int npl, nvx, nfc;
  opl pl[OP_MAXPL];
  ovx vx[OP_MAXV];
  ofc fc[OP_MAXPL];
} opoly;

/* 2D pieces (restricted VD): a convex polygon inside the supporting plane of
 * a triangle.  Vertex k lies on the support plane and on the planes of the
 * edges (k-1 -> k) and (k -> k+1). */
typedef struct {
  int npl, nv;
  opl pl[OP_MAXPL]; /* slot 0 is the supporting plane */
  int e[OP_MAXFV];  /* plane slot of the edge from vertex k to vertex k+1 */
  double y[OP_MAXFV][3];
} ogon;

/* Vertex of three planes by Cramer's rule, planes taken in key order. */
static int solve3(const opl *a, const opl *b, const opl *c, double *y) {
  const opl *q[3] = {a, b, c};
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (q[j]->key < q[i]->key) { const opl *t = q[i]; q[i] = q[j]; q[j] = t; }
  double c12[3], c20[3], c01[3];
  cross3(q[1]->n, q[2]->n, c12);
  cross3(q[2]->n, q[0]->n, c20);
  cross3(q[0]->n, q[1]->n, c01);
  double det = dot3(q[0]->n, c12);
  if (det == 0.0 || !isfinite(det)) return 3;
  for (int k = 0; k < 3; k++) y[k] = (q[0]->c * c12[k] + q[1]->c * c20[k] + q[2]->c * c01[k]) / det;
  return 0;
}

static void sort3slots(const opl *pl, int *p) {
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (pl[p[j]].key < pl[p[i]].key) { int t = p[i]; p[i] = p[j]; p[j] = t; }
}

/* H_ij relative to v_i: n.y <= c with n = v_j - v_i.  Voronoi (Eq. 1):
 * c = |n|^2 / 2.  Power diagram (Sec. 7.3) with weights w: |x - v_i|^2 - w_i
 * <= |x - v_j|^2 - w_j gives c = (|n|^2 + w_i - w_j) / 2. */
static void bisector_plane(const double *vi, const double *vj, int j, double wij, opl *h) {
  sub3(vj, vi, h->n);
  h->c = 0.5 * (dot3(h->n, h->n) + wij);
  h->key = j;
  h->label = j;
}

static int face_label(const int32_t *adj, int64_t a, int k, int f) {
  int32_t b = adj[a * k + f];
  return b >= 0 ? -(b + 1) : INT32_MIN + f;
}

/* Tetrahedron T_a as a polytope relative to site v (positively oriented
 * tets; local face f is opposite vertex f, loops counter-clockwise seen
 * from outside). */
static int init_tet(const double *verts, const int32_t *tet, const int32_t *adj, int64_t a,
                    const double *v, opoly *P) {
  static const int floop[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
  double q[4][3];
  for (int k = 0; k < 4; k++) sub3(&verts[3 * (int64_t)tet[k]], v, q[k]);
  P->npl = 4; P->nvx = 4; P->nfc = 4;
  for (int f = 0; f < 4; f++) {
    const double *A = q[floop[f][0]], *B = q[floop[f][1]], *C = q[floop[f][2]];
    double ab[3], ac[3];
    sub3(B, A, ab); sub3(C, A, ac);
    cross3(ab, ac, P->pl[f].n);
    P->pl[f].c = dot3(P->pl[f].n, A);
    P->pl[f].key = -1 - f;
    P->pl[f].label = face_label(adj, a, 4, f);
    P->fc[f].plane = f;
    P->fc[f].nv = 3;
    for (int t = 0; t < 3; t++) P->fc[f].v[t] = floop[f][t];
  }
  for (int k = 0; k < 4; k++) {
    int s = 0;
    for (int f = 0; f < 4; f++) if (f != k) P->vx[k].p[s++] = f;
    sort3slots(P->pl, P->vx[k].p);
    if (solve3(&P->pl[P->vx[k].p[0]], &P->pl[P->vx[k].p[1]], &P->pl[P->vx[k].p[2]], P->vx[k].y)) return 3;
  }
  return 0;
}

/* Cut polytope P by half-space h.  Returns 0 = unchanged, 1 = cut (result in
 * Q), 2 = empty, 3 = degenerate. */
static int clip3(const opoly *P, const opl *h, opoly *Q, double *margin) {
  double s[OP_MAXV];
  int any_out = 0, all_out = 1;
  double hn = sqrt(dot3(h->n, h->n));
  for (int v = 0; v < P->nvx; v++) {
    s[v] = dot3(h->n, P->vx[v].y) - h->c;
    if (s[v] > 0.0) any_out = 1; else all_out = 0;
  }
  if (!any_out) return 0;
  if (all_out) return 2;
  for (int v = 0; v < P->nvx; v++) {
    double sc = sqrt(dot3(P->vx[v].y, P->vx[v].y)) + hn;
    double mg = fabs(s[v]) / (hn * sc);
    if (mg < *margin) *margin = mg;
  }
  if (P->npl + 1 > OP_MAXPL) return 3;
  memcpy(Q->pl, P->pl, sizeof(opl) * P->npl);
  int H = P->npl;
  Q->pl[H] = *h;
  Q->npl = P->npl + 1;
  int remap[OP_MAXV];
  int nq = 0;
  for (int v = 0; v < P->nvx; v++) {
    if (s[v] <= 0.0) { Q->vx[nq] = P->vx[v]; remap[v] = nq++; } else remap[v] = -1;
  }
  /* new vertices on cut edges, shared by the two faces of the edge */
  int ek_a[OP_MAXV], ek_b[OP_MAXV], ek_v[OP_MAXV], nek = 0;
  int entry_of[OP_MAXPL], exit_of[OP_MAXPL];
  Q->nfc = 0;
  int ncut = 0;
  for (int f = 0; f < P->nfc; f++) {
    const ofc *F = &P->fc[f];
    ofc G;
    G.plane = F->plane;
    G.nv = 0;
    int ent = -1, ext = -1;
    for (int t = 0; t < F->nv; t++) {
      int va = F->v[t], vb = F->v[(t + 1) % F->nv];
      int ina = s[va] <= 0.0, inb = s[vb] <= 0.0;
      if (ina) {
        if (G.nv >= OP_MAXFV) return 3;
        G.v[G.nv++] = remap[va];
      }
      if (ina != inb) {
        int lo = va < vb ? va : vb, hi = va < vb ? vb : va, nv = -1;
        for (int e = 0; e < nek; e++)
          if (ek_a[e] == lo && ek_b[e] == hi) { nv = ek_v[e]; break; }
        if (nv < 0) {
          /* planes shared by va and vb: exactly two in general position */
          int sh[3], ns = 0;
          for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++)
              if (P->vx[va].p[x] == P->vx[vb].p[y]) sh[ns++] = P->vx[va].p[x];
          if (ns != 2) return 3;
          if (nq >= OP_MAXV) return 3;
          ovx *X = &Q->vx[nq];
          X->p[0] = sh[0]; X->p[1] = sh[1]; X->p[2] = H;
          sort3slots(Q->pl, X->p);
          if (solve3(&Q->pl[X->p[0]], &Q->pl[X->p[1]], &Q->pl[X->p[2]], X->y)) return 3;
          nv = nq++;
          ek_a[nek] = lo; ek_b[nek] = hi; ek_v[nek] = nv; nek++;
        }
        if (G.nv >= OP_MAXFV) return 3;
        G.v[G.nv++] = nv;
        if (ina) ext = nv; else ent = nv;
      }
    }
    if (G.nv >= 3) {
      Q->fc[Q->nfc++] = G;
      if (ent >= 0 || ext >= 0) {
        if (ent < 0 || ext < 0) return 3;
        entry_of[ncut] = ent; exit_of[ncut] = ext; ncut++;
      }
    } else if (G.nv > 0) {
      return 3; /* a face reduced to an edge or a point: not general position */
    }
  }
  if (ncut < 3) return 3;
  /* face on h: the cut edge of face f is traversed exit -> entry in f, so the
   * new face (seen from outside h) runs entry -> exit. */
  ofc N;
  N.plane = H;
  N.nv = 0;
  int start = entry_of[0], cur = start;
  for (int it = 0; it <= ncut; it++) {
    if (N.nv >= OP_MAXFV) return 3;
    N.v[N.nv++] = cur;
    int nxt = -1;
    for (int c = 0; c < ncut; c++) if (entry_of[c] == cur) { nxt = exit_of[c]; break; }
    if (nxt < 0) return 3;
    cur = nxt;
    if (cur == start) break;
  }
  if (cur != start || N.nv != ncut) return 3;
  Q->fc[Q->nfc++] = N;
  Q->nvx = nq;
  return 1;
}

/* Moments of a polytope relative to the site: volume, first moment and
 * integral of |y|^2, on a fan of tetrahedra (o, y0, yj, yj+1) whose apex o
 * is a vertex of the polytope.  Any apex gives the same sums in exact
 * arithmetic; an apex on the polytope keeps the rounding error of the volume
 * proportional to the polytope's own size, so a piece far smaller than its
 * distance to the site still gets a volume of the right sign. */
static void poly_moments3(const opoly *P, double *vol, double *mom, double *en) {
  double V = 0, M[3] = {0, 0, 0}, E = 0;
  const double *o = P->vx[0].y;
  for (int f = 0; f < P->nfc; f++) {
    const ofc *F = &P->fc[f];
    const double *a = P->vx[F->v[0]].y;
    double ao[3];
    sub3(a, o, ao);
    for (int t = 1; t + 1 < F->nv; t++) {
      const double *b = P->vx[F->v[t]].y, *c = P->vx[F->v[t + 1]].y;
      double bo[3], co[3], bc[3];
      sub3(b, o, bo);
      sub3(c, o, co);
      cross3(bo, co, bc);
      double v6 = dot3(ao, bc) / 6.0;
      double S[3] = {o[0] + a[0] + b[0] + c[0], o[1] + a[1] + b[1] + c[1], o[2] + a[2] + b[2] + c[2]};
      V += v6;
      for (int k = 0; k < 3; k++) M[k] += v6 * S[k] / 4.0;
      /* integral of |y|^2 over tet (o,a,b,c) = V/20 (sum |y_k|^2 + |sum y_k|^2) */
      E += v6 / 20.0 * (dot3(o, o) + dot3(a, a) + dot3(b, b) + dot3(c, c) + dot3(S, S));
    }
  }
  *vol = V;
  for (int k = 0; k < 3; k++) mom[k] = M[k];
  *en = E;
}

static double face_area3(const opoly *P, const ofc *F) {
  double A[3] = {0, 0, 0};
  const double *a = P->vx[F->v[0]].y;
  for (int t = 1; t + 1 < F->nv; t++) {
    double ab[3], ac[3], cr[3];
    sub3(P->vx[F->v[t]].y, a, ab);
    sub3(P->vx[F->v[t + 1]].y, a, ac);
    cross3(ab, ac, cr);
    for (int k = 0; k < 3; k++) A[k] += cr[k];
  }
  return 0.5 * sqrt(dot3(A, A));
}

/* ---- 2D ----------------------------------------------------------- */
static int init_tri(const double *verts, const int32_t *tri, const int32_t *adj, int64_t a,
                    const double *v, ogon *G) {
  double q[3][3];
  for (int k = 0; k < 3; k++) sub3(&verts[3 * (int64_t)tri[k]], v, q[k]);
  double ab[3], ac[3], N[3];
  sub3(q[1], q[0], ab); sub3(q[2], q[0], ac);
  cross3(ab, ac, N);
  G->npl = 4;
  opl *S = &G->pl[0];
  memcpy(S->n, N, sizeof N);
  S->c = dot3(N, q[0]);
  S->key = KEY_SUPPORT;
  S->label = LABEL_NONE;
  for (int e = 0; e < 3; e++) {
    const double *A = q[(e + 1) % 3], *B = q[(e + 2) % 3];
    double d[3];
    sub3(B, A, d);
    opl *L = &G->pl[1 + e];
    cross3(d, N, L->n);
    L->c = dot3(L->n, A);
    L->key = -1 - e;
    L->label = face_label(adj, a, 3, e);
  }
  G->nv = 3;
  for (int k = 0; k < 3; k++) {
    G->e[k] = 1 + (k + 2) % 3; /* edge from q_k to q_{k+1} is opposite q_{k+2} */
    int prev = 1 + (k + 1) % 3;
    if (solve3(&G->pl[0], &G->pl[prev], &G->pl[G->e[k]], G->y[k])) return 3;
  }
  return 0;
}

static int clip2(const ogon *P, const opl *h, ogon *Q, double *margin) {
  double s[OP_MAXFV];
  int any_out = 0, all_out = 1;
  double hn = sqrt(dot3(h->n, h->n));
  for (int v = 0; v < P->nv; v++) {
    s[v] = dot3(h->n, P->y[v]) - h->c;
    if (s[v] > 0.0) any_out = 1; else all_out = 0;
  }
  if (!any_out) return 0;
  if (all_out) return 2;
  for (int v = 0; v < P->nv; v++) {
    double sc = sqrt(dot3(P->y[v], P->y[v])) + hn;
    double mg = fabs(s[v]) / (hn * sc);
    if (mg < *margin) *margin = mg;
  }
  if (P->npl + 1 > OP_MAXPL) return 3;
  memcpy(Q->pl, P->pl, sizeof(opl) * P->npl);
  int H = P->npl;
  Q->pl[H] = *h;
  Q->npl = P->npl + 1;
  Q->nv = 0;
  for (int v = 0; v < P->nv; v++) {
    int w = (v + 1) % P->nv;
    int inv = s[v] <= 0.0, inw = s[w] <= 0.0;
    if (inv) {
      if (Q->nv >= OP_MAXFV) return 3;
      memcpy(Q->y[Q->nv], P->y[v], sizeof(double) * 3);
      Q->e[Q->nv] = P->e[v];
      Q->nv++;
    }
    if (inv != inw) {
      if (Q->nv >= OP_MAXFV) return 3;
      if (solve3(&Q->pl[0], &Q->pl[P->e[v]], &Q->pl[H], Q->y[Q->nv])) return 3;
      /* leaving: the edge after the new vertex runs along h; entering: along e[v] */
      Q->e[Q->nv] = inv ? H : P->e[v];
      Q->nv++;
    }
  }
  if (Q->nv < 3) return 3;
  return 1;
}

static void gon_moments(const ogon *P, double *area, double *mom, double *en) {
  const double *N = P->pl[0].n;
  double nn = sqrt(dot3(N, N));
  double A = 0, M[3] = {0, 0, 0}, E = 0;
  const double *a = P->y[0];
  for (int t = 1; t + 1 < P->nv; t++) {
    const double *b = P->y[t], *c = P->y[t + 1];
    double ab[3], ac[3], cr[3];
    sub3(b, a, ab); sub3(c, a, ac);
    cross3(ab, ac, cr);
    double ar = 0.5 * dot3(cr, N) / nn;
    double S[3] = {a[0] + b[0] + c[0], a[1] + b[1] + c[1], a[2] + b[2] + c[2]};
    A += ar;
    for (int k = 0; k < 3; k++) M[k] += ar * S[k] / 3.0;
    /* integral of |y|^2 over a triangle = A/12 (sum |y_k|^2 + |sum y_k|^2) */
    E += ar / 12.0 * (dot3(a, a) + dot3(b, b) + dot3(c, c) + dot3(S, S));
  }
  *area = A;
  for (int k = 0; k < 3; k++) mom[k] = M[k];
  *en = E;
}

/* ------------------------------------------------------------------ */
/* oracle-own uniform grid over the sites (for pruning only)            */
/* ------------------------------------------------------------------ */
typedef struct {
  double lo[3], h;
  int g[3];
  int32_t *start; /* [ncell+1] */
  int32_t *ids;   /* [n] */
} ogrid;

static int64_t ocell(const ogrid *G, int x, int y, int z) { return x + (int64_t)G->g[0] * (y + (int64_t)G->g[1] * z); }

static void ocoord(const ogrid *G, const double *p, int *c) {
  for (int k = 0; k < 3; k++) {
    double t = floor((p[k] - G->lo[k]) / G->h);
    int ci = t < 0 ? 0 : (t >= G->g[k] ? G->g[k] - 1 : (int)t);
    c[k] = ci;
  }
}

static int ogrid_build(ogrid *G, const double *sites, int64_t n, const double *verts, int64_t nv) {
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int64_t i = 0; i < n; i++)
    for (int k = 0; k < 3; k++) { double x = sites[3 * i + k]; if (x < lo[k]) lo[k] = x; if (x > hi[k]) hi[k] = x; }
  for (int64_t i = 0; i < nv; i++)
    for (int k = 0; k < 3; k++) { double x = verts[3 * i + k]; if (x < lo[k]) lo[k] = x; if (x > hi[k]) hi[k] = x; }
  double ext = 0;
  for (int k = 0; k < 3; k++) if (hi[k] - lo[k] > ext) ext = hi[k] - lo[k];
  if (ext <= 0) ext = 1;
  int gm = (int)ceil(cbrt((double)n / 2.0));
  if (gm < 1) gm = 1;
  G->h = ext / gm * (1.0 + 1e-12);
  for (int k = 0; k < 3; k++) {
    G->lo[k] = lo[k];
    G->g[k] = (int)ceil((hi[k] - lo[k]) / G->h);
    if (G->g[k] < 1) G->g[k] = 1;
  }
  int64_t nc = (int64_t)G->g[0] * G->g[1] * G->g[2];
  G->start = (int32_t *)calloc(nc + 1, sizeof(int32_t));
  G->ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  if (!G->start || !G->ids || !cid) { free(cid); return 2; }
  for (int64_t i = 0; i < n; i++) {
    int c[3];
    ocoord(G, &sites[3 * i], c);
    cid[i] = ocell(G, c[0], c[1], c[2]);
    G->start[cid[i] + 1]++;
  }
  for (int64_t c = 0; c < nc; c++) G->start[c + 1] += G->start[c];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (nc + 1));
  if (!fill) { free(cid); return 2; }
  memcpy(fill, G->start, sizeof(int32_t) * (nc + 1));
  for (int64_t i = 0; i < n; i++) G->ids[fill[cid[i]]++] = (int32_t)i;
  free(fill);
  free(cid);
  return 0;
}

static void ogrid_free(ogrid *G) { free(G->start); free(G->ids); }

/* distance from p to its nearest site (grid shells, exact) */
static double onn_dist(const ogrid *G, const double *sites, const double *p) {
  int c[3];
  ocoord(G, p, c);
  double best = DBL_MAX;
  int smax = G->g[0] + G->g[1] + G->g[2];
  for (int s = 0; s <= smax; s++) {
    int any = 0;
    for (int z = c[2] - s; z <= c[2] + s; z++) {
      if (z < 0 || z >= G->g[2]) continue;
      for (int y = c[1] - s; y <= c[1] + s; y++) {
        if (y < 0 || y >= G->g[1]) continue;
        for (int x = c[0] - s; x <= c[0] + s; x++) {
          if (x < 0 || x >= G->g[0]) continue;
          int cheb = abs(x - c[0]);
          if (abs(y - c[1]) > cheb) cheb = abs(y - c[1]);
          if (abs(z - c[2]) > cheb) cheb = abs(z - c[2]);
          if (cheb != s) continue;
          any = 1;
          int64_t ci = ocell(G, x, y, z);
          for (int32_t t = G->start[ci]; t < G->start[ci + 1]; t++) {
            const double *q = &sites[3 * (int64_t)G->ids[t]];
            double d[3];
            sub3(q, p, d);
            double dd = dot3(d, d);
            if (dd < best) best = dd;
          }
        }
      }
    }
    /* unvisited sites lie at least s*h away */
    if (best < DBL_MAX && sqrt(best) <= s * G->h) break;
    if (!any && s > 0 && best < DBL_MAX) break;
  }
  return sqrt(best);
}

/* ------------------------------------------------------------------ */
/* growable output buffers                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t np, cp;
  int32_t *site, *simp;
  double *mass, *mom, *en;
  int64_t *foff, *voff; /* local counts, converted later */
  int64_t nf, cf;
  int32_t *flab;
  double *fmeas;
  int64_t *fvoff; int64_t nfv, cfv; int32_t *fv;
  int64_t nv, cv;
  double *xyz;
  int32_t *vlab;
  int err;
  double margin;
} obuf;

#define GROW(ptr, cnt, cap, need, T)                                             \
  do {                                                                           \
    if ((need) > (cap)) {                                                        \
      int64_t nc_ = (cap) ? (cap) : 64;                                          \
      while (nc_ < (need)) nc_ *= 2;                                             \
      T *np_ = (T *)realloc((ptr), sizeof(T) * nc_);                             \
      if (!np_) { b->err = 2; return; }                                          \
      (ptr) = np_;                                                               \
      (cap) = nc_;                                                               \
    }                                                                            \
  } while (0)

static void obuf_piece_begin(obuf *b, int32_t site, int32_t simp, double mass, const double *mom, double en) {
  if (b->np + 1 > b->cp) {
    int64_t nc = b->cp ? b->cp * 2 : 64;
    int32_t *s1 = (int32_t *)realloc(b->site, sizeof(int32_t) * nc);
    if (s1) b->site = s1;
    int32_t *s2 = (int32_t *)realloc(b->simp, sizeof(int32_t) * nc);
    if (s2) b->simp = s2;
    double *d1 = (double *)realloc(b->mass, sizeof(double) * nc);
    if (d1) b->mass = d1;
    double *d2 = (double *)realloc(b->mom, sizeof(double) * 3 * nc);
    if (d2) b->mom = d2;
    double *d3 = (double *)realloc(b->en, sizeof(double) * nc);
    if (d3) b->en = d3;
    int64_t *o1 = (int64_t *)realloc(b->foff, sizeof(int64_t) * nc);
    if (o1) b->foff = o1;
    int64_t *o2 = (int64_t *)realloc(b->voff, sizeof(int64_t) * nc);
    if (o2) b->voff = o2;
    if (!s1 || !s2 || !d1 || !d2 || !d3 || !o1 || !o2) { b->err = 2; return; }
    b->cp = nc;
  }
  int64_t p = b->np++;
  b->site[p] = site; b->simp[p] = simp; b->mass[p] = mass; b->en[p] = en;
  for (int k = 0; k < 3; k++) b->mom[3 * p + k] = mom[k];
  b->foff[p] = b->nf;
  b->voff[p] = b->nv;
}

static void obuf_face(obuf *b, int32_t label, double meas, const int32_t *loop, int nl) {
  GROW(b->flab, b->nf, b->cf, b->nf + 1, int32_t);
  int64_t cap = b->cf;
  /* fmeas and fvoff share the face capacity */
  double *fm = (double *)realloc(b->fmeas, sizeof(double) * cap);
  int64_t *fo = (int64_t *)realloc(b->fvoff, sizeof(int64_t) * cap);
  if (!fm || !fo) { if (fm) b->fmeas = fm; if (fo) b->fvoff = fo; b->err = 2; return; }
  b->fmeas = fm; b->fvoff = fo;
  GROW(b->fv, b->nfv, b->cfv, b->nfv + nl, int32_t);
  b->flab[b->nf] = label;
  b->fmeas[b->nf] = meas;
  b->fvoff[b->nf] = b->nfv;
  memcpy(&b->fv[b->nfv], loop, sizeof(int32_t) * nl);
  b->nfv += nl;
  b->nf++;
}

static void obuf_vert(obuf *b, const double *xyz, const int32_t *lab) {
  if (b->nv + 1 > b->cv) {
    int64_t nc = b->cv ? b->cv * 2 : 256;
    double *x = (double *)realloc(b->xyz, sizeof(double) * 3 * nc);
    if (x) b->xyz = x;
    int32_t *l = (int32_t *)realloc(b->vlab, sizeof(int32_t) * 3 * nc);
    if (l) b->vlab = l;
    if (!x || !l) { b->err = 2; return; }
    b->cv = nc;
  }
  for (int k = 0; k < 3; k++) { b->xyz[3 * b->nv + k] = xyz[k]; b->vlab[3 * b->nv + k] = lab[k]; }
  b->nv++;
}

static void sort3i(int32_t *l) {
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (l[j] < l[i]) { int32_t t = l[i]; l[i] = l[j]; l[j] = t; }
}

static void emit_poly3(obuf *b, const opoly *P, int32_t site, int32_t simp, const double *v) {
  double vol, mom[3], en;
  poly_moments3(P, &vol, mom, &en);
  double am[3];
  for (int k = 0; k < 3; k++) am[k] = mom[k] + vol * v[k];
  obuf_piece_begin(b, site, simp, vol, am, en);
  if (b->err) return;
  for (int f = 0; f < P->nfc; f++) {
    int32_t loop[OP_MAXFV];
    for (int t = 0; t < P->fc[f].nv; t++) loop[t] = P->fc[f].v[t];
    obuf_face(b, P->pl[P->fc[f].plane].label, face_area3(P, &P->fc[f]), loop, P->fc[f].nv);
    if (b->err) return;
  }
  for (int x = 0; x < P->nvx; x++) {
    double xyz[3];
    int32_t lab[3];
    for (int k = 0; k < 3; k++) { xyz[k] = P->vx[x].y[k] + v[k]; lab[k] = P->pl[P->vx[x].p[k]].label; }
    sort3i(lab);
    obuf_vert(b, xyz, lab);
    if (b->err) return;
  }
}

static void emit_gon(obuf *b, const ogon *P, int32_t site, int32_t simp, const double *v) {
  double ar, mom[3], en;
  gon_moments(P, &ar, mom, &en);
  double am[3];
  for (int k = 0; k < 3; k++) am[k] = mom[k] + ar * v[k];
  obuf_piece_begin(b, site, simp, ar, am, en);
  if (b->err) return;
  for (int t = 0; t < P->nv; t++) {
    int w = (t + 1) % P->nv;
    double d[3];
    sub3(P->y[w], P->y[t], d);
    int32_t loop[2] = {t, w};
    obuf_face(b, P->pl[P->e[t]].label, sqrt(dot3(d, d)), loop, 2);
    if (b->err) return;
  }
  for (int t = 0; t < P->nv; t++) {
    double xyz[3];
    int32_t lab[3];
    int prev = P->e[(t + P->nv - 1) % P->nv];
    for (int k = 0; k < 3; k++) xyz[k] = P->y[t][k] + v[k];
    lab[0] = P->pl[prev].label; lab[1] = P->pl[P->e[t]].label; lab[2] = LABEL_NONE;
    sort3i(lab);
    obuf_vert(b, xyz, lab);
    if (b->err) return;
  }
}

/* ------------------------------------------------------------------ */
/* one (simplex, site) pair                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  const double *sites;
  int64_t n;
  const double *verts;
  const int32_t *simp, *adj;
  int dim, k;
  int brute;
  const ogrid *G;
  const double *w;     /* power weights (NULL: Voronoi) */
  double wmin, wmax;
} octx;

/* Clip the piece of site i in simplex a.  Returns 0 (empty), 1 (kept in
 * *P3 / *P2), or 3 (degenerate). */
static int carve_pair(const octx *C, int64_t a, int64_t i, opoly *bufA, opoly *bufB,
                      ogon *gA, ogon *gB, int *which, double *margin) {
  const double *v = &C->sites[3 * i];
  opoly *P = bufA, *Q = bufB;
  ogon *Pg = gA, *Qg = gB;
  int st;
  if (C->dim == 3) st = init_tet(C->verts, &C->simp[a * 4], C->adj, a, v, P);
  else st = init_tri(C->verts, &C->simp[a * 3], C->adj, a, v, Pg);
  if (st) return 3;
  opl h;
#define APPLY_J(jj)                                                               \
  do {                                                                            \
    bisector_plane(v, &C->sites[3 * (int64_t)(jj)], (int)(jj),                    \
                   C->w ? C->w[i] - C->w[(jj)] : 0.0, &h);                          \
    int r_;                                                                       \
    if (C->dim == 3) {                                                            \
      r_ = clip3(P, &h, Q, margin);                                               \
      if (r_ == 1) { opoly *t_ = P; P = Q; Q = t_; }                              \
    } else {                                                                      \
      r_ = clip2(Pg, &h, Qg, margin);                                             \
      if (r_ == 1) { ogon *t_ = Pg; Pg = Qg; Qg = t_; }                           \
    }                                                                             \
    if (r_ == 2) return 0;                                                        \
    if (r_ == 3) return 3;                                                        \
  } while (0)

  if (C->brute) {
    for (int64_t j = 0; j < C->n; j++) {
      if (j == i) continue;
      APPLY_J(j);
    }
  } else {
    const ogrid *G = C->G;
    int c[3];
    ocoord(G, v, c);
    int smax = G->g[0] + G->g[1] + G->g[2];
    for (int s = 0; s <= smax; s++) {
      int any = 0;
      for (int z = c[2] - s; z <= c[2] + s; z++) {
        if (z < 0 || z >= G->g[2]) continue;
        for (int y = c[1] - s; y <= c[1] + s; y++) {
          if (y < 0 || y >= G->g[1]) continue;
          for (int x = c[0] - s; x <= c[0] + s; x++) {
            if (x < 0 || x >= G->g[0]) continue;
            int cheb = abs(x - c[0]);
            if (abs(y - c[1]) > cheb) cheb = abs(y - c[1]);
            if (abs(z - c[2]) > cheb) cheb = abs(z - c[2]);
            if (cheb != s) continue;
            any = 1;
            int64_t ci = ocell(G, x, y, z);
            for (int32_t t = G->start[ci]; t < G->start[ci + 1]; t++) {
              int64_t j = G->ids[t];
              if (j == i) continue;
              APPLY_J(j);
            }
          }
        }
      }
      if (!any) break; /* the shell lies entirely outside the grid */
      /* security radius: every unvisited site is >= s*h from v_i; if that is
       * at least twice the largest |x - v_i| over the piece, each remaining
       * half-space contains the piece.  With power weights, a site at distance
       * d >= R from v_i has |x - v_j|^2 - w_j >= (d - R)^2 - w_max for x in the
       * piece, which is >= R^2 - w_i >= |x - v_i|^2 - w_i once
       * d >= R + sqrt(R^2 + w_max - w_i). */
      double R2 = 0;
      if (C->dim == 3) {
        for (int x = 0; x < P->nvx; x++) { double d = dot3(P->vx[x].y, P->vx[x].y); if (d > R2) R2 = d; }
      } else {
        for (int x = 0; x < Pg->nv; x++) { double d = dot3(Pg->y[x], Pg->y[x]); if (d > R2) R2 = d; }
      }
      double reach = 2.0 * sqrt(R2);
      if (C->w) {
        double t = R2 + C->wmax - C->w[i];
        reach = sqrt(R2) + (t > 0 ? sqrt(t) : 0.0);
      }
      if (s * G->h >= reach) break;
    }
  }
#undef APPLY_J
  if (C->dim == 3) {
    double vol, mom[3], en;
    poly_moments3(P, &vol, mom, &en);
    if (!(vol > 0.0)) return 0;
    if (P != bufA) *bufA = *P;
  } else {
    double ar, mom[3], en;
    gon_moments(Pg, &ar, mom, &en);
    if (!(ar > 0.0)) return 0;
    if (Pg != gA) *gA = *Pg;
  }
  *which = 0;
  return 1;
}

/* bounding box and diameter of simplex a */
static void simplex_box(const octx *C, int64_t a, double *lo, double *hi, double *diam) {
  for (int k = 0; k < 3; k++) { lo[k] = DBL_MAX; hi[k] = -DBL_MAX; }
  double dm = 0;
  for (int u = 0; u < C->k; u++) {
    const double *p = &C->verts[3 * (int64_t)C->simp[a * C->k + u]];
    for (int k = 0; k < 3; k++) { if (p[k] < lo[k]) lo[k] = p[k]; if (p[k] > hi[k]) hi[k] = p[k]; }
    for (int w = u + 1; w < C->k; w++) {
      const double *q = &C->verts[3 * (int64_t)C->simp[a * C->k + w]];
      double d[3];
      sub3(p, q, d);
      double dd = sqrt(dot3(d, d));
      if (dd > dm) dm = dd;
    }
  }
  *diam = dm;
}

static double box_dist(const double *lo, const double *hi, const double *p) {
  double d2 = 0;
  for (int k = 0; k < 3; k++) {
    double d = p[k] < lo[k] ? lo[k] - p[k] : (p[k] > hi[k] ? p[k] - hi[k] : 0.0);
    d2 += d * d;
  }
  return sqrt(d2);
}

/* ------------------------------------------------------------------ */
/* oracle-own uniform grid over the simplices' bounding boxes: finds the  */
/* candidate simplices of one site (sampled-site mode) without a scan of  */
/* all m simplices                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  double lo[3], h;
  int g[3];
  int32_t *start; /* [ncell+1] */
  int32_t *ids;   /* simplices overlapping each cell */
  double rmax;    /* largest Lipschitz radius r_a */
} osgrid;

static void oscoord(const osgrid *S, const double *p, int *c) {
  for (int k = 0; k < 3; k++) {
    double t = floor((p[k] - S->lo[k]) / S->h);
    c[k] = t < 0 ? 0 : (t >= S->g[k] ? S->g[k] - 1 : (int)t);
  }
}

static int64_t oscell(const osgrid *S, int x, int y, int z) { return x + (int64_t)S->g[0] * (y + (int64_t)S->g[1] * z); }

static int osgrid_build(osgrid *S, const octx *C, int64_t m, const double *ra) {
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  S->rmax = 0;
  for (int64_t a = 0; a < m; a++) {
    double l[3], h[3], dm;
    simplex_box(C, a, l, h, &dm);
    for (int k = 0; k < 3; k++) { if (l[k] < lo[k]) lo[k] = l[k]; if (h[k] > hi[k]) hi[k] = h[k]; }
    if (ra[a] > S->rmax) S->rmax = ra[a];
  }
  double ext = 0;
  for (int k = 0; k < 3; k++) if (hi[k] - lo[k] > ext) ext = hi[k] - lo[k];
  if (ext <= 0) ext = 1;
  int gm = (int)ceil(cbrt((double)m / 2.0));
  if (gm < 1) gm = 1;
  S->h = ext / gm * (1.0 + 1e-12);
  for (int k = 0; k < 3; k++) {
    S->lo[k] = lo[k];
    S->g[k] = (int)ceil((hi[k] - lo[k]) / S->h);
    if (S->g[k] < 1) S->g[k] = 1;
  }
  int64_t nc = (int64_t)S->g[0] * S->g[1] * S->g[2];
  S->start = (int32_t *)calloc(nc + 1, sizeof(int32_t));
  if (!S->start) return 2;
  /* two passes: count, then fill */
  for (int pass = 0; pass < 2; pass++) {
    int32_t *fill = NULL;
    if (pass == 1) {
      for (int64_t c = 0; c < nc; c++) S->start[c + 1] += S->start[c];
      S->ids = (int32_t *)malloc(sizeof(int32_t) * (S->start[nc] > 0 ? S->start[nc] : 1));
      fill = (int32_t *)malloc(sizeof(int32_t) * (nc + 1));
      if (!S->ids || !fill) { free(fill); return 2; }
      memcpy(fill, S->start, sizeof(int32_t) * (nc + 1));
    }
    for (int64_t a = 0; a < m; a++) {
      double l[3], h[3], dm;
      int c0[3], c1[3];
      simplex_box(C, a, l, h, &dm);
      oscoord(S, l, c0);
      oscoord(S, h, c1);
      for (int z = c0[2]; z <= c1[2]; z++)
        for (int y = c0[1]; y <= c1[1]; y++)
          for (int x = c0[0]; x <= c1[0]; x++) {
            int64_t c = oscell(S, x, y, z);
            if (pass == 0) S->start[c + 1]++;
            else S->ids[fill[c]++] = (int32_t)a;
          }
    }
    free(fill);
  }
  return 0;
}

static void osgrid_free(osgrid *S) { free(S->start); free(S->ids); }

/* ------------------------------------------------------------------ */
/* entry point                                                           */
/* ------------------------------------------------------------------ */
typedef struct { int32_t site, simp; int thread; int64_t idx; } pkey;
static int cmp_pkey(const void *x, const void *y) {
  const pkey *a = (const pkey *)x, *b = (const pkey *)y;
  if (a->site != b->site) return a->site < b->site ? -1 : 1;
  if (a->simp != b->simp) return a->simp < b->simp ? -1 : 1;
  return 0;
}

static void obuf_free(obuf *b) {
  free(b->site); free(b->simp); free(b->mass); free(b->mom); free(b->en);
  free(b->foff); free(b->voff); free(b->flab); free(b->fmeas); free(b->fvoff); free(b->fv);
  free(b->xyz); free(b->vlab);
}

int vdo_compute(const double *sites, int64_t n, const double *verts, int64_t nv,
                const int32_t *simp, const int32_t *adj, int64_t m, int simplex_dim,
                int brute, const int32_t *only_sites, int64_t n_only, int threads,
                vdo_result *out) {
  return vdo_compute_power(sites, NULL, n, verts, nv, simp, adj, m, simplex_dim, brute, only_sites, n_only,
                           threads, out);
}

int vdo_compute_power(const double *sites, const double *weights, int64_t n, const double *verts, int64_t nv,
                      const int32_t *simp, const int32_t *adj, int64_t m, int simplex_dim,
                      int brute, const int32_t *only_sites, int64_t n_only, int threads,
                      vdo_result *out) {
  memset(out, 0, sizeof *out);
  out->min_margin = DBL_MAX;
  if (n < 1 || m < 1 || (simplex_dim != 2 && simplex_dim != 3) || !sites || !verts || !simp || !adj)
    return 1;
  if (only_sites && brute) return 1;
  int k = simplex_dim + 1;
  for (int64_t a = 0; a < m * k; a++) if (simp[a] < 0 || simp[a] >= nv || adj[a] < -1 || adj[a] >= m) return 1;
  for (int64_t i = 0; i < 3 * n; i++) if (!isfinite(sites[i])) return 1;

  ogrid G;
  memset(&G, 0, sizeof G);
  if (ogrid_build(&G, sites, n, verts, nv)) { ogrid_free(&G); return 2; }
  octx C = {sites, n, verts, simp, adj, simplex_dim, k, brute, &G, weights, 0.0, 0.0};
  if (weights) {
    C.wmin = DBL_MAX;
    C.wmax = -DBL_MAX;
    for (int64_t i = 0; i < n; i++) {
      if (!isfinite(weights[i])) { ogrid_free(&G); return 1; }
      if (weights[i] < C.wmin) C.wmin = weights[i];
      if (weights[i] > C.wmax) C.wmax = weights[i];
    }
  }

#ifdef _OPENMP
  int nt = threads > 0 ? threads : omp_get_max_threads();
#else
  int nt = 1;
  (void)threads;
#endif
  obuf *bufs = (obuf *)calloc(nt, sizeof(obuf));
  if (!bufs) { ogrid_free(&G); return 2; }
  for (int t = 0; t < nt; t++) bufs[t].margin = DBL_MAX;
  int status = 0;

  /* Lipschitz bound: every point of T_a has its nearest site within
   * r_a = |p0 - nearest(p0)| + diam(T_a), so a site farther than r_a from
   * T_a cannot own any of it. */
  double *ra = NULL;
  if (!brute) {
    ra = (double *)malloc(sizeof(double) * m);
    if (!ra) { free(bufs); ogrid_free(&G); return 2; }
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
    for (int64_t a = 0; a < m; a++) {
      double lo[3], hi[3], dm;
      simplex_box(&C, a, lo, hi, &dm);
      ra[a] = onn_dist(&G, sites, &verts[3 * (int64_t)simp[a * k]]) + dm;
      /* power: some site k has |x - v_k|^2 - w_k <= r_a^2 - w_min on T_a, so
       * an owner i of x has |x - v_i|^2 <= r_a^2 - w_min + w_max */
      if (weights) ra[a] = sqrt(ra[a] * ra[a] - C.wmin + C.wmax);
    }
  }

  if (only_sites) {
    /* the candidate simplices of site i are those with dist(v_i, box_a) <= r_a
     * (the same Lipschitz filter as the full mode); they are found through a
     * grid over the simplices' boxes, within r_max of v_i */
    osgrid SG;
    memset(&SG, 0, sizeof SG);
    if (osgrid_build(&SG, &C, m, ra)) {
      osgrid_free(&SG); free(ra); free(bufs); ogrid_free(&G);
      return 2;
    }
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
      int tid = omp_get_thread_num();
#else
      int tid = 0;
#endif
      obuf *b = &bufs[tid];
      opoly *PA = (opoly *)malloc(sizeof(opoly)), *PB = (opoly *)malloc(sizeof(opoly));
      ogon *GA = (ogon *)malloc(sizeof(ogon)), *GB = (ogon *)malloc(sizeof(ogon));
      int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * m); /* last query that saw each simplex */
      if (!PA || !PB || !GA || !GB || !stamp) b->err = 2;
      else for (int64_t a = 0; a < m; a++) stamp[a] = -1;
#pragma omp for schedule(dynamic, 1)
      for (int64_t q = 0; q < n_only; q++) {
        int64_t i = only_sites[q];
        if (b->err || i < 0 || i >= n) { if (i < 0 || i >= n) b->err = 1; continue; }
        const double *v = &sites[3 * i];
        double qlo[3], qhi[3];
        for (int k = 0; k < 3; k++) { qlo[k] = v[k] - SG.rmax; qhi[k] = v[k] + SG.rmax; }
        int c0[3], c1[3];
        oscoord(&SG, qlo, c0);
        oscoord(&SG, qhi, c1);
        for (int z = c0[2]; z <= c1[2] && !b->err; z++)
          for (int y = c0[1]; y <= c1[1] && !b->err; y++)
            for (int x = c0[0]; x <= c1[0] && !b->err; x++) {
              int64_t ci = oscell(&SG, x, y, z);
              for (int32_t t = SG.start[ci]; t < SG.start[ci + 1]; t++) {
                int64_t a = SG.ids[t];
                if (stamp[a] == q) continue;
                stamp[a] = q;
                double lo[3], hi[3], dm;
                simplex_box(&C, a, lo, hi, &dm);
                if (box_dist(lo, hi, v) > ra[a]) continue;
                int which;
                int r = carve_pair(&C, a, i, PA, PB, GA, GB, &which, &b->margin);
                if (r == 3) { b->err = 3; break; }
                if (r == 1) {
                  if (simplex_dim == 3) emit_poly3(b, PA, (int32_t)i, (int32_t)a, v);
                  else emit_gon(b, GA, (int32_t)i, (int32_t)a, v);
                }
              }
            }
      }
      free(PA); free(PB); free(GA); free(GB); free(stamp);
    }
    osgrid_free(&SG);
  } else {
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
      int tid = omp_get_thread_num();
#else
      int tid = 0;
#endif
      obuf *b = &bufs[tid];
      opoly *PA = (opoly *)malloc(sizeof(opoly)), *PB = (opoly *)malloc(sizeof(opoly));
      ogon *GA = (ogon *)malloc(sizeof(ogon)), *GB = (ogon *)malloc(sizeof(ogon));
      if (!PA || !PB || !GA || !GB) b->err = 2;
#pragma omp for schedule(dynamic, 4)
      for (int64_t a = 0; a < m; a++) {
        if (b->err) continue;
        if (brute) {
          for (int64_t i = 0; i < n; i++) {
            int which;
            int r = carve_pair(&C, a, i, PA, PB, GA, GB, &which, &b->margin);
            if (r == 3) { b->err = 3; break; }
            if (r == 1) {
              if (simplex_dim == 3) emit_poly3(b, PA, (int32_t)i, (int32_t)a, &sites[3 * i]);
              else emit_gon(b, GA, (int32_t)i, (int32_t)a, &sites[3 * i]);
            }
          }
        } else {
          double lo[3], hi[3], dm;
          simplex_box(&C, a, lo, hi, &dm);
          double r = ra[a];
          double elo[3], ehi[3];
          for (int d = 0; d < 3; d++) { elo[d] = lo[d] - r; ehi[d] = hi[d] + r; }
          int c0[3], c1[3];
          ocoord(&G, elo, c0);
          ocoord(&G, ehi, c1);
          for (int z = c0[2]; z <= c1[2]; z++)
            for (int y = c0[1]; y <= c1[1]; y++)
              for (int x = c0[0]; x <= c1[0]; x++) {
                int64_t ci = ocell(&G, x, y, z);
                for (int32_t t = G.start[ci]; t < G.start[ci + 1]; t++) {
                  int64_t i = G.ids[t];
                  if (box_dist(lo, hi, &sites[3 * i]) > r) continue;
                  int which;
                  int rr = carve_pair(&C, a, i, PA, PB, GA, GB, &which, &b->margin);
                  if (rr == 3) { b->err = 3; break; }
                  if (rr == 1) {
                    if (simplex_dim == 3) emit_poly3(b, PA, (int32_t)i, (int32_t)a, &sites[3 * i]);
                    else emit_gon(b, GA, (int32_t)i, (int32_t)a, &sites[3 * i]);
                  }
                }
              }
        }
      }
      free(PA); free(PB); free(GA); free(GB);
    }
  }
  free(ra);
  ogrid_free(&G);
  for (int t = 0; t < nt; t++) if (bufs[t].err && !status) status = bufs[t].err;
  if (status) {
    for (int t = 0; t < nt; t++) obuf_free(&bufs[t]);
    free(bufs);
    return status;
  }

  /* merge, sorted by (site, simplex) */
  int64_t np = 0, nf = 0, nvv = 0, nfv = 0;
  for (int t = 0; t < nt; t++) { np += bufs[t].np; nf += bufs[t].nf; nvv += bufs[t].nv; nfv += bufs[t].nfv; }
  pkey *keys = (pkey *)malloc(sizeof(pkey) * (np ? np : 1));
  int64_t q = 0;
  for (int t = 0; t < nt; t++)
    for (int64_t p = 0; p < bufs[t].np; p++) {
      keys[q].site = bufs[t].site[p]; keys[q].simp = bufs[t].simp[p]; keys[q].thread = t; keys[q].idx = p; q++;
    }
  qsort(keys, np, sizeof(pkey), cmp_pkey);
  out->n_pieces = np;
  out->n_faces = nf;
  out->n_verts = nvv;
  out->piece_site = (int32_t *)malloc(sizeof(int32_t) * (np + 1));
  out->piece_simplex = (int32_t *)malloc(sizeof(int32_t) * (np + 1));
  out->piece_mass = (double *)malloc(sizeof(double) * (np + 1));
  out->piece_moment = (double *)malloc(sizeof(double) * 3 * (np + 1));
  out->piece_energy = (double *)malloc(sizeof(double) * (np + 1));
  out->piece_face_off = (int64_t *)malloc(sizeof(int64_t) * (np + 1));
  out->piece_vert_off = (int64_t *)malloc(sizeof(int64_t) * (np + 1));
  out->face_label = (int32_t *)malloc(sizeof(int32_t) * (nf + 1));
  out->face_measure = (double *)malloc(sizeof(double) * (nf + 1));
  out->face_vert_off = (int64_t *)malloc(sizeof(int64_t) * (nf + 1));
  out->face_vert = (int32_t *)malloc(sizeof(int32_t) * (nfv + 1));
  out->vert_xyz = (double *)malloc(sizeof(double) * 3 * (nvv + 1));
  out->vert_label = (int32_t *)malloc(sizeof(int32_t) * 3 * (nvv + 1));
  if (!keys || !out->piece_site || !out->piece_simplex || !out->piece_mass || !out->piece_moment ||
      !out->piece_energy || !out->piece_face_off || !out->piece_vert_off || !out->face_label ||
      !out->face_measure || !out->face_vert_off || !out->face_vert || !out->vert_xyz || !out->vert_label) {
    free(keys);
    for (int t = 0; t < nt; t++) obuf_free(&bufs[t]);
    free(bufs);
    vdo_free_result(out);
    return 2;
  }
  int64_t fo = 0, vo = 0, fvo = 0;
  for (int64_t p = 0; p < np; p++) {
    const obuf *b = &bufs[keys[p].thread];
    int64_t s = keys[p].idx;
    out->piece_site[p] = b->site[s];
    out->piece_simplex[p] = b->simp[s];
    out->piece_mass[p] = b->mass[s];
    for (int d = 0; d < 3; d++) out->piece_moment[3 * p + d] = b->mom[3 * s + d];
    out->piece_energy[p] = b->en[s];
    int64_t f0 = b->foff[s], f1 = (s + 1 < b->np) ? b->foff[s + 1] : b->nf;
    int64_t v0 = b->voff[s], v1 = (s + 1 < b->np) ? b->voff[s + 1] : b->nv;
    out->piece_face_off[p] = fo;
    out->piece_vert_off[p] = vo;
    for (int64_t f = f0; f < f1; f++) {
      out->face_label[fo] = b->flab[f];
      out->face_measure[fo] = b->fmeas[f];
      out->face_vert_off[fo] = fvo;
      int64_t e0 = b->fvoff[f], e1 = (f + 1 < b->nf) ? b->fvoff[f + 1] : b->nfv;
      for (int64_t e = e0; e < e1; e++) out->face_vert[fvo++] = b->fv[e];
      fo++;
    }
    for (int64_t v = v0; v < v1; v++) {
      for (int d = 0; d < 3; d++) {
        out->vert_xyz[3 * vo + d] = b->xyz[3 * v + d];
        out->vert_label[3 * vo + d] = b->vlab[3 * v + d];
      }
      vo++;
    }
  }
  out->piece_face_off[np] = fo;
  out->piece_vert_off[np] = vo;
  out->face_vert_off[nf] = fvo;
  out->n_face_verts = fvo;
  double mg = DBL_MAX;
  for (int t = 0; t < nt; t++) if (bufs[t].margin < mg) mg = bufs[t].margin;
  out->min_margin = mg;
  free(keys);
  for (int t = 0; t < nt; t++) obuf_free(&bufs[t]);
  free(bufs);
  return 0;
}

void vdo_free_result(vdo_result *r) {
  if (!r) return;
  free(r->piece_site); free(r->piece_simplex); free(r->piece_mass); free(r->piece_moment);
  free(r->piece_energy); free(r->piece_face_off); free(r->piece_vert_off); free(r->face_label);
  free(r->face_measure); free(r->face_vert_off); free(r->face_vert); free(r->vert_xyz);
  free(r->vert_label);
  memset(r, 0, sizeof *r);
}

/* ------------------------------------------------------------------ */
/* adjoint                                                              */
/* ------------------------------------------------------------------ */
/* Exact integrals over a triangle with vertices y0,y1,y2 (relative to the
 * site) of y, y y^T and |y|^2 y, from the barycentric monomial formula
 * int lambda_0^a lambda_1^b lambda_2^c dA = 2A a! b! c! / (a+b+c+2)!. */
static void tri_integrals(const double y[3][3], double A, double *I1, double I2[3][3], double *I3) {
  for (int p = 0; p < 3; p++) {
    I1[p] = 0;
    for (int k = 0; k < 3; k++) I1[p] += y[k][p];
    I1[p] *= A / 3.0;
  }
  for (int p = 0; p < 3; p++)
    for (int q = 0; q < 3; q++) {
      double s = 0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) s += (k == l ? 2.0 : 1.0) * y[k][p] * y[l][q];
      I2[p][q] = A / 12.0 * s;
    }
  for (int p = 0; p < 3; p++) {
    double s = 0;
    for (int k = 0; k < 3; k++)
      for (int l = 0; l < 3; l++)
        for (int mm = 0; mm < 3; mm++) {
          double c = (k == l && l == mm) ? 6.0 : ((k == l || l == mm || k == mm) ? 2.0 : 1.0);
          s += c * dot3(y[k], y[l]) * y[mm][p];
        }
    I3[p] = A / 60.0 * s;
  }
}

/* ------------------------------------------------------------------ */
/* density-weighted moments (Eq. 3 with a quadratic density)            */
/* ------------------------------------------------------------------ */
/* rho(x) = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 xy + c6 xz + c7 y^2 + c8 yz + c9 z^2 */
static double rho_at(const double *c, const double *x) {
  return c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[2] + c[4] * x[0] * x[0] + c[5] * x[0] * x[1] +
         c[6] * x[0] * x[2] + c[7] * x[1] * x[1] + c[8] * x[1] * x[2] + c[9] * x[2] * x[2];
}

/* Gauss-Legendre, 4 points on [0, 1] (exact to degree 7 in each variable) */
static const double GL4_T[4] = {0.5 - 0.5 * 0.8611363115940526, 0.5 - 0.5 * 0.3399810435848563,
                                0.5 + 0.5 * 0.3399810435848563, 0.5 + 0.5 * 0.8611363115940526};
static const double GL4_W[4] = {0.5 * 0.3478548451374538, 0.5 * 0.6521451548625461,
                                0.5 * 0.6521451548625461, 0.5 * 0.3478548451374538};

/* Integral over the triangle (P0, P1, P2) of f, by the conical product
 * (Duffy) rule: lambda1 = u, lambda2 = (1 - u) v, dA = 2 |A| (1 - u) du dv,
 * 4 x 4 Gauss points -- exact for polynomials of degree <= 6.  `area` is the
 * (signed) area; f(x, ctx, acc) adds weight * integrand to acc[0..nacc). */
typedef void (*vdo_integrand)(const double *x, double w, const void *ctx, double *acc);
static void tri_conical(const double *P0, const double *P1, const double *P2, double area, vdo_integrand f,
                        const void *ctx, double *acc) {
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) {
      double u = GL4_T[a], v = GL4_T[b];
      double l1 = u, l2 = (1 - u) * v, l0 = 1 - l1 - l2;
      double x[3];
      for (int d = 0; d < 3; d++) x[d] = l0 * P0[d] + l1 * P1[d] + l2 * P2[d];
      f(x, 2.0 * area * (1 - u) * GL4_W[a] * GL4_W[b], ctx, acc);
    }
}

/* Integral over the tetrahedron (P0..P3) of f: lambda1 = u, lambda2 = (1-u) v,
 * lambda3 = (1-u)(1-v) w, dV = 6 V (1-u)^2 (1-v) du dv dw, 4^3 Gauss points
 * -- exact for polynomials of degree <= 5. */
static void tet_conical(const double *P0, const double *P1, const double *P2, const double *P3, double vol,
                        vdo_integrand f, const void *ctx, double *acc) {
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++)
      for (int c = 0; c < 4; c++) {
        double u = GL4_T[a], v = GL4_T[b], w = GL4_T[c];
        double l1 = u, l2 = (1 - u) * v, l3 = (1 - u) * (1 - v) * w, l0 = 1 - l1 - l2 - l3;
        double x[3];
        for (int d = 0; d < 3; d++) x[d] = l0 * P0[d] + l1 * P1[d] + l2 * P2[d] + l3 * P3[d];
        f(x, 6.0 * vol * (1 - u) * (1 - u) * (1 - v) * GL4_W[a] * GL4_W[b] * GL4_W[c], ctx, acc);
      }
}

typedef struct {
  const double *c;  /* density coefficients */
  const double *v;  /* the site */
} rho_ctx;

/* acc += w rho(x) {1, x (3), |x - v|^2} */
static void rho_moments_integrand(const double *x, double w, const void *ctx, double *acc) {
  const rho_ctx *k = (const rho_ctx *)ctx;
  double wr = w * rho_at(k->c, x);
  double y[3];
  sub3(x, k->v, y);
  acc[0] += wr;
  acc[1] += wr * x[0]; acc[2] += wr * x[1]; acc[3] += wr * x[2];
  acc[4] += wr * dot3(y, y);
}

int vdo_density_moments(const vdo_result *r, const double *sites, const double *coef, int simplex_dim,
                        double *mass, double *moment, double *energy) {
  if (!r || !sites || !coef || !mass || !moment || !energy) return 1;
  for (int64_t p = 0; p < r->n_pieces; p++) {
    const double *v = &sites[3 * (int64_t)r->piece_site[p]];
    rho_ctx k = {coef, v};
    double acc[5] = {0, 0, 0, 0, 0};
    int64_t vb = r->piece_vert_off[p];
    const double *apex = &r->vert_xyz[3 * vb];
    for (int64_t f = r->piece_face_off[p]; f < r->piece_face_off[p + 1]; f++) {
      int64_t e0 = r->face_vert_off[f], e1 = r->face_vert_off[f + 1];
      if (simplex_dim == 3) {
        /* fan of tetrahedra (apex, face loop fan): positive volumes for
         * counter-clockwise loops seen from outside */
        const double *q0 = &r->vert_xyz[3 * (vb + r->face_vert[e0])];
        for (int64_t e = e0 + 1; e + 1 < e1; e++) {
          const double *q1 = &r->vert_xyz[3 * (vb + r->face_vert[e])];
          const double *q2 = &r->vert_xyz[3 * (vb + r->face_vert[e + 1])];
          double a[3], b[3], c[3], cr[3];
          sub3(q0, apex, a); sub3(q1, apex, b); sub3(q2, apex, c);
          cross3(b, c, cr);
          double vol = dot3(a, cr) / 6.0;
          if (vol != 0.0) tet_conical(apex, q0, q1, q2, vol, rho_moments_integrand, &k, acc);
        }
      } else {
        /* a polygon: its edges are the faces; fan of triangles (apex, edge) */
        const double *q0 = &r->vert_xyz[3 * (vb + r->face_vert[e0])];
        const double *q1 = &r->vert_xyz[3 * (vb + r->face_vert[e0 + 1])];
        double a[3], b[3], cr[3];
        sub3(q0, apex, a); sub3(q1, apex, b);
        cross3(a, b, cr);
        double ar = 0.5 * sqrt(dot3(cr, cr));
        if (ar > 0.0) tri_conical(apex, q0, q1, ar, rho_moments_integrand, &k, acc);
      }
    }
    mass[p] = acc[0];
    moment[3 * p] = acc[1]; moment[3 * p + 1] = acc[2]; moment[3 * p + 2] = acc[3];
    energy[p] = acc[4];
  }
  return 0;
}

/* integrand of the adjoint's face term with a density:
 * acc += w rho(x) (a0 + b.y + g |y|^2) y, y = x - v */
typedef struct {
  const double *c, *v, *b;
  double a0, g;
} face_ctx;
static void rho_face_integrand(const double *x, double w, const void *ctx, double *acc) {
  const face_ctx *k = (const face_ctx *)ctx;
  double y[3];
  sub3(x, k->v, y);
  double f = w * rho_at(k->c, x) * (k->a0 + dot3(k->b, y) + k->g * dot3(y, y));
  for (int d = 0; d < 3; d++) acc[d] += f * y[d];
}

int vdo_moments_backward(const vdo_result *r, const double *sites, int64_t n,
                         const double *mass, const double *cent,
                         const double *g_m, const double *g_c, const double *g_E,
                         const double *verts, const int32_t *simp, int simplex_dim,
                         double *g_sites) {
  return vdo_moments_backward_rho(r, sites, n, mass, cent, g_m, g_c, g_E, verts, simp, simplex_dim, NULL,
                                  g_sites);
}

int vdo_moments_backward_rho(const vdo_result *r, const double *sites, int64_t n,
                             const double *mass, const double *cent,
                             const double *g_m, const double *g_c, const double *g_E,
                             const double *verts, const int32_t *simp, int simplex_dim,
                             const double *rho, double *g_sites) {
  if (!r || !sites || !mass || !cent || !g_sites) return 1;
  double *al = (double *)calloc(n, sizeof(double));
  double *be = (double *)calloc(3 * n, sizeof(double));
  double *ga = (double *)calloc(n, sizeof(double));
  if (!al || !be || !ga) { free(al); free(be); free(ga); return 2; }
  for (int64_t k = 0; k < n; k++) {
    double gm = g_m ? g_m[k] : 0.0, gE = g_E ? g_E[k] : 0.0;
    double gc[3] = {0, 0, 0};
    if (g_c) for (int d = 0; d < 3; d++) gc[d] = g_c[3 * k + d];
    ga[k] = gE;
    if (mass[k] > 0) {
      al[k] = gm - dot3(gc, &cent[3 * k]) / mass[k];
      for (int d = 0; d < 3; d++) be[3 * k + d] = gc[d] / mass[k];
    }
  }
  for (int64_t i = 0; i < n; i++) {
    for (int d = 0; d < 3; d++) g_sites[3 * i + d] = 0.0;
    if (mass[i] > 0)
      for (int d = 0; d < 3; d++) g_sites[3 * i + d] = 2.0 * ga[i] * mass[i] * (sites[3 * i + d] - cent[3 * i + d]);
  }
  for (int64_t p = 0; p < r->n_pieces; p++) {
    int64_t i = r->piece_site[p];
    const double *vi = &sites[3 * i];
    int64_t vbase = r->piece_vert_off[p];
    double Ntri[3] = {0, 0, 0};
    if (simplex_dim == 2) {
      const int32_t *t = &simp[3 * (int64_t)r->piece_simplex[p]];
      double ab[3], ac[3];
      sub3(&verts[3 * (int64_t)t[1]], &verts[3 * (int64_t)t[0]], ab);
      sub3(&verts[3 * (int64_t)t[2]], &verts[3 * (int64_t)t[0]], ac);
      cross3(ab, ac, Ntri);
      double nn = sqrt(dot3(Ntri, Ntri));
      for (int d = 0; d < 3; d++) Ntri[d] /= nn;
    }
    for (int64_t f = r->piece_face_off[p]; f < r->piece_face_off[p + 1]; f++) {
      int32_t k = r->face_label[f];
      if (k < 0) continue;
      const double *vk = &sites[3 * (int64_t)k];
      double nk[3];
      sub3(vk, vi, nk);
      double dik = sqrt(dot3(nk, nk));
      double bdiff[3];
      for (int d = 0; d < 3; d++) bdiff[d] = be[3 * i + d] - be[3 * k + d];
      double a0 = (al[i] - al[k]) + dot3(bdiff, vi);
      double gdiff = ga[i] - ga[k];
      int64_t e0 = r->face_vert_off[f], e1 = r->face_vert_off[f + 1];
      double contrib[3] = {0, 0, 0};
      if (simplex_dim == 3) {
        double y0[3];
        sub3(&r->vert_xyz[3 * (vbase + r->face_vert[e0])], vi, y0);
        for (int64_t e = e0 + 1; e + 1 < e1; e++) {
          double y[3][3];
          memcpy(y[0], y0, sizeof y0);
          sub3(&r->vert_xyz[3 * (vbase + r->face_vert[e])], vi, y[1]);
          sub3(&r->vert_xyz[3 * (vbase + r->face_vert[e + 1])], vi, y[2]);
          double ab[3], ac[3], cr[3];
          sub3(y[1], y[0], ab); sub3(y[2], y[0], ac);
          cross3(ab, ac, cr);
          /* oriented area: the loop is counter-clockwise around the outward
           * normal of cell i, which points towards v_k */
          double A = 0.5 * dot3(cr, nk) / dik;
          if (rho) {
            /* with a density the integrand rho (a0 + b.y + g|y|^2) y has
             * degree 5: the conical product rule on the triangle */
            double P[3][3], acc[3] = {0, 0, 0};
            for (int t = 0; t < 3; t++)
              for (int d = 0; d < 3; d++) P[t][d] = vi[d] + y[t][d];
            face_ctx fc = {rho, vi, bdiff, a0, gdiff};
            tri_conical(P[0], P[1], P[2], A, rho_face_integrand, &fc, acc);
            for (int q = 0; q < 3; q++) contrib[q] += acc[q] / dik;
            continue;
          }
          double I1[3], I2[3][3], I3[3];
          tri_integrals(y, A, I1, I2, I3);
          for (int q = 0; q < 3; q++) {
            double bI2 = 0;
            for (int s = 0; s < 3; s++) bI2 += bdiff[s] * I2[s][q];
            contrib[q] += (a0 * I1[q] + bI2 + gdiff * I3[q]) / dik;
          }
        }
      } else {
        /* segment on triangle T: in-plane normal speed is V / s with
         * s = |n - (n.N) N| (n unit bisector normal, N unit triangle normal);
         * Simpson's rule is exact for the cubic integrand. */
        double nh[3] = {nk[0] / dik, nk[1] / dik, nk[2] / dik};
        double nN = dot3(nh, Ntri);
        double sv[3] = {nh[0] - nN * Ntri[0], nh[1] - nN * Ntri[1], nh[2] - nN * Ntri[2]};
        double sfac = sqrt(dot3(sv, sv));
        double yA[3], yB[3], yM[3];
        sub3(&r->vert_xyz[3 * (vbase + r->face_vert[e0])], vi, yA);
        sub3(&r->vert_xyz[3 * (vbase + r->face_vert[e0 + 1])], vi, yB);
        for (int d = 0; d < 3; d++) yM[d] = 0.5 * (yA[d] + yB[d]);
        double dl[3];
        sub3(yB, yA, dl);
        double len = sqrt(dot3(dl, dl));
        if (rho) {
          /* with a density the integrand has degree 5: Boole's rule (five
           * equally spaced points, weights 7, 32, 12, 32, 7 over 90) */
          const double bw[5] = {7.0 / 90.0, 32.0 / 90.0, 12.0 / 90.0, 32.0 / 90.0, 7.0 / 90.0};
          for (int t = 0; t < 5; t++) {
            double y[3], x[3];
            for (int d = 0; d < 3; d++) { y[d] = yA[d] + 0.25 * t * dl[d]; x[d] = vi[d] + y[d]; }
            double f = rho_at(rho, x) * (a0 + dot3(bdiff, y) + gdiff * dot3(y, y));
            for (int q = 0; q < 3; q++) contrib[q] += bw[t] * len * f * y[q] / (dik * sfac);
          }
        } else {
          const double *pts[3] = {yA, yM, yB};
          const double w[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
          for (int t = 0; t < 3; t++) {
            const double *y = pts[t];
            double f = a0 + dot3(bdiff, y) + gdiff * dot3(y, y);
            for (int q = 0; q < 3; q++) contrib[q] += w[t] * len * f * y[q] / (dik * sfac);
          }
        }
      }
      for (int q = 0; q < 3; q++) g_sites[3 * i + q] += contrib[q];
    }
  }
  free(al); free(be); free(ga);
  return 0;
}
