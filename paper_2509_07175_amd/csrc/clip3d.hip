// clip3d.hip -- clipped Voronoi cells in a tetrahedral domain, one wavefront
// per site.
//
// Carving (shared by both modes) follows Alg. 1 / Alg. 3:
//   * a corner is classified by the point-in-cell test (Sec. 4.1, Eq. 2): it is
//     inside Omega_i iff its nearest site is v_i or a site named by the flag of
//     one of the corner's planes.  Corners are tested lazily, up to four at a
//     time (one 16-lane group per query): the loop only needs *some* outside
//     corner, and corners that a later clip removes are never tested;
//   * for an outside corner the search edge is an edge from a tested-inside
//     neighbour (Alg. 1) or else the virtual edge from v_i (Alg. 3); it is
//     optionally shortened by lambda*delta steps (Sec. 6.1), then the bisector
//     is found by the edge-based search (Sec. 4.2), where a search point also
//     counts as inside when its nearest site is named by the flag of a plane
//     through the search edge;
//   * the clip removes only R_p, the connected outside component that contains
//     the chosen outside corner (Sec. 6.3).
//
// Modes (vd_options.carve_mode):
//   0 per-simplex: the tetrahedra of the cell are visited breadth-first through
//     negative face flags from the tetrahedron containing v_i (the propagation
//     of Alg. 5) and each piece T_a cap Omega_i is carved as above.
//   1 cell-first: the cell is carved once from the padded bounding box of the
//     domain (the simple-domain kernel of Sec. 5.2, which Alg. 5 uses for its
//     interior sites); every corner of the result is certified inside Omega_i,
//     so its bisector facets F are exactly the half-spaces that bound the cell
//     inside the box.  The same propagation then visits the tetrahedra and
//     each piece is T_a cut by the half-spaces of F: T_a cap Omega_i =
//     T_a cap cell, with no further point-in-cell test.
//
// Polytope layout in LDS (the dual triangle mesh of Sec. 6.3): planes (normal,
// offset, flag) and corners; a corner stores its three planes in
// counter-clockwise order seen from outside (det of the outward normals > 0),
// the corner across each of its three dual edges, its coordinates relative to
// v_i and its test state.  Lane l owns corner slots l and l+64, so the flood
// fill of R_p, the fan of the new face and compaction are wave-parallel;
// tested/inside/removed sets are 128-bit ballot masks.
//
// Moments of a piece: a fan of tetrahedra (corner 0 of the piece, foot of the
// face plane, corner, next corner around the face), three per corner, reduced across the
// wave with butterfly shuffles (fixed order, no floating-point atomics).
#include <type_traits>

#include "vd_arena.h"

namespace {

constexpr int kMaxIters = 4096;  // queries + clips of one polytope
constexpr int kBoxBase = VD_BND_BASE + 16;  // flags of the bounding-box planes (never emitted)

// The carved cell kept in LDS for the piece phase, over the site cache's
// arrays: the cache is not read after the carve unless a piece falls back to
// a carve of its own, which then switches the cache off and queries the grid.
// Cells with more planes or corners go to the wave's global save area.
constexpr int kLF = 32;  // planes
constexpr int kLC = 64;  // corners
struct LdsCell {
  double pn[kLF][4];
  double cy[kLC][3];
  int plab[kLF];
  int cpl[kLC], cnb[kLC];
};
static_assert(sizeof(LdsCell) <= offsetof(SiteCache, step), "the LDS cell overlays only the cache's arrays");

struct __align__(16) WaveLds {
  double pn[VD_P_MAX][4];    // plane: outward normal (relative coords), offset
  double cy[VD_C_MAX][3];    // corner coordinates relative to v_i
  int plab[VD_P_MAX];        // plane flag: sorted site >= 0, -(b+1), boundary/box code
  int cpl[VD_C_MAX];         // corner planes a | b << 8 | c << 16 (CCW from outside)
  int cnb[VD_C_MAX];         // corner across a->b | across b->c << 8 | across c->a << 16
  int cst[VD_C_MAX];         // bit 0 inside, bit 1 tested, bits 8.. nearest site + 1
  unsigned char byFirst[VD_P_MAX], bySecond[VD_P_MAX];
  int tq[VD_Q_MAX];          // tetrahedra of this site, breadth-first
  int nbl[VD_NB_MAX];        // neighbours found so far (sorted positions)
  union {
    int pfirst[VD_P_MAX];    // lowest corner slot on each plane (face walks, after a carve)
    int psl[VD_P_MAX];       // site cache slot of each bisector plane's site, or -1 (during a carve)
  };
  WaveArena ar;              // output chunks, queue position, statistics
  union {
    SiteCache K;             // sites around v_i for the nearest-site queries (carve)
    LdsCell LC;              // the carved cell (piece phase)
  };
  // per-site sums and neighbour masks (uniform; kept here rather than in
  // registers that would be live across the whole carve)
  double acc[5];             // volume, first moment (relative to v_i), energy
  unsigned long long cellpos, nbmask;
};

struct Stats {
  long long queries = 0, cands = 0, clips = 0, grid = 0;  // grid: queries not answered by the site cache
};

__device__ __forceinline__ int p8(int packed, int e) { return (packed >> (8 * e)) & 0xff; }
__device__ __forceinline__ int pack3(int a, int b, int c) { return a | (b << 8) | (c << 16); }
__device__ __forceinline__ uint64_t low_mask(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1ull); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }


struct SiteCtx {
  double vx, vy, vz, delta;
  double h, w;  // power diagram: lifted coordinate and weight of the site (else 0)
  int si;
};

// Vertex of three planes by Cramer's rule, planes taken in ascending flag order
// so a vertex does not depend on the order in which its planes were created.
__device__ __forceinline__ void solve3(const WaveLds &S, int a, int b, int c, double *y) {
  int q[3] = {a, b, c};
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i + 1; j < 3; j++)
      if (S.plab[q[j]] < S.plab[q[i]]) { int t = q[i]; q[i] = q[j]; q[j] = t; }
  const double *n0 = S.pn[q[0]], *n1 = S.pn[q[1]], *n2 = S.pn[q[2]];
  const double c12[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2], n1[0] * n2[1] - n1[1] * n2[0]};
  const double c20[3] = {n2[1] * n0[2] - n2[2] * n0[1], n2[2] * n0[0] - n2[0] * n0[2], n2[0] * n0[1] - n2[1] * n0[0]};
  const double c01[3] = {n0[1] * n1[2] - n0[2] * n1[1], n0[2] * n1[0] - n0[0] * n1[2], n0[0] * n1[1] - n0[1] * n1[0]};
  const double det = n0[0] * c12[0] + n0[1] * c12[1] + n0[2] * c12[2];
  const double id = 1.0 / det;
#pragma unroll
  for (int k = 0; k < 3; k++) y[k] = (n0[3] * c12[k] + n1[3] * c20[k] + n2[3] * c01[k]) * id;
}

// Drop planes that no corner references (keeps slot order).  Returns the new
// plane count.
__device__ int compact_planes(WaveLds &S, int npl, int nc) {
  const int l = vd_lane();
  uint64_t used = 0;
  for (int s = l; s < nc; s += 64) {
    const int pl = S.cpl[s];
    used |= (1ull << p8(pl, 0)) | (1ull << p8(pl, 1)) | (1ull << p8(pl, 2));
  }
  used = wave_or64(used);
  const int newnpl = __popcll(used);
  double pv[4] = {0, 0, 0, 0};
  int lab = 0, sl = -1;
  const bool mine = l < npl && ((used >> l) & 1ull);
  if (mine) { for (int k = 0; k < 4; k++) pv[k] = S.pn[l][k]; lab = S.plab[l]; sl = S.psl[l]; }
  int cp[2] = {0, 0};
  for (int h = 0; h < 2; h++) {
    const int s = l + 64 * h;
    if (s < nc) cp[h] = S.cpl[s];
  }
  __syncthreads();
  if (mine) {
    const int ni = __popcll(used & low_mask(l));
    for (int k = 0; k < 4; k++) S.pn[ni][k] = pv[k];
    S.plab[ni] = lab;
    S.psl[ni] = sl;
  }
  for (int h = 0; h < 2; h++) {
    const int s = l + 64 * h;
    if (s < nc) {
      const int a = __popcll(used & low_mask(p8(cp[h], 0)));
      const int b = __popcll(used & low_mask(p8(cp[h], 1)));
      const int c = __popcll(used & low_mask(p8(cp[h], 2)));
      S.cpl[s] = pack3(a, b, c);
    }
  }
  __syncthreads();
  return newnpl;
}

// Clip by plane slot P, removing R_p: the connected set of corners strictly
// outside P that contains corner pt (Sec. 6.3); pt < 0 removes every corner
// outside P (a cut of a convex polytope).  New corners are created on every dual edge
// leaving R_p and form the fan of the new face.
// Returns 0 (nothing outside: unchanged), 1 empty, 2 capacity, 3 degenerate,
// 4 cut (nc updated).
// W: the polytope may hold more than 64 corners (two slots per lane); the
// narrow instance (nc <= 64 on entry, the common case) keeps one slot per
// lane and one 64-bit mask per set.
template <bool MON, bool W>
__device__ int clip_poly_w(WaveLds &S, int P, int pt, int &nc, int ps, int kcert) {
  constexpr int NH = W ? 2 : 1;
  // bit s of the 128-bit set (lo, hi); narrow: every index is below 64
  auto bit = [](uint64_t lo, uint64_t hi, int s) { return W ? bit128(lo, hi, s) : ((lo >> s) & 1ull) != 0; };
  const int l = vd_lane();
  const double nx = S.pn[P][0], ny = S.pn[P][1], nz = S.pn[P][2], c = S.pn[P][3];
  int pl[2] = {0, 0}, nb[2] = {0, 0}, cs[2] = {0, 0};
  double y[2][3] = {{0, 0, 0}, {0, 0, 0}};
  bool v[2] = {false, false}, o[2] = {false, false};
  double sd[2] = {-1.0, -1.0};
  for (int h = 0; h < NH; h++) {
    const int s = l + 64 * h;
    v[h] = s < nc;
    if (v[h]) {
      pl[h] = S.cpl[s]; nb[h] = S.cnb[s]; cs[h] = S.cst[s];
      y[h][0] = S.cy[s][0]; y[h][1] = S.cy[s][1]; y[h][2] = S.cy[s][2];
      sd[h] = nx * y[h][0] + ny * y[h][1] + nz * y[h][2] - c;
    }
    o[h] = v[h] && sd[h] > 0.0;
  }
  if (MON) {
    margin_track(S.ar, v[0], sd[0], fabs(nx * y[0][0]) + fabs(ny * y[0][1]) + fabs(nz * y[0][2]) + fabs(c), v[1],
                 sd[1], fabs(nx * y[1][0]) + fabs(ny * y[1][1]) + fabs(nz * y[1][2]) + fabs(c));
    count_add(S.ar.classified, nc);
  }
  const uint64_t olo = __ballot(o[0]), ohi = W ? __ballot(o[1]) : 0ull;
  if (!(olo | ohi)) return pt < 0 ? 0 : 3;
  uint64_t Rlo, Rhi;
  if (pt < 0) {
    // a cut of a convex polytope: every outside corner goes (an outside set
    // that rounding made disconnected gives a non-simple boundary, caught below)
    Rlo = olo;
    Rhi = ohi;
  } else {
    if (!bit(olo, ohi, pt)) return 3;
    Rlo = pt < 64 ? (1ull << pt) : 0ull;
    Rhi = (W && pt >= 64) ? (1ull << (pt - 64)) : 0ull;
  }
  for (int it = 0; pt >= 0 && it < VD_C_MAX; it++) {
    bool j[2] = {false, false};
    for (int h = 0; h < NH; h++) {
      const int s = l + 64 * h;
      j[h] = o[h] && !bit(Rlo, Rhi, s) &&
             (bit(Rlo, Rhi, p8(nb[h], 0)) || bit(Rlo, Rhi, p8(nb[h], 1)) || bit(Rlo, Rhi, p8(nb[h], 2)));
    }
    const uint64_t a = __ballot(j[0]), b = W ? __ballot(j[1]) : 0ull;
    if (!(a | b)) break;
    Rlo |= a;
    Rhi |= b;
  }
  const int nR = __popcll(Rlo) + __popcll(Rhi);
  if (MON && pt >= 0) {
    // tests spent on corners this clip removes, besides the one that led to it
    const uint64_t tlo = __ballot(v[0] && (cs[0] & 2)), thi = W ? __ballot(v[1] && (cs[1] & 2)) : 0ull;
    const int w = __popcll(tlo & Rlo) + __popcll(thi & Rhi) - (bit(tlo, thi, pt) ? 1 : 0);
    count_add(S.ar.wasted, w);
  }
  if (nR >= nc) return 1;
  bool r[2] = {false, false};
  int em[2] = {0, 0};
  for (int h = 0; h < NH; h++) {
    const int s = l + 64 * h;
    r[h] = v[h] && bit(Rlo, Rhi, s);
    if (r[h])
      for (int e = 0; e < 3; e++)
        if (!bit(Rlo, Rhi, p8(nb[h], e))) em[h] |= 1 << e;
  }
  const int cnt = __popc(em[0]) + __popc(em[1]);
  const int inc = wave_incl_scan(cnt);
  const int nnew = __builtin_amdgcn_readlane(inc, 63);
  const int base = inc - cnt;
  const int nsurv = nc - nR;
  if (nnew < 3) return 3;
  if (nsurv + nnew > VD_C_MAX) return 2;
  const uint64_t vlo = low_mask(nc < 64 ? nc : 64), vhi = W ? low_mask(nc > 64 ? nc - 64 : 0) : 0ull;
  const uint64_t Slo = vlo & ~Rlo, Shi = vhi & ~Rhi;
  // every plane is "first" (resp. "second") of at most one new corner when the
  // boundary of R_p is a simple loop; the tables give the fan adjacency.  A
  // plane that is first (second) of two new corners shows as fewer distinct
  // first (second) planes than new corners.
  __syncthreads();
  uint64_t fm = 0, sm = 0;
  {
    int t = base;
    for (int h = 0; h < NH; h++)
      for (int e = 0; e < 3; e++)
        if (em[h] & (1 << e)) {
          const int u = p8(pl[h], e), w = p8(pl[h], (e + 1) % 3);
          S.byFirst[u] = (unsigned char)(nsurv + t);
          S.bySecond[w] = (unsigned char)(nsurv + t);
          fm |= 1ull << u;
          sm |= 1ull << w;
          t++;
        }
  }
  fm = wave_or64(fm);
  sm = wave_or64(sm);
  if (__popcll(fm) != nnew || __popcll(sm) != nnew) return 3;
  __syncthreads();
  // all old corner data sits in registers: write the new layout
  bool nf = false;
  {
    // new slot of every surviving corner (lane l: slots l and l + 64), and of
    // the three neighbours of each corner, fetched from their owning lanes
    const int nlo = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(Slo >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)Slo, 0u));
    const int nhi = W ? __popcll(Slo) + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(Shi >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)Shi, 0u))
                      : 0;
    int nbn[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int h = 0; h < NH; h++)
#pragma unroll
      for (int e = 0; e < 3; e++) {
        const int m = p8(nb[h], e);
        int x = __shfl(nlo, m & 63, 64);
        if (W && nc > 64) {
          const int y = __shfl(nhi, m & 63, 64);
          x = m < 64 ? x : y;
        }
        nbn[h][e] = x;
      }
    int t = base;
#pragma unroll
    for (int h = 0; h < NH; h++) {
      if (v[h] && !r[h]) {
        const int ns = h ? nhi : nlo;
        int nbo[3];
        for (int e = 0; e < 3; e++) {
          const int m = p8(nb[h], e);
          nbo[e] = bit(Rlo, Rhi, m) ? S.byFirst[p8(pl[h], (e + 1) % 3)] : nbn[h][e];
        }
        S.cpl[ns] = pl[h];
        S.cnb[ns] = pack3(nbo[0], nbo[1], nbo[2]);
        S.cst[ns] = cs[h];
        S.cy[ns][0] = y[h][0]; S.cy[ns][1] = y[h][1]; S.cy[ns][2] = y[h][2];
      }
      if (r[h])
#pragma unroll
        for (int e = 0; e < 3; e++)
          if (em[h] & (1 << e)) {
            const int u = p8(pl[h], e), w = p8(pl[h], (e + 1) % 3);
            const int ns = nsurv + t;
            S.cpl[ns] = pack3(u, w, P);
            S.cnb[ns] = pack3(nbn[h][e], S.byFirst[w], S.bySecond[u]);
            // the corner on the search edge (pt, ps) is the point the search's
            // last query tested, with the same flags: already known inside
            S.cst[ns] = (ps >= 0 && l + 64 * h == pt && p8(nb[h], e) == ps) ? (3 | ((kcert + 1) << 8)) : 0;
            t++;
          }
    }
  }
  __syncthreads();
  // coordinates of the new corners, one per lane (a removed corner may own up
  // to three of them)
  for (int t = l; t < nnew; t += 64) {
    const int ns = nsurv + t;
    const int cp = S.cpl[ns];
    double yy[3];
    solve3(S, p8(cp, 0), p8(cp, 1), p8(cp, 2), yy);
    nf = nf || !isfinite(yy[0] + yy[1] + yy[2]);
    S.cy[ns][0] = yy[0]; S.cy[ns][1] = yy[1]; S.cy[ns][2] = yy[2];
  }
  __syncthreads();
  nc = nsurv + nnew;
  if (MON) count_add(S.ar.newc, nnew);
  // three planes without a common point (e.g. all containing one direction)
  // give a non-finite corner: report the cut as degenerate
  if (__ballot(nf)) return 3;
  return 4;
}

template <bool MON>
__device__ __forceinline__ int clip_poly(WaveLds &S, int P, int pt, int &nc, int ps = -1, int kcert = -1) {
  return nc <= 64 ? clip_poly_w<MON, false>(S, P, pt, nc, ps, kcert) : clip_poly_w<MON, true>(S, P, pt, nc, ps, kcert);
}

__device__ __forceinline__ void state_masks(const WaveLds &S, int nc, uint64_t &tlo, uint64_t &thi,
                                            uint64_t &ilo, uint64_t &ihi) {
  const int l = vd_lane();
  const int a = l < nc ? S.cst[l] : 0;
  tlo = __ballot(a & 2);
  ilo = __ballot(a & 1);
  thi = ihi = 0ull;
  if (nc > 64) {  // the second corner slot of each lane is in use
    const int b = l + 64 < nc ? S.cst[l + 64] : 0;
    thi = __ballot(b & 2);
    ihi = __ballot(b & 1);
  }
}

// Alg. 1 / Alg. 3 on the polytope in LDS until every corner is certified inside
// Omega_i.  Written as a loop with a single nearest-site query per iteration:
//   TEST    up to four untested corners, one 16-lane group each (taken when no
//           tested corner is known to be outside);
//   LAMBDA  a point A + lambda*delta*u of the improved search (Sec. 6.1);
//   SEARCH  the crossing of the search edge with B_ij (Sec. 4.2).
// Returns 0 (done, non-empty), 1 (empty), 2 capacity, 3 degenerate.
struct CarveParams {
  int improved, straddle, max_iters;
};

// POW: power diagram (Sec. 7.3).  The sites are lifted to (v_j, h_j) with
// h_j = sqrt(eta - w_j) and the cell is the restricted Voronoi cell of the
// lifted site on the hyperplane of the domain: corners are tested as points
// of that hyperplane (4th coordinate 0), the virtual search edge starts at the
// lifted site (v_i, h_i), whose 4D cell always contains it, and a search point
// on it has a 4th coordinate between h_i and 0.  The clip plane is the power
// plane n.y <= (|n|^2 + w_i - w_j)/2 (the lifted bisector on the hyperplane).
template <bool MON, bool POW>
__device__ int carve(WaveLds &S, const GridView &G, const CarveParams C, const SiteCtx &X, int &npl, int &nc,
                     Stats &st) {
  enum { PICK = 0, TEST, LAMBDA, SEARCH };
  const int l = vd_lane();
  const int grp = l >> 4;
  int mode = PICK;
  int pt = -1, j = -1, ef0 = -2, ef1 = -2, lam = 2, nstep = 0;
  int ps_edge = -1;   // inside end of the search edge when it is an edge of P
  bool qon = false;   // the search point lies strictly inside its edge
  int tslot = -1, nbatch = 0;
  int jsl = -1, efs0 = -1, efs1 = -1;  // cache slots of j and of the edge's sites (-1: none)
  double A0 = 0, A1 = 0, A2 = 0, g0 = 0, g1 = 0, g2 = 0, u0 = 0, u1 = 0, u2 = 0, L = 0;
  double n0 = 0, n1 = 0, n2 = 0, nc3 = 0;
  double q0 = 0, q1 = 0, q2 = 0;  // query point relative to v_i (per group for TEST)
  double A4 = 0, g4 = 0, q4 = 0;   // POW: 4th coordinates of the edge ends and of the query
  // crossing of [A, g] with B_ij (j = current candidate)
  auto bisector_point = [&]() {
    // the site's coordinates from the LDS cache when it holds them (exact copies)
    if (jsl >= 0) {
      n0 = S.K.x[jsl] - X.vx; n1 = S.K.y[jsl] - X.vy; n2 = S.K.z[jsl] - X.vz;
    } else {
      n0 = GL(G.sx)[j] - X.vx; n1 = GL(G.sy)[j] - X.vy; n2 = GL(G.sz)[j] - X.vz;
    }
    const double e0 = g0 - A0, e1 = g1 - A1, e2 = g2 - A2;
    double den, num;
    if (POW) {
      // 4D bisector of the lifted sites, relative to (v_i, h_i)
      const double n4 = GL(G.sh)[j] - X.h, e4 = g4 - A4;
      den = n0 * e0 + n1 * e1 + n2 * e2 + n4 * e4;
      num = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2 + n4 * n4) - (n0 * A0 + n1 * A1 + n2 * A2 + n4 * (A4 - X.h));
      nc3 = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2 + X.w - GL(G.sw)[j]);
    } else {
      nc3 = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2);
      den = n0 * e0 + n1 * e1 + n2 * e2;
      num = nc3 - (n0 * A0 + n1 * A1 + n2 * A2);
    }
    qon = den > 0.0 && num > 0.0 && num < den;
    double t = den > 0.0 ? num / den : 1.0;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    q0 = A0 + t * e0; q1 = A1 + t * e1; q2 = A2 + t * e2;
    if (POW) q4 = A4 + t * (g4 - A4);
  };
  for (int it = 0; it < kMaxIters; it++) {
    if (mode == PICK) {
      uint64_t tlo, thi, ilo, ihi;
      state_masks(S, nc, tlo, thi, ilo, ihi);
      const uint64_t olo = tlo & ~ilo, ohi = thi & ~ihi;
      if (!(olo | ohi)) {
        // no known outside corner: test the next untested ones
        const uint64_t vlo = low_mask(nc < 64 ? nc : 64), vhi = low_mask(nc > 64 ? nc - 64 : 0);
        const uint64_t ulo = vlo & ~tlo, uhi = vhi & ~thi;
        if (!(ulo | uhi)) return 0;
        // newest corners first (highest slots: the corners of the latest
        // faces, nearest to v_i): fewer of them are cut away after their test
        // than of the older, farther ones
        tslot = -1;
        nbatch = 0;
        uint64_t m = uhi;
        for (int h = 1; h >= 0; h--) {
          while (m && nbatch < 4) {
            const int b = 63 - __clzll((long long)m);
            if (nbatch == grp) tslot = b + 64 * h;
            nbatch++;
            m &= ~(1ull << b);
          }
          m = ulo;
        }
        const int s = tslot >= 0 ? tslot : (ulo ? __ffsll((unsigned long long)ulo) - 1
                                                : 64 + __ffsll((unsigned long long)uhi) - 1);
        q0 = S.cy[s][0]; q1 = S.cy[s][1]; q2 = S.cy[s][2];
        mode = TEST;
      } else {
        // ---- the search edge: from a tested-inside neighbour (Alg. 1) or v_i (Alg. 3)
        pt = -1;
        int ps = -1;
        if (C.straddle) {
          bool cand[2];
          for (int h = 0; h < 2; h++) {
            const int s = l + 64 * h;
            cand[h] = false;
            if (bit128(olo, ohi, s)) {
              const int nbp = S.cnb[s];
              cand[h] = bit128(ilo, ihi, p8(nbp, 0)) || bit128(ilo, ihi, p8(nbp, 1)) || bit128(ilo, ihi, p8(nbp, 2));
            }
          }
          const uint64_t clo = __ballot(cand[0]), chi = __ballot(cand[1]);
          if (clo | chi) {
            pt = clo ? __ffsll((unsigned long long)clo) - 1 : 64 + __ffsll((unsigned long long)chi) - 1;
            const int nbp = uni(S.cnb[pt]);
            for (int e = 0; e < 3; e++)
              if (bit128(ilo, ihi, p8(nbp, e))) { ps = p8(nbp, e); break; }
          }
        }
        if (pt < 0) pt = olo ? __ffsll((unsigned long long)olo) - 1 : 64 + __ffsll((unsigned long long)ohi) - 1;
        ps_edge = ps;
        A0 = A1 = A2 = 0;
        A4 = ps >= 0 ? 0.0 : X.h;  // from a corner on the hyperplane, or from the lifted site
        g4 = 0.0;
        if (ps >= 0) { A0 = S.cy[ps][0]; A1 = S.cy[ps][1]; A2 = S.cy[ps][2]; }
        g0 = S.cy[pt][0]; g1 = S.cy[pt][1]; g2 = S.cy[pt][2];
        j = uni((S.cst[pt] >> 8) - 1);
        if (j < 0 || j == X.si) return 3;
        jsl = POW ? -1 : cache_slot(S.K, j);
        // flags of a point on the edge p_s p_t: the two planes through the edge
        ef0 = ef1 = -2;
        efs0 = efs1 = -1;
        if (ps >= 0) {
          const int a0 = uni(S.cpl[ps]), b0 = uni(S.cpl[pt]);
          int ne = 0;
          for (int x = 0; x < 3; x++) {
            const int px = p8(a0, x);
            if (px == p8(b0, 0) || px == p8(b0, 1) || px == p8(b0, 2)) {
              const int lab = S.plab[px];
              if (ne == 0) { ef0 = lab >= 0 ? lab : -2; efs0 = lab >= 0 ? S.psl[px] : -1; }
              else { ef1 = lab >= 0 ? lab : -2; efs1 = lab >= 0 ? S.psl[px] : -1; }
              ne++;
            }
          }
          ef0 = uni(ef0); ef1 = uni(ef1);
          efs0 = uni(efs0); efs1 = uni(efs1);
        }
        nstep = 0;
        const double d0 = g0 - A0, d1 = g1 - A1, d2 = g2 - A2;
        L = C.improved ? sqrt(d0 * d0 + d1 * d1 + d2 * d2) : 0.0;
        if (C.improved && L > 0 && 2.0 * X.delta < L) {
          u0 = d0 / L; u1 = d1 / L; u2 = d2 / L;
          lam = 2;
          mode = LAMBDA;
        } else {
          bisector_point();
          mode = SEARCH;
        }
      }
    }
    // ---- the one nearest-site query of this iteration ----
    // LAMBDA: the four 16-lane groups test lambda .. lambda+3 at once; the
    // smallest one found outside is the step the sequential search would stop at
    bool lv = true;
    if (mode == LAMBDA) {
      const int lg = lam + grp;
      lv = lg < 2 + C.max_iters && lg * X.delta < L;
      const double tt = (lv ? lg : lam) * X.delta;
      q0 = A0 + tt * u0; q1 = A1 + tt * u1; q2 = A2 + tt * u2;
    }
    const int gs = (mode == TEST || mode == LAMBDA) ? 16 : 64;
    const double qx = X.vx + q0, qy = X.vy + q1, qz = X.vz + q2;
    const double dx = qx - X.vx, dy = qy - X.vy, dz = qz - X.vz;
    // sites the test treats like v_i: flags of the corner's planes (TEST), the
    // candidate and the search edge's planes (SEARCH), the edge's planes (LAMBDA)
    int e0 = ef0, e1 = ef1, e2 = mode == SEARCH ? j : -1;
    int es0 = efs0, es1 = efs1, es2 = mode == SEARCH ? jsl : -1;
    if (mode == TEST) {
      const int tpl = S.cpl[tslot >= 0 ? tslot : 0];
      e0 = S.plab[p8(tpl, 0)]; e1 = S.plab[p8(tpl, 1)]; e2 = S.plab[p8(tpl, 2)];
      es0 = S.psl[p8(tpl, 0)]; es1 = S.psl[p8(tpl, 1)]; es2 = S.psl[p8(tpl, 2)];
    }
    bool on_grid;
    if (MON) count_add(S.ar.rounds, 1);
    int kq;
    if (POW) {
      // lifted query on the grid; corners lie on the hyperplane
      const double qw = mode == SEARCH ? q4 : 0.0, dw = qw - X.h;
      kq = nn_query<true>(G, gs, qx, qy, qz, dx * dx + dy * dy + dz * dz + dw * dw, X.si, st.cands, qw);
      on_grid = true;
    } else {
      kq = nn_cached(S.K, G, gs, qx, qy, qz, dx * dx + dy * dy + dz * dz, X.si, e0 < 0 ? -1 : e0, e1 < 0 ? -1 : e1,
                     e2 < 0 ? -1 : e2, e0 < 0 ? -1 : es0, e1 < 0 ? -1 : es1, e2 < 0 ? -1 : es2, st.cands, on_grid);
    }
    if (mode == TEST) {
      st.queries += nbatch;
      st.grid += __popcll(__ballot(on_grid && (l & 15) == 0 && grp < nbatch));
      const int pl = tslot >= 0 ? S.cpl[tslot] : 0;
      const bool in = (kq == X.si) || (kq == S.plab[p8(pl, 0)]) || (kq == S.plab[p8(pl, 1)]) ||
                      (kq == S.plab[p8(pl, 2)]);
      __syncthreads();
      if (tslot >= 0 && (l & 15) == 0) S.cst[tslot] = (in ? 1 : 0) | 2 | ((kq + 1) << 8);
      __syncthreads();
      mode = PICK;
      continue;
    }
    if (mode == LAMBDA) {
      const bool lead = (l & 15) == 0;
      st.queries += __popcll(__ballot(lv && lead));
      st.grid += __popcll(__ballot(lv && lead && on_grid));
      const uint64_t hit = __ballot(lv && lead && kq != X.si && kq != ef0 && kq != ef1);
      if (hit) {
        const int src = __ffsll((unsigned long long)hit) - 1;  // lowest group found outside
        j = __builtin_amdgcn_readlane(kq, src);
        jsl = POW ? -1 : cache_slot(S.K, j);
        g0 = readlane_d(q0, src); g1 = readlane_d(q1, src); g2 = readlane_d(q2, src);
      } else {
        lam += 4;
        if (lam < 2 + C.max_iters && lam * X.delta < L) continue;
      }
      bisector_point();
      mode = SEARCH;
      continue;
    }
    st.queries++;
    st.grid += on_grid ? 1 : 0;
    const int k = uni(kq);
    // SEARCH: q lies on the boundary of Omega_i -> B_ij is a face of the cell
    if (!(k == X.si || k == j || k == ef0 || k == ef1)) {
      if (++nstep >= C.max_iters) return 3;
      j = k;
      jsl = POW ? -1 : cache_slot(S.K, j);
      g0 = q0; g1 = q1; g2 = q2;
      g4 = q4;
      bisector_point();
      continue;
    }
    // ---- clip by B_ij ----
    if (npl >= VD_P_MAX) {
      npl = compact_planes(S, npl, nc);
      if (npl >= VD_P_MAX) return 2;
    }
    const int P = npl++;
    __syncthreads();
    if (l == 0) {
      S.pn[P][0] = n0; S.pn[P][1] = n1; S.pn[P][2] = n2; S.pn[P][3] = nc3;
      S.plab[P] = j;
      S.psl[P] = jsl;
    }
    __syncthreads();
    const int rc = clip_poly<MON>(S, P, pt, nc, ps_edge >= 0 && qon ? ps_edge : -1, k);
    st.clips++;
    if (rc == 1) return 1;
    if (rc != 4) return rc == 0 ? 3 : rc;
    mode = PICK;
  }
  return 3;
}

// Plane of face f of T_a (opposite vertex f), outward, relative to v_i, and
// its flag.  Face loops {1,2,3},{0,3,2},{0,1,3},{0,2,1} are packed 2 bits per
// vertex, 6 bits per face (no indexed local arrays).
__device__ __forceinline__ void tet_plane(const DomainView &D, const SiteCtx &X, int a, int f, double *pl,
                                          int &lab) {
  const auto tv = &GL(D.simp)[(long long)a * 4];
  const unsigned loops = (1u | 2u << 2 | 3u << 4) | (0u | 3u << 2 | 2u << 4) << 6 |
                         (0u | 1u << 2 | 3u << 4) << 12 | (0u | 2u << 2 | 1u << 4) << 18;
  const unsigned lf = loops >> (6 * f);
  const auto pA = &GL(D.verts)[3 * (long long)tv[lf & 3]];
  const auto pB = &GL(D.verts)[3 * (long long)tv[(lf >> 2) & 3]];
  const auto pC = &GL(D.verts)[3 * (long long)tv[(lf >> 4) & 3]];
  const double A0 = pA[0] - X.vx, A1 = pA[1] - X.vy, A2 = pA[2] - X.vz;
  const double ab0 = pB[0] - pA[0], ab1 = pB[1] - pA[1], ab2 = pB[2] - pA[2];
  const double ac0 = pC[0] - pA[0], ac1 = pC[1] - pA[1], ac2 = pC[2] - pA[2];
  const double n0 = ab1 * ac2 - ab2 * ac1, n1 = ab2 * ac0 - ab0 * ac2, n2 = ab0 * ac1 - ab1 * ac0;
  pl[0] = n0; pl[1] = n1; pl[2] = n2;
  pl[3] = n0 * A0 + n1 * A1 + n2 * A2;
  const int b = GL(D.adj)[(long long)a * 4 + f];
  lab = b >= 0 ? -(b + 1) : VD_BND_BASE + f;
}

// P <- T_a: 4 planes (face f opposite vertex f), 4 corners.  Lane l < 4
// builds plane l and corner l; the fixed topology of a positively oriented
// tetrahedron is packed in constants.
__device__ void init_tet(WaveLds &S, const DomainView &D, const SiteCtx &X, int a, int tested) {
  const int l = vd_lane();
  if (l < 4) {
    double pl[4];
    int lab;
    tet_plane(D, X, a, l, pl, lab);
    S.pn[l][0] = pl[0]; S.pn[l][1] = pl[1]; S.pn[l][2] = pl[2]; S.pn[l][3] = pl[3];
    S.plab[l] = lab;
    S.psl[l] = -1;
    // corner l = vertex l: planes counter-clockwise from outside
    // {1,3,2},{0,2,3},{0,3,1},{0,1,2}; neighbours {2,1,3},{3,0,2},{1,0,3},{2,0,1}
    S.cpl[l] = l == 0 ? pack3(1, 3, 2) : (l == 1 ? pack3(0, 2, 3) : (l == 2 ? pack3(0, 3, 1) : pack3(0, 1, 2)));
    S.cnb[l] = l == 0 ? pack3(2, 1, 3) : (l == 1 ? pack3(3, 0, 2) : (l == 2 ? pack3(1, 0, 3) : pack3(2, 0, 1)));
    S.cst[l] = tested ? 3 : 0;
    const auto p = &GL(D.verts)[3 * (long long)GL(D.simp)[(long long)a * 4 + l]];
    S.cy[l][0] = p[0] - X.vx; S.cy[l][1] = p[1] - X.vy; S.cy[l][2] = p[2] - X.vz;
  }
  __syncthreads();
}

static_assert(VD_C_MAX * 3 >= VD_CACHE_SCRATCH, "the corner array doubles as the site cache's sort scratch");

// cell-first: keep the carved cell (npl planes, nc corners) in this wave's
// part of a global buffer (it stays in the L2 of the wave's XCD) ...
struct SavedCell {
  __attribute__((address_space(1))) double *pn, *cy;
  __attribute__((address_space(1))) int *plab, *cpl, *cnb;
};
__device__ __forceinline__ SavedCell saved_cell(const CellsDev &C) {
  SavedCell B;
  double *base = C.saved + (long long)blockIdx.x * VD_SAVE_DOUBLES;
  B.pn = GL(base);
  B.cy = GL(base + VD_F_MAX * 4);
  int *ib = reinterpret_cast<int *>(base + VD_F_MAX * 4 + VD_CB_MAX * 3);
  B.plab = GL(ib);
  B.cpl = GL(ib + VD_F_MAX);
  B.cnb = GL(ib + VD_F_MAX + VD_CB_MAX);
  return B;
}

__device__ void save_cell(WaveLds &S, const CellsDev &C, int npl, int nc) {
  const int l = vd_lane();
  const SavedCell B = saved_cell(C);
  if (l < npl) {
    for (int k = 0; k < 4; k++) B.pn[4 * l + k] = S.pn[l][k];
    B.plab[l] = S.plab[l];
  }
  for (int s = l; s < nc; s += 64) {
    B.cpl[s] = S.cpl[s];
    B.cnb[s] = S.cnb[s];
    for (int k = 0; k < 3; k++) B.cy[3 * s + k] = S.cy[s][k];
  }
  __threadfence_block();  // the wave reads it back: stores complete first
}

// ... and start a piece from it: the cell plus the four planes of T_a in
// slots npl .. npl+3 (not yet cut)
__device__ void restore_cell(WaveLds &S, const CellsDev &C, int npl, int nc, const DomainView &D, const SiteCtx &X,
                             int a) {
  const int l = vd_lane();
  const SavedCell B = saved_cell(C);
  if (l < npl) {
    for (int k = 0; k < 4; k++) S.pn[l][k] = B.pn[4 * l + k];
    S.plab[l] = B.plab[l];
  } else if (l < npl + 4) {
    double pl[4];
    int lab;
    tet_plane(D, X, a, l - npl, pl, lab);
    for (int k = 0; k < 4; k++) S.pn[l][k] = pl[k];
    S.plab[l] = lab;
  }
  if (l < npl + 4) S.psl[l] = -1;  // a restored cell is only cut, never queried
  for (int s = l; s < nc; s += 64) {
    S.cpl[s] = B.cpl[s];
    S.cnb[s] = B.cnb[s];
    S.cst[s] = 3;
    for (int k = 0; k < 3; k++) S.cy[s][k] = B.cy[3 * s + k];
  }
  __syncthreads();
}

// the cell in LDS (npl <= kLF planes, nc <= kLC corners) over the cache
__device__ void save_cell_lds(WaveLds &S, int npl, int nc) {
  const int l = vd_lane();
  __syncthreads();
  double p4[4] = {0, 0, 0, 0};
  int lab = 0;
  if (l < npl) {
    for (int k = 0; k < 4; k++) p4[k] = S.pn[l][k];
    lab = S.plab[l];
  }
  int cp = 0, cn = 0;
  double y0 = 0, y1 = 0, y2 = 0;
  if (l < nc) { cp = S.cpl[l]; cn = S.cnb[l]; y0 = S.cy[l][0]; y1 = S.cy[l][1]; y2 = S.cy[l][2]; }
  __syncthreads();  // the cache is read no more
  if (l < npl) {
    for (int k = 0; k < 4; k++) S.LC.pn[l][k] = p4[k];
    S.LC.plab[l] = lab;
  }
  if (l < nc) { S.LC.cpl[l] = cp; S.LC.cnb[l] = cn; S.LC.cy[l][0] = y0; S.LC.cy[l][1] = y1; S.LC.cy[l][2] = y2; }
  __syncthreads();
}

// start a piece from the LDS cell: the cell plus the four planes of T_a in
// slots npl .. npl+3 (not yet cut)
__device__ void restore_cell_lds(WaveLds &S, int npl, int nc, const DomainView &D, const SiteCtx &X, int a) {
  const int l = vd_lane();
  if (l < npl) {
    for (int k = 0; k < 4; k++) S.pn[l][k] = S.LC.pn[l][k];
    S.plab[l] = S.LC.plab[l];
  } else if (l < npl + 4) {
    double pl[4];
    int lab;
    tet_plane(D, X, a, l - npl, pl, lab);
    for (int k = 0; k < 4; k++) S.pn[l][k] = pl[k];
    S.plab[l] = lab;
  }
  if (l < npl + 4) S.psl[l] = -1;  // a restored cell is only cut, never queried
  if (l < nc) {
    S.cpl[l] = S.LC.cpl[l];
    S.cnb[l] = S.LC.cnb[l];
    S.cst[l] = 3;
    S.cy[l][0] = S.LC.cy[l][0]; S.cy[l][1] = S.LC.cy[l][1]; S.cy[l][2] = S.LC.cy[l][2];
  }
  __syncthreads();
}

// P <- box [lo, hi] (planes x-,x+,y-,y+,z-,z+; corner (bx,by,bz) = 4bx+2by+bz)
__device__ void init_box(WaveLds &S, const SiteCtx &X, const double *lo, const double *hi) {
  const int l = vd_lane();
  if (l < 6) {
    const int ax = l >> 1, side = l & 1;
    const double vc = ax == 0 ? X.vx : (ax == 1 ? X.vy : X.vz);
    const double lov = ax == 0 ? lo[0] : (ax == 1 ? lo[1] : lo[2]);
    const double hiv = ax == 0 ? hi[0] : (ax == 1 ? hi[1] : hi[2]);
    S.pn[l][0] = ax == 0 ? (side ? 1.0 : -1.0) : 0.0;
    S.pn[l][1] = ax == 1 ? (side ? 1.0 : -1.0) : 0.0;
    S.pn[l][2] = ax == 2 ? (side ? 1.0 : -1.0) : 0.0;
    S.pn[l][3] = side ? hiv - vc : vc - lov;
    S.plab[l] = kBoxBase + l;
    S.psl[l] = -1;
  }
  if (l < 8) {
    // planes / neighbours of corner l, 4 bits per entry (12 bits per corner)
    const unsigned long long CP = 0x240ull | 0x520ull << 12 | 0x430ull << 24 | 0x350ull << 36 | 0x421ull << 48;
    const unsigned long long CP2 = 0x251ull | 0x341ull << 12 | 0x531ull << 24;
    const unsigned long long CN = 0x142ull | 0x350ull << 12 | 0x063ull << 24 | 0x271ull << 36 | 0x605ull << 48;
    const unsigned long long CN2 = 0x417ull | 0x724ull << 12 | 0x536ull << 24;
    const unsigned cpl = l < 5 ? (unsigned)((CP >> (12 * l)) & 0xfff) : (unsigned)((CP2 >> (12 * (l - 5))) & 0xfff);
    const unsigned cnb = l < 5 ? (unsigned)((CN >> (12 * l)) & 0xfff) : (unsigned)((CN2 >> (12 * (l - 5))) & 0xfff);
    S.cpl[l] = pack3(cpl & 15, (cpl >> 4) & 15, (cpl >> 8) & 15);
    S.cnb[l] = pack3(cnb & 15, (cnb >> 4) & 15, (cnb >> 8) & 15);
    S.cst[l] = 0;
    S.cy[l][0] = ((l >> 2) & 1 ? hi[0] : lo[0]) - X.vx;
    S.cy[l][1] = ((l >> 1) & 1 ? hi[1] : lo[1]) - X.vy;
    S.cy[l][2] = (l & 1 ? hi[2] : lo[2]) - X.vz;
  }
  __syncthreads();
}

__device__ __forceinline__ int convert_label(const GridView &G, int lab) { return lab >= 0 ? GL(G.perm)[lab] : lab; }

// Face moments of the bisector faces of the piece in LDS, for the adjoint:
// for face x on B_ik, I0 = int y dA/d, I1 = int y y^T dA/d, I2 = int |y|^2 y dA/d
// with y = x - v_i and d = |v_k - v_i|.  Lane x walks around face x from its
// lowest corner (a fixed order, so the sums are reproducible) and integrates
// the fan of triangles (foot of the plane, corner, next corner): linear and
// quadratic terms in closed form, the cubic term with the degree-3 rule of
// Strang and Fix (centroid -27/48, points (3/5,1/5,1/5) 25/48); with a density
// every integrand carries it and one degree-5 rule takes all twelve.
template <bool DENS>
__device__ void face_moments(WaveLds &S, int nc, int npl, uint64_t fmask, const CellsDev &C, const GridView &G,
                             const SiteCtx &X, long long pidx) {
  const int l = vd_lane();
  __syncthreads();
  if (l < npl) S.pfirst[l] = 0x7fffffff;
  __syncthreads();
  for (int s = l; s < nc; s += 64) {
    const int pl = S.cpl[s];
    atomicMin(&S.pfirst[p8(pl, 0)], s);
    atomicMin(&S.pfirst[p8(pl, 1)], s);
    atomicMin(&S.pfirst[p8(pl, 2)], s);
  }
  __syncthreads();
  const bool mine = l < npl && ((fmask >> l) & 1ull) && S.plab[l] >= 0;
  const uint64_t pos = __ballot(mine);
  const int npos = __popcll(pos);
  const long long base = arena_take(S.ar, C, AR_FINT, npos);
  const bool fits = base + npos <= C.cap_fint;
  if (l == 0 && pidx < C.cap_piece) {
    GL(C.piece_fint_start)[pidx] = base;
    GL(C.piece_nfint)[pidx] = fits ? npos : 0;
    if (!fits) S.ar.dropped++;
  }
  if (!mine) return;
  const int x = l;
  const double n0 = S.pn[x][0], n1 = S.pn[x][1], n2 = S.pn[x][2], cc = S.pn[x][3];
  const double nn = n0 * n0 + n1 * n1 + n2 * n2;
  const double d = sqrt(nn), f = cc / nn;
  const double h0 = n0 / d, h1 = n1 / d, h2 = n2 / d;
  const double r0 = n0 * f, r1 = n1 * f, r2 = n2 * f;
  double I[12];
  for (int k = 0; k < 12; k++) I[k] = 0.0;
  const int start = S.pfirst[x];
  int T = start;
  for (int step = 0; step < VD_C_MAX; step++) {
    const int pl = S.cpl[T];
    const int e = p8(pl, 0) == x ? 0 : (p8(pl, 1) == x ? 1 : 2);
    const int nx = p8(S.cnb[T], (e + 2) % 3);
    const double a0 = S.cy[T][0], a1 = S.cy[T][1], a2 = S.cy[T][2];
    const double b0 = S.cy[nx][0], b1 = S.cy[nx][1], b2 = S.cy[nx][2];
    const double u0 = a0 - r0, u1 = a1 - r1, u2 = a2 - r2, w0 = b0 - r0, w1 = b1 - r1, w2 = b2 - r2;
    const double A = 0.5 * ((u1 * w2 - u2 * w1) * h0 + (u2 * w0 - u0 * w2) * h1 + (u0 * w1 - u1 * w0) * h2);
    if (DENS) {
      // weighted by the density: one degree-5 rule for all twelve integrals
      const double P0[3] = {r0, r1, r2}, P1[3] = {a0, a1, a2}, P2[3] = {b0, b1, b2};
      tri_density_face(C.dens, X.vx, X.vy, X.vz, P0, P1, P2, A, I);
      T = nx;
      if (T == start) break;
      continue;
    }
    const double s0 = r0 + a0 + b0, s1 = r1 + a1 + b1, s2 = r2 + a2 + b2;
    I[0] += A * s0 / 3.0; I[1] += A * s1 / 3.0; I[2] += A * s2 / 3.0;
    const double q = A / 12.0;
    I[3] += q * (r0 * r0 + a0 * a0 + b0 * b0 + s0 * s0);
    I[4] += q * (r0 * r1 + a0 * a1 + b0 * b1 + s0 * s1);
    I[5] += q * (r0 * r2 + a0 * a2 + b0 * b2 + s0 * s2);
    I[6] += q * (r1 * r1 + a1 * a1 + b1 * b1 + s1 * s1);
    I[7] += q * (r1 * r2 + a1 * a2 + b1 * b2 + s1 * s2);
    I[8] += q * (r2 * r2 + a2 * a2 + b2 * b2 + s2 * s2);
    // cubic |y|^2 y: degree-3 rule on (r, a, b)
    const double c0 = s0 / 3.0, c1 = s1 / 3.0, c2 = s2 / 3.0;
    double t0 = -27.0 / 48.0 * (c0 * c0 + c1 * c1 + c2 * c2);
    double acc0 = t0 * c0, acc1 = t0 * c1, acc2 = t0 * c2;
#pragma unroll
    for (int v = 0; v < 3; v++) {
      // point 3/5 at vertex v, 1/5 at the other two
      const double p0 = 0.2 * s0 + 0.4 * (v == 0 ? r0 : (v == 1 ? a0 : b0));
      const double p1 = 0.2 * s1 + 0.4 * (v == 0 ? r1 : (v == 1 ? a1 : b1));
      const double p2 = 0.2 * s2 + 0.4 * (v == 0 ? r2 : (v == 1 ? a2 : b2));
      const double w = 25.0 / 48.0 * (p0 * p0 + p1 * p1 + p2 * p2);
      acc0 += w * p0; acc1 += w * p1; acc2 += w * p2;
    }
    I[9] += A * acc0; I[10] += A * acc1; I[11] += A * acc2;
    T = nx;
    if (T == start) break;
  }
  const long long r = base + __popcll(pos & low_mask(l));
  if (r < C.cap_fint) {
    const double id = 1.0 / d;
    for (int k = 0; k < 12; k++) GL(C.fint)[12 * r + k] = I[k] * id;
    GL(C.fint_lab)[r] = GL(G.perm)[S.plab[x]];
  }
}

// Entries VD_Q_MAX.. of a site's simplex queue live in this wave's part of a
// global buffer (cells that meet more simplices than the LDS queue holds).
// Out of line: the common case never touches them.
__device__ __forceinline__ int spill_get(const CellsDev &C, int i) {
  return GL(C.tq_spill)[(long long)blockIdx.x * C.q_spill + i - VD_Q_MAX];
}
__device__ __forceinline__ bool spill_has(const CellsDev &C, int b, int nt) {
  const int*q = C.tq_spill + (long long)blockIdx.x * C.q_spill - VD_Q_MAX;
  bool have = false;
  for (int e = VD_Q_MAX + vd_lane(); e < nt; e += 64) have = have || (q[e] == b);
  return have;
}
__device__ __forceinline__ void spill_put(const CellsDev &C, int i, int b) {
  if (vd_lane() == 0) GL(C.tq_spill)[(long long)blockIdx.x * C.q_spill + i - VD_Q_MAX] = b;
}

// Appends simplex b to the site's breadth-first queue unless it is there
// already.  Returns false when the queue is full.
__device__ __forceinline__ bool tq_push(WaveLds &S, const CellsDev &C, int &nt, int b) {
  const int l = vd_lane();
  bool have = false;
  const int nl = nt < VD_Q_MAX ? nt : VD_Q_MAX;
  for (int e = l; e < nl; e += 64) have = have || (S.tq[e] == b);
  if (nt > VD_Q_MAX) have = have || spill_has(C, b, nt);
  if (__ballot(have)) return true;
  if (nt >= VD_Q_MAX + C.q_spill) return false;
  __syncthreads();
  if (nt < VD_Q_MAX) {
    if (l == 0) S.tq[nt] = b;
  } else {
    spill_put(C, nt, b);  // large cells: the queue continues in global memory
  }
  nt++;
  __syncthreads();
  return true;
}

// The lowest-index tetrahedron containing q (the whole wave scans the point's
// location cell), or -1.
__device__ int locate_wave(const DomainView &D, double qx, double qy, double qz) {
  if (!D.lstart) return -1;
  const double q[3] = {qx, qy, qz};
  int cc[3];
  for (int k = 0; k < 3; k++) cc[k] = cell_coord(q[k], GL(D.lgeom)[k], GL(D.lgeom)[6 + k], D.lg[k]);
  const int c = cc[0] + D.lg[0] * (cc[1] + D.lg[1] * cc[2]);
  int best = 0x7fffffff;
  for (int t = GL(D.lstart)[c] + vd_lane(); t < GL(D.lstart)[c + 1]; t += 64) {
    const int a = GL(D.litems)[t];
    if (a < best && tet_contains(D, a, q)) best = a;
  }
  const int b = (int)wave_min((double)best);
  return b == 0x7fffffff ? -1 : b;
}

// Is q in M?  One lane scans q's location cell (the tolerance of tet_contains
// counts a point on the boundary as inside).
__device__ bool in_domain(const DomainView &D, double qx, double qy, double qz) {
  const double q[3] = {qx, qy, qz};
  int cc[3];
  for (int k = 0; k < 3; k++) cc[k] = cell_coord(q[k], GL(D.lgeom)[k], GL(D.lgeom)[6 + k], D.lg[k]);
  const int c = cc[0] + D.lg[0] * (cc[1] + D.lg[1] * cc[2]);
  for (int t = GL(D.lstart)[c]; t < GL(D.lstart)[c + 1]; t++)
    if (tet_contains(D, GL(D.litems)[t], q)) return true;
  return false;
}

// Do all nc corners of the polytope in S lie in M?  (Whole wave.)
__device__ __forceinline__ bool cell_in_domain(const WaveLds &S, const DomainView &D, const SiteCtx &X, int nc) {
  bool out = false;
  for (int x = vd_lane(); x < nc; x += 64)
    out = out || !in_domain(D, X.vx + S.cy[x][0], X.vy + S.cy[x][1], X.vz + S.cy[x][2]);
  return !__ballot(out);
}

// Gabriel neighbours among the first kGabriel cache entries (distance-bucket
// order): a site v_j whose ball on the diameter [v_i, v_j] holds no other site
// (and lies inside the cached radius, so every site that could be in it is
// cached) has the midpoint of v_i v_j on the face of Omega_i towards it, so
// the bisector B_ij is a face plane of the cell and a valid clip (Alg. 1 only
// clips by faces).  The polytope (the box) is clipped by every such bisector
// before the carve, which then finds the other faces by its tests and
// searches.  Returns 0, or a clip's failure (the caller then carves the box
// without these clips).  Lanes c and c + 32 hold candidate c and scan the two
// halves of the cached sites; the halves' results are then merged through LDS.
constexpr int kGabriel = 24;
static_assert(kGabriel <= 32, "a candidate per lane of each half-wave");

// Merges the two half-wave scans of a candidate: the deepest site (the lower
// position on a tie, as one scan in position order would take) and whether
// both halves found the ball empty.  The lanes swap their results through the
// 64 rows at ex (whole wave; the rows are free while the function runs).
__device__ __forceinline__ void merge_halves(double (*ex)[3], double &depth, int &deep, bool &empty) {
  const int l = vd_lane();
  const bool lo = l < 32;
  __syncthreads();
  ex[l][0] = depth;
  ex[l][1] = (double)deep;
  ex[l][2] = empty ? 1.0 : 0.0;
  __syncthreads();
  const double od = ex[l ^ 32][0];
  const int ok = (int)ex[l ^ 32][1];
  const bool oe = ex[l ^ 32][2] != 0.0;
  __syncthreads();
  const double dlo = lo ? depth : od, dhi = lo ? od : depth;
  const int klo = lo ? deep : ok, khi = lo ? ok : deep;
  depth = dhi < dlo ? dhi : dlo;
  deep = dhi < dlo ? khi : klo;
  empty = empty && oe;
}

template <bool MON>
__device__ int gabriel_clips(WaveLds &S, const SiteCtx &X, int &npl, int &nc, Stats &st) {
  const int l = vd_lane();
  const int cl = l & 31;  // this lane's candidate
  const bool upper = l >= 32;
  const int n = S.K.cnt;
  const int T = n < kGabriel ? n : kGabriel;
  if (T <= 0) return 0;
  // sites nearer to v_i than the farthest candidate lie below position E
  const int kbT = S.K.kb[T - 1];
  int E = n;
  {
    const uint64_t a = __ballot(l < n && S.K.kb[l] > kbT);
    const uint64_t b = __ballot(l + 64 < n && S.K.kb[l + 64] > kbT);
    if (a) E = __ffsll((unsigned long long)a) - 1;
    else if (b) E = 64 + __ffsll((unsigned long long)b) - 1;
  }
  const double rc2 = S.K.rc * S.K.rc;
  double jx = 0, jy = 0, jz = 0, dj2 = 0;
  bool gab = false;
  if (cl < T) {
    jx = S.K.x[cl] - X.vx; jy = S.K.y[cl] - X.vy; jz = S.K.z[cl] - X.vz;
    dj2 = jx * jx + jy * jy + jz * jz;
    gab = dj2 > 0.0 && dj2 < rc2 * (1.0 - 1e-9);
  }
  const double mx = 0.5 * jx, my = 0.5 * jy, mz = 0.5 * jz, r2 = 0.25 * dj2 * (1.0 + 1e-9);
  const bool cand = gab;
  int kin = -1;          // the site deepest inside the diametral ball
  double kdepth = 1e300;
  // corner rows 64-127 are unused until the first clip below (the box has 8)
  double(*const ex)[3] = &S.cy[64];
  static_assert(VD_C_MAX >= 128, "64 free corner rows for the merge");
  const int hE = (E + 1) >> 1;
  for (int k = upper ? hE : 0, kend = upper ? E : hE; k < kend; k++) {
    const double kx = S.K.x[k] - X.vx, ky = S.K.y[k] - X.vy, kz = S.K.z[k] - X.vz;
    const double ex = kx - mx, ey = ky - my, ez = kz - mz;
    const bool self = kx == 0.0 && ky == 0.0 && kz == 0.0;
    const double e2 = ex * ex + ey * ey + ez * ez;
    if (k != cl && !self && e2 <= r2) {
      gab = false;
      if (e2 < kdepth) { kdepth = e2; kin = k; }
    }
  }
  merge_halves(ex, kdepth, kin, gab);
  // A non-Gabriel v_j is still a Delaunay neighbour when the smallest sphere
  // through v_i, v_j and the site v_k deepest in its diametral ball holds no
  // other site: its centre (the circumcentre of the three) is then a point of
  // the Voronoi edge of i, j, k, which lies on the face towards v_j.  Only
  // spheres up to 1.4 times the diametral ball's (squared radius) are tried:
  // larger ones rarely come out empty and cost a longer scan.
  bool tri = false;
  double cx = 0, cy = 0, cz = 0, R2 = 0;
  if (cand && !gab && kin >= 0) {
    const double ax = jx, ay = jy, az = jz;
    const double bx = S.K.x[kin] - X.vx, by = S.K.y[kin] - X.vy, bz = S.K.z[kin] - X.vz;
    const double wx = ay * bz - az * by, wy = az * bx - ax * bz, wz = ax * by - ay * bx;
    const double w2 = wx * wx + wy * wy + wz * wz, a2 = dj2, b2 = bx * bx + by * by + bz * bz;
    if (w2 > 1e-12 * a2 * b2) {
      // c = (|a|^2 (b x w) + |b|^2 (w x a)) / (2 |w|^2), w = a x b
      const double iw = 0.5 / w2;
      cx = (a2 * (by * wz - bz * wy) + b2 * (wy * az - wz * ay)) * iw;
      cy = (a2 * (bz * wx - bx * wz) + b2 * (wz * ax - wx * az)) * iw;
      cz = (a2 * (bx * wy - by * wx) + b2 * (wx * ay - wy * ax)) * iw;
      R2 = cx * cx + cy * cy + cz * cz;
      tri = 4.0 * R2 < rc2 * (1.0 - 1e-9) && R2 < 0.35 * a2;
    }
  }
  if (__ballot(tri)) {
    // sites within 2 R of v_i lie below the first bucket beyond (2 R)^2
    const double lim = -wave_min(tri ? -4.0 * R2 : 0.0);
    int E2 = n;
    {
      const uint64_t a = __ballot(l < n && (double)S.K.kb[l] * S.K.step > lim);
      const uint64_t b = __ballot(l + 64 < n && (double)S.K.kb[l + 64] * S.K.step > lim);
      if (a) E2 = __ffsll((unsigned long long)a) - 1;
      else if (b) E2 = 64 + __ffsll((unsigned long long)b) - 1;
    }
    const double R2in = R2 * (1.0 + 1e-9);
    const int h2 = (E2 + 1) >> 1;
    for (int k = upper ? h2 : 0, kend = upper ? E2 : h2; k < kend; k++) {
      const double kx = S.K.x[k] - X.vx, ky = S.K.y[k] - X.vy, kz = S.K.z[k] - X.vz;
      const double ex = kx - cx, ey = ky - cy, ez = kz - cz;
      const bool self = kx == 0.0 && ky == 0.0 && kz == 0.0;
      if (k != cl && k != kin && !self && ex * ex + ey * ey + ez * ez <= R2in) tri = false;
    }
    {
      double dd = 0.0;
      int dk = 0;
      merge_halves(ex, dd, dk, tri);
    }
    gab = gab || tri;
  }
  gab = gab && !upper;  // the lower half clips
  for (uint64_t m = __ballot(gab); m; m &= m - 1) {
    const int c = __ffsll((unsigned long long)m) - 1;
    if (npl >= VD_P_MAX) return 2;
    const int P = npl++;
    __syncthreads();
    if (l == c) {
      S.pn[P][0] = jx; S.pn[P][1] = jy; S.pn[P][2] = jz; S.pn[P][3] = 0.5 * dj2;
      S.plab[P] = S.K.p[c];
      S.psl[P] = c;
    }
    __syncthreads();
    const int rc = clip_poly<MON>(S, P, -1, nc);
    if (rc == 4) st.clips++;
    else if (rc != 0) return rc;
  }
  return 0;
}

// Neighbour e of the site's list: the first VD_NB_MAX in LDS, the rest in this
// wave's part of a global buffer.
__device__ __forceinline__ int nb_get(const WaveLds &S, const CellsDev &C, int e) {
  return e < VD_NB_MAX ? S.nbl[e] : GL(C.nb_spill)[(long long)blockIdx.x * C.nbs_cap + e - VD_NB_MAX];
}

// Appends neighbour lab unless it is listed already.  Returns false when the
// list is full (the synchronous clip then grows the buffer and runs again).
__device__ __forceinline__ bool nb_push(WaveLds &S, const CellsDev &C, int &nnb, int lab) {
  const int l = vd_lane();
  bool have = false;
  const int nl = nnb < VD_NB_MAX ? nnb : VD_NB_MAX;
  for (int e = l; e < nl; e += 64) have = have || (S.nbl[e] == lab);
  for (int e = VD_NB_MAX + l; e < nnb; e += 64) have = have || (nb_get(S, C, e) == lab);
  if (__ballot(have)) return true;
  if (nnb >= VD_NB_MAX + C.nbs_cap) return false;
  __syncthreads();
  if (l == 0) {
    if (nnb < VD_NB_MAX) S.nbl[nnb] = lab;
    else GL(C.nb_spill)[(long long)blockIdx.x * C.nbs_cap + nnb - VD_NB_MAX] = lab;
  }
  nnb++;
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// One site: its pieces, per-site sums and neighbour list.  The tetrahedra of
// the cell are visited breadth-first through negative face flags from the
// tetrahedron containing v_i (the propagation of Alg. 5).
//   cell-first (C.mode = 1): Omega_i cap box is carved once (Sec. 5.2); every
//     corner of the result is certified by a point-in-cell test, so
//     T_a cap Omega_i = T_a cap cell: the saved cell cut by the (at most four)
//     planes of T_a.  A cell too large to save falls back to the other mode.
//   per-simplex (C.mode = 0): each piece is carved from T_a by point-in-cell
//     tests and the bisector search.
// The carve has one call site: the first job of a cell-first site is the cell.
// ---------------------------------------------------------------------------
template <bool MON, bool DENS, bool POW, bool CORNERS>
__device__ void do_site(WaveLds &S, const GridView &G0, const DomainView &D0, const CellsDev &C, int si) {
  const int l = vd_lane();
  // The views are re-read from memory (scalar loads) in each piece iteration
  // rather than held in scalar registers across the whole site: the opaque
  // pointer copies below keep the compiler from hoisting their fields.
  const GridView *Gp = &G0;
  const DomainView *Dp = &D0;
  const GridView &G = G0;
  const DomainView &D = D0;
  SiteCtx X;
  X.vx = GL(G.sx)[si]; X.vy = GL(G.sy)[si]; X.vz = GL(G.sz)[si];
  X.delta = GL(G.delta)[si];
  X.h = POW ? GL(G.sh)[si] : 0.0;
  X.w = POW ? GL(G.sw)[si] : 0.0;
  X.si = si;
  const int orig = GL(G.perm)[si];
  const int seed = GL(C.seed)[si];
  const CarveParams P = {C.improved, C.straddle, C.max_iters};
  Stats st;
  int err = 0;  // 2 capacity, 3 degenerate, 4 outside M without boundary seeds
  int where = 0;  // failing stage (VD_STAGE_*)
  int nt = 0, head = 0, nnb = 0, npieces = 0, npl0 = 0, nc0 = 0;
  bool cell_job = C.mode == 1, saved = false, saved_lds = false;
  // pieces cut from the saved cell: their bisector faces are cell planes, so
  // the neighbours found are a mask over the cell's plane slots (cellpos: the
  // slots whose flag is a site), turned into a list once per site
  if (l == 0) {
    for (int k = 0; k < 5; k++) S.acc[k] = 0.0;
    S.cellpos = 0ull;
    S.nbmask = 0ull;
  }
  int cell_lab = 0;  // lane x: the flag of the cell's plane x

  if (C.cache) {
    cache_fill(S.K, G, X.vx, X.vy, X.vz, &S.cy[0][0]);  // the corner array is free until the carve
  } else {
    if (l == 0) S.K.cnt = -1;
  }
  if (seed >= 0 && seed < D.m) {
    if (l == 0) S.tq[0] = seed;
    nt = 1;
  }
  __syncthreads();
  long long nbseed = 0;  // boundary triangles the cell meets (when computed)
  if (C.bseed_off) {
    // Alg. 5: every boundary triangle the cell meets seeds the tetrahedron
    // behind it, which reaches the parts of Omega_i cap M that are not
    // connected to the site's own tetrahedron (or all of them, for a site
    // outside M)
    const long long q0 = GL(C.bseed_off)[orig], q1 = GL(C.bseed_off)[orig + 1];
    nbseed = q1 - q0;
    for (long long q = q0; q < q1; q++) {
      const int t = GL(C.btet)[GL(C.bseed_tri)[GL(C.bseed_pid)[q]]];
      if (!tq_push(S, C, nt, t)) { err = 2; where = VD_STAGE_SIMPLICES; break; }
    }
  } else if (!nt && !POW) {
    err = 4;  // outside every tetrahedron, and no boundary seeds to find its cell
  }
  if (!nt && !POW) cell_job = false;
  for (;;) {
    asm volatile("" : "+s"(Gp), "+s"(Dp));
    const GridView &G = *Gp;
    const DomainView &D = *Dp;
    int a = -1, npl = 4, nc = 4;
    bool empty = false, need_carve = true;
    if (cell_job) {
      init_box(S, X, D.box_lo, D.box_hi);
      npl = 6;
      nc = 8;
    } else {
      if (head >= nt || err) break;
      a = head < VD_Q_MAX ? S.tq[head] : spill_get(C, head);
      head++;
      if (saved) {
        if (saved_lds) restore_cell_lds(S, npl0, nc0, D, X, a);
        else restore_cell(S, C, npl0, nc0, D, X, a);
        npl = npl0 + 4;
        nc = nc0;
        need_carve = false;
#pragma unroll 1
        for (int f = 0; f < 4; f++) {
          const int rc = clip_poly<MON>(S, npl0 + f, -1, nc);
          if (rc == 4) st.clips++;
          else if (rc == 1) { empty = true; break; }
          else if (rc == 2) { err = rc; where = VD_STAGE_PIECE_CUT; break; }
          else if (rc == 3) { need_carve = true; break; }  // degenerate cut: carve this piece from T_a
        }
        if (need_carve && !err) {
          if (saved_lds && l == 0) S.K.cnt = -1;  // the cell sits over the cache: query the grid
          init_tet(S, D, X, a, 0);
          npl = 4;
          nc = 4;
        }
      } else {
        init_tet(S, D, X, a, 0);
      }
    }
    if (need_carve) {
      if (cell_job && !POW && S.K.cnt > 0 && gabriel_clips<MON>(S, X, npl, nc, st)) {
        init_box(S, X, D.box_lo, D.box_hi);  // a failed clip: carve the box as it is
        npl = 6;
        nc = 8;
      }
      const int rc = carve<MON, POW>(S, G, P, X, npl, nc, st);
      if (cell_job) {
        cell_job = false;
        if (POW && rc == 1) { head = nt; continue; }     // an empty power cell: no pieces
        if (rc == 1 || rc == 3) { err = 3; where = VD_STAGE_CELL; continue; }  // the site lies in the box
        if (rc == 2) continue;                           // too large: carve per simplex
        npl = compact_planes(S, npl, nc);
        // Alg. 5's interior sites.  whole == 1: a cell that meets no boundary
        // triangle lies inside M or outside it as a whole (it contains v_i,
        // which is in M; a power cell is judged by the mean of its corners).
        // whole == 2 (a convex M holding every site): a cell whose corners all
        // lie in M lies in M.  Such a cell is one piece, cut by no tetrahedron.
        if (C.whole && nbseed == 0 && (!CORNERS || cell_in_domain(S, D, X, nc))) {
          bool inside = true;
          if (POW) {
            double c0 = 0, c1 = 0, c2 = 0;
            for (int x = l; x < nc; x += 64) { c0 += S.cy[x][0]; c1 += S.cy[x][1]; c2 += S.cy[x][2]; }
            c0 = wave_sum(c0) / nc; c1 = wave_sum(c1) / nc; c2 = wave_sum(c2) / nc;
            inside = locate_wave(D, X.vx + c0, X.vy + c1, X.vz + c2) >= 0;
          }
          head = nt;  // no tetrahedron to visit
          if (!inside) continue;
          // fall through: the moments and the emission of the piece (a = -1)
        } else {
          if (npl <= VD_F_MAX && npl + 4 <= VD_P_MAX && nc <= VD_CB_MAX) {
            saved_lds = npl <= kLF && nc <= kLC;
            if (saved_lds) save_cell_lds(S, npl, nc);
            else save_cell(S, C, npl, nc);
            npl0 = npl;
            nc0 = nc;
            saved = true;
            {
              const uint64_t cp = __ballot(l < npl && S.plab[l] >= 0);
              if (l == 0) S.cellpos = cp;
            }
            cell_lab = l < npl ? S.plab[l] : 0;
            if (POW) {
              // a power cell need not contain its site: seed the tetrahedron
              // holding the mean of the cell's corners (a point of the cell);
              // parts of the cell that reach the boundary of M are seeded from
              // the boundary surface
              double c0 = 0, c1 = 0, c2 = 0;
              for (int x = l; x < nc; x += 64) { c0 += S.cy[x][0]; c1 += S.cy[x][1]; c2 += S.cy[x][2]; }
              c0 = wave_sum(c0) / nc; c1 = wave_sum(c1) / nc; c2 = wave_sum(c2) / nc;
              const int t = locate_wave(D, X.vx + c0, X.vy + c1, X.vz + c2);
              if (t >= 0 && !tq_push(S, C, nt, t)) { err = 2; where = VD_STAGE_SIMPLICES; }
            }
          }
          continue;
        }
      }
      if (rc == 1) empty = true;
      else if (rc) { err = rc; where = VD_STAGE_PIECE_CARVE; }
    }
    if (err) break;
    if (empty) continue;
    // ---- moments of the piece: fan of tetrahedra (o, foot of plane x seen
    // from o, corner, next corner) with the apex o at corner 0, so that the
    // volume's rounding error scales with the piece and not with its distance
    // to v_i (a tip of the cell in a far tetrahedron keeps a positive volume)
    double pv = 0, pmx = 0, pmy = 0, pmz = 0, pe = 0;
    double dm = 0, dmx = 0, dmy = 0, dmz = 0, de = 0;  // density-weighted (DENS)
    uint64_t fmask = 0;
    const double o0 = S.cy[0][0], o1 = S.cy[0][1], o2 = S.cy[0][2];
    const double oo = o0 * o0 + o1 * o1 + o2 * o2;
#pragma unroll 1
    for (int h = 0; h < 2; h++) {
      const int s = l + 64 * h;
      if (s >= nc) continue;
      const int pl = S.cpl[s], nb = S.cnb[s];
      const double Y0 = S.cy[s][0], Y1 = S.cy[s][1], Y2 = S.cy[s][2];
      const double y0 = Y0 - o0, y1 = Y1 - o1, y2 = Y2 - o2;
      const double YY = Y0 * Y0 + Y1 * Y1 + Y2 * Y2;
      fmask |= (1ull << p8(pl, 0)) | (1ull << p8(pl, 1)) | (1ull << p8(pl, 2));
      // plane p8(pl,e) continues around its face to the corner across edge (e+2)%3
#pragma unroll 1
      for (int e = 0; e < 3; e++) {
        const int x = p8(pl, e);
        const int nx_ = p8(nb, (e + 2) % 3);
        const double n0 = S.pn[x][0], n1 = S.pn[x][1], n2 = S.pn[x][2], cc = S.pn[x][3];
        const double f = (cc - (n0 * o0 + n1 * o1 + n2 * o2)) / (n0 * n0 + n1 * n1 + n2 * n2);
        const double r0 = n0 * f, r1 = n1 * f, r2 = n2 * f;
        const double Z0 = S.cy[nx_][0], Z1 = S.cy[nx_][1], Z2 = S.cy[nx_][2];
        const double z0 = Z0 - o0, z1 = Z1 - o1, z2 = Z2 - o2;
        const double det = r0 * (y1 * z2 - y2 * z1) - r1 * (y0 * z2 - y2 * z0) + r2 * (y0 * z1 - y1 * z0);
        const double vol = det / 6.0;
        // the tetrahedron's corners relative to v_i: o, o + r, Y, Z
        const double R0 = o0 + r0, R1 = o1 + r1, R2 = o2 + r2;
        const double s0 = o0 + R0 + Y0 + Z0, s1 = o1 + R1 + Y1 + Z1, s2 = o2 + R2 + Y2 + Z2;
        pv += vol;
        pmx += vol * s0 * 0.25; pmy += vol * s1 * 0.25; pmz += vol * s2 * 0.25;
        pe += vol * (1.0 / 20.0) *
              (oo + R0 * R0 + R1 * R1 + R2 * R2 + YY + Z0 * Z0 + Z1 * Z1 + Z2 * Z2 + s0 * s0 + s1 * s1 + s2 * s2);
        if (DENS) {
          const double V0[3] = {o0, o1, o2}, V1[3] = {R0, R1, R2}, V2[3] = {Y0, Y1, Y2}, V3[3] = {Z0, Z1, Z2};
          tet_density_moments(C.dens, X.vx, X.vy, X.vz, V0, V1, V2, V3, vol, dm, dmx, dmy, dmz, de);
        }
      }
    }
    pv = wave_sum(pv); pmx = wave_sum(pmx); pmy = wave_sum(pmy); pmz = wave_sum(pmz); pe = wave_sum(pe);
    fmask = wave_or64(fmask);
    // a piece exists when its volume is positive; with a density its moments
    // are the weighted ones
    if (!(pv > 0.0)) continue;
    if (DENS) {
      pv = wave_sum(dm); pmx = wave_sum(dmx); pmy = wave_sum(dmy); pmz = wave_sum(dmz); pe = wave_sum(de);
    }
    if (l == 0) { S.acc[0] += pv; S.acc[1] += pmx; S.acc[2] += pmy; S.acc[3] += pmz; S.acc[4] += pe; }
    if (MON) count_add(S.ar.fantets, 3 * nc);
    // ---- emit the piece ----
    const int nface = __popcll(fmask);
    const long long pidx = arena_take(S.ar, C, AR_PIECE, 1);
    long long fo = 0, vo = 0;
    if (C.emit) {
      fo = arena_take(S.ar, C, AR_FACE, nface);
      vo = arena_take(S.ar, C, AR_VERT, nc);
    }
    if (C.want_grad) face_moments<DENS>(S, nc, npl, fmask, C, G, X, pidx);
    // a record that does not fit its arena is dropped and counted; the per-site
    // counts below only count what was written, so the CSR built from them
    // stays inside the arenas (the clip then reports VD_ERR_CAPACITY)
    const bool fits_fv = C.emit && fo + nface <= C.cap_face && vo + nc <= C.cap_vert;
    if (pidx < C.cap_piece) {
      if (l == 0) {
        GL(C.piece_site)[pidx] = orig;
        GL(C.piece_simplex)[pidx] = a;
        GL(C.piece_nface)[pidx] = nface;
        GL(C.piece_nvert)[pidx] = nc;
        GL(C.piece_mass)[pidx] = pv;
        GL(C.piece_mom)[3 * pidx + 0] = pmx + pv * X.vx;
        GL(C.piece_mom)[3 * pidx + 1] = pmy + pv * X.vy;
        GL(C.piece_mom)[3 * pidx + 2] = pmz + pv * X.vz;
        GL(C.piece_energy)[pidx] = pe;
        GL(C.piece_fstart)[pidx] = fits_fv ? fo : -1;
        GL(C.piece_vstart)[pidx] = fits_fv ? vo : -1;
        S.ar.pieces++;
        if (fits_fv) { S.ar.faces += nface; S.ar.verts += nc; }
        if (C.emit && !fits_fv) S.ar.dropped++;
      }
      npieces++;
      if (fits_fv) {
        // caller-index flag of plane l, read once; corners fetch theirs from the plane's lane
        const int lab = l < npl && ((fmask >> l) & 1ull) ? convert_label(G, S.plab[l]) : 0;
        if (l < npl && ((fmask >> l) & 1ull)) GL(C.face_label)[fo + __popcll(fmask & low_mask(l))] = lab;
        for (int h = 0; h < 2; h++) {
          if (64 * h >= nc) break;
          const int s = l + 64 * h;
          const int pl = s < nc ? S.cpl[s] : 0;
          const int l0 = __shfl(lab, p8(pl, 0), 64), l1 = __shfl(lab, p8(pl, 1), 64), l2 = __shfl(lab, p8(pl, 2), 64);
          if (s < nc) {
            GL(C.vert_xyz)[3 * (vo + s) + 0] = S.cy[s][0] + X.vx;
            GL(C.vert_xyz)[3 * (vo + s) + 1] = S.cy[s][1] + X.vy;
            GL(C.vert_xyz)[3 * (vo + s) + 2] = S.cy[s][2] + X.vz;
            GL(C.vert_label)[3 * (vo + s) + 0] = l0;
            GL(C.vert_label)[3 * (vo + s) + 1] = l1;
            GL(C.vert_label)[3 * (vo + s) + 2] = l2;
          }
        }
      }
    } else if (l == 0) {
      S.ar.dropped++;
    }
    // ---- propagate: neighbours (positive flags), tetrahedra (negative flags) ----
    // A piece cut from the saved cell adds its cell planes to the mask; only
    // the four planes of T_a can lead to other tetrahedra.
    const bool from_cell = saved && !need_carve;
    if (from_cell && l == 0) S.nbmask |= fmask & S.cellpos;
    for (uint64_t m = from_cell ? fmask & (15ull << npl0) : fmask; m; m &= m - 1) {
      const int x = __ffsll((unsigned long long)m) - 1;
      const int lab = uni(S.plab[x]);
      if (lab >= 0) {
        if (!nb_push(S, C, nnb, lab)) { err = 2; where = VD_STAGE_NEIGHBOURS; break; }
      } else if (a >= 0 && lab > VD_BND_BASE + 3) {  // a whole cell (a = -1) has no tetrahedron planes
        if (!tq_push(S, C, nt, -lab - 1)) { err = 2; where = VD_STAGE_SIMPLICES; break; }
      }
    }
    __syncthreads();
  }
  // neighbours of the pieces cut from the saved cell
  __syncthreads();
  for (uint64_t m = S.nbmask; m && !err; m &= m - 1) {
    const int lab = __builtin_amdgcn_readlane(cell_lab, __ffsll((unsigned long long)m) - 1);
    if (!nb_push(S, C, nnb, lab)) { err = 2; where = VD_STAGE_NEIGHBOURS; break; }
  }
  // ---- per-site results ----
  const long long ns0 = arena_take(S.ar, C, AR_NBR, nnb);
  if (l == 0) {
    const double Mv = S.acc[0];
    GL(C.mass)[orig] = Mv;
    GL(C.mom)[3 * (long long)orig + 0] = S.acc[1] + Mv * X.vx;
    GL(C.mom)[3 * (long long)orig + 1] = S.acc[2] + Mv * X.vy;
    GL(C.mom)[3 * (long long)orig + 2] = S.acc[3] + Mv * X.vz;
    GL(C.energy)[orig] = S.acc[4];
    const bool nfit = ns0 + nnb <= C.cap_nbr;
    GL(C.pcount)[orig] = npieces;
    GL(C.ncount)[orig] = nfit ? nnb : 0;
    GL(C.nstart)[orig] = ns0;
    if (nfit) S.ar.nbrs += nnb;
    else S.ar.dropped++;
    S.ar.queries += st.queries;
    S.ar.cands += st.cands;
    S.ar.clips += st.clips;
    S.ar.gridq += st.grid;
    if (err) {
      atomicAdd(&C.cnt[err == 2 ? CNT_ERR_CAP : (err == 4 ? CNT_ERR_LOC : CNT_ERR_DEG)], 1ull);
      atomicMin((int *)&C.cnt[CNT_BAD_SITE], orig);
      if (where) atomicOr((unsigned long long *)&C.cnt[CNT_STAGES], 1ull << where);
    }
  }
  __syncthreads();
  if (ns0 + nnb <= C.cap_nbr) {
    // neighbours in ascending caller index: rank sort (up to 64 from the
    // lanes' registers, more from memory)
    if (nnb <= 64) {
      const int me = l < nnb ? GL(G.perm)[S.nbl[l]] : 0;
      int rk = 0;
      for (int o = 0; o < nnb; o++) rk += (__builtin_amdgcn_readlane(me, o) < me) ? 1 : 0;
      if (l < nnb) GL(C.nbr_arena)[ns0 + rk] = me;
    } else {
      for (int e = l; e < nnb; e += 64) {
        const int me = GL(G.perm)[nb_get(S, C, e)];
        int rk = 0;
        for (int o = 0; o < nnb; o++) rk += (GL(G.perm)[nb_get(S, C, o)] < me) ? 1 : 0;
        GL(C.nbr_arena)[ns0 + rk] = me;
      }
    }
  }
  __syncthreads();
}

// Persistent: every workgroup (one wave) takes sites from the queues until
// all are done.  Three waves per SIMD: 168 VGPRs (a few values spill around
// the carve) and 12.8 KB of LDS per wave (the carved cell is kept over the
// site cache when it fits, else in a global buffer); the third wave hides
// more LDS and memory latency than that costs.
// MON: the work counters and margin tracking of vd_options.monitor; DENS: the
// density-weighted moments of vd_options.use_density; POW: power diagrams;
// CORNERS: the interior split by the cells' corners (whole_interior on a
// convex domain).  Each is compiled in only for the instances that use it, so
// the default instance carries none of them.
template <bool MON, bool DENS, bool POW, bool CORNERS>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 3))) site_kernel(GridView G, DomainView D, const CellsDev *__restrict__ Cp) {
  __shared__ WaveLds S;
  const CellsDev &C = *Cp;
  arena_init(S.ar);
  for (;;) {
    const int si = queue_next(S.ar, C, G.n);
    if (si < 0) break;
    // the site's own diagram (a batch) or the only one; one call site keeps
    // the per-site code inlined once
    const int b = G.nb > 1 ? diagram_of(G.site_off, G.nb, si) : 0;
    do_site<MON, DENS, POW, CORNERS>(S, G.views[b], D.views[b], C, si);
  }
  arena_close(S.ar, C);
}

struct QueueStarts {
  long long off[VD_QUEUES];
  int given;
};
__global__ void queue_init(int *q, long long n, QueueStarts qs) {
  const int k = threadIdx.x;
  const long long q8 = (n + VD_QUEUES - 1) / VD_QUEUES;
  if (k < VD_QUEUES) q[k * VD_QSTRIDE] = (int)(qs.given ? qs.off[k] : (k * q8 < n ? k * q8 : n));
}

int resident_workgroups() {
  static int cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int &w = cache[dev];
  if (!w) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, site_kernel<false, false, false, false>, 64, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
    w = per_cu * ncu;
  }
  return w;
}

}  // namespace

int vd_sites3d_workgroups(long long n) {
  const int w = resident_workgroups();
  return (int)(n < w ? (n > 0 ? n : 1) : w);
}

// qoff: the first position of each queue in the batch's work order, or NULL
void vd_launch_queue_init(int *queue, long long n, const long long *qoff, hipStream_t st) {
  QueueStarts qs{};
  qs.given = qoff ? 1 : 0;
  if (qoff)
    for (int k = 0; k < VD_QUEUES; k++) qs.off[k] = qoff[k];
  hipLaunchKernelGGL(queue_init, dim3(1), dim3(64), 0, st, queue, n, qs);
}

void vd_launch_sites3d(const GridView &G, const DomainView &D, const CellsDev *Cdev, int workgroups, bool monitor,
                       bool density, bool power, bool corners, hipStream_t st) {
  const dim3 grid(workgroups), block(64);
  if (power) {  // power diagrams: no density, interior split by the boundary diagram
    if (monitor) hipLaunchKernelGGL((site_kernel<true, false, true, false>), grid, block, 0, st, G, D, Cdev);
    else hipLaunchKernelGGL((site_kernel<false, false, true, false>), grid, block, 0, st, G, D, Cdev);
  } else if (corners) {
    if (monitor && density) hipLaunchKernelGGL((site_kernel<true, true, false, true>), grid, block, 0, st, G, D, Cdev);
    else if (monitor) hipLaunchKernelGGL((site_kernel<true, false, false, true>), grid, block, 0, st, G, D, Cdev);
    else if (density) hipLaunchKernelGGL((site_kernel<false, true, false, true>), grid, block, 0, st, G, D, Cdev);
    else hipLaunchKernelGGL((site_kernel<false, false, false, true>), grid, block, 0, st, G, D, Cdev);
  } else if (monitor && density) {
    hipLaunchKernelGGL((site_kernel<true, true, false, false>), grid, block, 0, st, G, D, Cdev);
  } else if (monitor) {
    hipLaunchKernelGGL((site_kernel<true, false, false, false>), grid, block, 0, st, G, D, Cdev);
  } else if (density) {
    hipLaunchKernelGGL((site_kernel<false, true, false, false>), grid, block, 0, st, G, D, Cdev);
  } else {
    hipLaunchKernelGGL((site_kernel<false, false, false, false>), grid, block, 0, st, G, D, Cdev);
  }
}
