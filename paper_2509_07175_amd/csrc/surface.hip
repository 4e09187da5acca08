// surface.hip -- restricted Voronoi diagram on a triangle mesh (Alg. 4).
//
// One wavefront per triangle T_a.  The first site is the nearest site of the
// triangle's centroid; further sites come from the positive edge flags of the
// pieces already carved (the propagation of Alg. 4, kept inside the wave:
// the triangle's site list lives in LDS, so no global pair lists or atomic
// labels are needed).  Each piece T_a cap Omega_i is a convex polygon in the
// plane of T_a, carved by point-in-cell tests (Sec. 4.1) and the edge-based
// bisector search (Sec. 4.2) along straddling polygon edges (Alg. 1) or the
// virtual edge from v_i (Alg. 3, v_i is generally off the plane), removing
// only the run of outside vertices that contains the chosen one (the 2D
// form of R_p, Sec. 6.3).
//
// Polygon layout in LDS: lane t owns vertex t (up to 64); vertex t lies on the
// supporting plane and on the planes of the edges t-1 -> t and t -> t+1.
// The nearest-site queries of a triangle's pieces go to an LDS cache of the
// sites around its centroid (the 3D kernel's cache, with its exact witness
// and coverage tests), and to the grid when the cache cannot decide.
// Per-site sums (mass, centroid, energy, neighbours) are formed afterwards
// from the pieces in a fixed order (site_reduce), so results do not depend on
// the order in which waves finish.
#include "vd_arena.h"

namespace {

constexpr int kSP = 64;        // planes of one polygon
constexpr int kSV = 64;        // vertices of one polygon (one per lane)
constexpr int kSS = 128;       // sites of one triangle held in LDS (more spill to global memory)
constexpr int kMaxIters = 4096;

struct __align__(16) TriLds {
  double pn[kSP][4];  // slot 0 supporting plane, 1..3 triangle edges, then bisectors
  double vy[kSV][3];  // vertex coordinates relative to the current site
  int plab[kSP];
  int ve[kSV];        // plane slot of the edge from vertex t to vertex t+1
  int vst[kSV];       // bit 0 inside, bit 1 tested, bits 8.. nearest site + 1
  int sq[kSS];        // first sites of this triangle (sorted positions), breadth-first
  int sqf[kSS];       // the site whose piece's edge flag listed each of them (-1: the seed) ...
  int sqf2[kSS];      // ... and a second one that flagged it before its turn (-1: none)
  WaveArena ar;       // output chunks, queue position, statistics
  SiteCache K;        // sites around the triangle's centroid for the nearest-site queries
};
static_assert(offsetof(TriLds, vy) == offsetof(TriLds, pn) + sizeof(double) * kSP * 4 &&
                  kSP * 4 + kSV * 3 >= VD_CACHE_SCRATCH,
              "the polygon arrays double as the site cache's fill scratch");

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t lowm(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1ull); }

struct SStats {
  long long queries = 0, cands = 0, clips = 0;
};

// vertex of the supporting plane and two planes (Cramer, planes in flag order)
__device__ __forceinline__ void solve_s(const TriLds &S, int a, int b, double *y) {
  int q[3] = {0, a, b};
  if (S.plab[q[2]] < S.plab[q[1]]) { int t = q[1]; q[1] = q[2]; q[2] = t; }
  const double *n0 = S.pn[q[0]], *n1 = S.pn[q[1]], *n2 = S.pn[q[2]];
  const double c12[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2], n1[0] * n2[1] - n1[1] * n2[0]};
  const double c20[3] = {n2[1] * n0[2] - n2[2] * n0[1], n2[2] * n0[0] - n2[0] * n0[2], n2[0] * n0[1] - n2[1] * n0[0]};
  const double c01[3] = {n0[1] * n1[2] - n0[2] * n1[1], n0[2] * n1[0] - n0[0] * n1[2], n0[0] * n1[1] - n0[1] * n1[0]};
  const double det = n0[0] * c12[0] + n0[1] * c12[1] + n0[2] * c12[2];
  const double id = 1.0 / det;
  for (int k = 0; k < 3; k++) y[k] = (n0[3] * c12[k] + n1[3] * c20[k] + n2[3] * c01[k]) * id;
}

// P <- T_a relative to site v (slot 0 = supporting plane)
__device__ void init_tri(TriLds &S, const DomainView &D, int a, double vx, double vy, double vz) {
  const int l = vd_lane();
  const auto tv = &GL(D.simp)[(long long)a * 3];
  const auto p0 = &GL(D.verts)[3 * (long long)tv[0]], p1 = &GL(D.verts)[3 * (long long)tv[1]],
               p2 = &GL(D.verts)[3 * (long long)tv[2]];
  const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  if (l == 0) {
    S.pn[0][0] = N[0]; S.pn[0][1] = N[1]; S.pn[0][2] = N[2];
    S.pn[0][3] = N[0] * (p0[0] - vx) + N[1] * (p0[1] - vy) + N[2] * (p0[2] - vz);
    S.plab[0] = 2147483647;
  }
  if (l >= 1 && l <= 3) {
    const int e = l - 1;  // edge opposite vertex e: from q_{e+1} to q_{e+2}
    const auto A = &GL(D.verts)[3 * (long long)tv[(e + 1) % 3]], B = &GL(D.verts)[3 * (long long)tv[(e + 2) % 3]];
    const double d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double n[3] = {d[1] * N[2] - d[2] * N[1], d[2] * N[0] - d[0] * N[2], d[0] * N[1] - d[1] * N[0]};
    S.pn[l][0] = n[0]; S.pn[l][1] = n[1]; S.pn[l][2] = n[2];
    S.pn[l][3] = n[0] * (A[0] - vx) + n[1] * (A[1] - vy) + n[2] * (A[2] - vz);
    const int b = GL(D.adj)[(long long)a * 3 + e];
    S.plab[l] = b >= 0 ? -(b + 1) : VD_BND_BASE + e;
  }
  if (l < 3) {
    const auto p = &GL(D.verts)[3 * (long long)tv[l]];
    S.vy[l][0] = p[0] - vx; S.vy[l][1] = p[1] - vy; S.vy[l][2] = p[2] - vz;
    S.ve[l] = 1 + (l + 2) % 3;  // edge from q_l to q_{l+1} is opposite q_{l+2}
    S.vst[l] = 0;
  }
  __syncthreads();
}

// Drop planes no edge references (slot 0 stays).  Returns the new count.
__device__ int compact_s(TriLds &S, int npl, int nv) {
  const int l = vd_lane();
  uint64_t used = 1ull;
  if (l < nv) used |= 1ull << S.ve[l];
  used = wave_or64(used);
  double pv[4] = {0, 0, 0, 0};
  int lab = 0;
  const bool mine = l < npl && ((used >> l) & 1ull);
  if (mine) { for (int k = 0; k < 4; k++) pv[k] = S.pn[l][k]; lab = S.plab[l]; }
  const int e = l < nv ? S.ve[l] : 0;
  __syncthreads();
  if (mine) {
    const int ni = __popcll(used & lowm(l));
    for (int k = 0; k < 4; k++) S.pn[ni][k] = pv[k];
    S.plab[ni] = lab;
  }
  if (l < nv) S.ve[l] = __popcll(used & lowm(e));
  __syncthreads();
  return __popcll(used);
}

// Clip the polygon by plane slot P, removing the run of consecutive outside
// vertices that contains vertex pt (pt < 0: the farthest outside vertex).
// Returns 0 unchanged, 1 empty, 2 capacity, 3 degenerate, 4 cut.
__device__ int clip_s(TriLds &S, bool mon, int P, int pt, int &nv) {
  const int l = vd_lane();
  const double nx = S.pn[P][0], ny = S.pn[P][1], nz = S.pn[P][2], c = S.pn[P][3];
  double y0 = 0, y1 = 0, y2 = 0, sd = -1.0;
  int e = 0, st = 0;
  const bool v = l < nv;
  if (v) {
    y0 = S.vy[l][0]; y1 = S.vy[l][1]; y2 = S.vy[l][2];
    e = S.ve[l]; st = S.vst[l];
    sd = nx * y0 + ny * y1 + nz * y2 - c;
  }
  if (mon) {
    margin_track(S.ar, v, sd, fabs(nx * y0) + fabs(ny * y1) + fabs(nz * y2) + fabs(c), false, 0.0, 1.0);
    count_add(S.ar.classified, nv);
  }
  const uint64_t O = __ballot(v && sd > 0.0);
  if (!O) return pt < 0 ? 0 : 3;
  if (pt < 0) {
    double b = -sd;
    int bi = l;
    group_argmin(b, bi, 64);
    pt = uni(bi);
  } else if (!((O >> pt) & 1ull)) {
    return 3;
  }
  // the run [a, b] of outside vertices around pt (cyclic)
  int a = pt, b = pt, len = 1;
  while (len < nv && ((O >> ((a + nv - 1) % nv)) & 1ull)) { a = (a + nv - 1) % nv; len++; }
  while (len < nv && ((O >> ((b + 1) % nv)) & 1ull)) { b = (b + 1) % nv; len++; }
  if (len >= nv) return 1;
  const int keep = nv - len;
  if (keep + 2 > kSV) return 2;
  const int am1 = (a + nv - 1) % nv;
  const int eA = uni(S.ve[am1]), eB = uni(S.ve[b]);
  __syncthreads();
  // kept vertex t moves to (t - b - 1) mod nv; new vertices at keep, keep+1
  const int k = (l - b - 1 + 2 * nv) % nv;
  const bool kept = v && k < keep;
  if (kept) {
    S.vy[k][0] = y0; S.vy[k][1] = y1; S.vy[k][2] = y2;
    S.ve[k] = e;
    S.vst[k] = st;
  }
  __syncthreads();
  if (l == 0 || l == 1) {
    double yy[3];
    if (l == 0) solve_s(S, eA, P, yy); else solve_s(S, P, eB, yy);
    const int t = keep + l;
    S.vy[t][0] = yy[0]; S.vy[t][1] = yy[1]; S.vy[t][2] = yy[2];
    S.ve[t] = l == 0 ? P : eB;
    S.vst[t] = 0;
  }
  __syncthreads();
  nv = keep + 2;
  if (mon) count_add(S.ar.newc, 2);
  return 4;
}

struct SParams {
  int improved, straddle, max_iters;
  bool monitor;  // count work and track predicate margins
};

// Carve the polygon until every vertex is certified inside Omega_i (TEST /
// LAMBDA / SEARCH queries as in the 3D kernel).  Returns 0, 1 empty, 2, 3.
// POW: power diagram, as in the 3D kernel: the lifted site (v_i, h_i) starts
// the virtual search edges, polygon vertices lie on the hyperplane (4th
// coordinate 0) and the clip plane is the power plane.
template <bool POW>
__device__ int carve_s(TriLds &S, const GridView &G, const SParams C, int si, double vx, double vy, double vz,
                       double delta, int &npl, int &nv, SStats &ss) {
  enum { PICK = 0, TEST, LAMBDA, SEARCH };
  const int l = vd_lane();
  const int grp = l >> 4;
  int mode = PICK;
  int pt = -1, j = -1, ef0 = -2, lam = 2, nstep = 0, tslot = -1, nbatch = 0;
  double A0 = 0, A1 = 0, A2 = 0, g0 = 0, g1 = 0, g2 = 0, u0 = 0, u1 = 0, u2 = 0, L = 0;
  double n0 = 0, n1 = 0, n2 = 0, nc3 = 0, q0 = 0, q1 = 0, q2 = 0;
  const double hi_ = POW ? GL(G.sh)[si] : 0.0, wi_ = POW ? GL(G.sw)[si] : 0.0;
  double A4 = 0, g4 = 0, q4 = 0;  // POW: 4th coordinates
  auto bisector_point = [&]() {
    n0 = GL(G.sx)[j] - vx; n1 = GL(G.sy)[j] - vy; n2 = GL(G.sz)[j] - vz;
    const double e0 = g0 - A0, e1 = g1 - A1, e2 = g2 - A2;
    double den, num;
    if (POW) {
      const double n4 = GL(G.sh)[j] - hi_, e4 = g4 - A4;
      den = n0 * e0 + n1 * e1 + n2 * e2 + n4 * e4;
      num = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2 + n4 * n4) - (n0 * A0 + n1 * A1 + n2 * A2 + n4 * (A4 - hi_));
      nc3 = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2 + wi_ - GL(G.sw)[j]);
    } else {
      nc3 = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2);
      den = n0 * e0 + n1 * e1 + n2 * e2;
      num = nc3 - (n0 * A0 + n1 * A1 + n2 * A2);
    }
    double t = den > 0.0 ? num / den : 1.0;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    q0 = A0 + t * e0; q1 = A1 + t * e1; q2 = A2 + t * e2;
    if (POW) q4 = A4 + t * (g4 - A4);
  };
  for (int it = 0; it < kMaxIters; it++) {
    if (mode == PICK) {
      const int vs = l < nv ? S.vst[l] : 0;
      const uint64_t T = __ballot(vs & 2), I = __ballot(vs & 1);
      const uint64_t O = T & ~I;
      if (!O) {
        const uint64_t U = lowm(nv) & ~T;
        if (!U) return 0;
        tslot = -1;
        nbatch = 0;
        uint64_t m = U;
        while (m && nbatch < 4) {
          const int b = __ffsll((unsigned long long)m) - 1;
          if (nbatch == grp) tslot = b;
          nbatch++;
          m &= m - 1;
        }
        const int s = tslot >= 0 ? tslot : __ffsll((unsigned long long)U) - 1;
        q0 = S.vy[s][0]; q1 = S.vy[s][1]; q2 = S.vy[s][2];
        mode = TEST;
      } else {
        pt = -1;
        int ps = -1, edge = -1;
        if (C.straddle) {
          // outside vertex with an inside neighbour along the polygon
          const bool out = (O >> l) & 1ull;
          const int prv = (l + nv - 1) % (nv > 0 ? nv : 1), nxt = (l + 1) % (nv > 0 ? nv : 1);
          const bool cand = out && (((I >> prv) & 1ull) || ((I >> nxt) & 1ull));
          const uint64_t Cm = __ballot(cand);
          if (Cm) {
            pt = __ffsll((unsigned long long)Cm) - 1;
            const int pp = (pt + nv - 1) % nv, pn_ = (pt + 1) % nv;
            if ((I >> pp) & 1ull) { ps = pp; edge = pp; } else { ps = pn_; edge = pt; }
          }
        }
        if (pt < 0) pt = __ffsll((unsigned long long)O) - 1;
        A0 = A1 = A2 = 0;
        A4 = ps >= 0 ? 0.0 : hi_;
        g4 = 0.0;
        if (ps >= 0) { A0 = S.vy[ps][0]; A1 = S.vy[ps][1]; A2 = S.vy[ps][2]; }
        g0 = S.vy[pt][0]; g1 = S.vy[pt][1]; g2 = S.vy[pt][2];
        j = uni((S.vst[pt] >> 8) - 1);
        if (j < 0 || j == si) return 3;
        ef0 = -2;
        if (edge >= 0) {
          const int lab = uni(S.plab[uni(S.ve[edge])]);
          ef0 = lab >= 0 ? lab : -2;
        }
        nstep = 0;
        const double d0 = g0 - A0, d1 = g1 - A1, d2 = g2 - A2;
        L = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (C.improved && L > 0 && 2.0 * delta < L) {
          u0 = d0 / L; u1 = d1 / L; u2 = d2 / L;
          lam = 2;
          q0 = A0 + 2.0 * delta * u0; q1 = A1 + 2.0 * delta * u1; q2 = A2 + 2.0 * delta * u2;
          mode = LAMBDA;
        } else {
          bisector_point();
          mode = SEARCH;
        }
      }
    }
    const int gs = mode == TEST ? 16 : 64;
    const double qx = vx + q0, qy = vy + q1, qz = vz + q2;
    const double dx = qx - vx, dy = qy - vy, dz = qz - vz;
    if (C.monitor) count_add(S.ar.rounds, 1);
    int kq;
    if (POW) {
      const double qw = mode == SEARCH ? q4 : 0.0, dw = qw - hi_;
      kq = nn_query<true>(G, gs, qx, qy, qz, dx * dx + dy * dy + dz * dz + dw * dw, si, ss.cands, qw);
    } else {
      // sites the test treats like v_i: the flags of the vertex's two edges
      // (TEST), the edge's flag (LAMBDA), and the candidate (SEARCH)
      int e0 = ef0, e1 = -1, e2 = mode == SEARCH ? j : -1;
      if (mode == TEST) {
        const int ts = tslot >= 0 ? tslot : 0;
        e0 = S.plab[S.ve[(ts + nv - 1) % nv]];
        e1 = S.plab[S.ve[ts]];
      }
      bool on_grid;
      kq = nn_cached(S.K, G, gs, qx, qy, qz, dx * dx + dy * dy + dz * dz, si, e0 < 0 ? -1 : e0, e1 < 0 ? -1 : e1,
                     e2 < 0 ? -1 : e2, -1, -1, -1, ss.cands, on_grid);
    }
    if (mode == TEST) {
      ss.queries += nbatch;
      bool in = false;
      if (tslot >= 0) {
        const int prv = (tslot + nv - 1) % nv;
        in = (kq == si) || (kq == S.plab[S.ve[prv]]) || (kq == S.plab[S.ve[tslot]]);
      }
      __syncthreads();
      if (tslot >= 0 && (l & 15) == 0) S.vst[tslot] = (in ? 1 : 0) | 2 | ((kq + 1) << 8);
      __syncthreads();
      mode = PICK;
      continue;
    }
    ss.queries++;
    const int k = uni(kq);
    if (mode == LAMBDA) {
      if (k != si && k != ef0) {
        j = k; g0 = q0; g1 = q1; g2 = q2;
      } else {
        lam++;
        if (lam < 2 + C.max_iters && lam * delta < L) {
          const double tt = lam * delta;
          q0 = A0 + tt * u0; q1 = A1 + tt * u1; q2 = A2 + tt * u2;
          continue;
        }
      }
      bisector_point();
      mode = SEARCH;
      continue;
    }
    if (!(k == si || k == j || k == ef0)) {
      if (++nstep >= C.max_iters) return 3;
      j = k;
      g0 = q0; g1 = q1; g2 = q2;
      g4 = q4;
      bisector_point();
      continue;
    }
    if (npl >= kSP) {
      npl = compact_s(S, npl, nv);
      if (npl >= kSP) return 2;
    }
    const int P = npl++;
    __syncthreads();
    if (l == 0) {
      S.pn[P][0] = n0; S.pn[P][1] = n1; S.pn[P][2] = n2; S.pn[P][3] = nc3;
      S.plab[P] = j;
    }
    __syncthreads();
    const int rc = clip_s(S, C.monitor, P, pt, nv);
    ss.clips++;
    if (rc == 1) return 1;
    if (rc != 4) return rc == 0 ? 3 : rc;
    mode = PICK;
  }
  return 3;
}

__device__ __forceinline__ int conv(const GridView &G, int lab) { return lab >= 0 ? GL(G.perm)[lab] : lab; }

// The triangle's site list: entries below kSS in LDS, the rest in this wave's
// part of the global overflow buffer (C.sq_cap entries; a clip that runs out
// reports VD_STAGE_TRIANGLE_SITES and is re-run with a larger buffer).
__device__ __forceinline__ int sq_get(const TriLds &S, const CellsDev &C, int e) {
  return e < kSS ? S.sq[e] : GL(C.sq_spill)[(long long)blockIdx.x * C.sq_cap + (e - kSS)];
}

// Is site j in the list?  (The whole wave scans; the answer is wave-uniform.)
// Position of site j in the list, or -1.  (The whole wave scans; the answer
// is wave-uniform.)
__device__ __forceinline__ int sq_find(const TriLds &S, const CellsDev &C, int nsq, int j) {
  for (int e0 = 0; e0 < nsq; e0 += 64) {
    const int e = e0 + vd_lane();
    const uint64_t m = __ballot(e < nsq && sq_get(S, C, e) == j);
    if (m) return e0 + __ffsll((unsigned long long)m) - 1;
  }
  return -1;
}

// Append site j; false when the overflow buffer is full.
__device__ __forceinline__ bool sq_push(TriLds &S, const CellsDev &C, int &nsq, int j, int from) {
  if (nsq >= kSS + C.sq_cap) return false;
  __syncthreads();
  if (vd_lane() == 0) {
    if (nsq < kSS) {
      S.sq[nsq] = j;
      S.sqf[nsq] = from;
      S.sqf2[nsq] = -1;
    }
    else GL(C.sq_spill)[(long long)blockIdx.x * C.sq_cap + (nsq - kSS)] = j;
  }
  nsq++;
  __syncthreads();
  return true;
}

// Gabriel neighbours of site si among the first kGabrielS cache entries: the
// ball on the diameter [v_si, v_j] lies inside the cached region (every site
// that could be in it is cached) and holds no other site, so the midpoint of
// v_si v_j lies on the face of the cell of si towards v_j, and B(si, j) is a
// face plane, a valid clip.  Returns the mask of their cache slots (known
// bisectors `skip0`, `skip1` left out).
constexpr int kGabrielS = 16;
__device__ uint64_t gabriel_mask_s(const TriLds &S, int si, double vx, double vy, double vz, int skip0, int skip1) {
  const int l = vd_lane();
  const int n = S.K.cnt;
  const int T = n < kGabrielS ? n : kGabrielS;
  if (T <= 0) return 0ull;
  double ax = 0, ay = 0, az = 0, r2 = 0, mx = 0, my = 0, mz = 0;
  bool gab = false;
  double reach2 = 0.0;
  if (l < T) {
    const int pj = S.K.p[l];
    ax = S.K.x[l] - vx; ay = S.K.y[l] - vy; az = S.K.z[l] - vz;
    const double a2 = ax * ax + ay * ay + az * az;
    mx = vx + 0.5 * ax; my = vy + 0.5 * ay; mz = vz + 0.5 * az;
    r2 = 0.25 * a2;
    const double dx = mx - S.K.vx, dy = my - S.K.vy, dz = mz - S.K.vz;
    const double reach = (sqrt(dx * dx + dy * dy + dz * dz) + sqrt(r2)) * (1.0 + 1e-9);
    gab = pj != si && pj != skip0 && pj != skip1 && a2 > 0.0 && reach < S.K.rc;
    reach2 = gab ? reach * reach : 0.0;
  }
  if (!__ballot(gab)) return 0ull;
  // sites within reach of the centre lie below the first bucket beyond it
  const double lim = -wave_min(-reach2);
  int E = n;
  {
    const uint64_t a = __ballot(l < n && (double)S.K.kb[l] * S.K.step > lim);
    const uint64_t b = __ballot(l + 64 < n && (double)S.K.kb[l + 64] * S.K.step > lim);
    if (a) E = __ffsll((unsigned long long)a) - 1;
    else if (b) E = 64 + __ffsll((unsigned long long)b) - 1;
  }
  const double r2in = r2 * (1.0 + 1e-9);
  for (int k = 0; k < E; k++) {
    const double ex = S.K.x[k] - mx, ey = S.K.y[k] - my, ez = S.K.z[k] - mz;
    if (k != l && S.K.p[k] != si && ex * ex + ey * ey + ez * ez <= r2in) gab = false;
  }
  return __ballot(gab);
}

template <bool DENS, bool POW>
__device__ void do_triangle(TriLds &S, const GridView &G, const DomainView &D, const CellsDev &C, int a) {
  const int l = vd_lane();
  const SParams P = {C.improved, C.straddle, C.max_iters, C.monitor != 0};
  SStats ss;
  int err = 0;
  // seed: nearest site of the centroid (Alg. 4)
  int nsq = 0, head = 0;
  {
    const auto tv = &GL(D.simp)[(long long)a * 3];
    const auto p0 = &GL(D.verts)[3 * (long long)tv[0]], p1 = &GL(D.verts)[3 * (long long)tv[1]],
                 p2 = &GL(D.verts)[3 * (long long)tv[2]];
    const double cx = (p0[0] + p1[0] + p2[0]) / 3.0, cy = (p0[1] + p1[1] + p2[1]) / 3.0,
                 cz = (p0[2] + p1[2] + p2[2]) / 3.0;
    // the sites around the centroid, for the queries of every piece of T_a
    // (the polygon arrays are free until the first piece)
    if (!POW && C.cache) {
      cache_fill(S.K, G, cx, cy, cz, &S.pn[0][0]);
    } else {
      if (l == 0) S.K.cnt = -1;
      __syncthreads();
    }
    const int k = uni(nn_query<POW>(G, 64, cx, cy, cz, 1e300, -1, ss.cands, 0.0));
    ss.queries++;
    if (k >= 0) {
      if (l == 0) {
        S.sq[0] = k;
        S.sqf[0] = S.sqf2[0] = -1;
      }
      nsq = 1;
    } else {
      err = 3;
    }
  }
  __syncthreads();
  int where = VD_STAGE_TRIANGLE;
  while (head < nsq && !err) {
    const int si = uni(sq_get(S, C, head));
    const int from = head < kSS ? uni(S.sqf[head]) : -1, from2 = head < kSS ? uni(S.sqf2[head]) : -1;
    head++;
    const double vx = GL(G.sx)[si], vy = GL(G.sy)[si], vz = GL(G.sz)[si], delta = GL(G.delta)[si];
    init_tri(S, D, a, vx, vy, vz);
    int npl = 4, nv = 3;
    int rc = 0;
    // the pieces already carved in T_a that have an edge on a bisector with si
    // (the one that listed si, and one more that flagged it before its turn):
    // those bisectors bound this piece too, so clip by them before the carve
    // instead of finding them by tests and searches
    for (int f = 0; f < 2 && rc == 0; f++) {
      const int nb = f == 0 ? from : from2;
      if (nb < 0) continue;
      __syncthreads();
      if (l == 0) {
        const double n0 = GL(G.sx)[nb] - vx, n1 = GL(G.sy)[nb] - vy, n2 = GL(G.sz)[nb] - vz;
        S.pn[npl][0] = n0; S.pn[npl][1] = n1; S.pn[npl][2] = n2;
        S.pn[npl][3] = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2 + (POW ? GL(G.sw)[si] - GL(G.sw)[nb] : 0.0));
        S.plab[npl] = nb;
      }
      __syncthreads();
      rc = clip_s(S, C.monitor, npl, -1, nv);
      npl++;
      if (rc == 4) ss.clips++;
      if (rc == 4 || rc == 0) {
        rc = 0;
      } else if (rc != 1) {
        // a degenerate cut: carve the piece from T_a alone
        init_tri(S, D, a, vx, vy, vz);
        npl = 4;
        nv = 3;
        rc = 0;
        break;
      }
    }
    if (!POW && rc == 0 && nv > 0) {
      // and by the bisectors of the site's Gabriel neighbours (those that do
      // not cross the piece leave it unchanged)
      for (uint64_t m = gabriel_mask_s(S, si, vx, vy, vz, from, from2); m && rc == 0; m &= m - 1) {
        const int c = __ffsll((unsigned long long)m) - 1;
        if (npl >= kSP) break;
        __syncthreads();
        if (l == 0) {
          const double n0 = S.K.x[c] - vx, n1 = S.K.y[c] - vy, n2 = S.K.z[c] - vz;
          S.pn[npl][0] = n0; S.pn[npl][1] = n1; S.pn[npl][2] = n2;
          S.pn[npl][3] = 0.5 * (n0 * n0 + n1 * n1 + n2 * n2);
          S.plab[npl] = S.K.p[c];
        }
        __syncthreads();
        rc = clip_s(S, C.monitor, npl, -1, nv);
        npl++;
        if (rc == 4) ss.clips++;
        if (rc == 4 || rc == 0) {
          rc = 0;
        } else if (rc != 1) {
          init_tri(S, D, a, vx, vy, vz);  // a degenerate cut: carve from T_a alone
          npl = 4;
          nv = 3;
          rc = 0;
          break;
        }
      }
    }
    if (rc == 0) rc = carve_s<POW>(S, G, P, si, vx, vy, vz, delta, npl, nv, ss);
    if (rc == 1) continue;
    if (rc) { err = rc; break; }
    // ---- moments: fan from corner 0 of the piece, so that the area's rounding
    // error scales with the piece and not with its distance to v_i ----
    const double N0 = S.pn[0][0], N1 = S.pn[0][1], N2 = S.pn[0][2];
    const double inrm = 1.0 / sqrt(N0 * N0 + N1 * N1 + N2 * N2);
    const double o0 = S.vy[0][0], o1 = S.vy[0][1], o2 = S.vy[0][2];
    double pa = 0, pmx = 0, pmy = 0, pmz = 0, pe = 0;
    double dm = 0, dmx = 0, dmy = 0, dmz = 0, de = 0;  // density-weighted (DENS)
    if (l < nv) {
      const int t2 = (l + 1) % nv;
      const double y0 = S.vy[l][0], y1 = S.vy[l][1], y2 = S.vy[l][2];
      const double z0 = S.vy[t2][0], z1 = S.vy[t2][1], z2 = S.vy[t2][2];
      const double a0 = y0 - o0, a1 = y1 - o1, a2 = y2 - o2;
      const double b0 = z0 - o0, b1 = z1 - o1, b2 = z2 - o2;
      const double cr0 = a1 * b2 - a2 * b1, cr1 = a2 * b0 - a0 * b2, cr2 = a0 * b1 - a1 * b0;
      const double ar = 0.5 * (cr0 * N0 + cr1 * N1 + cr2 * N2) * inrm;
      const double s0 = o0 + y0 + z0, s1 = o1 + y1 + z1, s2 = o2 + y2 + z2;
      pa = ar;
      pmx = ar * s0 / 3.0; pmy = ar * s1 / 3.0; pmz = ar * s2 / 3.0;
      pe = ar / 12.0 * (o0 * o0 + o1 * o1 + o2 * o2 + y0 * y0 + y1 * y1 + y2 * y2 + z0 * z0 + z1 * z1 + z2 * z2 +
                        s0 * s0 + s1 * s1 + s2 * s2);
      if (DENS) {
        const double P0[3] = {o0, o1, o2}, P1[3] = {y0, y1, y2}, P2[3] = {z0, z1, z2};
        tri_density_moments(C.dens, vx, vy, vz, P0, P1, P2, ar, dm, dmx, dmy, dmz, de);
      }
    }
    pa = wave_sum(pa); pmx = wave_sum(pmx); pmy = wave_sum(pmy); pmz = wave_sum(pmz); pe = wave_sum(pe);
    if (C.monitor) count_add(S.ar.fantets, nv);
    // a piece exists when its area is positive; with a density its moments are
    // the weighted ones
    if (!(pa > 0.0)) continue;
    if (DENS) {
      pa = wave_sum(dm); pmx = wave_sum(dmx); pmy = wave_sum(dmy); pmz = wave_sum(dmz); pe = wave_sum(de);
    }
    const int orig = GL(G.perm)[si];
    const long long pidx = arena_take(S.ar, C, AR_PIECE, 1);
    const long long fo = arena_take(S.ar, C, AR_FACE, nv);
    const long long vo = arena_take(S.ar, C, AR_VERT, nv);
    // only records that fit are counted: the per-site CSR built from the
    // counts then stays inside the arenas (the clip reports the overflow)
    const bool fits_fv = fo + nv <= C.cap_face && vo + nv <= C.cap_vert;
    if (l == 0 && pidx < C.cap_piece && fits_fv)
      __hip_atomic_fetch_add(GL(C.pcount) + orig, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (l == 0 && !(pidx < C.cap_piece && fits_fv)) S.ar.dropped++;
    if (C.want_grad) {
      // segment moments of the bisector edges: a point of the edge moves in
      // the plane of T_a with speed (x - v_i).dv / (d s), s = |n - (n.N)N|
      // (n, N unit normals of the bisector and of T_a); 2-point Gauss-Legendre
      // is exact for the cubic integrand
      const int lab = l < nv ? S.plab[S.ve[l]] : -1;
      const uint64_t pos = __ballot(lab >= 0);
      const int npos = __popcll(pos);
      const long long base = arena_take(S.ar, C, AR_FINT, npos);
      const bool ffits = base + npos <= C.cap_fint;
      if (l == 0 && pidx < C.cap_piece) {
        GL(C.piece_fint_start)[pidx] = base;
        GL(C.piece_nfint)[pidx] = ffits ? npos : 0;
        if (!ffits) S.ar.dropped++;
      }
      const long long r = base + __popcll(pos & lowm(l));
      if (lab >= 0 && r < C.cap_fint) {
        const int t2 = (l + 1) % nv;
        const double n0 = GL(G.sx)[lab] - vx, n1 = GL(G.sy)[lab] - vy, n2 = GL(G.sz)[lab] - vz;
        const double d = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        const double h0 = n0 / d, h1 = n1 / d, h2 = n2 / d;
        const double M0 = N0 * inrm, M1 = N1 * inrm, M2 = N2 * inrm;
        const double hn = h0 * M0 + h1 * M1 + h2 * M2;
        const double e0 = h0 - hn * M0, e1 = h1 - hn * M1, e2 = h2 - hn * M2;
        const double sfac = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        const double a0 = S.vy[l][0], a1 = S.vy[l][1], a2 = S.vy[l][2];
        const double b0 = S.vy[t2][0], b1 = S.vy[t2][1], b2 = S.vy[t2][2];
        const double ln = sqrt((b0 - a0) * (b0 - a0) + (b1 - a1) * (b1 - a1) + (b2 - a2) * (b2 - a2));
        double I[12];
        for (int k = 0; k < 12; k++) I[k] = 0.0;
        // Gauss-Legendre: 2 points (exact for the cubic integrand), or 3 with a
        // density (quadratic times cubic)
        const double gq = 0.5 / sqrt(3.0), g3 = 0.5 * sqrt(0.6);
        const int ng = DENS ? 3 : 2;
        for (int g = 0; g < ng; g++) {
          const double xi = ng == 2 ? (g == 0 ? 0.5 - gq : 0.5 + gq) : (g == 0 ? 0.5 - g3 : (g == 1 ? 0.5 : 0.5 + g3));
          const double y0 = a0 + xi * (b0 - a0), y1 = a1 + xi * (b1 - a1), y2 = a2 + xi * (b2 - a2);
          const double w = (ng == 2 ? 0.5 : (g == 1 ? 8.0 / 18.0 : 5.0 / 18.0)) * ln *
                           (DENS ? density_at(C.dens, vx + y0, vy + y1, vz + y2) : 1.0);
          const double yy = y0 * y0 + y1 * y1 + y2 * y2;
          I[0] += w * y0; I[1] += w * y1; I[2] += w * y2;
          I[3] += w * y0 * y0; I[4] += w * y0 * y1; I[5] += w * y0 * y2;
          I[6] += w * y1 * y1; I[7] += w * y1 * y2; I[8] += w * y2 * y2;
          I[9] += w * yy * y0; I[10] += w * yy * y1; I[11] += w * yy * y2;
        }
        const double sc = 1.0 / (d * sfac);
        for (int k = 0; k < 12; k++) GL(C.fint)[12 * r + k] = I[k] * sc;
        GL(C.fint_lab)[r] = GL(G.perm)[lab];
      }
    }
    if (pidx < C.cap_piece) {
      if (l == 0) {
        // a piece whose edges did not fit is written as an unused slot
        GL(C.piece_site)[pidx] = fits_fv ? orig : -1;
        GL(C.piece_simplex)[pidx] = a;
        GL(C.piece_nface)[pidx] = nv;
        GL(C.piece_nvert)[pidx] = nv;
        GL(C.piece_mass)[pidx] = pa;
        GL(C.piece_mom)[3 * pidx + 0] = pmx + pa * vx;
        GL(C.piece_mom)[3 * pidx + 1] = pmy + pa * vy;
        GL(C.piece_mom)[3 * pidx + 2] = pmz + pa * vz;
        GL(C.piece_energy)[pidx] = pe;
        GL(C.piece_fstart)[pidx] = fo;
        GL(C.piece_vstart)[pidx] = vo;
        if (fits_fv) {
          S.ar.pieces++;
          S.ar.faces += nv;
          S.ar.verts += nv;
        }
      }
      if (fits_fv && l < nv) {
        const int prv = (l + nv - 1) % nv;
        GL(C.face_label)[fo + l] = conv(G, S.plab[S.ve[l]]);
        GL(C.vert_xyz)[3 * (vo + l) + 0] = S.vy[l][0] + vx;
        GL(C.vert_xyz)[3 * (vo + l) + 1] = S.vy[l][1] + vy;
        GL(C.vert_xyz)[3 * (vo + l) + 2] = S.vy[l][2] + vz;
        GL(C.vert_label)[3 * (vo + l) + 0] = conv(G, S.plab[S.ve[prv]]);
        GL(C.vert_label)[3 * (vo + l) + 1] = conv(G, S.plab[S.ve[l]]);
        GL(C.vert_label)[3 * (vo + l) + 2] = 2147483647;
      }
    }
    // ---- propagate over positive edge flags (Alg. 4) ----
    const int lab = l < nv ? S.plab[S.ve[l]] : -1;
    uint64_t pos = __ballot(lab >= 0);
    for (; pos; pos &= pos - 1) {
      const int t = __ffsll((unsigned long long)pos) - 1;
      const int j = __builtin_amdgcn_readlane(lab, t);
      const int at = sq_find(S, C, nsq, j);
      if (at < 0) {
        if (!sq_push(S, C, nsq, j, si)) {
          err = 2;
          where = VD_STAGE_TRIANGLE_SITES;
          break;
        }
      } else if (at >= head && at < kSS && l == 0 && S.sqf2[at] < 0 && S.sqf[at] != si) {
        S.sqf2[at] = si;  // a second known edge of j's piece, not yet carved
      }
    }
    __syncthreads();
  }
  if (l == 0) {
    S.ar.queries += ss.queries;
    S.ar.clips += ss.clips;
    S.ar.cands += ss.cands;
    if (err) {
      atomicAdd(&C.cnt[err == 2 ? CNT_ERR_CAP : CNT_ERR_DEG], 1ull);
      atomicMin((int *)&C.cnt[CNT_BAD_SITE], a);
      atomicOr((unsigned long long *)&C.cnt[CNT_STAGES], 1ull << where);
    }
  }
  __syncthreads();
}

// Persistent: every workgroup (one wave) takes triangles from the queues.
// Four waves per SIMD (128 VGPRs, a few spilled values): the polygon carve is
// latency-bound, and the extra wave hides more of it than the spills cost.
template <bool DENS, bool POW>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) surface_kernel(GridView G, DomainView D, const CellsDev *__restrict__ Cp) {
  __shared__ TriLds S;
  const CellsDev &C = *Cp;
  arena_init(S.ar);
  for (;;) {
    const int a = queue_next(S.ar, C, D.m);
    if (a < 0) break;
    // the triangle's own diagram (a batch) or the only one
    const int b = D.nb > 1 ? diagram_of(D.simp_off, D.nb, a) : 0;
    do_triangle<DENS, POW>(S, G.views[b], D.views[b], C, a);
  }
  arena_close(S.ar, C);
}

// Per-site sums over the site's pieces (CSR order: ascending simplex) and the
// sorted, de-duplicated positive edge flags as neighbour list: site_reduce
// writes the sums and the list length, site_nbrs the list at its CSR offset.
// Up to kNbLocal neighbours are gathered in registers; more are counted and
// written in place.
constexpr int kB = 256;
constexpr int kNbLocal = 96;

__device__ __forceinline__ int site_neighbours(const CellsDev &C, const long long *__restrict__ poff,
                                               const int *__restrict__ pid, long long i, int *nb, int &overflow) {
  int cnt = 0;
  for (long long q = poff[i]; q < poff[i + 1]; q++) {
    const int p = pid[q];
    const long long f0 = GL(C.piece_fstart)[p];
    for (int f = 0; f < GL(C.piece_nface)[p]; f++) {
      const int lab = GL(C.face_label)[f0 + f];
      if (lab < 0) continue;
      int k = 0;
      while (k < cnt && nb[k] < lab) k++;
      if (k < cnt && nb[k] == lab) continue;
      if (cnt >= kNbLocal) { overflow = 1; continue; }
      for (int x = cnt; x > k; x--) nb[x] = nb[x - 1];
      nb[k] = lab;
      cnt++;
    }
  }
  return cnt;
}

// A site with more than kNbLocal distinct neighbours: its edge flags are
// walked in place (no list): `first` tells whether the flag of edge (q, f)
// does not occur on an earlier edge of the site.  The count costs a square
// of the site's edges, which only such sites pay.
__device__ __forceinline__ int edge_label(const CellsDev &C, const int *__restrict__ pid, long long q, int f) {
  return GL(C.face_label)[GL(C.piece_fstart)[pid[q]] + f];
}
__device__ bool first_occurrence(const CellsDev &C, const long long *__restrict__ poff, const int *__restrict__ pid,
                                 long long i, long long q, int f, int lab) {
  for (long long q2 = poff[i]; q2 <= q; q2++) {
    const int nf = q2 < q ? GL(C.piece_nface)[pid[q2]] : f;
    for (int f2 = 0; f2 < nf; f2++)
      if (edge_label(C, pid, q2, f2) == lab) return false;
  }
  return true;
}
// Distinct neighbours of site i; with out != NULL they are also written there
// (unsorted).
__device__ int site_neighbours_wide(const CellsDev &C, const long long *__restrict__ poff, const int *__restrict__ pid,
                                    long long i, int *out) {
  int cnt = 0;
  for (long long q = poff[i]; q < poff[i + 1]; q++) {
    const int nf = GL(C.piece_nface)[pid[q]];
    for (int f = 0; f < nf; f++) {
      const int lab = edge_label(C, pid, q, f);
      if (lab < 0 || !first_occurrence(C, poff, pid, i, q, f, lab)) continue;
      if (out) out[cnt] = lab;
      cnt++;
    }
  }
  return cnt;
}

__global__ void __launch_bounds__(kB) site_reduce(long long n, const long long *__restrict__ poff,
                                                  const int *__restrict__ pid, const CellsDev *__restrict__ Cp) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const CellsDev &C = *Cp;
  double m = 0, mx = 0, my = 0, mz = 0, e = 0;
  for (long long q = poff[i]; q < poff[i + 1]; q++) {
    const int p = pid[q];
    m += GL(C.piece_mass)[p];
    mx += GL(C.piece_mom)[3 * (long long)p + 0];
    my += GL(C.piece_mom)[3 * (long long)p + 1];
    mz += GL(C.piece_mom)[3 * (long long)p + 2];
    e += GL(C.piece_energy)[p];
  }
  GL(C.mass)[i] = m;
  GL(C.mom)[3 * i + 0] = mx;
  GL(C.mom)[3 * i + 1] = my;
  GL(C.mom)[3 * i + 2] = mz;
  GL(C.energy)[i] = e;
  int nb[kNbLocal];
  int overflow = 0;
  const int cnt = site_neighbours(C, poff, pid, i, nb, overflow);
  GL(C.ncount)[i] = overflow ? site_neighbours_wide(C, poff, pid, i, nullptr) : cnt;
}

// cap: entries of nbr.  A no-sync clip keeps the size of the synchronous clip
// before it; lists past the end are not written and the overflow is counted
// (the clip then reports VD_ERR_CAPACITY).
__global__ void __launch_bounds__(kB) site_nbrs(long long n, const long long *__restrict__ poff,
                                                const int *__restrict__ pid, const long long *__restrict__ noff,
                                                int *__restrict__ nbr, long long cap, const CellsDev *__restrict__ Cp) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  int nb[kNbLocal];
  int overflow = 0;
  const CellsDev &C = *Cp;
  int cnt = site_neighbours(C, poff, pid, i, nb, overflow);
  if (overflow) cnt = site_neighbours_wide(C, poff, pid, i, nullptr);
  const long long o = noff[i];
  if (o + cnt > cap) {
    atomicAdd(&Cp->cnt[CNT_OVERFLOW], 1ull);
    return;
  }
  if (!overflow) {
    for (int k = 0; k < cnt; k++) nbr[o + k] = nb[k];
    return;
  }
  // a wide site: the distinct flags in place, then sorted in place
  int *out = nbr + o;
  site_neighbours_wide(C, poff, pid, i, out);
  for (int k = 1; k < cnt; k++) {
    const int v = out[k];
    int y = k - 1;
    while (y >= 0 && out[y] > v) { out[y + 1] = out[y]; y--; }
    out[y + 1] = v;
  }
}

int resident_workgroups() {
  static int cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int &w = cache[dev];
  if (!w) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, surface_kernel<false, false>, 64, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
    w = per_cu * ncu;
  }
  return w;
}

}  // namespace

int vd_surface_workgroups(long long m) {
  const int w = resident_workgroups();
  return (int)(m < w ? (m > 0 ? m : 1) : w);
}

void vd_launch_surface(const GridView &G, const DomainView &D, const CellsDev *Cdev, int workgroups, bool density,
                       bool power, hipStream_t st) {
  const dim3 grid((unsigned)workgroups), block(64);
  if (power) hipLaunchKernelGGL((surface_kernel<false, true>), grid, block, 0, st, G, D, Cdev);
  else if (density) hipLaunchKernelGGL((surface_kernel<true, false>), grid, block, 0, st, G, D, Cdev);
  else hipLaunchKernelGGL((surface_kernel<false, false>), grid, block, 0, st, G, D, Cdev);
}

void vd_launch_site_reduce(long long n, const long long *poff, const int *pid, const CellsDev *Cdev,
                           hipStream_t st) {
  const unsigned nb = (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1);
  hipLaunchKernelGGL(site_reduce, dim3(nb), dim3(kB), 0, st, n, poff, pid, Cdev);
}

void vd_launch_site_nbrs(long long n, const long long *poff, const int *pid, const long long *noff, int *nbr,
                         long long cap, const CellsDev *Cdev, hipStream_t st) {
  const unsigned nb = (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1);
  hipLaunchKernelGGL(site_nbrs, dim3(nb), dim3(kB), 0, st, n, poff, pid, noff, nbr, cap, Cdev);
}
