// clip3d.hip -- clipped Voronoi cells in a tetrahedral domain, one wavefront
// per site.
//
// For site v_i the wave visits the tetrahedra of its cell breadth-first through
// negative face flags, starting at the tetrahedron that contains v_i (the
// propagation of Alg. 5).  Each piece P_{a,i} = T_a cap Omega_i is carved as in
// Alg. 1 / Alg. 3:
//   * every corner is classified by the point-in-cell test (Sec. 4.1, Eq. 2):
//     inside iff its nearest site is v_i or one of the sites named by the flags
//     of the faces through the corner;
//   * while some corner is outside, a search edge is chosen: an edge from an
//     inside corner to an outside one (Alg. 1), else the virtual edge from v_i
//     to the lowest outside corner (Alg. 3);
//   * the edge is shortened by lambda*delta steps (Sec. 6.1) and the bisector
//     is found by the edge-based search (Sec. 4.2);
//   * the clip removes only R_p, the connected outside component containing the
//     chosen outside corner (Sec. 6.3).
//
// Polytope layout in LDS (the dual triangle mesh of Sec. 6.3): planes (normal,
// offset, flag) and corners; a corner stores its three planes in
// counter-clockwise order seen from outside (det of the outward normals > 0),
// the corner across each of its three dual edges, its coordinates relative to
// v_i and its in/out flag.  Lane l owns corner slots l and l+64, so
// classification, flood fill of R_p, the fan of the new face and compaction
// are wave-parallel; inside/outside/removed sets are 128-bit ballot masks.
//
// Moments of a piece: a fan of tetrahedra (v_i, foot of the face plane,
// corner, next corner around the face), three per corner, reduced across the
// wave with butterfly shuffles (fixed order, no floating-point atomics).
#include "vd_internal.h"

namespace {

constexpr int kMaxClips = 256;

struct __align__(16) WaveLds {
  double pn[VD_P_MAX][4];    // plane: outward normal (relative coords), offset
  double cy[VD_C_MAX][3];    // corner coordinates relative to v_i
  int plab[VD_P_MAX];        // plane flag: sorted site >= 0, -(b+1), or boundary code
  int cpl[VD_C_MAX];         // corner planes a | b << 8 | c << 16 (CCW from outside)
  int cnb[VD_C_MAX];         // corner across a->b | across b->c << 8 | across c->a << 16
  int cnn[VD_C_MAX];         // nearest site found by the corner's point-in-cell test
  int cflg[VD_C_MAX];        // bit 0: inside
  unsigned char byFirst[VD_P_MAX], bySecond[VD_P_MAX];
  int tq[VD_Q_MAX];          // tetrahedra of this site, breadth-first
  int pid[VD_Q_MAX];         // arena index of each emitted piece
  int nbl[VD_NB_MAX];        // neighbours found so far (sorted positions)
};

__device__ __forceinline__ int p8(int packed, int e) { return (packed >> (8 * e)) & 0xff; }
__device__ __forceinline__ int pack3(int a, int b, int c) { return a | (b << 8) | (c << 16); }

__device__ __forceinline__ uint64_t low_mask(int k) {  // bits [0, k), k in [0, 64]
  return k >= 64 ? ~0ull : ((1ull << k) - 1ull);
}

struct Stats {
  long long queries = 0, cands = 0, clips = 0;
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

// Point-in-cell test of corner s (Sec. 4.1): nearest site of the corner, inside
// iff it is the site itself or a site named by a flag of the corner's planes.
__device__ __forceinline__ bool classify(WaveLds &S, const GridView &G, int s, int si, double vx,
                                         double vy, double vz, Stats &st) {
  const double y0 = S.cy[s][0], y1 = S.cy[s][1], y2 = S.cy[s][2];
  const double qx = vx + y0, qy = vy + y1, qz = vz + y2;
  const double dx = qx - vx, dy = qy - vy, dz = qz - vz;
  double d2;
  const int k = nn_query(G, qx, qy, qz, dx * dx + dy * dy + dz * dz, si, d2, st.cands);
  st.queries++;
  const int pl = S.cpl[s];
  const bool in = (k == si) || (k == S.plab[p8(pl, 0)]) || (k == S.plab[p8(pl, 1)]) || (k == S.plab[p8(pl, 2)]);
  __syncthreads();
  if (vd_lane() == 0) { S.cnn[s] = k; S.cflg[s] = in ? 1 : 0; }
  __syncthreads();
  return in;
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
  // new index of plane x = number of used planes below x
  double pv[4] = {0, 0, 0, 0};
  int lab = 0;
  const bool mine = l < npl && ((used >> l) & 1ull);
  if (mine) { for (int k = 0; k < 4; k++) pv[k] = S.pn[l][k]; lab = S.plab[l]; }
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
  }
  for (int h = 0; h < 2; h++) {
    const int s = l + 64 * h;
    if (s < nc) {
      int a = p8(cp[h], 0), b = p8(cp[h], 1), c = p8(cp[h], 2);
      a = __popcll(used & low_mask(a));
      b = __popcll(used & low_mask(b));
      c = __popcll(used & low_mask(c));
      S.cpl[s] = pack3(a, b, c);
    }
  }
  __syncthreads();
  return newnpl;
}

// Clip by plane slot P, removing R_p: the connected set of corners strictly
// outside P that contains corner pt (Sec. 6.3).  New corners are created on
// every dual edge leaving R_p and form the fan of the new face.
// Returns 0 ok, 1 empty, 2 capacity, 3 degenerate.  On success nc and nsurv
// (corners kept; new corners are slots [nsurv, nc)) are updated.
__device__ int clip_poly(WaveLds &S, int P, int pt, int &nc, int &nsurv_out) {
  const int l = vd_lane();
  const double nx = S.pn[P][0], ny = S.pn[P][1], nz = S.pn[P][2], c = S.pn[P][3];
  int pl[2] = {0, 0}, nb[2] = {0, 0}, fl[2] = {0, 0}, nn[2] = {0, 0};
  double y[2][3] = {{0, 0, 0}, {0, 0, 0}};
  bool v[2], o[2];
  for (int h = 0; h < 2; h++) {
    const int s = l + 64 * h;
    v[h] = s < nc;
    if (v[h]) {
      pl[h] = S.cpl[s]; nb[h] = S.cnb[s]; fl[h] = S.cflg[s]; nn[h] = S.cnn[s];
      y[h][0] = S.cy[s][0]; y[h][1] = S.cy[s][1]; y[h][2] = S.cy[s][2];
    }
    o[h] = v[h] && (nx * y[h][0] + ny * y[h][1] + nz * y[h][2] - c > 0.0);
  }
  const uint64_t olo = __ballot(o[0]), ohi = __ballot(o[1]);
  if (!bit128(olo, ohi, pt)) return 3;
  uint64_t Rlo = pt < 64 ? (1ull << pt) : 0ull, Rhi = pt >= 64 ? (1ull << (pt - 64)) : 0ull;
  for (int it = 0; it < VD_C_MAX; it++) {
    bool j[2];
    for (int h = 0; h < 2; h++) {
      const int s = l + 64 * h;
      j[h] = o[h] && !bit128(Rlo, Rhi, s) &&
             (bit128(Rlo, Rhi, p8(nb[h], 0)) || bit128(Rlo, Rhi, p8(nb[h], 1)) || bit128(Rlo, Rhi, p8(nb[h], 2)));
    }
    const uint64_t a = __ballot(j[0]), b = __ballot(j[1]);
    if (!(a | b)) break;
    Rlo |= a;
    Rhi |= b;
  }
  const int nR = __popcll(Rlo) + __popcll(Rhi);
  if (nR >= nc) return 1;
  bool r[2];
  int em[2] = {0, 0};  // boundary edges of removed corners
  for (int h = 0; h < 2; h++) {
    const int s = l + 64 * h;
    r[h] = v[h] && bit128(Rlo, Rhi, s);
    if (r[h])
      for (int e = 0; e < 3; e++)
        if (!bit128(Rlo, Rhi, p8(nb[h], e))) em[h] |= 1 << e;
  }
  const int cnt = __popc(em[0]) + __popc(em[1]);
  const int inc = wave_incl_scan(cnt);
  const int nnew = __shfl(inc, 63, 64);
  const int base = inc - cnt;
  const int nsurv = nc - nR;
  if (nnew < 3) return 3;
  if (nsurv + nnew > VD_C_MAX) return 2;
  const uint64_t vlo = low_mask(nc < 64 ? nc : 64), vhi = low_mask(nc > 64 ? nc - 64 : 0);
  const uint64_t Slo = vlo & ~Rlo, Shi = vhi & ~Rhi;
  auto rank = [&](int s) -> int {
    return s < 64 ? __popcll(Slo & low_mask(s)) : __popcll(Slo) + __popcll(Shi & low_mask(s - 64));
  };
  // every plane is "first" (resp. "second") of at most one new corner when the
  // boundary of R_p is a simple loop; the tables give the fan adjacency
  __syncthreads();
  {
    int t = base;
    for (int h = 0; h < 2; h++)
      for (int e = 0; e < 3; e++)
        if (em[h] & (1 << e)) {
          const int u = p8(pl[h], e), w = p8(pl[h], (e + 1) % 3);
          S.byFirst[u] = (unsigned char)(nsurv + t);
          S.bySecond[w] = (unsigned char)(nsurv + t);
          t++;
        }
  }
  __syncthreads();
  bool bad = false;
  {
    int t = base;
    for (int h = 0; h < 2; h++)
      for (int e = 0; e < 3; e++)
        if (em[h] & (1 << e)) {
          const int u = p8(pl[h], e), w = p8(pl[h], (e + 1) % 3);
          if (S.byFirst[u] != nsurv + t || S.bySecond[w] != nsurv + t) bad = true;
          t++;
        }
  }
  if (__ballot(bad)) return 3;
  // all old corner data sits in registers: write the new layout
  {
    int t = base;
    for (int h = 0; h < 2; h++) {
      const int s = l + 64 * h;
      if (v[h] && !r[h]) {
        const int ns = rank(s);
        int nbo[3];
        for (int e = 0; e < 3; e++) {
          const int m = p8(nb[h], e);
          nbo[e] = bit128(Rlo, Rhi, m) ? S.byFirst[p8(pl[h], (e + 1) % 3)] : rank(m);
        }
        S.cpl[ns] = pl[h];
        S.cnb[ns] = pack3(nbo[0], nbo[1], nbo[2]);
        S.cflg[ns] = fl[h];
        S.cnn[ns] = nn[h];
        S.cy[ns][0] = y[h][0]; S.cy[ns][1] = y[h][1]; S.cy[ns][2] = y[h][2];
      }
      if (r[h])
        for (int e = 0; e < 3; e++)
          if (em[h] & (1 << e)) {
            const int u = p8(pl[h], e), w = p8(pl[h], (e + 1) % 3);
            const int ns = nsurv + t;
            const int m = p8(nb[h], e);
            S.cpl[ns] = pack3(u, w, P);
            S.cnb[ns] = pack3(rank(m), S.byFirst[w], S.bySecond[u]);
            S.cflg[ns] = 0;
            S.cnn[ns] = -1;
            double yy[3];
            solve3(S, u, w, P, yy);
            S.cy[ns][0] = yy[0]; S.cy[ns][1] = yy[1]; S.cy[ns][2] = yy[2];
            t++;
          }
    }
  }
  __syncthreads();
  nc = nsurv + nnew;
  nsurv_out = nsurv;
  return 0;
}

__device__ __forceinline__ void masks_inside(const WaveLds &S, int nc, uint64_t &ilo, uint64_t &ihi) {
  const int l = vd_lane();
  const bool a = l < nc && (S.cflg[l] & 1);
  const bool b = l + 64 < nc && (S.cflg[l + 64] & 1);
  ilo = __ballot(a);
  ihi = __ballot(b);
}

__device__ __forceinline__ int convert_label(const GridView &G, int lab) {
  return lab >= 0 ? G.perm[lab] : lab;
}

__global__ void __launch_bounds__(64) clip3d_kernel(GridView G, DomainView D, CellsDev C) {
  __shared__ WaveLds S;
  const int l = vd_lane();
  // consecutive sorted sites go to the same XCD (workgroup b runs on XCD b % 8)
  const int q8 = gridDim.x >> 3;
  const int si = (blockIdx.x & 7) * q8 + (blockIdx.x >> 3);
  if (si >= G.n) return;
  const double vx = G.sx[si], vy = G.sy[si], vz = G.sz[si];
  const int orig = G.perm[si];
  const double delta = G.delta[si];
  const int seed = C.seed[si];
  Stats st;
  int err = 0;  // 2 capacity, 3 degenerate
  int nt = 0, head = 0, nnb = 0, npieces = 0;
  double Mv = 0, Mx = 0, My = 0, Mz = 0, Me = 0;
  if (seed >= 0 && seed < D.m) {
    if (l == 0) S.tq[0] = seed;
    nt = 1;
  }
  __syncthreads();
  while (head < nt && !err) {
    const int a = S.tq[head++];
    // ---- P <- T_a (4 planes, 4 corners) ----
    {
      const int *tv = &D.simp[(long long)a * 4];
      double q[4][3];
      for (int k = 0; k < 4; k++) {
        const double *p = &D.verts[3 * (long long)tv[k]];
        q[k][0] = p[0] - vx; q[k][1] = p[1] - vy; q[k][2] = p[2] - vz;
      }
      if (l < 4) {
        // face f = l opposite vertex f, counter-clockwise from outside
        const int L[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
        const double *A = q[L[l][0]], *B = q[L[l][1]], *Cc = q[L[l][2]];
        const double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        const double ac[3] = {Cc[0] - A[0], Cc[1] - A[1], Cc[2] - A[2]};
        const double n[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
        S.pn[l][0] = n[0]; S.pn[l][1] = n[1]; S.pn[l][2] = n[2];
        S.pn[l][3] = n[0] * A[0] + n[1] * A[1] + n[2] * A[2];
        const int b = D.adj[(long long)a * 4 + l];
        S.plab[l] = b >= 0 ? -(b + 1) : VD_BND_BASE + l;
        // corner l = vertex l; planes CCW from outside and neighbours across
        // the dual edges (fixed for positively oriented tetrahedra)
        const int CP[4] = {pack3(1, 3, 2), pack3(0, 2, 3), pack3(0, 3, 1), pack3(0, 1, 2)};
        const int CN[4] = {pack3(2, 1, 3), pack3(3, 0, 2), pack3(1, 0, 3), pack3(2, 0, 1)};
        S.cpl[l] = CP[l];
        S.cnb[l] = CN[l];
        S.cflg[l] = 0;
        S.cnn[l] = -1;
        S.cy[l][0] = q[l][0]; S.cy[l][1] = q[l][1]; S.cy[l][2] = q[l][2];
      }
    }
    __syncthreads();
    int npl = 4, nc = 4;
    for (int s = 0; s < 4; s++) classify(S, G, s, si, vx, vy, vz, st);
    bool empty = false;
    for (int it = 0;; it++) {
      if (it >= kMaxClips) { err = 3; break; }
      uint64_t ilo, ihi;
      masks_inside(S, nc, ilo, ihi);
      const uint64_t vlo = low_mask(nc < 64 ? nc : 64), vhi = low_mask(nc > 64 ? nc - 64 : 0);
      const uint64_t olo = vlo & ~ilo, ohi = vhi & ~ihi;
      if (!(olo | ohi)) break;
      // ---- choose the search edge ----
      int pt = -1, ps = -1;
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
          const int nbp = S.cnb[pt];
          for (int e = 0; e < 3; e++)
            if (bit128(ilo, ihi, p8(nbp, e))) { ps = p8(nbp, e); break; }
        }
      }
      if (pt < 0) pt = olo ? __ffsll((unsigned long long)olo) - 1 : 64 + __ffsll((unsigned long long)ohi) - 1;
      double A[3] = {0, 0, 0};
      if (ps >= 0) { A[0] = S.cy[ps][0]; A[1] = S.cy[ps][1]; A[2] = S.cy[ps][2]; }
      double g[3] = {S.cy[pt][0], S.cy[pt][1], S.cy[pt][2]};
      int j = S.cnn[pt];
      // Flags of a point on the edge p_s p_t: the two planes of the edge
      // (Sec. 4.1 flag rule).  A search point whose nearest site is named by
      // one of them lies on that face of Omega_i, i.e. inside.
      int ef0 = -2, ef1 = -2;
      if (ps >= 0) {
        const int a0 = S.cpl[ps], b0 = S.cpl[pt];
        int ne = 0;
        for (int x = 0; x < 3; x++) {
          const int px = p8(a0, x);
          if (px == p8(b0, 0) || px == p8(b0, 1) || px == p8(b0, 2)) {
            const int lab = S.plab[px];
            if (ne == 0) ef0 = lab >= 0 ? lab : -2; else ef1 = lab >= 0 ? lab : -2;
            ne++;
          }
        }
      }
      // ---- improved search (Sec. 6.1): g = A + lambda*delta*u, lambda = 2, 3, ...
      if (C.improved) {
        const double d0 = g[0] - A[0], d1 = g[1] - A[1], d2 = g[2] - A[2];
        const double L = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (L > 0) {
          const double u0 = d0 / L, u1 = d1 / L, u2 = d2 / L;
          for (int lam = 2; lam < 2 + C.max_iters && lam * delta < L; lam++) {
            const double t = lam * delta;
            const double gx = A[0] + t * u0, gy = A[1] + t * u1, gz = A[2] + t * u2;
            const double qx = vx + gx, qy = vy + gy, qz = vz + gz;
            const double ex = qx - vx, ey = qy - vy, ez = qz - vz;
            double dd;
            const int k = nn_query(G, qx, qy, qz, ex * ex + ey * ey + ez * ez, si, dd, st.cands);
            st.queries++;
            if (k != si && k != ef0 && k != ef1) { j = k; g[0] = gx; g[1] = gy; g[2] = gz; break; }
          }
        }
      }
      // ---- edge-based bisector search (Sec. 4.2) on [A, g] ----
      if (j < 0 || j == si) { err = 3; break; }
      double nj[4];
      for (int stp = 0;; stp++) {
        if (stp >= C.max_iters) { err = 3; break; }
        nj[0] = G.sx[j] - vx; nj[1] = G.sy[j] - vy; nj[2] = G.sz[j] - vz;
        nj[3] = 0.5 * (nj[0] * nj[0] + nj[1] * nj[1] + nj[2] * nj[2]);
        const double e0 = g[0] - A[0], e1 = g[1] - A[1], e2 = g[2] - A[2];
        const double den = nj[0] * e0 + nj[1] * e1 + nj[2] * e2;
        const double num = nj[3] - (nj[0] * A[0] + nj[1] * A[1] + nj[2] * A[2]);
        double t = den > 0.0 ? num / den : 1.0;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        const double qx = vx + (A[0] + t * e0), qy = vy + (A[1] + t * e1), qz = vz + (A[2] + t * e2);
        const double ex = qx - vx, ey = qy - vy, ez = qz - vz;
        double dd;
        const int k = nn_query(G, qx, qy, qz, ex * ex + ey * ey + ez * ez, si, dd, st.cands);
        st.queries++;
        // q lies on the boundary of Omega_i: B_ij is a face of the cell
        if (k == si || k == j || k == ef0 || k == ef1) break;
        j = k;
        g[0] = A[0] + t * e0; g[1] = A[1] + t * e1; g[2] = A[2] + t * e2;
      }
      if (err) break;
      // ---- clip by B_ij ----
      if (npl >= VD_P_MAX) {
        npl = compact_planes(S, npl, nc);
        if (npl >= VD_P_MAX) { err = 2; break; }
      }
      const int P = npl++;
      __syncthreads();
      if (l == 0) {
        S.pn[P][0] = nj[0]; S.pn[P][1] = nj[1]; S.pn[P][2] = nj[2]; S.pn[P][3] = nj[3];
        S.plab[P] = j;
      }
      __syncthreads();
      int nsurv = nc;
      const int rc = clip_poly(S, P, pt, nc, nsurv);
      st.clips++;
      if (rc == 1) { empty = true; break; }
      if (rc) { err = rc; break; }
      for (int s = nsurv; s < nc; s++) classify(S, G, s, si, vx, vy, vz, st);
    }
    if (err) break;
    if (empty || nc == 0) continue;
    // ---- moments of the piece ----
    double pv = 0, pmx = 0, pmy = 0, pmz = 0, pe = 0;
    uint64_t fmask = 0;
    for (int h = 0; h < 2; h++) {
      const int s = l + 64 * h;
      if (s >= nc) continue;
      const int pl = S.cpl[s], nb = S.cnb[s];
      const double y0 = S.cy[s][0], y1 = S.cy[s][1], y2 = S.cy[s][2];
      fmask |= (1ull << p8(pl, 0)) | (1ull << p8(pl, 1)) | (1ull << p8(pl, 2));
      // plane p8(pl,e) continues around the face to the corner across edge (e+2)%3
      for (int e = 0; e < 3; e++) {
        const int x = p8(pl, e);
        const int nx_ = p8(nb, (e + 2) % 3);
        const double n0 = S.pn[x][0], n1 = S.pn[x][1], n2 = S.pn[x][2], cc = S.pn[x][3];
        const double f = cc / (n0 * n0 + n1 * n1 + n2 * n2);
        const double r0 = n0 * f, r1 = n1 * f, r2 = n2 * f;
        const double z0 = S.cy[nx_][0], z1 = S.cy[nx_][1], z2 = S.cy[nx_][2];
        const double det = r0 * (y1 * z2 - y2 * z1) - r1 * (y0 * z2 - y2 * z0) + r2 * (y0 * z1 - y1 * z0);
        const double vol = det / 6.0;
        const double s0 = r0 + y0 + z0, s1 = r1 + y1 + z1, s2 = r2 + y2 + z2;
        pv += vol;
        pmx += vol * s0 * 0.25; pmy += vol * s1 * 0.25; pmz += vol * s2 * 0.25;
        pe += vol * (1.0 / 20.0) *
              (r0 * r0 + r1 * r1 + r2 * r2 + y0 * y0 + y1 * y1 + y2 * y2 + z0 * z0 + z1 * z1 + z2 * z2 +
               s0 * s0 + s1 * s1 + s2 * s2);
      }
    }
    pv = wave_sum(pv); pmx = wave_sum(pmx); pmy = wave_sum(pmy); pmz = wave_sum(pmz); pe = wave_sum(pe);
    fmask = wave_or64(fmask);
    if (!(pv > 0.0)) continue;
    Mv += pv; Mx += pmx; My += pmy; Mz += pmz; Me += pe;
    // ---- emit the piece ----
    const int nface = __popcll(fmask);
    long long pidx = 0, fo = 0, vo = 0;
    if (l == 0) {
      pidx = (long long)atomicAdd(&C.cnt[CNT_PIECES], 1ull);
      if (C.emit) {
        fo = (long long)atomicAdd(&C.cnt[CNT_FACES], (unsigned long long)nface);
        vo = (long long)atomicAdd(&C.cnt[CNT_VERTS], (unsigned long long)nc);
      }
    }
    pidx = __shfl(pidx, 0, 64);
    fo = __shfl(fo, 0, 64);
    vo = __shfl(vo, 0, 64);
    if (pidx < C.cap_piece) {
      if (l == 0) {
        C.piece_site[pidx] = orig;
        C.piece_simplex[pidx] = a;
        C.piece_nface[pidx] = nface;
        C.piece_nvert[pidx] = nc;
        C.piece_mass[pidx] = pv;
        C.piece_mom[3 * pidx + 0] = pmx + pv * vx;
        C.piece_mom[3 * pidx + 1] = pmy + pv * vy;
        C.piece_mom[3 * pidx + 2] = pmz + pv * vz;
        C.piece_energy[pidx] = pe;
        C.piece_fstart[pidx] = C.emit ? fo : -1;
        C.piece_vstart[pidx] = C.emit ? vo : -1;
      }
      if (C.emit && fo + nface <= C.cap_face && vo + nc <= C.cap_vert) {
        if (l < npl && ((fmask >> l) & 1ull))
          C.face_label[fo + __popcll(fmask & low_mask(l))] = convert_label(G, S.plab[l]);
        for (int h = 0; h < 2; h++) {
          const int s = l + 64 * h;
          if (s < nc) {
            const int pl = S.cpl[s];
            C.vert_xyz[3 * (vo + s) + 0] = S.cy[s][0] + vx;
            C.vert_xyz[3 * (vo + s) + 1] = S.cy[s][1] + vy;
            C.vert_xyz[3 * (vo + s) + 2] = S.cy[s][2] + vz;
            for (int e = 0; e < 3; e++) C.vert_label[3 * (vo + s) + e] = convert_label(G, S.plab[p8(pl, e)]);
          }
        }
      }
    }
    if (l == 0) S.pid[npieces] = (int)pidx;
    npieces++;
    // ---- propagate: neighbours (positive flags), tetrahedra (negative flags) ----
    for (uint64_t m = fmask; m; m &= m - 1) {
      const int x = __ffsll((unsigned long long)m) - 1;
      const int lab = S.plab[x];
      if (lab >= 0) {
        const bool have = (l < nnb && S.nbl[l] == lab) || (l + 64 < nnb && S.nbl[l + 64] == lab);
        if (!__ballot(have)) {
          if (nnb >= VD_NB_MAX) { err = 2; break; }
          __syncthreads();
          if (l == 0) S.nbl[nnb] = lab;
          nnb++;
          __syncthreads();
        }
      } else if (lab > VD_BND_BASE + 3) {
        const int b = -lab - 1;
        bool have = false;
        for (int e = l; e < nt; e += 64) have = have || (S.tq[e] == b);
        if (!__ballot(have)) {
          if (nt >= VD_Q_MAX) { err = 2; break; }
          __syncthreads();
          if (l == 0) S.tq[nt] = b;
          nt++;
          __syncthreads();
        }
      }
    }
    __syncthreads();
  }
  // ---- per-site results ----
  if (l == 0) {
    C.mass[orig] = Mv;
    C.mom[3 * (long long)orig + 0] = Mx + Mv * vx;
    C.mom[3 * (long long)orig + 1] = My + Mv * vy;
    C.mom[3 * (long long)orig + 2] = Mz + Mv * vz;
    C.energy[orig] = Me;
    C.pcount[orig] = npieces;
    C.ncount[orig] = nnb;
  }
  long long ps0 = 0, ns0 = 0;
  if (l == 0) {
    ps0 = (long long)atomicAdd(&C.cnt[CNT_PLIST], (unsigned long long)npieces);
    ns0 = (long long)atomicAdd(&C.cnt[CNT_NBRS], (unsigned long long)nnb);
    C.pstart[orig] = ps0;
    C.nstart[orig] = ns0;
  }
  ps0 = __shfl(ps0, 0, 64);
  ns0 = __shfl(ns0, 0, 64);
  __syncthreads();
  if (ps0 + npieces <= C.cap_plist)
    for (int e = l; e < npieces; e += 64) C.plist[ps0 + e] = S.pid[e];
  if (ns0 + nnb <= C.cap_nbr) {
    // neighbours in ascending caller index: rank sort
    for (int h = 0; h < 2; h++) {
      const int e = l + 64 * h;
      if (e < nnb) {
        const int me = G.perm[S.nbl[e]];
        int rk = 0;
        for (int o = 0; o < nnb; o++) rk += (G.perm[S.nbl[o]] < me) ? 1 : 0;
        C.nbr_arena[ns0 + rk] = me;
      }
    }
  }
  if (l == 0) {
    atomicAdd(&C.cnt[CNT_QUERIES], (unsigned long long)st.queries);
    atomicAdd(&C.cnt[CNT_CLIPS], (unsigned long long)st.clips);
    atomicAdd(&C.cnt[CNT_CANDS], (unsigned long long)st.cands);
    if (err) {
      atomicAdd(&C.cnt[err == 2 ? CNT_ERR_CAP : CNT_ERR_DEG], 1ull);
      atomicMin((int *)&C.cnt[CNT_BAD_SITE], orig);
    }
  }
}

}  // namespace

void vd_launch_clip3d(const GridView &G, const DomainView &D, const CellsDev &C, hipStream_t st) {
  const unsigned q8 = (unsigned)((G.n + 7) / 8);
  hipLaunchKernelGGL(clip3d_kernel, dim3(q8 * 8), dim3(64), 0, st, G, D, C);
}
