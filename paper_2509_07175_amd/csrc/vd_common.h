// vd_common.h -- device-side building blocks shared by the kernels.
//
// gfx950 (CDNA4), wave64.  Geometry is float64 throughout (FP64 vector ALU is
// full rate on this chip); nothing here is a dense contraction, so no MFMA.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define VD_WAVE 64

// The views' arrays are device allocations: device code reads and writes them
// through global (address space 1) pointers, so the accesses are global_*
// instructions.  Through the generic pointers of the view structs they would
// be flat_* accesses, which also count against the LDS wait counter: every
// wait for an LDS result would then wait for outstanding memory loads too.
#define GL(p) ((__attribute__((address_space(1))) std::remove_pointer_t<decltype(p)> *)(p))
#define VD_BND_BASE (-2147483647 - 1)

// Device view of the nearest-site grid (Sec. 6.2).  Sites are stored in cell
// order; "sorted position" indexes sx/sy/sz/delta, perm maps it back to the
// caller's index.  geom = {lo[3], h[3], ih[3]} lives in device memory because
// the bounding box is reduced on the device.
//
// A batch of independent diagrams is one disjoint union: diagram b owns the
// sorted positions [site_off[b], site_off[b+1]) and its own block of grid
// cells; views[b] is its view (its cstart points into the shared offsets, so
// positions stay global).  A plain grid is the batch of one, views = NULL.
struct GridView {
  int n;       // sites of this view (all sites for the batch view)
  int g[3];
  const double *geom;
  const double *sx, *sy, *sz;
  const int *cstart;  // [g0*g1*g2 + 1]
  const int *perm;    // sorted position -> caller index
  const double *delta;  // half nearest-other-site distance, by sorted position
  const double *sw, *sh;  // power diagram (Sec. 7.3): weight w and lifted coordinate
                          // h = sqrt(eta - w) by sorted position; NULL for Voronoi
  int nb;                      // diagrams (1: plain)
  const GridView *views;       // [nb] per-diagram views (nb > 1)
  const long long *site_off;   // [nb + 1] sorted-position offsets (nb > 1)
};

// diagram of the uniform item x: largest b with off[b] <= x
__device__ __forceinline__ int diagram_of(const long long *off, int nb, long long x) {
  int lo = 0, hi = nb;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ GridView grid_of(const GridView &G, long long si) {
  return G.nb > 1 ? G.views[diagram_of(G.site_off, G.nb, si)] : G;
}

__device__ __forceinline__ int vd_lane() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// lanes below this one
__device__ __forceinline__ unsigned long long low_mask_lt(int l) { return (1ull << l) - 1ull; }

__device__ __forceinline__ bool bit128(uint64_t lo, uint64_t hi, int s) {
  return s < 64 ? ((lo >> s) & 1ull) : ((hi >> (s - 64)) & 1ull);
}

// ---------------------------------------------------------------------------
// Wave primitives on DPP (row = 16 lanes) and lane reads.  The reductions
// combine within rows with quad_perm / row_half_mirror / row_mirror moves and
// across the four rows with v_readlane, so they cost a few VALU latencies
// instead of one LDS round trip (ds_bpermute) per step.  Every lane of the
// wave must be active (of the row, for the row_ variants).
// ---------------------------------------------------------------------------
#define VD_DPP_QUAD_XOR1 0xB1   // quad_perm [1,0,3,2]
#define VD_DPP_QUAD_XOR2 0x4E   // quad_perm [2,3,0,1]
#define VD_DPP_ROW_HALF_MIRROR 0x141
#define VD_DPP_ROW_MIRROR 0x140
#define VD_DPP_ROW_SHR(k) (0x110 + (k))
#define VD_DPP_ROW_BCAST15 0x142
#define VD_DPP_ROW_BCAST31 0x143

// lanes whose source is outside the row get `old`
template <int CTRL>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double old, double v) {
  const uint64_t o = (uint64_t)__double_as_longlong(old), b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
// permutations within a row (quad_perm, row mirrors): every lane has a source,
// so no `old` value has to be kept in the destination register
template <int CTRL>
__device__ __forceinline__ int perm_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ double perm_d(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ long long readlane_ll(long long v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (long long)(((uint64_t)hi << 32) | lo);
}

// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += dpp_i<VD_DPP_ROW_SHR(1)>(0, v);
  v += dpp_i<VD_DPP_ROW_SHR(2)>(0, v);
  v += dpp_i<VD_DPP_ROW_SHR(4)>(0, v);
  v += dpp_i<VD_DPP_ROW_SHR(8)>(0, v);
  v += __builtin_amdgcn_update_dpp(0, v, VD_DPP_ROW_BCAST15, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, VD_DPP_ROW_BCAST31, 0xc, 0xf, false);
  return v;
}

// inclusive prefix sum within each row of 16 lanes
__device__ __forceinline__ int row_incl_scan(int v) {
  v += dpp_i<VD_DPP_ROW_SHR(1)>(0, v);
  v += dpp_i<VD_DPP_ROW_SHR(2)>(0, v);
  v += dpp_i<VD_DPP_ROW_SHR(4)>(0, v);
  v += dpp_i<VD_DPP_ROW_SHR(8)>(0, v);
  return v;
}

// sum over the wave, the same value in every lane (fixed combination order)
__device__ __forceinline__ double wave_sum(double v) {
  v += perm_d<VD_DPP_QUAD_XOR1>(v);
  v += perm_d<VD_DPP_QUAD_XOR2>(v);
  v += perm_d<VD_DPP_ROW_HALF_MIRROR>(v);
  v += perm_d<VD_DPP_ROW_MIRROR>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// minimum over the wave, the same value in every lane
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, perm_d<VD_DPP_QUAD_XOR1>(v));
  v = fmin(v, perm_d<VD_DPP_QUAD_XOR2>(v));
  v = fmin(v, perm_d<VD_DPP_ROW_HALF_MIRROR>(v));
  v = fmin(v, perm_d<VD_DPP_ROW_MIRROR>(v));
  return fmin(fmin(readlane_d(v, 0), readlane_d(v, 16)), fmin(readlane_d(v, 32), readlane_d(v, 48)));
}

__device__ __forceinline__ int wave_isum(int v) {
  v += perm_i<VD_DPP_QUAD_XOR1>(v);
  v += perm_i<VD_DPP_QUAD_XOR2>(v);
  v += perm_i<VD_DPP_ROW_HALF_MIRROR>(v);
  v += perm_i<VD_DPP_ROW_MIRROR>(v);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo |= perm_i<VD_DPP_QUAD_XOR1>(lo); hi |= perm_i<VD_DPP_QUAD_XOR1>(hi);
  lo |= perm_i<VD_DPP_QUAD_XOR2>(lo); hi |= perm_i<VD_DPP_QUAD_XOR2>(hi);
  lo |= perm_i<VD_DPP_ROW_HALF_MIRROR>(lo); hi |= perm_i<VD_DPP_ROW_HALF_MIRROR>(hi);
  lo |= perm_i<VD_DPP_ROW_MIRROR>(lo); hi |= perm_i<VD_DPP_ROW_MIRROR>(hi);
  const uint32_t L = (uint32_t)(__builtin_amdgcn_readlane(lo, 0) | __builtin_amdgcn_readlane(lo, 16) |
                                __builtin_amdgcn_readlane(lo, 32) | __builtin_amdgcn_readlane(lo, 48));
  const uint32_t H = (uint32_t)(__builtin_amdgcn_readlane(hi, 0) | __builtin_amdgcn_readlane(hi, 16) |
                                __builtin_amdgcn_readlane(hi, 32) | __builtin_amdgcn_readlane(hi, 48));
  return ((uint64_t)H << 32) | L;
}

// (d, k) <- the lexicographic minimum of (d, k) and (od, ok).  Bitwise, not
// short-circuit, logic and selects: no branch, no exec-mask juggling.
__device__ __forceinline__ void lexmin(double &d, int &k, double od, int ok) {
  const bool take = (od < d) | ((od == d) & (ok < k));
  d = take ? od : d;
  k = take ? ok : k;
}

// Lexicographic (distance^2, sorted position) minimum within each row of 16
// lanes; every lane of the row ends with the row's result.
template <int CTRL>
__device__ __forceinline__ void argmin_step(double &d, int &k) {
  const double od = perm_d<CTRL>(d);
  const int ok = perm_i<CTRL>(k);
  lexmin(d, k, od, ok);
}
__device__ __forceinline__ void row_argmin(double &d, int &k) {
  argmin_step<VD_DPP_QUAD_XOR1>(d, k);
  argmin_step<VD_DPP_QUAD_XOR2>(d, k);
  argmin_step<VD_DPP_ROW_HALF_MIRROR>(d, k);
  argmin_step<VD_DPP_ROW_MIRROR>(d, k);
}

// ... over the wave; every lane ends with the result
__device__ __forceinline__ void wave_argmin(double &d, int &k) {
  row_argmin(d, k);
  double bd = readlane_d(d, 0);
  int bk = __builtin_amdgcn_readlane(k, 0);
#pragma unroll
  for (int r = 1; r < 4; r++) {
    const double od = readlane_d(d, 16 * r);
    const int ok = __builtin_amdgcn_readlane(k, 16 * r);
    lexmin(bd, bk, od, ok);
  }
  d = bd;
  k = bk;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int cell_coord(double x, double lo, double ih, int g) {
  double t = floor((x - lo) * ih);
  if (!(t > 0.0)) return 0;  // also catches NaN
  if (t >= (double)(g - 1)) return g - 1;
  return (int)t;
}

// ---------------------------------------------------------------------------
// nearest-site query by a group of gs lanes (gs = 64: the whole wave; gs = 16:
// four independent queries per wave).  q and the known candidate (r2, k0) are
// uniform within a group.  The candidate box is split into x-rows; a row of
// consecutive cells is one contiguous range of sorted sites, so the group
// flattens all rows into one candidate list (coalesced SoA loads).
// ---------------------------------------------------------------------------
// POW: power diagram, the sites lifted to (v_j, h_j) and the query to (q, qw):
// the distance is |q - v_j|^2 + (qw - h_j)^2, never below the 3D one, so the
// boxes trimmed to the 3D ball of the best distance still hold every nearer site.
template <bool POW = false>
__device__ __forceinline__ void scan_box(const GridView &G, int gs, int x0, int x1, int y0, int y1, int z0,
                                         int z1, double qx, double qy, double qz, double &bd, int &bk,
                                         long long &ncand, double qw = 0.0) {
  const int gl = vd_lane() & (gs - 1);
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  const int R = ny * (z1 - z0 + 1);
  for (int r0 = 0; r0 < R; r0 += gs) {
    const int r = r0 + gl;
    int st = 0, cnt = 0;
    if (r < R) {
      const int yy = y0 + r % ny, zz = z0 + r / ny;
      const int c0 = x0 + G.g[0] * (yy + G.g[1] * zz);
      st = GL(G.cstart)[c0];
      cnt = GL(G.cstart)[c0 + nx] - st;
    }
    const int inc = gs == 64 ? wave_incl_scan(cnt) : row_incl_scan(cnt);
    const int excl = inc - cnt;
    const int total = gs == 64 ? __builtin_amdgcn_readlane(inc, 63) : __shfl(inc, gs - 1, gs);
    const int nrows = (R - r0) < gs ? (R - r0) : gs;
    ncand += total;
    for (int base = 0; base < total; base += gs) {
      const int t = base + gl;
      int rr = 0;
      for (int step = gs >> 1; step >= 1; step >>= 1) {
        const int cand = rr + step;
        const int v = __shfl(excl, cand & (gs - 1), gs);
        if (cand < nrows && v <= t) rr = cand;
      }
      const int rst = __shfl(st, rr, gs);
      const int rex = __shfl(excl, rr, gs);
      if (t < total) {
        const int p = rst + (t - rex);
        const double dx = qx - GL(G.sx)[p], dy = qy - GL(G.sy)[p], dz = qz - GL(G.sz)[p];
        double d = dx * dx + dy * dy + dz * dz;
        if (POW) {
          const double dw = qw - GL(G.sh)[p];
          d += dw * dw;
        }
        lexmin(bd, bk, d, p);
      }
    }
  }
}

__device__ __forceinline__ void group_argmin(double &d, int &k, int gs) {
  if (gs == 64) wave_argmin(d, k);
  else row_argmin(d, k);  // gs == 16: a group is a DPP row
}

template <bool POW = false>
__device__ __forceinline__ int nn_query(const GridView &G, int gs, double qx, double qy, double qz, double r2,
                                        int k0, long long &ncand, double qw = 0.0) {
  const double lox = GL(G.geom)[0], loy = GL(G.geom)[1], loz = GL(G.geom)[2];
  const double ihx = GL(G.geom)[6], ihy = GL(G.geom)[7], ihz = GL(G.geom)[8];
  const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
  double bd = r2;
  int bk = k0;
  const int cx = cell_coord(qx, lox, ihx, gx), cy = cell_coord(qy, loy, ihy, gy), cz = cell_coord(qz, loz, ihz, gz);
  // Boxes of growing half-width R (in cells) around q's cell, each trimmed to
  // the ball of the best distance so far; stop once that ball lies inside the
  // scanned box (every site closer than the best has then been seen).  R = 1
  // is the usual 3x3x3 block; far query points double R.
  int R = 1;
  for (int round = 0; round < 32; round++) {
    const double r = sqrt(bd);
    const int X0 = cell_coord(qx - r, lox, ihx, gx), X1 = cell_coord(qx + r, lox, ihx, gx);
    const int Y0 = cell_coord(qy - r, loy, ihy, gy), Y1 = cell_coord(qy + r, loy, ihy, gy);
    const int Z0 = cell_coord(qz - r, loz, ihz, gz), Z1 = cell_coord(qz + r, loz, ihz, gz);
    const int x0 = max(cx - R, X0), x1 = min(cx + R, X1);
    const int y0 = max(cy - R, Y0), y1 = min(cy + R, Y1);
    const int z0 = max(cz - R, Z0), z1 = min(cz + R, Z1);
    scan_box<POW>(G, gs, x0, x1, y0, y1, z0, z1, qx, qy, qz, bd, bk, ncand, qw);
    group_argmin(bd, bk, gs);
    const double rn = sqrt(bd);
    const bool inside = cell_coord(qx - rn, lox, ihx, gx) >= x0 && cell_coord(qx + rn, lox, ihx, gx) <= x1 &&
                        cell_coord(qy - rn, loy, ihy, gy) >= y0 && cell_coord(qy + rn, loy, ihy, gy) <= y1 &&
                        cell_coord(qz - rn, loz, ihz, gz) >= z0 && cell_coord(qz + rn, loz, ihz, gz) <= z1;
    if (inside) break;
    R *= 2;
  }
  return bk;
}

// Single-lane nearest site of q, excluding sorted position `excl` (-1: none).
// Rings of cells around q's cell until the ring distance exceeds the best.
__device__ __forceinline__ int nn_thread(const GridView &G, double qx, double qy, double qz, int excl,
                                         double &out_d2) {
  const double lox = GL(G.geom)[0], loy = GL(G.geom)[1], loz = GL(G.geom)[2];
  const double hx = GL(G.geom)[3], hy = GL(G.geom)[4], hz = GL(G.geom)[5];
  const double ihx = GL(G.geom)[6], ihy = GL(G.geom)[7], ihz = GL(G.geom)[8];
  const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
  const int cx = cell_coord(qx, lox, ihx, gx), cy = cell_coord(qy, loy, ihy, gy),
            cz = cell_coord(qz, loz, ihz, gz);
  double bd = 1e300;
  int bk = -1;
  const double hmin = fmin(hx, fmin(hy, hz));
  const int smax = gx + gy + gz;
  for (int s = 0; s <= smax; s++) {
    bool any = false;
    for (int z = cz - s; z <= cz + s; z++) {
      if (z < 0 || z >= gz) continue;
      for (int y = cy - s; y <= cy + s; y++) {
        if (y < 0 || y >= gy) continue;
        // rows strictly inside the ring only touch it at x = cx - s and cx + s
        const bool edge = (z == cz - s || z == cz + s || y == cy - s || y == cy + s);
        const int step = edge ? 1 : 2 * s;
        for (int x = cx - s; x <= cx + s; x += step) {
          if (x < 0 || x >= gx) continue;
          any = true;
          const int c = x + gx * (y + gy * z);
          for (int p = GL(G.cstart)[c]; p < GL(G.cstart)[c + 1]; p++) {
            if (p == excl) continue;
            const double dx = qx - GL(G.sx)[p], dy = qy - GL(G.sy)[p], dz = qz - GL(G.sz)[p];
            const double d = dx * dx + dy * dy + dz * dz;
            lexmin(bd, bk, d, p);
          }
        }
      }
    }
    // sites in rings > s lie at least s*hmin away
    if (bk >= 0 && sqrt(bd) <= s * hmin) break;
    if (!any && s > 0 && bk >= 0) break;
  }
  out_d2 = bd;
  return bk;
}

// ---------------------------------------------------------------------------
// Per-wave LDS copy of the sites in a block of grid cells around the site v
// being carved, ordered by distance to v in 64 buckets of squared distance
// (bucket k: k*step <= d^2 < (k+1)*step; the last one is unbounded), in
// block order within a bucket.  Every site within rc of v is held
// (rc = distance from v to the block's boundary, less a margin for the
// rounding of cell assignment).  A query q only scans entries up to distance
// |q - v| + d from v, judged by the bucket bound of the next entry (d = best
// distance so far: farther sites cannot be
// nearer to q), and its answer is exact, with the same tie-break, when
// |q - v| + d < rc; otherwise the grid query continues from that best
// candidate.  The block is the largest one (half-width <= 8 cells) whose sites
// fit, sized from the density of the 3x3x3 block around the site.
// ---------------------------------------------------------------------------
#define VD_CACHE 128
#define VD_CACHE_SCRATCH 288  // doubles of scratch cache_fill needs (bucket starts, bucket sets)

struct SiteCache {
  double x[VD_CACHE], y[VD_CACHE], z[VD_CACHE];
  int p[VD_CACHE];
  unsigned char kb[VD_CACHE];  // distance bucket of each entry (non-decreasing)
  double step;        // bucket width in squared distance
  double vx, vy, vz;  // the site
  double rc;          // radius around the site within which every site is held
  int cnt;            // sites held; -1 = none for this site
  int b[6];           // the cell block x0, x1, y0, y1, z0, z1
};


// sites in the cell block (whole wave)
__device__ __forceinline__ int block_count(const GridView &G, int x0, int x1, int y0, int y1, int z0, int z1) {
  const int l = vd_lane();
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1, R = ny * (z1 - z0 + 1);
  int c = 0;
  for (int r = l; r < R; r += 64) {
    const int c0 = x0 + G.g[0] * ((y0 + r % ny) + G.g[1] * (z0 + r / ny));
    c += GL(G.cstart)[c0 + nx] - GL(G.cstart)[c0];
  }
  return wave_isum(c);
}

// scratch: VD_CACHE_SCRATCH doubles of LDS the caller does not use during the call
// Calls f(p, t) for every site of the cell block, p its sorted position and t
// its index in block order (rows of x-cells, contiguous site ranges); the
// whole wave takes part, lane l handling t = l, l + 64, ...
template <class F>
__device__ __forceinline__ void for_block_sites(const GridView &G, int x0, int x1, int y0, int y1, int z0, int z1,
                                                F f) {
  const int l = vd_lane();
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1, R = ny * (z1 - z0 + 1);
  int off = 0;
  for (int r0 = 0; r0 < R; r0 += 64) {
    const int rr = r0 + l;
    int st = 0, cnt = 0;
    if (rr < R) {
      const int c0 = x0 + G.g[0] * ((y0 + rr % ny) + G.g[1] * (z0 + rr / ny));
      st = GL(G.cstart)[c0];
      cnt = GL(G.cstart)[c0 + nx] - st;
    }
    const int inc = wave_incl_scan(cnt);
    const int excl = inc - cnt;
    const int total = __builtin_amdgcn_readlane(inc, 63);
    const int nrows = (R - r0) < 64 ? (R - r0) : 64;
    for (int base = 0; base < total; base += 64) {
      const int t = base + l;
      int w = 0;
      for (int step = 32; step >= 1; step >>= 1) {
        const int cand = w + step;
        const int v = __shfl(excl, cand & 63, 64);
        if (cand < nrows && v <= t) w = cand;
      }
      const int rst = __shfl(st, w, 64);
      const int rex = __shfl(excl, w, 64);
      f(t < total ? rst + (t - rex) : -1, off + t);
    }
    off += total;
  }
}

// The block is sized from the density of the 3x3x3 block around v so that it
// holds about 2.5 VD_CACHE sites.  Its sites are counted in 64 buckets of
// squared distance to v.  If more than VD_CACHE of them are in the block, only
// a prefix of buckets that fits is kept (every site with d^2 < T^2, rc = T).
// The kept sites are stored in bucket order (a counting sort; within a bucket
// in block order, so the cache is the same on every run).
__device__ void cache_fill(SiteCache &K, const GridView &G, double vx, double vy, double vz, double *scratch) {
  const int l = vd_lane();
  const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
  const int cx = cell_coord(vx, GL(G.geom)[0], GL(G.geom)[6], gx);
  const int cy = cell_coord(vy, GL(G.geom)[1], GL(G.geom)[7], gy);
  const int cz = cell_coord(vz, GL(G.geom)[2], GL(G.geom)[8], gz);
  auto cells = [&](int r) {
    return (long long)(min(cx + r, gx - 1) - max(cx - r, 0) + 1) * (min(cy + r, gy - 1) - max(cy - r, 0) + 1) *
           (min(cz + r, gz - 1) - max(cz - r, 0) + 1);
  };
  auto count = [&](int r) {
    return block_count(G, max(cx - r, 0), min(cx + r, gx - 1), max(cy - r, 0), min(cy + r, gy - 1),
                       max(cz - r, 0), min(cz + r, gz - 1));
  };
  constexpr int kMaxBlock = 4 * VD_CACHE;  // candidates read at most
  const int c1 = count(1);
  int r = 1;
  const double dens = (double)c1 / (double)cells(1);
  while (r < 8 && (c1 == 0 || dens * (double)cells(r + 1) <= 2.5 * VD_CACHE)) r++;
  int c = r == 1 ? c1 : count(r);
  while (c > kMaxBlock && r > 0) c = count(--r);
  __syncthreads();
  if (c > kMaxBlock) {
    if (l == 0) K.cnt = -1;
    __syncthreads();
    return;
  }
  const int x0 = max(cx - r, 0), x1 = min(cx + r, gx - 1), y0 = max(cy - r, 0), y1 = min(cy + r, gy - 1);
  const int z0 = max(cz - r, 0), z1 = min(cz + r, gz - 1);
  // distance from v to the block boundary (a side at the grid's edge is open),
  // less a margin for the rounding of cell assignment
  double rcb = 1e300;
  {
    const auto lo = GL(G.geom), h = GL(G.geom) + 3;
    if (x0 > 0) rcb = fmin(rcb, vx - (lo[0] + x0 * h[0]));
    if (x1 < gx - 1) rcb = fmin(rcb, lo[0] + (x1 + 1) * h[0] - vx);
    if (y0 > 0) rcb = fmin(rcb, vy - (lo[1] + y0 * h[1]));
    if (y1 < gy - 1) rcb = fmin(rcb, lo[1] + (y1 + 1) * h[1] - vy);
    if (z0 > 0) rcb = fmin(rcb, vz - (lo[2] + z0 * h[2]));
    if (z1 < gz - 1) rcb = fmin(rcb, lo[2] + (z1 + 1) * h[2] - vz);
    rcb -= 1e-9 * fmin(h[0], fmin(h[1], h[2]));
    if (rcb < 0.0) rcb = 0.0;
  }
  auto d2of = [&](int p) {
    const double ax = GL(G.sx)[p] - vx, ay = GL(G.sy)[p] - vy, az = GL(G.sz)[p] - vz;
    return ax * ax + ay * ay + az * az;
  };
  // buckets of squared distance: NB - 1 of width step over [0, rc2), the last
  // one beyond.  Range: the block's inscribed ball when some sites may have to
  // go, else (and for sides open at the grid's edge) a ball holding the block.
  constexpr int NB = 64;
  const bool select = c > VD_CACHE;
  const double hm = fmax(GL(G.geom)[3], fmax(GL(G.geom)[4], GL(G.geom)[5]));
  const double rcw2 = 3.0 * ((r + 1) * hm) * ((r + 1) * hm);
  const double rc2 = select ? fmin(rcb * rcb, rcw2) : rcw2;
  const double step = rc2 / (NB - 1);
  const double istep = rc2 > 0.0 ? (NB - 1) / rc2 : 0.0;
  auto bucket = [&](double d2) {
    int k = rc2 > 0.0 ? (int)fmin((double)(NB - 1), floor(d2 * istep)) : NB - 1;
    if (k < NB - 1 && d2 >= (k + 1) * step) k++;
    if (k > 0 && d2 < k * step) k--;
    return k;
  };
  // scratch: bucket counts (then starts), and per bucket a 256-bit set of the
  // entries in it (stable order within a bucket)
  int *hist = reinterpret_cast<int *>(scratch);
  unsigned long long *bits = reinterpret_cast<unsigned long long *>(scratch) + NB / 2;
  hist[l] = 0;
#pragma unroll
  for (int w = 0; w < 4; w++) bits[l * 4 + w] = 0ull;
  __syncthreads();
  for_block_sites(G, x0, x1, y0, y1, z0, z1, [&](int p, int) {
    if (p >= 0) atomicAdd(&hist[bucket(d2of(p))], 1);
  });
  __syncthreads();
  const int cnt = hist[l];
  const int cum = wave_incl_scan(cnt);
  // buckets 0 .. B-1 are kept (cum is non-decreasing, so the fitting lanes are a prefix)
  const int B = select ? __popcll(__ballot(l < NB - 1 && cum <= VD_CACHE)) : NB;
  const double keep2 = B * step;
  __syncthreads();
  hist[l] = cum - cnt;
  __syncthreads();
  // kept sites in block order, with their buckets
  int off = 0;
  for_block_sites(G, x0, x1, y0, y1, z0, z1, [&](int p, int) {
    int k = NB;
    if (p >= 0) k = bucket(d2of(p));
    const bool take = k < B;
    const int pos = off + wave_incl_scan(take ? 1 : 0) - (take ? 1 : 0);
    if (take) {
      K.x[pos] = GL(G.sx)[p];
      K.y[pos] = GL(G.sy)[p];
      K.z[pos] = GL(G.sz)[p];
      K.p[pos] = p;
      K.kb[pos] = (unsigned char)k;
    }
    off += __popcll(__ballot(take));
  });
  __syncthreads();
  // counting sort by bucket: position = bucket start + earlier entries of the bucket
  double ex[4], ey[4], ez[4];
  int ep[4], ek[4];
#pragma unroll
  for (int h = 0; h < 4; h++) {
    const int t = l + 64 * h;
    ex[h] = ey[h] = ez[h] = 0.0; ep[h] = 0; ek[h] = 0;
    if (t < off) {
      ex[h] = K.x[t]; ey[h] = K.y[t]; ez[h] = K.z[t]; ep[h] = K.p[t]; ek[h] = K.kb[t];
      atomicOr(&bits[ek[h] * 4 + h], 1ull << l);
    }
  }
  __syncthreads();
  int rk[4];
#pragma unroll
  for (int h = 0; h < 4; h++) {
    rk[h] = 0;
    if (l + 64 * h < off) {
      int r0 = hist[ek[h]];
      for (int w = 0; w < h; w++) r0 += __popcll(bits[ek[h] * 4 + w]);
      rk[h] = r0 + __popcll(bits[ek[h] * 4 + h] & low_mask_lt(l));
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 4; h++) {
    if (l + 64 * h < off) {
      K.x[rk[h]] = ex[h]; K.y[rk[h]] = ey[h]; K.z[rk[h]] = ez[h]; K.p[rk[h]] = ep[h];
      K.kb[rk[h]] = (unsigned char)ek[h];
    }
  }
  if (l == 0) {
    // every site within rc of v is held; the block test holds only when the
    // whole block was kept
    K.rc = select ? fmin(rcb, sqrt(keep2) * (1.0 - 1e-12)) : rcb;
    K.step = step;
    K.vx = vx; K.vy = vy; K.vz = vz;
    K.cnt = off;
    K.b[0] = x0; K.b[1] = x1; K.b[2] = y0; K.b[3] = y1; K.b[4] = z0; K.b[5] = z1;
    if (select) { K.b[0] = 1; K.b[1] = 0; }  // an empty x-range: never inside
  }
  __syncthreads();
}

// Point-in-cell query of q (group of gs lanes, q uniform in the group) for the
// site k0 at squared distance r2 from q, where the sites e0, e1, e2 (-1: none)
// are those the caller treats like k0 (the flags of the planes through q).
// Returns either the nearest site of q (ties to the lowest sorted position) or
// a witness: a cached site strictly nearer to q than k0 and every e.  A witness
// decides the caller's test as the nearest site would (the nearest site is
// then none of k0, e0, e1, e2), and it is a valid next site for the bisector
// search, which only needs a site nearer to its outer point than v_i.
// Distances are computed by one formula everywhere, so "strictly nearer"
// holds for the nearest site too.
// sqrt(x) to about 1e-13 relative (hardware reciprocal square root and one
// Newton step), for bounds that carry a wider margin of their own
__device__ __forceinline__ double sqrt_bound(double x) {
  if (!(x > 0.0)) return 0.0;
  const double r = __builtin_amdgcn_rsq(x);
  const double s0 = x * r;
  return fma(0.5 * r, fma(-s0, s0, x), s0);
}

__device__ __forceinline__ double sq_dist(const GridView &G, int e, double qx, double qy, double qz) {
  const double dx = qx - GL(G.sx)[e], dy = qy - GL(G.sy)[e], dz = qz - GL(G.sz)[e];
  return dx * dx + dy * dy + dz * dz;
}

// Squared distance from q to site e, from its cache slot `slot` when it has
// one (the cache holds exact copies of the coordinates, so both give the same
// value), else from the grid's arrays.
__device__ __forceinline__ double sq_dist_at(const SiteCache &K, const GridView &G, int e, int slot, double qx,
                                             double qy, double qz) {
  if (slot >= 0) {
    const double dx = qx - K.x[slot], dy = qy - K.y[slot], dz = qz - K.z[slot];
    return dx * dx + dy * dy + dz * dz;
  }
  return sq_dist(G, e, qx, qy, qz);
}

// Cache slot of site k (sorted position), or -1: the whole wave compares the
// held positions (at most VD_CACHE, two per lane).
__device__ __forceinline__ int cache_slot(const SiteCache &K, int k) {
  const int n = K.cnt, l = vd_lane();
  if (n <= 0 || k < 0) return -1;
  const bool a = l < n && K.p[l] == k;
  const bool b = l + 64 < n && K.p[l + 64] == k;
  const uint64_t ma = __ballot(a), mb = __ballot(b);
  if (ma) return __ffsll((unsigned long long)ma) - 1;
  if (mb) return 64 + __ffsll((unsigned long long)mb) - 1;
  return -1;
}

// es0..es2: the cache slots of e0..e2 (-1: not cached, or no such site).
__device__ __forceinline__ int nn_cached(const SiteCache &K, const GridView &G, int gs, double qx, double qy,
                                         double qz, double r2, int k0, int e0, int e1, int e2, int es0, int es1,
                                         int es2, long long &ncand, bool &on_grid) {
  const int n = K.cnt;
  on_grid = false;
  if (n >= 0) {
    const int gl = vd_lane() & (gs - 1);
    const double wx = qx - K.vx, wy = qy - K.vy, wz = qz - K.vz;
    const double dq = sqrt(wx * wx + wy * wy + wz * wz);
    double wit = r2;
    if (e0 >= 0) wit = fmin(wit, sq_dist_at(K, G, e0, es0, qx, qy, qz));
    if (e1 >= 0) wit = fmin(wit, sq_dist_at(K, G, e1, es1, qx, qy, qz));
    if (e2 >= 0) wit = fmin(wit, sq_dist_at(K, G, e2, es2, qx, qy, qz));
    double bd = r2;
    int bk = k0;
    for (int base = 0; base < n; base += gs) {
      const int t = base + gl;
      if (t < n) {
        const double dx = qx - K.x[t], dy = qy - K.y[t], dz = qz - K.z[t];
        const double d = dx * dx + dy * dy + dz * dz;
        const int p = K.p[t];
        lexmin(bd, bk, d, p);
      }
      group_argmin(bd, bk, gs);
      ncand += (n - base) < gs ? (n - base) : gs;
      if (bd < wit) return bk;  // witness
      const int u = base + gs;
      if (u >= n) break;
      // entries from u on lie at least sqrt(kb[u] * step) from v: stop once
      // that exceeds |q - v| + d
      const double reach = (dq + sqrt_bound(bd)) * (1.0 + 1e-9);
      if ((double)K.kb[u] * K.step * (1.0 - 1e-12) > reach * reach) break;
    }
    const double rn = sqrt(bd);
    if ((dq + rn) * (1.0 + 1e-12) < K.rc) return bk;
    // or the ball of q lies inside the block (same cell arithmetic as the
    // grid's binning): every site in it is cached, and every cached site in
    // it lies within |q - v| + d of v, so it was scanned
    {
      const double r = rn * (1.0 + 1e-12);
      const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
      if (cell_coord(qx - r, GL(G.geom)[0], GL(G.geom)[6], gx) >= K.b[0] && cell_coord(qx + r, GL(G.geom)[0], GL(G.geom)[6], gx) <= K.b[1] &&
          cell_coord(qy - r, GL(G.geom)[1], GL(G.geom)[7], gy) >= K.b[2] && cell_coord(qy + r, GL(G.geom)[1], GL(G.geom)[7], gy) <= K.b[3] &&
          cell_coord(qz - r, GL(G.geom)[2], GL(G.geom)[8], gz) >= K.b[4] && cell_coord(qz + r, GL(G.geom)[2], GL(G.geom)[8], gz) <= K.b[5])
        return bk;
    }
    r2 = bd;
    k0 = bk;
  }
  on_grid = true;
  return nn_query(G, gs, qx, qy, qz, r2, k0, ncand);
}

