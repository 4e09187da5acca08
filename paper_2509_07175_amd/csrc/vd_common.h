// vd_common.h -- device-side building blocks shared by the kernels.
//
// gfx950 (CDNA4), wave64.  Geometry is float64 throughout (FP64 vector ALU is
// full rate on this chip); nothing here is a dense contraction, so no MFMA.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define VD_WAVE 64
#define VD_BND_BASE (-2147483647 - 1)

// Device view of the nearest-site grid (Sec. 6.2).  Sites are stored in cell
// order; "sorted position" indexes sx/sy/sz/delta, perm maps it back to the
// caller's index.  geom = {lo[3], h[3], ih[3]} lives in device memory because
// the bounding box is reduced on the device.
struct GridView {
  int n;
  int g[3];
  const double *geom;
  const double *sx, *sy, *sz;
  const int *cstart;  // [g0*g1*g2 + 1]
  const int *perm;    // sorted position -> caller index
  const double *delta;  // half nearest-other-site distance, by sorted position
};

__device__ __forceinline__ int vd_lane() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ bool bit128(uint64_t lo, uint64_t hi, int s) {
  return s < 64 ? ((lo >> s) & 1ull) : ((hi >> (s - 64)) & 1ull);
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = vd_lane();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int o = __shfl_up(v, d, 64);
    if (l >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo |= (unsigned)__shfl_xor((int)lo, m, 64);
    hi |= (unsigned)__shfl_xor((int)hi, m, 64);
    v = ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// Lexicographic (distance^2, sorted position) minimum over the wave; every
// lane ends with the result.
__device__ __forceinline__ void wave_argmin(double &d, int &k) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    double od = __shfl_xor(d, m, 64);
    int ok = __shfl_xor(k, m, 64);
    if (od < d || (od == d && ok < k)) { d = od; k = ok; }
  }
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
__device__ __forceinline__ void scan_box(const GridView &G, int gs, int x0, int x1, int y0, int y1, int z0,
                                         int z1, double qx, double qy, double qz, double &bd, int &bk,
                                         long long &ncand) {
  const int gl = vd_lane() & (gs - 1);
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  const int R = ny * (z1 - z0 + 1);
  for (int r0 = 0; r0 < R; r0 += gs) {
    const int r = r0 + gl;
    int st = 0, cnt = 0;
    if (r < R) {
      const int yy = y0 + r % ny, zz = z0 + r / ny;
      const int c0 = x0 + G.g[0] * (yy + G.g[1] * zz);
      st = G.cstart[c0];
      cnt = G.cstart[c0 + nx] - st;
    }
    int inc = cnt;
    for (int d = 1; d < gs; d <<= 1) {
      const int o = __shfl_up(inc, d, gs);
      if (gl >= d) inc += o;
    }
    const int excl = inc - cnt;
    const int total = __shfl(inc, gs - 1, gs);
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
        const double dx = qx - G.sx[p], dy = qy - G.sy[p], dz = qz - G.sz[p];
        const double d = dx * dx + dy * dy + dz * dz;
        if (d < bd || (d == bd && p < bk)) { bd = d; bk = p; }
      }
    }
  }
}

__device__ __forceinline__ void group_argmin(double &d, int &k, int gs) {
  for (int m = gs >> 1; m >= 1; m >>= 1) {
    const double od = __shfl_xor(d, m, 64);
    const int ok = __shfl_xor(k, m, 64);
    if (od < d || (od == d && ok < k)) { d = od; k = ok; }
  }
}

__device__ __forceinline__ int nn_query(const GridView &G, int gs, double qx, double qy, double qz, double r2,
                                        int k0, long long &ncand) {
  const double lox = G.geom[0], loy = G.geom[1], loz = G.geom[2];
  const double ihx = G.geom[6], ihy = G.geom[7], ihz = G.geom[8];
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
    scan_box(G, gs, x0, x1, y0, y1, z0, z1, qx, qy, qz, bd, bk, ncand);
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
  const double lox = G.geom[0], loy = G.geom[1], loz = G.geom[2];
  const double hx = G.geom[3], hy = G.geom[4], hz = G.geom[5];
  const double ihx = G.geom[6], ihy = G.geom[7], ihz = G.geom[8];
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
          for (int p = G.cstart[c]; p < G.cstart[c + 1]; p++) {
            if (p == excl) continue;
            const double dx = qx - G.sx[p], dy = qy - G.sy[p], dz = qz - G.sz[p];
            const double d = dx * dx + dy * dy + dz * dz;
            if (d < bd || (d == bd && p < bk)) { bd = d; bk = p; }
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
// Per-wave LDS copy of the sites in a block of grid cells around the site
// being carved.  A query whose ball (centre q, radius = best distance found in
// the copy) lies inside the block has its exact answer, with the same
// tie-break, from the copy alone; otherwise the grid query continues from that
// best candidate.  The block is the largest one (half-width <= 8 cells) whose
// sites fit, sized from the density of the 3x3x3 block around the site.
// ---------------------------------------------------------------------------
#define VD_CACHE 224

struct SiteCache {
  double x[VD_CACHE], y[VD_CACHE], z[VD_CACHE];
  int p[VD_CACHE];
  int cnt;   // sites held; -1 = none for this site
  int b[6];  // cell block x0, x1, y0, y1, z0, z1
};

__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// sites in the cell block (whole wave)
__device__ __forceinline__ int block_count(const GridView &G, int x0, int x1, int y0, int y1, int z0, int z1) {
  const int l = vd_lane();
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1, R = ny * (z1 - z0 + 1);
  int c = 0;
  for (int r = l; r < R; r += 64) {
    const int c0 = x0 + G.g[0] * ((y0 + r % ny) + G.g[1] * (z0 + r / ny));
    c += G.cstart[c0 + nx] - G.cstart[c0];
  }
  return wave_isum(c);
}

__device__ void cache_fill(SiteCache &K, const GridView &G, double vx, double vy, double vz) {
  const int l = vd_lane();
  const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
  const int cx = cell_coord(vx, G.geom[0], G.geom[6], gx);
  const int cy = cell_coord(vy, G.geom[1], G.geom[7], gy);
  const int cz = cell_coord(vz, G.geom[2], G.geom[8], gz);
  auto cells = [&](int r) {
    return (long long)(min(cx + r, gx - 1) - max(cx - r, 0) + 1) * (min(cy + r, gy - 1) - max(cy - r, 0) + 1) *
           (min(cz + r, gz - 1) - max(cz - r, 0) + 1);
  };
  auto count = [&](int r) {
    return block_count(G, max(cx - r, 0), min(cx + r, gx - 1), max(cy - r, 0), min(cy + r, gy - 1),
                       max(cz - r, 0), min(cz + r, gz - 1));
  };
  const int c1 = count(1);
  int r = 1;
  const double dens = (double)c1 / (double)cells(1);
  while (r < 8 && (c1 == 0 || dens * (double)cells(r + 1) <= 0.7 * VD_CACHE)) r++;
  int c = r == 1 ? c1 : count(r);
  while (c > VD_CACHE && r > 0) c = count(--r);
  __syncthreads();
  if (c > VD_CACHE) {
    if (l == 0) K.cnt = -1;
    __syncthreads();
    return;
  }
  const int x0 = max(cx - r, 0), x1 = min(cx + r, gx - 1), y0 = max(cy - r, 0), y1 = min(cy + r, gy - 1);
  const int z0 = max(cz - r, 0), z1 = min(cz + r, gz - 1);
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1, R = ny * (z1 - z0 + 1);
  int off = 0;
  for (int r0 = 0; r0 < R; r0 += 64) {
    const int rr = r0 + l;
    int st = 0, cnt = 0;
    if (rr < R) {
      const int c0 = x0 + gx * ((y0 + rr % ny) + gy * (z0 + rr / ny));
      st = G.cstart[c0];
      cnt = G.cstart[c0 + nx] - st;
    }
    const int inc = wave_incl_scan(cnt);
    const int excl = inc - cnt;
    const int total = __shfl(inc, 63, 64);
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
      if (t < total) {
        const int p = rst + (t - rex);
        K.x[off + t] = G.sx[p];
        K.y[off + t] = G.sy[p];
        K.z[off + t] = G.sz[p];
        K.p[off + t] = p;
      }
    }
    off += total;
  }
  if (l == 0) {
    K.cnt = off;
    K.b[0] = x0; K.b[1] = x1; K.b[2] = y0; K.b[3] = y1; K.b[4] = z0; K.b[5] = z1;
  }
  __syncthreads();
}

// nearest site of q (group of gs lanes, q uniform in the group), seeded with
// the candidate (r2, k0); exact, ties to the lowest sorted position
__device__ __forceinline__ int nn_cached(const SiteCache &K, const GridView &G, int gs, double qx, double qy,
                                         double qz, double r2, int k0, long long &ncand) {
  const int n = K.cnt;
  if (n >= 0) {
    const int gl = vd_lane() & (gs - 1);
    double bd = r2;
    int bk = k0;
    for (int t = gl; t < n; t += gs) {
      const double dx = qx - K.x[t], dy = qy - K.y[t], dz = qz - K.z[t];
      const double d = dx * dx + dy * dy + dz * dz;
      const int p = K.p[t];
      if (d < bd || (d == bd && p < bk)) { bd = d; bk = p; }
    }
    group_argmin(bd, bk, gs);
    ncand += n;
    const double rn = sqrt(bd);
    const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
    const bool inside = cell_coord(qx - rn, G.geom[0], G.geom[6], gx) >= K.b[0] &&
                        cell_coord(qx + rn, G.geom[0], G.geom[6], gx) <= K.b[1] &&
                        cell_coord(qy - rn, G.geom[1], G.geom[7], gy) >= K.b[2] &&
                        cell_coord(qy + rn, G.geom[1], G.geom[7], gy) <= K.b[3] &&
                        cell_coord(qz - rn, G.geom[2], G.geom[8], gz) >= K.b[4] &&
                        cell_coord(qz + rn, G.geom[2], G.geom[8], gz) <= K.b[5];
    if (inside) return bk;
    r2 = bd;
    k0 = bk;
  }
  return nn_query(G, gs, qx, qy, qz, r2, k0, ncand);
}

