// cells.hip -- output compaction and per-site moments.
//
// The clip kernels write pieces and per-site lists into chunks of shared
// arenas, so records sit anywhere in their arenas (unused piece slots carry
// site -1).  Finalize turns them into CSR: an exclusive scan of the per-site
// counts, then each site's list copied (neighbours) or ranked (pieces, by
// simplex) into place.  Moments convert
// the per-site mass / first moment / energy sums (accumulated in a fixed order
// inside each wave) into mass, centroid and energy.
#include <algorithm>
#include <climits>

#include "vd_internal.h"
#include "vd_scan.h"

namespace {

constexpr int kB = 256;
inline unsigned blocks(long long n) { return (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1); }

// Per-site lists from their arena runs into CSR: a 16-lane group copies one
// site's list (consecutive lanes, consecutive entries), four sites per wave.
constexpr int kGroup = 16;
__global__ void __launch_bounds__(kB) gather_lists(long long n, const int *__restrict__ count,
                                                   const long long *__restrict__ start,
                                                   const int *__restrict__ arena,
                                                   const long long *__restrict__ off,
                                                   int *__restrict__ out) {
  const long long t = (long long)blockIdx.x * kB + threadIdx.x;
  const long long i = t / kGroup;
  const int gl = (int)(t % kGroup);
  if (i >= n) return;
  const long long o = off[i], s = start[i];
  const int c = count[i];
  for (int k = gl; k < c; k += kGroup) out[o + k] = arena[s + k];
}

// 3D pieces: a site's pieces fill a run of consecutive slots of its wave's
// piece chunk, unless the chunk ran out during the site (then two or more
// runs).  Counts each site's runs (nrun) and keeps a run's first slot in the
// low half of run[s].  Slots in use: the arena's high-water mark (read on the
// device, so the launch needs no host copy of it), at most its capacity.
__global__ void __launch_bounds__(kB) piece_runs(const unsigned long long *__restrict__ cnt, long long cap,
                                                 const int *__restrict__ site, int *__restrict__ nrun,
                                                 unsigned long long *__restrict__ run) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  const long long used = (long long)cnt[CNT_PIECES];
  if (p >= (used < cap ? used : cap)) return;
  const int s = site[p];
  if (s < 0 || (p > 0 && site[p - 1] == s)) return;  // unused slot, or not the first of a run
  atomicAdd(&nrun[s], 1);
  run[s] = (unsigned long long)p;
}

// Pieces grouped by site (counting sort): every piece, or (nrun given) only
// those of sites with more than one run, whose positions are counted in the
// high half of run[s].
__global__ void __launch_bounds__(kB) scatter_pieces(const unsigned long long *__restrict__ cnt, long long cap,
                                                     const int *__restrict__ site,
                                                     const long long *__restrict__ off, int *__restrict__ fill,
                                                     const int *__restrict__ nrun, unsigned long long *__restrict__ run,
                                                     int *__restrict__ out) {
  const long long p = (long long)blockIdx.x * kB + threadIdx.x;
  const long long used = (long long)cnt[CNT_PIECES];
  if (p >= (used < cap ? used : cap)) return;
  const int s = site[p];
  if (s < 0) return;  // unused slot of a wave's chunk
  if (!nrun) {
    out[off[s] + atomicAdd(&fill[s], 1)] = (int)p;
  } else if (nrun[s] > 1) {
    out[off[s] + (long long)(atomicAdd(&run[s], 1ull << 32) >> 32)] = (int)p;
  }
}

// Each site's pieces by ascending simplex index into the CSR `out`: a piece's
// position is the number of the site's pieces with a smaller key (a site has
// at most one piece per simplex; equal keys would keep their source order).
// A site's pieces come from its single run of slots (r >= 0: slots r, r+1,
// ...) or from `in` at its CSR offset (grouped by scatter_pieces).  Sites have
// from one to a few hundred pieces, so a 16-lane group ranks a site of up to
// 16 pieces by lane shuffles, four sites per wave, and the whole wave takes
// the larger ones, 64 pieces at a time against all of the site's keys.
constexpr int kSortWaves = kB / 64;
constexpr int kSmall = 16;
__device__ __forceinline__ int piece_at(long long r, const int *__restrict__ in, long long a, int x) {
  return r >= 0 ? (int)(r + x) : in[a + x];
}

__device__ __forceinline__ void rank_segment_wave(long long a, long long r, int k, const int *__restrict__ simplex,
                                                  const int *__restrict__ in, int *__restrict__ out) {
  const int l = threadIdx.x & 63;
  for (int x0 = 0; x0 < k; x0 += 64) {
    const int x = x0 + l;
    int id = 0, key = INT_MAX;
    if (x < k) {
      id = piece_at(r, in, a, x);
      key = simplex[id];
    }
    int rk = 0;
    for (int y0 = 0; y0 < k; y0 += 64) {
      int ky = key;
      if (y0 != x0) ky = y0 + l < k ? simplex[piece_at(r, in, a, y0 + l)] : INT_MAX;
      const int lim = k - y0 < 64 ? k - y0 : 64;
      for (int o = 0; o < lim; o++) {
        const int kk = __builtin_amdgcn_readlane(ky, o);
        rk += (kk < key || (kk == key && y0 + o < x)) ? 1 : 0;
      }
    }
    if (x < k) out[a + rk] = id;
  }
}

__device__ __forceinline__ long long readlane64(long long v, int src) {
  return ((long long)__builtin_amdgcn_readlane((int)(v >> 32), src) << 32) |
         (unsigned)__builtin_amdgcn_readlane((int)v, src);
}

// nrun / run: the runs of piece_runs (3D), or NULL (every site from `in`)
__global__ void __launch_bounds__(kB) sort_segments(long long n, const long long *__restrict__ off,
                                                    const int *__restrict__ simplex, const int *__restrict__ nrun,
                                                    const unsigned long long *__restrict__ run,
                                                    const int *__restrict__ in, int *__restrict__ out) {
  const int l = threadIdx.x & 63, g = l / kSmall, gl = l % kSmall;
  const long long nw = (long long)gridDim.x * kSortWaves;
  for (long long s0 = ((long long)blockIdx.x * kSortWaves + threadIdx.x / 64) * 4; s0 < n; s0 += 4 * nw) {
    const long long s = s0 + g;
    long long a = 0, r = -1;
    int k = 0;
    if (s < n) {
      a = off[s];
      k = (int)(off[s + 1] - a);
      if (nrun && k > 0 && nrun[s] == 1) r = (long long)(run[s] & 0xffffffffull);
    }
    const bool small = k <= kSmall;
    int id = 0, key = INT_MAX;
    if (small && gl < k) {
      id = piece_at(r, in, a, gl);
      key = simplex[id];
    }
    int rk = 0;
#pragma unroll
    for (int o = 0; o < kSmall; o++) {
      const int kk = __shfl(key, (l & ~(kSmall - 1)) + o, 64);
      rk += (kk < key || (kk == key && o < gl)) ? 1 : 0;
    }
    if (small && gl < k) out[a + rk] = id;
    for (uint64_t big = __ballot(!small && gl == 0); big; big &= big - 1) {
      const int src = __ffsll((unsigned long long)big) - 1;
      rank_segment_wave(readlane64(a, src), readlane64(r, src), __builtin_amdgcn_readlane(k, src), simplex, in, out);
    }
  }
}

__global__ void __launch_bounds__(kB) moments_kernel(long long n, const int *__restrict__ rank,
                                                     const double *__restrict__ sx, const double *__restrict__ sy,
                                                     const double *__restrict__ sz, const double *__restrict__ mass,
                                                     const double *__restrict__ mom, const double *__restrict__ en,
                                                     double *__restrict__ out_m, double *__restrict__ out_c,
                                                     double *__restrict__ out_e) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const double m = mass[i];
  if (out_m) out_m[i] = m;
  if (out_c) {
    if (m > 0.0) {
      const double im = 1.0 / m;
      out_c[3 * i + 0] = mom[3 * i + 0] * im;
      out_c[3 * i + 1] = mom[3 * i + 1] * im;
      out_c[3 * i + 2] = mom[3 * i + 2] * im;
    } else {
      const int p = rank[i];
      out_c[3 * i + 0] = sx[p];
      out_c[3 * i + 1] = sy[p];
      out_c[3 * i + 2] = sz[p];
    }
  }
  if (out_e) out_e[i] = m > 0.0 ? en[i] : 0.0;
}

}  // namespace

void vd_launch_fill_int(int *p, long long n, int v, hipStream_t st);

void vd_launch_finalize(vd_cells c, hipStream_t st) {
  const long long n = c->n;
  const CellsDev &d = c->d;
  // slots to scan: the high-water mark when the host has read it, else the capacity
  const long long npieces = c->pending ? d.cap_piece : std::min<long long>((long long)c->host_cnt[CNT_PIECES], d.cap_piece);
  const unsigned long long *cnt = (const unsigned long long *)d.cnt;
  const long long groups = (n + 4 * kSortWaves - 1) / (4 * kSortWaves);
  const unsigned nsort = (unsigned)std::max<long long>(1, std::min<long long>(groups, 8192));
  vdscan::exclusive_scan<int, long long>(d.pcount, n, c->piece_off, c->scan_tmp, st);
  vd_launch_fill_int(c->fillc, n, 0, st);
  if (c->dim == 3) {
    // each site's pieces from its run of slots, ranked by simplex; the few
    // sites whose pieces span runs are grouped first
    unsigned long long *run = reinterpret_cast<unsigned long long *>(d.pstart);
    hipLaunchKernelGGL(piece_runs, dim3(blocks(npieces)), dim3(kB), 0, st, cnt, (long long)d.cap_piece,
                       (const int *)d.piece_site, c->fillc, run);
    hipLaunchKernelGGL(scatter_pieces, dim3(blocks(npieces)), dim3(kB), 0, st, cnt, (long long)d.cap_piece,
                       (const int *)d.piece_site, (const long long *)c->piece_off, c->fillc,
                       (const int *)c->fillc, run, c->pid_tmp);
    hipLaunchKernelGGL(sort_segments, dim3(nsort), dim3(kB), 0, st, n, (const long long *)c->piece_off,
                       (const int *)d.piece_simplex, (const int *)c->fillc, (const unsigned long long *)run,
                       (const int *)c->pid_tmp, c->piece_id);
    vdscan::exclusive_scan<int, long long>(d.ncount, n, c->nbr_off, c->scan_tmp, st);
    hipLaunchKernelGGL(gather_lists, dim3(blocks(n * kGroup)), dim3(kB), 0, st, n, (const int *)d.ncount,
                       (const long long *)d.nstart, (const int *)d.nbr_arena, (const long long *)c->nbr_off,
                       c->nbr);
    return;
  }
  // surfaces (pieces are emitted per triangle): counting sort of the pieces
  // by site, then by simplex inside each site
  hipLaunchKernelGGL(scatter_pieces, dim3(blocks(npieces)), dim3(kB), 0, st, cnt, (long long)d.cap_piece,
                     (const int *)d.piece_site, (const long long *)c->piece_off, c->fillc, (const int *)nullptr,
                     (unsigned long long *)nullptr, c->pid_tmp);
  hipLaunchKernelGGL(sort_segments, dim3(nsort), dim3(kB), 0, st, n, (const long long *)c->piece_off,
                     (const int *)d.piece_simplex, (const int *)nullptr, (const unsigned long long *)nullptr,
                     (const int *)c->pid_tmp, c->piece_id);
  // per-site sums and neighbour lists from the pieces, in CSR order
  vd_launch_site_reduce(n, c->piece_off, c->piece_id, c->d_dev, st);
  vdscan::exclusive_scan<int, long long>(d.ncount, n, c->nbr_off, c->scan_tmp, st);
  vd_launch_site_nbrs(n, c->piece_off, c->piece_id, c->nbr_off, c->nbr, c->cap_nbr_csr, c->d_dev, st);
}

void vd_launch_moments(const vd_cells_s *c, const GridView &G, double *mass, double *cent, double *energy,
                       hipStream_t st) {
  const long long n = c->n;
  vd_grid g = c->grid;
  hipLaunchKernelGGL(moments_kernel, dim3(blocks(n)), dim3(kB), 0, st, n, (const int *)g->rank,
                     G.sx, G.sy, G.sz, (const double *)c->d.mass, (const double *)c->d.mom,
                     (const double *)c->d.energy, mass, cent, energy);
}
