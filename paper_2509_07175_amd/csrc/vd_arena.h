// vd_arena.h -- per-wave output allocation and the work queue of the
// persistent clip kernels.
//
// A persistent wave processes many sites (or triangles).  Its output records
// go to arenas shared by all waves; instead of one global atomic per record
// (which serialises every wave on a handful of addresses), a wave reserves a
// chunk of C.chunk[r] slots with one atomic and hands out slots from it.  The
// unused tail of the last piece chunk is marked piece_site = -1 when the wave
// ends; face/vertex/neighbour/face-moment records are reached through offsets
// only, so their holes need no marking.
//
// Work items come from VD_QUEUES queues, queue k owning the k-th eighth of the
// items in order; workgroup b starts on queue b % 8 (the XCD it runs on when
// workgroups are dealt round-robin over the 8 XCDs), so an XCD works through a
// contiguous block of grid-ordered sites and keeps their neighbourhoods in its
// L2.  A wave whose queue is exhausted moves on to the next queue.  A batch
// can instead give each queue a list of positions (C.order), so that every
// queue starts with its most expensive diagrams.
#pragma once
#include "vd_internal.h"

struct WaveArena {
  long long cur[AR_N], end[AR_N];
  unsigned long long queries, cands, clips, gridq;
  unsigned long long pieces, faces, verts, nbrs;  // records written (real counts)
  unsigned long long dropped;                     // records that did not fit their arena
  // work counters of the clips (lane 0 updates them in LDS, so they cost no
  // registers across the carve)
  unsigned long long rounds, classified, newc, wasted, fantets, lowmargin;
  double minmargin;                               // smallest relative classification margin
  int qi;                                         // queues tried so far
};

__device__ __forceinline__ void arena_init(WaveArena &A) {
  if (vd_lane() == 0) {
    for (int r = 0; r < AR_N; r++) A.cur[r] = A.end[r] = 0;
    A.queries = A.cands = A.clips = A.gridq = 0;
    A.pieces = A.faces = A.verts = A.nbrs = 0;
    A.dropped = 0;
    A.rounds = A.classified = A.newc = A.wasted = A.fantets = A.lowmargin = 0;
    A.minmargin = 1.0;
    A.qi = 0;
  }
}

// k slots of arena r for this wave (k and r uniform); returns the first slot.
// The returned range may reach past the arena's capacity: callers check.
__device__ __forceinline__ long long arena_take(WaveArena &A, const CellsDev &C, int r, long long k) {
  long long o = 0;
  if (vd_lane() == 0) {
    long long cur = A.cur[r];
    if (cur + k > A.end[r]) {
      const long long t = k > C.chunk[r] ? k : C.chunk[r];
      cur = (long long)__hip_atomic_fetch_add(GL(C.cnt) + r, (unsigned long long)t, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
      A.end[r] = cur + t;
    }
    A.cur[r] = cur + k;
    o = cur;
  }
  return readlane_ll(o, 0);
}

// Next work item in [0, n), or -1 when every queue is exhausted.
__device__ __forceinline__ int queue_next(WaveArena &A, const CellsDev &C, long long n) {
  int r = -1;
  if (vd_lane() == 0) {
    const long long q8 = (n + VD_QUEUES - 1) / VD_QUEUES;
    const int x = (int)(blockIdx.x % VD_QUEUES);
    for (; A.qi < VD_QUEUES; A.qi++) {
      const int k = (x + A.qi) % VD_QUEUES;
      const long long beg = C.order ? C.qoff[k] : k * q8;
      const long long end = C.order ? C.qoff[k + 1] : ((k + 1) * q8 < n ? (k + 1) * q8 : n);
      if (beg >= end) continue;
      const int v = __hip_atomic_fetch_add(GL(C.queue) + k * VD_QSTRIDE, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v < end) { r = C.order ? GL(C.order)[v] : v; break; }
    }
  }
  return __builtin_amdgcn_readlane(r, 0);
}

// End of a persistent wave: mark the unused tail of its piece chunk and add
// its statistics to the global counters.
__device__ __forceinline__ void arena_close(WaveArena &A, const CellsDev &C) {
  const int l = vd_lane();
  const long long a = A.cur[AR_PIECE], b = A.end[AR_PIECE] < C.cap_piece ? A.end[AR_PIECE] : C.cap_piece;
  for (long long p = a + l; p < b; p += 64) GL(C.piece_site)[p] = -1;
  if (l == 0) {
    atomicAdd(&C.cnt[CNT_QUERIES], A.queries);
    atomicAdd(&C.cnt[CNT_CANDS], A.cands);
    atomicAdd(&C.cnt[CNT_CLIPS], A.clips);
    atomicAdd(&C.cnt[CNT_GRIDQ], A.gridq);
    atomicAdd(&C.cnt[CNT_REAL_PIECES], A.pieces);
    atomicAdd(&C.cnt[CNT_REAL_FACES], A.faces);
    atomicAdd(&C.cnt[CNT_REAL_VERTS], A.verts);
    atomicAdd(&C.cnt[CNT_REAL_NBRS], A.nbrs);
    if (A.dropped) atomicAdd(&C.cnt[CNT_OVERFLOW], A.dropped);
    atomicAdd(&C.cnt[CNT_ROUNDS], A.rounds);
    atomicAdd(&C.cnt[CNT_CLASSIFIED], A.classified);
    atomicAdd(&C.cnt[CNT_NEWCORNERS], A.newc);
    atomicAdd(&C.cnt[CNT_WASTED], A.wasted);
    atomicAdd(&C.cnt[CNT_FANTETS], A.fantets);
    if (A.lowmargin) atomicAdd(&C.cnt[CNT_LOWMARGIN], A.lowmargin);
    atomicMin(&C.cnt[CNT_MINMARGIN], (unsigned long long)__double_as_longlong(A.minmargin));
  }
}

// Adds v to a work counter of the wave's LDS totals: an LDS atomic from lane 0
// whose result is unused, so nothing waits for it and no register stays live.
__device__ __forceinline__ void count_add(unsigned long long &ctr, unsigned long long v) {
  if (vd_lane() == 0) __hip_atomic_fetch_add(&ctr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Relative margin of the classification of corners y against the plane
// n.y = c: |n.y - c| / (|n0 y0| + |n1 y1| + |n2 y2| + |c|), the signed distance
// over the magnitude its rounding error scales with.  Each lane brings up to two
// corners (valid flag, signed distance, scale).  Lane 0 keeps the wave's minimum
// and the count of margins below 1e-12 (near-degenerate decisions); the
// division is only taken when some corner is within 1e-3 of its plane.
__device__ __forceinline__ void margin_track(WaveArena &A, bool v0, double sd0, double sc0, bool v1, double sd1,
                                             double sc1) {
  const bool n0 = v0 && fabs(sd0) < 1e-3 * sc0, n1 = v1 && fabs(sd1) < 1e-3 * sc1;
  if (__ballot(n0 || n1)) {
    const int nlow = __popcll(__ballot(v0 && fabs(sd0) < 1e-12 * sc0)) + __popcll(__ballot(v1 && fabs(sd1) < 1e-12 * sc1));
    double r = n0 ? fabs(sd0) / sc0 : 1.0;
    if (n1) r = fmin(r, fabs(sd1) / sc1);
    r = wave_min(r);
    if (vd_lane() == 0) {
      A.lowmargin += nlow;
      if (r < A.minmargin) A.minmargin = r;
    }
  }
}
