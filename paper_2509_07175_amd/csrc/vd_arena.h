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
// L2.  A wave whose queue is exhausted moves on to the next queue.
#pragma once
#include "vd_internal.h"

struct WaveArena {
  long long cur[AR_N], end[AR_N];
  unsigned long long queries, cands, clips, gridq;
  unsigned long long pieces, faces, verts, nbrs;  // records written (real counts)
  int qi;                                         // queues tried so far
};

__device__ __forceinline__ void arena_init(WaveArena &A) {
  if (vd_lane() == 0) {
    for (int r = 0; r < AR_N; r++) A.cur[r] = A.end[r] = 0;
    A.queries = A.cands = A.clips = A.gridq = 0;
    A.pieces = A.faces = A.verts = A.nbrs = 0;
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
      const long long end = (k + 1) * q8 < n ? (k + 1) * q8 : n;
      if (k * q8 >= end) continue;
      const int v = __hip_atomic_fetch_add(GL(C.queue) + k * VD_QSTRIDE, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v < end) { r = v; break; }
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
  }
}
