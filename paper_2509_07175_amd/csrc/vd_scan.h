// vd_scan.h -- device-wide exclusive prefix sum (three launches, no host sync).
//
// Tile = 1024 elements per 256-thread block.  Pass 1 scans each tile in LDS and
// writes the tile total; pass 2 scans the tile totals in one block (looping over
// chunks of 1024); pass 3 adds the tile offsets.  out[n] receives the grand
// total, so out has n+1 entries.  Used for counting-sort offsets and CSR
// offsets; it is bandwidth-bound and far from the hot path.
#pragma once
#include <hip/hip_runtime.h>

namespace vdscan {

constexpr int kThreads = 256;
constexpr int kTile = 1024;

template <typename TIn, typename TOut>
__global__ void __launch_bounds__(kThreads) tile_scan(const TIn *in, long long n, TOut *out,
                                                      TOut *tile_sum) {
  __shared__ TOut s[kTile];
  const long long base = (long long)blockIdx.x * kTile;
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    const long long i = base + k;
    s[k] = i < n ? (TOut)in[i] : (TOut)0;
  }
  __syncthreads();
  // each thread owns 4 consecutive elements
  TOut loc[4];
  TOut run = 0;
  for (int j = 0; j < 4; j++) { loc[j] = run; run += s[threadIdx.x * 4 + j]; }
  __syncthreads();
  __shared__ TOut t[kThreads];
  t[threadIdx.x] = run;
  __syncthreads();
  for (int d = 1; d < kThreads; d <<= 1) {
    TOut v = threadIdx.x >= (unsigned)d ? t[threadIdx.x - d] : (TOut)0;
    __syncthreads();
    t[threadIdx.x] += v;
    __syncthreads();
  }
  const TOut off = t[threadIdx.x] - run;
  for (int j = 0; j < 4; j++) {
    const long long i = base + threadIdx.x * 4 + j;
    if (i < n) out[i] = off + loc[j];
  }
  if (threadIdx.x == kThreads - 1) tile_sum[blockIdx.x] = t[kThreads - 1];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) sums_scan(T *tile_sum, long long ntiles, T *total_out) {
  __shared__ T t[kThreads];
  T carry = 0;
  for (long long b = 0; b < ntiles; b += kThreads) {
    const long long i = b + threadIdx.x;
    const T v = i < ntiles ? tile_sum[i] : (T)0;
    t[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
      T u = threadIdx.x >= (unsigned)d ? t[threadIdx.x - d] : (T)0;
      __syncthreads();
      t[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < ntiles) tile_sum[i] = carry + t[threadIdx.x] - v;
    const T last = t[kThreads - 1];
    __syncthreads();
    carry += last;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) add_offsets(T *out, long long n, const T *tile_sum) {
  const long long base = (long long)blockIdx.x * kTile;
  const T off = tile_sum[blockIdx.x];
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    const long long i = base + k;
    if (i < n) out[i] += off;
  }
}

inline long long tiles(long long n) { return (n + kTile - 1) / kTile; }

// out[0..n] = exclusive scan of in[0..n), out[n] = total.
// tmp must hold tiles(n) elements of TOut.
template <typename TIn, typename TOut>
inline void exclusive_scan(const TIn *in, long long n, TOut *out, TOut *tmp, hipStream_t st) {
  const long long nt = tiles(n) > 0 ? tiles(n) : 1;
  hipLaunchKernelGGL((tile_scan<TIn, TOut>), dim3((unsigned)nt), dim3(kThreads), 0, st, in, n, out, tmp);
  hipLaunchKernelGGL((sums_scan<TOut>), dim3(1), dim3(kThreads), 0, st, tmp, nt, out + n);
  hipLaunchKernelGGL((add_offsets<TOut>), dim3((unsigned)nt), dim3(kThreads), 0, st, out, n, tmp);
}

}  // namespace vdscan
