// peak_probe.hip -- measured ceilings of the chip for the roofline report.
//
// Not part of the Voronoi path: a stand-alone library (libvd_probe.so) that
// bench.py loads to put measured peaks next to the published ones.
//   vd_probe_fma_f64: every lane runs eight independent chains of FP64 fused
//     multiply-adds (v_fma_f64), enough to cover the FMA latency; the grid
//     fills every SIMD several times over.  FLOPs = 2 per FMA.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ void __launch_bounds__(256) fma_chains(int iters, double a, double b, double *out) {
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; k++) x[k] = (double)(threadIdx.x + k) * 1e-3;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int k = 0; k < 8; k++) x[k] = fma(x[k], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; k++) s += x[k];
  // keep the chains live: the store happens only for a value the chains never reach
  if (s == 12345.678) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// Runs `blocks` workgroups of 256 lanes, `iters` iterations of 8 FMAs per lane,
// timed with HIP events on a private stream.  Writes the elapsed milliseconds
// to *ms and returns 0, or a HIP error code.  out: device scratch of
// blocks * 256 doubles (never written in practice).
extern "C" int vd_probe_fma_f64(int blocks, int iters, double *out, float *ms, double *flops) {
  if (blocks <= 0 || iters <= 0 || !out || !ms || !flops) return (int)hipErrorInvalidValue;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t rc = hipStreamCreate(&st);
  if (rc == hipSuccess) rc = hipEventCreate(&e0);
  if (rc == hipSuccess) rc = hipEventCreate(&e1);
  if (rc == hipSuccess) {
    hipLaunchKernelGGL(fma_chains, dim3(blocks), dim3(256), 0, st, iters, 0.999999, 1e-7, out);  // warm-up
    rc = hipEventRecord(e0, st);
  }
  if (rc == hipSuccess) {
    hipLaunchKernelGGL(fma_chains, dim3(blocks), dim3(256), 0, st, iters, 0.999999, 1e-7, out);
    rc = hipGetLastError();
  }
  if (rc == hipSuccess) rc = hipEventRecord(e1, st);
  if (rc == hipSuccess) rc = hipEventSynchronize(e1);
  if (rc == hipSuccess) rc = hipEventElapsedTime(ms, e0, e1);
  *flops = 2.0 * 8.0 * (double)iters * (double)blocks * 256.0;
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (st) hipStreamDestroy(st);
  return (int)rc;
}
