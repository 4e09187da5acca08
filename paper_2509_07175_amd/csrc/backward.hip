// backward.hip -- adjoint of the per-site moments (pull-based, no atomics).
//
// For L = sum_k gm_k m_k + gc_k.c_k + gE_k E_k the derivative with respect to
// site v_i at fixed combinatorics is
//   2 gE_i m_i (v_i - c_i)
//   + sum over the bisector faces F_ik of the cell of
//       (a_i - a_k + (b_i - b_k).v_i) I0 + (b_i - b_k).I1 + (gE_i - gE_k) I2
// with a_k = gm_k - gc_k.c_k / m_k, b_k = gc_k / m_k and the face moments
// I0 = int y/d, I1 = int y y^T/d, I2 = int |y|^2 y/d (y = x - v_i) stored by the
// forward pass.  This follows from Eq. 1 and Eq. 3: moving v_i moves the face
// on the bisector of v_i and v_k with normal speed (x - v_i).dv_i / |v_k - v_i|
// (Reynolds transport), the energy integrands of the two cells agree on the
// face, and the interior of cell i contributes -2 int (x - v_i) gE_i.
// One thread per site reads its own faces (pieces in CSR order) and the
// weights of its neighbours; nothing is scattered.  After a no-sync clip that
// dropped records the gradient is NaN (the clip's status is VD_ERR_CAPACITY).
#include "vd_internal.h"

namespace {

constexpr int kB = 256;
inline unsigned blocks(long long n) { return (unsigned)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1); }

// w[5i..] = {a_i, b_i (3), gE_i}
__global__ void __launch_bounds__(kB) adjoint_weights(long long n, const double *__restrict__ mass,
                                                      const double *__restrict__ mom,
                                                      const double *__restrict__ gm, const double *__restrict__ gc,
                                                      const double *__restrict__ ge, double *__restrict__ w) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const double m = mass[i];
  double a = 0, b0 = 0, b1 = 0, b2 = 0;
  if (m > 0.0) {
    const double im = 1.0 / m;
    const double c0 = mom[3 * i] * im, c1 = mom[3 * i + 1] * im, c2 = mom[3 * i + 2] * im;
    const double g0 = gc ? gc[3 * i] : 0.0, g1 = gc ? gc[3 * i + 1] : 0.0, g2 = gc ? gc[3 * i + 2] : 0.0;
    a = (gm ? gm[i] : 0.0) - (g0 * c0 + g1 * c1 + g2 * c2) * im;
    b0 = g0 * im; b1 = g1 * im; b2 = g2 * im;
  }
  w[5 * i + 0] = a;
  w[5 * i + 1] = b0;
  w[5 * i + 2] = b1;
  w[5 * i + 3] = b2;
  w[5 * i + 4] = (m > 0.0 && ge) ? ge[i] : 0.0;
}

__global__ void __launch_bounds__(kB) adjoint_gather(long long n, const int *__restrict__ rank,
                                                     const double *__restrict__ sx, const double *__restrict__ sy,
                                                     const double *__restrict__ sz, const double *__restrict__ mass,
                                                     const double *__restrict__ mom, const double *__restrict__ w,
                                                     const long long *__restrict__ poff, const int *__restrict__ pid,
                                                     const long long *__restrict__ fstart, const int *__restrict__ nfint,
                                                     const double *__restrict__ fint, const int *__restrict__ flab,
                                                     const unsigned long long *__restrict__ cnt,
                                                     double *__restrict__ out) {
  const long long i = (long long)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  if (cnt[CNT_OVERFLOW]) {
    // a no-sync clip dropped records (face moments among them): no gradient
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    out[3 * i + 0] = out[3 * i + 1] = out[3 * i + 2] = nan;
    return;
  }
  const int p = rank[i];
  const double v0 = sx[p], v1 = sy[p], v2 = sz[p];
  const double m = mass[i];
  const double ai = w[5 * i], bi0 = w[5 * i + 1], bi1 = w[5 * i + 2], bi2 = w[5 * i + 3], gi = w[5 * i + 4];
  double o0 = 0, o1 = 0, o2 = 0;
  if (m > 0.0) {
    const double im = 1.0 / m;
    o0 = 2.0 * gi * (m * v0 - mom[3 * i + 0]);
    o1 = 2.0 * gi * (m * v1 - mom[3 * i + 1]);
    o2 = 2.0 * gi * (m * v2 - mom[3 * i + 2]);
    (void)im;
  }
  for (long long q = poff[i]; q < poff[i + 1]; q++) {
    const int pc = pid[q];
    const long long r0 = fstart[pc];
    const int nr = nfint[pc];
    for (int r = 0; r < nr; r++) {
      const long long rr = r0 + r;
      const int k = flab[rr];
      const double *I = &fint[12 * rr];
      const double b0 = bi0 - w[5 * (long long)k + 1], b1 = bi1 - w[5 * (long long)k + 2],
                   b2 = bi2 - w[5 * (long long)k + 3];
      const double a0 = (ai - w[5 * (long long)k]) + b0 * v0 + b1 * v1 + b2 * v2;
      const double g = gi - w[5 * (long long)k + 4];
      o0 += a0 * I[0] + (b0 * I[3] + b1 * I[4] + b2 * I[5]) + g * I[9];
      o1 += a0 * I[1] + (b0 * I[4] + b1 * I[6] + b2 * I[7]) + g * I[10];
      o2 += a0 * I[2] + (b0 * I[5] + b1 * I[7] + b2 * I[8]) + g * I[11];
    }
  }
  out[3 * i + 0] = o0;
  out[3 * i + 1] = o1;
  out[3 * i + 2] = o2;
}

}  // namespace

void vd_launch_backward(const vd_cells_s *c, const GridView &G, const double *gm, const double *gc, const double *ge,
                        double *gs, double *work, hipStream_t st) {
  const long long n = c->n;
  const CellsDev &d = c->d;
  hipLaunchKernelGGL(adjoint_weights, dim3(blocks(n)), dim3(kB), 0, st, n, (const double *)d.mass,
                     (const double *)d.mom, gm, gc, ge, work);
  hipLaunchKernelGGL(adjoint_gather, dim3(blocks(n)), dim3(kB), 0, st, n, (const int *)c->grid->rank, G.sx, G.sy,
                     G.sz, (const double *)d.mass, (const double *)d.mom, (const double *)work,
                     (const long long *)c->piece_off, (const int *)c->piece_id,
                     (const long long *)d.piece_fint_start, (const int *)d.piece_nfint, (const double *)d.fint,
                     (const int *)d.fint_lab, (const unsigned long long *)d.cnt, gs);
}
