// Vector kernels of the overlap solvers whose scalar coefficients stay on the device.
//
// The inner products of a Krylov iteration (FP64 sums, written by the projection kernels into
// small device slots) feed the next vector update directly: each kernel reads its coefficient from
// device memory, so an iteration is a chain of launches on one stream with no host round trip.
// A coefficient that would divide by a non-positive or non-finite curvature is replaced by zero
// and raises a flag word the host reads later (the iteration then stands still instead of
// producing NaN).
#pragma once

#include "common.hpp"

namespace ovl {

// flag bits of the solver state word
enum : int { SOLVE_FLAG_CURVATURE = 1 };

// CG step on the normal equations:  a = rr / Re<p, q>,  x += a p,  r -= a q
template <class C, class SE>
__global__ void __launch_bounds__(256)
    cg_xr_kernel(SE *__restrict__ x, SE *__restrict__ r, const SE *__restrict__ p,
                 const SE *__restrict__ q, const double2 *__restrict__ rr,
                 const double2 *__restrict__ pq, int *__restrict__ flag, int64_t n) {
  const double den = pq->x;
  const bool ok = den > 0.0 && isfinite(den) && isfinite(rr->x);
  const double a = ok ? rr->x / den : 0.0;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!ok && k == 0) *flag |= SOLVE_FLAG_CURVATURE;
  if (k >= n) return;
  const C ac = C(a);
  const cx<C> pv = load_c<C>(p, k), qv = load_c<C>(q, k);
  const cx<C> xv = load_c<C>(x, k), rv = load_c<C>(r, k);
  store_c<C>(x, k, mk<C>(fma(ac, pv.re, xv.re), fma(ac, pv.im, xv.im)));
  store_c<C>(r, k, mk<C>(fma(-ac, qv.re, rv.re), fma(-ac, qv.im, rv.im)));
}

// p = r + beta p,  beta = rr_new / rr_old  (0 when rr_old is 0)
template <class C, class SE>
__global__ void __launch_bounds__(256)
    cg_p_kernel(SE *__restrict__ p, const SE *__restrict__ r, const double2 *__restrict__ rr_new,
                const double2 *__restrict__ rr_old, int64_t n) {
  const double o = rr_old->x;
  const double beta = (o > 0.0 && isfinite(o)) ? rr_new->x / o : 0.0;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const C b = C(beta);
  const cx<C> pv = load_c<C>(p, k), rv = load_c<C>(r, k);
  store_c<C>(p, k, mk<C>(fma(b, pv.re, rv.re), fma(b, pv.im, rv.im)));
}

// Generalised conjugate residual (GMRESR) step, FP64:
//   c /= ||c||, z /= ||c||  with nrm2 = <c, c>  (both untouched when ||c|| is 0 or not finite)
__global__ void __launch_bounds__(256)
    gcr_normalise_kernel(double2 *__restrict__ c, double2 *__restrict__ z,
                         const double2 *__restrict__ nrm2, int *__restrict__ flag, int64_t n) {
  const double s2 = nrm2->x;
  const bool ok = s2 > 0.0 && isfinite(s2);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!ok && k == 0) *flag |= SOLVE_FLAG_CURVATURE;
  if (k >= n || !ok) return;
  const double s = 1.0 / sqrt(s2);
  const double2 cv = c[k], zv = z[k];
  c[k] = make_double2(cv.x * s, cv.y * s);
  z[k] = make_double2(zv.x * s, zv.y * s);
}

//   a = <c, r>,  x += a z,  r -= a c   (a complex, from the device slot)
__global__ void __launch_bounds__(256)
    gcr_update_kernel(double2 *__restrict__ x, double2 *__restrict__ r, const double2 *__restrict__ z,
                      const double2 *__restrict__ c, const double2 *__restrict__ alpha, int64_t n) {
  const double2 a = *alpha;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double2 zv = z[k], cv = c[k], xv = x[k], rv = r[k];
  x[k] = make_double2(xv.x + a.x * zv.x - a.y * zv.y, xv.y + a.x * zv.y + a.y * zv.x);
  r[k] = make_double2(rv.x - (a.x * cv.x - a.y * cv.y), rv.y - (a.x * cv.y + a.y * cv.x));
}

//   v -= sum_{i < m} beta_i B_i  for B a block of m FP64 vectors (n elements each, contiguous),
//   beta from the device (one complex per vector); up to two vectors updated with the same
//   coefficients (c against the C basis, z against the Z basis).
__global__ void __launch_bounds__(256)
    gcr_orth_kernel(double2 *__restrict__ v, const double2 *__restrict__ B, int m,
                    const double2 *__restrict__ beta, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2 acc = v[k];
  for (int i = 0; i < m; ++i) {
    const double2 b = beta[i], e = B[(int64_t)i * n + k];
    acc.x -= b.x * e.x - b.y * e.y;
    acc.y -= b.x * e.y + b.y * e.x;
  }
  v[k] = acc;
}

}  // namespace ovl
