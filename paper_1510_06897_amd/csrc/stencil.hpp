// Spin projection of the Wilson stencil (Sec. 2, eq. 2) with compile-time direction, used by the
// link-derivative kernel.
//
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^+, 0]] with A_k = -i sigma_k (k = x, y, z) and
// A_t = 1.  For psi = (u, d) (upper / lower spin pairs):
//   (1 - gamma_mu) psi = (h, -A_mu^+ h),  h = u - A_mu d,
//   (1 + gamma_mu) psi = (h, +A_mu^+ h),  h = u + A_mu d.
#pragma once

#include "common.hpp"

namespace ovl {

// h = u -+ A_mu d for the projector (1 - gamma_mu) (MINUS = true) or (1 + gamma_mu)
template <int MU, bool MINUS, class C>
__device__ __forceinline__ void project(const cx<C> u[2][3], const cx<C> d[2][3], cx<C> h[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 0) {  // A = -i sigma_1: A d = (-i d1, -i d0)
      h[0][c] = MINUS ? u[0][c] + mul_i(d[1][c]) : u[0][c] - mul_i(d[1][c]);
      h[1][c] = MINUS ? u[1][c] + mul_i(d[0][c]) : u[1][c] - mul_i(d[0][c]);
    } else if (MU == 1) {  // A = -i sigma_2: A d = (-d1, d0)
      h[0][c] = MINUS ? u[0][c] + d[1][c] : u[0][c] - d[1][c];
      h[1][c] = MINUS ? u[1][c] - d[0][c] : u[1][c] + d[0][c];
    } else if (MU == 2) {  // A = -i sigma_3: A d = (-i d0, i d1)
      h[0][c] = MINUS ? u[0][c] + mul_i(d[0][c]) : u[0][c] - mul_i(d[0][c]);
      h[1][c] = MINUS ? u[1][c] - mul_i(d[1][c]) : u[1][c] + mul_i(d[1][c]);
    } else {  // A = 1
      h[0][c] = MINUS ? u[0][c] - d[0][c] : u[0][c] + d[0][c];
      h[1][c] = MINUS ? u[1][c] - d[1][c] : u[1][c] + d[1][c];
    }
  }
}

// load the 12 spin-colour components of one site (component stride cs bytes), split into spin
// pairs; g5 applies gamma5 = diag(1, 1, -1, -1) on the fly
template <class C, class SE>
__device__ __forceinline__ void load_spinor(rsrc_t v, uint32_t cs, uint32_t site, bool g5,
                                            cx<C> u[2][3], cx<C> d[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) u[s][c] = bld<C, SE>(v, (s * 3 + c) * cs, site);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<C> x = bld<C, SE>(v, ((s + 2) * 3 + c) * cs, site);
      d[s][c] = g5 ? -x : x;
    }
}

}  // namespace ovl
