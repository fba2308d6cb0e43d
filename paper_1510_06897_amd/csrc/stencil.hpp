// Wilson hopping stencil on one lattice site, in half-spinor form (Sec. 2, eq. 2).
//
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^+, 0]] with A_k = -i sigma_k (k = x, y, z) and
// A_t = 1.  For psi = (u, d) (upper / lower spin pairs):
//   (1 - gamma_mu) psi = (h, -A_mu^+ h),  h = u - A_mu d,
//   (1 + gamma_mu) psi = (h, +A_mu^+ h),  h = u + A_mu d,
// so each hop moves a 2-spin x 3-colour half-spinor through one SU(3) matrix and rebuilds the
// lower spin pair from it: 12 complex multiply-adds per colour matrix instead of 24.
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

// acc[upper] += r, acc[lower] += -+A_mu^+ r
template <int MU, bool MINUS, class C>
__device__ __forceinline__ void reconstruct_add(cx<C> acc[12], const cx<C> r[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0 * 3 + c] = acc[0 * 3 + c] + r[0][c];
    acc[1 * 3 + c] = acc[1 * 3 + c] + r[1][c];
    cx<C> l0, l1;
    if (MU == 0) {  // A^+ r = (i r1, i r0)
      l0 = mul_i(r[1][c]);
      l1 = mul_i(r[0][c]);
    } else if (MU == 1) {  // A^+ r = (r1, -r0)
      l0 = r[1][c];
      l1 = -r[0][c];
    } else if (MU == 2) {  // A^+ r = (i r0, -i r1)
      l0 = mul_i(r[0][c]);
      l1 = mul_mi(r[1][c]);
    } else {
      l0 = r[0][c];
      l1 = r[1][c];
    }
    if (MINUS) {
      acc[2 * 3 + c] = acc[2 * 3 + c] - l0;
      acc[3 * 3 + c] = acc[3 * 3 + c] - l1;
    } else {
      acc[2 * 3 + c] = acc[2 * 3 + c] + l0;
      acc[3 * 3 + c] = acc[3 * 3 + c] + l1;
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

// links of one direction: resource over U_mu[a][b][V], component stride ls bytes
// acc += (1 - gamma_mu) U_mu(x) v(x + mu) + (1 + gamma_mu) U_mu(x - mu)^+ v(x - mu)
template <int MU, class C, class SE, class LE>
__device__ __forceinline__ void hop_dir(cx<C> acc[12], rsrc_t v, uint32_t cs, rsrc_t Um,
                                        uint32_t ls, uint32_t site, uint32_t fwd, uint32_t bwd,
                                        bool g5) {
  {
    cx<C> u[2][3], d[2][3], h[2][3], r[2][3];
    load_spinor<C, SE>(v, cs, fwd, g5, u, d);
    project<MU, true>(u, d, h);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[0][a] = mk<C>(0, 0);
      r[1][a] = mk<C>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const cx<C> m = bld<C, LE>(Um, (a * 3 + b) * ls, site);
        r[0][a] = cmadd(r[0][a], m, h[0][b]);
        r[1][a] = cmadd(r[1][a], m, h[1][b]);
      }
    }
    reconstruct_add<MU, true>(acc, r);
  }
  {
    cx<C> u[2][3], d[2][3], h[2][3], r[2][3];
    load_spinor<C, SE>(v, cs, bwd, g5, u, d);
    project<MU, false>(u, d, h);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[0][a] = mk<C>(0, 0);
      r[1][a] = mk<C>(0, 0);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        // (U^+)_{ab} = conj(U_{ba}) at the backward site
        const cx<C> m = bld<C, LE>(Um, (b * 3 + a) * ls, bwd);
        r[0][a] = cjmadd(r[0][a], m, h[0][b]);
        r[1][a] = cjmadd(r[1][a], m, h[1][b]);
      }
    reconstruct_add<MU, false>(acc, r);
  }
}

// per-direction link resources of a gauge field stored as [4][3][3][V] elements of LE
template <class LE>
struct LinkRes {
  rsrc_t u[4];
  uint32_t ls;  // component stride in bytes
};
template <class LE>
__device__ __forceinline__ LinkRes<LE> link_res(const void *U, int V) {
  LinkRes<LE> r;
  r.ls = (uint32_t)V * elem_traits<LE>::bytes;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
    r.u[mu] = make_rsrc(reinterpret_cast<const LE *>(U) + (int64_t)mu * 9 * V, 9u * r.ls);
  return r;
}

// acc (12 complex, zeroed by the caller) += hopping term of eq. 2 at `site`
template <class C, class SE, class LE>
__device__ __forceinline__ void hop_site(cx<C> acc[12], rsrc_t v, const LinkRes<LE> &U,
                                         const Geom &g, int site, bool g5) {
  int fwd[4], bwd[4];
  neighbours(g, site, fwd, bwd);
  const uint32_t cs = (uint32_t)g.V * elem_traits<SE>::bytes;
  // a rolled loop over directions: loads of one direction cannot be hoisted above the arithmetic
  // of the previous one, which bounds the live registers to one neighbour pair and its links
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    switch (mu) {
      case 0: hop_dir<0, C, SE, LE>(acc, v, cs, U.u[0], U.ls, site, fwd[0], bwd[0], g5); break;
      case 1: hop_dir<1, C, SE, LE>(acc, v, cs, U.u[1], U.ls, site, fwd[1], bwd[1], g5); break;
      case 2: hop_dir<2, C, SE, LE>(acc, v, cs, U.u[2], U.ls, site, fwd[2], bwd[2], g5); break;
      default: hop_dir<3, C, SE, LE>(acc, v, cs, U.u[3], U.ls, site, fwd[3], bwd[3], g5); break;
    }
  }
}

}  // namespace ovl
