// Direction-split Wilson hopping stencil (Sec. 2, eq. 2): four threads per lattice site.
//
// A workgroup of 4 * SPB threads covers SPB consecutive sites; thread t handles direction
// mu = t / SPB for site t % SPB.  It loads the neighbour spinors at x + mu and x - mu and the two
// links U_mu(x), U_mu(x - mu), projects each neighbour to a half-spinor, multiplies by the link
// and rebuilds the lower spin pair.  The four directional partial sums of a site are then added
// through LDS, after which thread (mu, site) owns spin component s = mu of the result.  Every
// memory instruction of a wave reads consecutive sites of one direction (fully coalesced), each
// thread waits on two memory round trips instead of eight, and a lattice gets 4x the threads.
//
// The spin structure of direction mu enters through per-thread coefficients:
//   (1 - gamma_mu) psi:  h0 = u0 + z0 d[p], h1 = u1 + z1 d[1-p],
//                        lower0 = w0 r[p], lower1 = w1 r[1-p]   (r = U h),
//   (1 + gamma_mu) psi:  the same with z and w negated,
// where p, z, w follow from gamma_mu = [[0, A_mu], [A_mu^+, 0]], A_k = -i sigma_k, A_t = 1.
#pragma once

#include "common.hpp"

namespace ovl {

template <class C>
struct DirCoef {
  bool p;
  cx<C> z0, z1, w0, w1;
};

template <class C>
__device__ __forceinline__ DirCoef<C> dir_coef(int mu) {
  DirCoef<C> k;
  k.p = mu < 2;
  k.z0 = mk<C>(mu == 1 ? 1 : (mu == 3 ? -1 : 0), (mu == 0 || mu == 2) ? 1 : 0);
  k.z1 = mk<C>((mu == 1 || mu == 3) ? -1 : 0, mu == 0 ? 1 : (mu == 2 ? -1 : 0));
  k.w0 = mk<C>((mu == 1 || mu == 3) ? -1 : 0, (mu == 0 || mu == 2) ? -1 : 0);
  k.w1 = mk<C>(mu == 1 ? 1 : (mu == 3 ? -1 : 0), mu == 0 ? -1 : (mu == 2 ? 1 : 0));
  return k;
}

// z * d for z in {+-1, +-i}
template <class C>
__device__ __forceinline__ cx<C> zmul(cx<C> z, cx<C> d) {
  return mk<C>(z.re * d.re - z.im * d.im, z.re * d.im + z.im * d.re);
}

// one link (component stride ls bytes, element lsite): all three rows, or with r12 the first
// two, the third completed as for an SU(3) matrix (uniform per launch)
template <class C, class LE>
__device__ __forceinline__ void load_link3(rsrc_t Um, uint32_t ls, uint32_t lsite, bool r12,
                                           cx<C> m[3][3]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) m[a][b] = bld<C, LE>(Um, (a * 3 + b) * ls, lsite);
  if (r12) {
    su3_row2(m);
  } else {
#pragma unroll
    for (int b = 0; b < 3; ++b) m[2][b] = bld<C, LE>(Um, (6 + b) * ls, lsite);
  }
}

template <class C, bool DAG>
__device__ __forceinline__ void hop_apply(cx<C> acc[12], const cx<C> u[2][3], const cx<C> d[2][3],
                                          const cx<C> m[3][3], const DirCoef<C> &k, C sgn);

// one hop: acc += (1 -+ gamma_mu) M h, M = U (forward) or U^+ (backward), neighbour at `nb`,
// link read at `ls_site`; sgn = +1 for (1 - gamma_mu), -1 for (1 + gamma_mu)
template <class C, class SE, class LE, bool DAG>
__device__ __forceinline__ void quad_hop(cx<C> acc[12], rsrc_t v, uint32_t cs, rsrc_t Um,
                                         uint32_t ls, uint32_t nb, uint32_t lsite,
                                         const DirCoef<C> &k, C sgn, bool g5, bool r12) {
  cx<C> u[2][3], d[2][3];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      u[s][c] = bld<C, SE>(v, (s * 3 + c) * cs, nb);
      cx<C> x = bld<C, SE>(v, ((s + 2) * 3 + c) * cs, nb);
      d[s][c] = g5 ? -x : x;
    }
  cx<C> m[3][3];
  load_link3<C, LE>(Um, ls, lsite, r12, m);
  hop_apply<C, DAG>(acc, u, d, m, k, sgn);
}

// the arithmetic of one hop on loaded data: acc += (1 -+ gamma_mu) M h
template <class C, bool DAG>
__device__ __forceinline__ void hop_apply(cx<C> acc[12], const cx<C> u[2][3], const cx<C> d[2][3],
                                          const cx<C> m[3][3], const DirCoef<C> &k, C sgn) {
  const cx<C> z0 = scale(k.z0, sgn), z1 = scale(k.z1, sgn);
  const cx<C> w0 = scale(k.w0, sgn), w1 = scale(k.w1, sgn);
  cx<C> h[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<C> dA = k.p ? d[1][c] : d[0][c];
    const cx<C> dB = k.p ? d[0][c] : d[1][c];
    h[0][c] = u[0][c] + zmul(z0, dA);
    h[1][c] = u[1][c] + zmul(z1, dB);
  }
  cx<C> r[2][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[0][a] = mk<C>(0, 0);
    r[1][a] = mk<C>(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (DAG) {  // (U^+)_{ab} = conj(U_{ba})
        r[0][a] = cjmadd(r[0][a], m[b][a], h[0][b]);
        r[1][a] = cjmadd(r[1][a], m[b][a], h[1][b]);
      } else {
        r[0][a] = cmadd(r[0][a], m[a][b], h[0][b]);
        r[1][a] = cmadd(r[1][a], m[a][b], h[1][b]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = acc[c] + r[0][c];
    acc[3 + c] = acc[3 + c] + r[1][c];
    const cx<C> rA = k.p ? r[1][c] : r[0][c];
    const cx<C> rB = k.p ? r[0][c] : r[1][c];
    acc[6 + c] = acc[6 + c] + zmul(w0, rA);
    acc[9 + c] = acc[9 + c] + zmul(w1, rB);
  }
}

// The same hop with the direction fixed at compile time (kernels whose waves each take one
// direction): z, w in {+-1, +-i} become additions with swapped or negated components instead of
// complex products by a per-thread coefficient, and the gamma5 of the input (s5 = -1: the lower
// spin pair negated, uniform per launch) folds into those additions.  Bitwise the same sums as
// hop_apply on the gamma5-applied input (the products there are exact).
template <int MU>
struct DirK {
  static constexpr bool p = MU < 2;
  static constexpr int z0r = MU == 1 ? 1 : (MU == 3 ? -1 : 0), z0i = (MU == 0 || MU == 2) ? 1 : 0;
  static constexpr int z1r = (MU == 1 || MU == 3) ? -1 : 0, z1i = MU == 0 ? 1 : (MU == 2 ? -1 : 0);
  static constexpr int w0r = (MU == 1 || MU == 3) ? -1 : 0, w0i = (MU == 0 || MU == 2) ? -1 : 0;
  static constexpr int w1r = MU == 1 ? 1 : (MU == 3 ? -1 : 0), w1i = MU == 0 ? -1 : (MU == 2 ? 1 : 0);
};
// z x for a compile-time z in {+-1, +-i}
template <int ZR, int ZI, class C>
__device__ __forceinline__ cx<C> zc(cx<C> x) {
  static_assert(ZR * ZR + ZI * ZI == 1, "z must be +-1 or +-i");
  if constexpr (ZR == 1) return x;
  else if constexpr (ZR == -1) return mk<C>(-x.re, -x.im);
  else if constexpr (ZI == 1) return mk<C>(-x.im, x.re);
  else return mk<C>(x.im, -x.re);
}
// u + s (z x), s = +-1 at run time
template <int ZR, int ZI, class C>
__device__ __forceinline__ cx<C> add_szx(cx<C> u, C s, cx<C> x) {
  const cx<C> y = zc<ZR, ZI>(x);
  return mk<C>(fma(s, y.re, u.re), fma(s, y.im, u.im));
}

// acc += (1 - SG gamma_MU) M h for the raw neighbour (u, d) (d not yet multiplied by s5)
template <class C, bool DAG, int MU, int SG>
__device__ __forceinline__ void hop_apply_k(cx<C> acc[12], const cx<C> u[2][3], const cx<C> d[2][3],
                                            const cx<C> m[3][3], C s5) {
  using K = DirK<MU>;
  cx<C> h[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<C> dA = K::p ? d[1][c] : d[0][c];
    const cx<C> dB = K::p ? d[0][c] : d[1][c];
    h[0][c] = add_szx<SG * K::z0r, SG * K::z0i>(u[0][c], s5, dA);
    h[1][c] = add_szx<SG * K::z1r, SG * K::z1i>(u[1][c], s5, dB);
  }
  cx<C> r[2][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[0][a] = mk<C>(0, 0);
    r[1][a] = mk<C>(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (DAG) {
        r[0][a] = cjmadd(r[0][a], m[b][a], h[0][b]);
        r[1][a] = cjmadd(r[1][a], m[b][a], h[1][b]);
      } else {
        r[0][a] = cmadd(r[0][a], m[a][b], h[0][b]);
        r[1][a] = cmadd(r[1][a], m[a][b], h[1][b]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = acc[c] + r[0][c];
    acc[3 + c] = acc[3 + c] + r[1][c];
    const cx<C> rA = K::p ? r[1][c] : r[0][c];
    const cx<C> rB = K::p ? r[0][c] : r[1][c];
    acc[6 + c] = acc[6 + c] + zc<SG * K::w0r, SG * K::w0i>(rA);
    acc[9 + c] = acc[9 + c] + zc<SG * K::w1r, SG * K::w1i>(rB);
  }
}

// one hop whose direction is chosen per lane (dag = backward: M = U^+, sgn = -1), so that the
// forward and the backward hops of a wave run the same instructions
template <class C, class SE, class LE>
__device__ __forceinline__ void quad_hop_sel(cx<C> acc[12], rsrc_t v, uint32_t cs, rsrc_t Um,
                                             uint32_t ls, uint32_t nb, uint32_t lsite,
                                             const DirCoef<C> &k, bool dag, bool g5,
                                             bool r12) {
  cx<C> u[2][3], d[2][3];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      u[s][c] = bld<C, SE>(v, (s * 3 + c) * cs, nb);
      cx<C> x = bld<C, SE>(v, ((s + 2) * 3 + c) * cs, nb);
      d[s][c] = g5 ? -x : x;
    }
  cx<C> m[3][3], mm[3][3];
  load_link3<C, LE>(Um, ls, lsite, r12, m);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) mm[a][b] = dag ? mk<C>(m[b][a].re, -m[b][a].im) : m[a][b];
  hop_apply<C, false>(acc, u, d, mm, k, dag ? C(-1) : C(1));
}

// h = projection of (u, d) by (1 - gamma_mu) (sgn = +1) or (1 + gamma_mu) (sgn = -1)
template <class C>
__device__ __forceinline__ void dir_project(const cx<C> u[2][3], const cx<C> d[2][3],
                                            const DirCoef<C> &k, C sgn, cx<C> h[2][3]) {
  const cx<C> z0 = scale(k.z0, sgn), z1 = scale(k.z1, sgn);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<C> dA = k.p ? d[1][c] : d[0][c];
    const cx<C> dB = k.p ? d[0][c] : d[1][c];
    h[0][c] = u[0][c] + zmul(z0, dA);
    h[1][c] = u[1][c] + zmul(z1, dB);
  }
}

// dir_project with the direction fixed at compile time, and a uniform run-time switch over it
template <class C, int MU, int SG>
__device__ __forceinline__ void dir_project_k(const cx<C> u[2][3], const cx<C> d[2][3],
                                              cx<C> h[2][3]) {
  using K = DirK<MU>;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<C> dA = K::p ? d[1][c] : d[0][c];
    const cx<C> dB = K::p ? d[0][c] : d[1][c];
    h[0][c] = u[0][c] + zc<SG * K::z0r, SG * K::z0i>(dA);
    h[1][c] = u[1][c] + zc<SG * K::z1r, SG * K::z1i>(dB);
  }
}
template <class C, int SG>
__device__ __forceinline__ void dir_project_sw(int mu, const cx<C> u[2][3], const cx<C> d[2][3],
                                               cx<C> h[2][3]) {
  switch (mu) {
    case 0: dir_project_k<C, 0, SG>(u, d, h); break;
    case 1: dir_project_k<C, 1, SG>(u, d, h); break;
    case 2: dir_project_k<C, 2, SG>(u, d, h); break;
    default: dir_project_k<C, 3, SG>(u, d, h); break;
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

// Extents, strides and coordinates as named scalars.  The direction-split kernel selects one of
// four values per thread; with arrays the compiler turns those selects into dynamically indexed
// private memory, so everything here is plain scalars.
struct Ext4 {
  int lx, ly, lz, lt;  // extents
  int sy, sz, st;      // strides of y, z, t in the site index (x has stride 1)
  int V;
};
struct Coord4 {
  int x, y, z, t;
};

__device__ __forceinline__ Ext4 ext_of(const Geom &g) {
  Ext4 e;
  e.lx = g.L[0];
  e.ly = g.L[1];
  e.lz = g.L[2];
  e.lt = g.L[3];
  e.sy = g.stride[1];
  e.sz = g.stride[2];
  e.st = g.stride[3];
  e.V = g.V;
  return e;
}

__device__ __forceinline__ Coord4 coords_of(const Ext4 &e, int s) {
  Coord4 c;
  c.x = s % e.lx;
  int r = s / e.lx;
  c.y = r % e.ly;
  r /= e.ly;
  c.z = r % e.lz;
  c.t = r / e.lz;
  return c;
}

// neighbour sites of `site` along mu (periodic)
__device__ __forceinline__ void dir_neighbours(const Ext4 &e, const Coord4 &c, int site, int mu,
                                               int &fwd, int &bwd) {
  const int st = mu == 0 ? 1 : mu == 1 ? e.sy : mu == 2 ? e.sz : e.st;
  const int L = mu == 0 ? e.lx : mu == 1 ? e.ly : mu == 2 ? e.lz : e.lt;
  const int x = mu == 0 ? c.x : mu == 1 ? c.y : mu == 2 ? c.z : c.t;
  const int wrap = (L - 1) * st;
  fwd = (x + 1 == L) ? site - wrap : site + st;
  bwd = (x == 0) ? site + wrap : site - st;
}

}  // namespace ovl
