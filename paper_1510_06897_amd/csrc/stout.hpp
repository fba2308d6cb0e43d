// Stout smearing of the gauge links on the device and its chain-rule derivative (FP64).
//
// The links entering K are smoothed by three steps of over-improved stout smearing with
// rho = 0.1 and eps = -0.25 (Sec. 2).  One step replaces every link at once by
//   U'_mu(x) = exp(M) U_mu(x),   M = TA(Omega) = (Omega - Omega^+)/2 - tr(Omega - Omega^+)/6,
//   Omega = C_mu(x) U_mu(x)^+,
// where C_mu(x) sums the paths from x to x + mu that close a loop with the link: the three-link
// plaquette staples with weight rho c_p and the five-link staples of the 2 x 1 rectangles with
// weight rho c_r, c_p = (5 - 2 eps)/3, c_r = -(1 - eps)/12 (the over-improved gauge action; eps = 1
// leaves the plaquette alone: plain stout smearing).
//
// Links are read and written in the caller layout U[mu][a][b][site] (complex double), so one
// wave reads one matrix element of 64 consecutive sites per load; the path factors are read
// through raw buffer resources (lane offset site * 16 bytes, element offset in a scalar register),
// so a field must span less than 4 GiB.  A thread owns one link
// (site, mu); the workgroup's 256 threads share mu, so the path loops below are uniform over a
// wave.  exp(M) is a Taylor series after scaling M to norm <= 1/2, followed by squaring; the
// derivative of exp comes from the same series for the Frechet derivative (the directional
// derivative of every power, carried along the squarings).
#pragma once

#include "common.hpp"

namespace ovl {

// ---------------------------------------------------------------------------------------------
// 3 x 3 complex FP64 matrices in registers
struct M3 {
  cx<double> e[3][3];
};

__device__ __forceinline__ M3 m3_zero() {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = mk<double>(0.0, 0.0);
  return r;
}
__device__ __forceinline__ M3 m3_unit() {
  M3 r = m3_zero();
#pragma unroll
  for (int i = 0; i < 3; ++i) r.e[i][i] = mk<double>(1.0, 0.0);
  return r;
}
// A B
__device__ __forceinline__ M3 m3_mul(const M3 &a, const M3 &b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cmadd(s, a.e[i][k], b.e[k][j]);
      r.e[i][j] = s;
    }
  return r;
}
// A^+ B
__device__ __forceinline__ M3 m3_dmul(const M3 &a, const M3 &b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cjmadd(s, a.e[k][i], b.e[k][j]);
      r.e[i][j] = s;
    }
  return r;
}
// A B^+
__device__ __forceinline__ M3 m3_muld(const M3 &a, const M3 &b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cjmadd(s, b.e[j][k], a.e[i][k]);
      r.e[i][j] = s;
    }
  return r;
}
__device__ __forceinline__ M3 m3_dag(const M3 &a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = mk<double>(a.e[j][i].re, -a.e[j][i].im);
  return r;
}
// a + s b
__device__ __forceinline__ M3 m3_axpy(const M3 &a, double s, const M3 &b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      r.e[i][j] = mk<double>(fma(s, b.e[i][j].re, a.e[i][j].re), fma(s, b.e[i][j].im, a.e[i][j].im));
  return r;
}
__device__ __forceinline__ M3 m3_scale(const M3 &a, double s) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = scale(a.e[i][j], s);
  return r;
}
__device__ __forceinline__ double m3_frob(const M3 &a) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += a.e[i][j].re * a.e[i][j].re + a.e[i][j].im * a.e[i][j].im;
  return sqrt(s);
}

// element (a, b) of link `dir` at `site`: U[dir][a][b][site]
__device__ __forceinline__ M3 load_m3(const double2 *__restrict__ U, int dir, int site, int V) {
  M3 r;
  const double2 *p = U + (int64_t)dir * 9 * V + site;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 v = p[(int64_t)(3 * i + j) * V];
      r.e[i][j] = mk<double>(v.x, v.y);
    }
  return r;
}
__device__ __forceinline__ void store_m3(double2 *__restrict__ U, int dir, int site, int V,
                                         const M3 &m) {
  double2 *p = U + (int64_t)dir * 9 * V + site;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) p[(int64_t)(3 * i + j) * V] = make_double2(m.e[i][j].re, m.e[i][j].im);
}

// ---------------------------------------------------------------------------------------------
// exp(A) and the Frechet derivative L(A, F) = d/dt exp(A + t F) at t = 0.
//   Scale: X = A / 2^s with ||X||_F <= 1/2.  Series: T_0 = 1, T_{k+1} = X T_k / (k + 1) gives
//   exp(X) = sum T_k; the derivative of X^k along F obeys D_{k+1} = F X^k + X D_k, so with
//   S_k = D_k / k!:  S_1 = F, S_{k+1} = (F T_k + X S_k) / (k + 1) and L(X, F) = sum S_k.
//   Square: exp(2Y) = exp(Y)^2 and L(2Y, 2G) = L(Y, G) exp(Y) + exp(Y) L(Y, G).
// 18 terms leave a remainder below 0.5^19 / 19! (1e-23) of the scaled series.
constexpr int kExpTerms = 18;

__device__ __forceinline__ int exp_scaling(const M3 &a) {
  double n = m3_frob(a);
  int s = 0;
  while (n > 0.5 && s < 40) {
    n *= 0.5;
    ++s;
  }
  return s;
}

__device__ inline M3 m3_exp(const M3 &a) {
  const int s = exp_scaling(a);
  const M3 x = m3_scale(a, ldexp(1.0, -s));
  M3 e = m3_unit(), t = m3_unit();
  for (int k = 1; k <= kExpTerms; ++k) {
    t = m3_scale(m3_mul(x, t), 1.0 / k);
    e = m3_axpy(e, 1.0, t);
  }
  for (int i = 0; i < s; ++i) e = m3_mul(e, e);
  return e;
}

// exp(A) into *e and L(A, F) into *l
__device__ inline void m3_exp_frechet(const M3 &a, const M3 &f, M3 *e_out, M3 *l_out) {
  const int s = exp_scaling(a);
  const double sc = ldexp(1.0, -s);
  const M3 x = m3_scale(a, sc), g = m3_scale(f, sc);
  M3 e = m3_unit(), t = m3_unit();
  M3 l = m3_zero(), d = m3_zero();
  for (int k = 1; k <= kExpTerms; ++k) {
    // S_k = (F T_{k-1} + X S_{k-1}) / k, T_k = X T_{k-1} / k  (S_0 = 0, T_0 = 1)
    const M3 dn = m3_scale(m3_axpy(m3_mul(g, t), 1.0, m3_mul(x, d)), 1.0 / k);
    t = m3_scale(m3_mul(x, t), 1.0 / k);
    d = dn;
    e = m3_axpy(e, 1.0, t);
    l = m3_axpy(l, 1.0, d);
  }
  for (int i = 0; i < s; ++i) {
    l = m3_axpy(m3_mul(l, e), 1.0, m3_mul(e, l));
    e = m3_mul(e, e);
  }
  *e_out = e;
  *l_out = l;
}

// traceless anti-Hermitian part: (W - W^+)/2 - tr(W - W^+)/6
__device__ __forceinline__ M3 m3_ta(const M3 &w) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      r.e[i][j] = mk<double>(0.5 * (w.e[i][j].re - w.e[j][i].re), 0.5 * (w.e[i][j].im + w.e[j][i].im));
  const double tr_im = (r.e[0][0].im + r.e[1][1].im + r.e[2][2].im) / 3.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) r.e[i][i].im -= tr_im;
  return r;
}

// ---------------------------------------------------------------------------------------------
// Staple paths.  For a link along mu, a plane mu-nu (nu != mu) and an orientation s = +1 or -1 of
// nu, four paths lead from x to x + mu:
//   shape 0  plaquette            (nu,s)  (mu,+)  (nu,-s)
//   shape 1  2 x 1, link first    (nu,s)  (mu,+)  (mu,+)  (nu,-s) (mu,-)
//   shape 2  2 x 1, link second   (mu,-)  (nu,s)  (mu,+)  (mu,+)  (nu,-s)
//   shape 3  1 x 2                (nu,s)  (nu,s)  (mu,+)  (nu,-s) (nu,-s)
// A step (d,+) from position z takes the factor U_d(x + z) and moves to z + e_d; a step (d,-)
// moves to z - e_d and takes U_d(x + z - e_d)^+.  Together with the link these are the 6
// plaquettes and 18 rectangles that contain it.
__device__ __forceinline__ int path_len(int shape) { return shape == 0 ? 3 : 5; }

__device__ __forceinline__ void path_step(int mu, int nu, int s, int shape, int k, int &dir,
                                          int &sgn) {
  // (direction selector, sign) per position: 0 = mu, 1 = nu; sign in units of s for nu
  int sel, sg;
  switch (shape) {
    case 0: sel = (k == 1) ? 0 : 1; sg = (k == 0) ? 1 : (k == 1 ? 1 : -1); break;
    case 1: sel = (k == 1 || k == 2 || k == 4) ? 0 : 1; sg = (k == 3 || k == 4) ? -1 : 1; break;
    case 2: sel = (k == 1 || k == 4) ? 1 : 0; sg = (k == 0 || k == 4) ? -1 : 1; break;
    default: sel = (k == 2) ? 0 : 1; sg = (k >= 3) ? -1 : 1; break;
  }
  dir = sel == 0 ? mu : nu;
  sgn = sel == 0 ? sg : sg * s;
}

struct SiteCoord {
  int c[4];
};
__device__ __forceinline__ SiteCoord site_coord(int site, const Geom &g) {
  SiteCoord r;
  int v = site;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    r.c[d] = v % g.L[d];
    v /= g.L[d];
  }
  return r;
}

// Positions on the paths of link (x, mu) in the plane (mu, nu): a path moves along mu and nu only,
// so a position is x + a e_mu + b e_nu (|a|, |b| <= 2) and its site index takes two periodic wraps.
struct PlaneAddr {
  int rest;    // site index of x without its mu and nu parts
  int xm, xn;  // coordinates of x along mu and nu
  int lm, ln;  // extents along mu and nu
  int sm, sn;  // strides along mu and nu
};
__device__ __forceinline__ PlaneAddr plane_addr(const SiteCoord &x, int site, int mu, int nu,
                                                const Geom &g) {
  PlaneAddr p;
  p.xm = x.c[mu];
  p.xn = x.c[nu];
  p.lm = g.L[mu];
  p.ln = g.L[nu];
  p.sm = g.stride[mu];
  p.sn = g.stride[nu];
  p.rest = site - p.xm * p.sm - p.xn * p.sn;
  return p;
}
// v mod L for -2 L <= v < 3 L (two conditional steps each way also cover extent 1)
__device__ __forceinline__ int wrap2(int v, int L) {
  v += v < 0 ? L : 0;
  v += v < 0 ? L : 0;
  v -= v >= L ? L : 0;
  v -= v >= L ? L : 0;
  return v;
}
__device__ __forceinline__ int plane_site(const PlaneAddr &p, int a, int b) {
  return p.rest + wrap2(p.xm + a, p.lm) * p.sm + wrap2(p.xn + b, p.ln) * p.sn;
}

// link field U[dir][a][b][site] read through a buffer resource
__device__ __forceinline__ M3 load_m3r(rsrc_t r, int dir, int site, int V) {
  M3 m;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      m.e[i][j] = bld<double, double2>(r, (uint32_t)((dir * 9 + 3 * i + j) * V) * 16u, site);
  return m;
}

// Path step k of (shape, s): along mu (along = 0) or nu (1), forward (fwd) or backward, from
// the path_step table.  A forward step at position (a, b) takes U_dir(x + a e_mu + b e_nu) and
// moves on; a backward step moves first and takes the link there, daggered.
__device__ __forceinline__ void path_move(int shape, int k, int s, int &along, bool &fwd) {
  int dir, sgn;
  path_step(0, 1, s, shape, k, dir, sgn);
  along = dir;
  fwd = sgn > 0;
}
__device__ __forceinline__ M3 path_factor(rsrc_t U, const PlaneAddr &pa, int &a, int &b,
                                          int along, bool fwd, int mu, int nu, int V) {
  const int dir = along == 0 ? mu : nu;
  int &z = along == 0 ? a : b;
  if (fwd) {
    const M3 f = load_m3r(U, dir, plane_site(pa, a, b), V);
    z += 1;
    return f;
  }
  z -= 1;
  return m3_dag(load_m3r(U, dir, plane_site(pa, a, b), V));
}

// C_mu(x) = sum over the paths of their products, plaquette paths weighted wp, rectangles wr
__device__ inline M3 staple_sum(rsrc_t U, const SiteCoord &x, int site, int mu, double wp,
                                double wr, const Geom &g) {
  M3 c = m3_zero();
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const PlaneAddr pa = plane_addr(x, site, mu, nu, g);
    for (int s = 1; s >= -1; s -= 2) {
      // shapes 0 and 1 share their first two factors (nu,s)(mu,+): the plaquette closes from
      // there, the rectangle goes on from the same product and position
      int a = 0, b = 0, along;
      bool fwd;
      path_move(0, 0, s, along, fwd);
      M3 p = path_factor(U, pa, a, b, along, fwd, mu, nu, g.V);
      path_move(0, 1, s, along, fwd);
      p = m3_mul(p, path_factor(U, pa, a, b, along, fwd, mu, nu, g.V));
      if (wp != 0.0) {
        int a0 = a, b0 = b;
        path_move(0, 2, s, along, fwd);
        c = m3_axpy(c, wp, m3_mul(p, path_factor(U, pa, a0, b0, along, fwd, mu, nu, g.V)));
      }
      if (wr == 0.0) continue;
      for (int k = 2; k < path_len(1); ++k) {
        path_move(1, k, s, along, fwd);
        p = m3_mul(p, path_factor(U, pa, a, b, along, fwd, mu, nu, g.V));
      }
      c = m3_axpy(c, wr, p);
      for (int shape = 2; shape < 4; ++shape) {
        a = b = 0;
        path_move(shape, 0, s, along, fwd);
        p = path_factor(U, pa, a, b, along, fwd, mu, nu, g.V);
        for (int k = 1; k < path_len(shape); ++k) {
          path_move(shape, k, s, along, fwd);
          p = m3_mul(p, path_factor(U, pa, a, b, along, fwd, mu, nu, g.V));
        }
        c = m3_axpy(c, wr, p);
      }
    }
  }
  return c;
}

// One smearing step: out_mu(x) = exp(TA(C_mu(x) U_mu(x)^+)) U_mu(x).  Grid (ceil(V / 256), 4).
// C_out (nullable) receives the staple sums for the chain rule.
__global__ void __launch_bounds__(256)
    stout_step_kernel(const double2 *__restrict__ U, double2 *__restrict__ out,
                      double2 *__restrict__ C_out, double wp, double wr, Geom g) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int mu = blockIdx.y;
  if (site >= g.V) return;
  const SiteCoord x = site_coord(site, g);
  const M3 c = staple_sum(make_rsrc(U, 576u * (uint32_t)g.V), x, site, mu, wp, wr, g);
  if (C_out) store_m3(C_out, mu, site, g.V, c);
  const M3 u = load_m3(U, mu, site, g.V);
  const M3 e = m3_exp(m3_ta(m3_muld(c, u)));
  store_m3(out, mu, site, g.V, m3_mul(e, u));
}

// Backward of one step, the part local to each link.  With G' = dL/dRe U' + i dL/dIm U' of the
// step's output (same convention throughout):
//   dL/dE = G' U^+,  dL/dM = L(M^+, dL/dE)  (the adjoint of the Frechet derivative of exp at M),
//   dL/dOmega = (g - g^+)/2 - (i/3) Im tr(g) for g = dL/dM  (M = TA(Omega)),
//   Gamma = dL/dC = dL/dOmega U,   direct = E^+ G' + (dL/dOmega)^+ C.
// Writes Gamma and the direct part of dL/dU.  C_in (nullable): the level's staple sums.
__global__ void __launch_bounds__(256)
    stout_back_local_kernel(const double2 *__restrict__ U, const double2 *__restrict__ C_in,
                            const double2 *__restrict__ gout, double2 *__restrict__ gamma,
                            double2 *__restrict__ direct, double wp, double wr, Geom g) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int mu = blockIdx.y;
  if (site >= g.V) return;
  // the staple sums of this level from the forward pass when available
  const M3 c = C_in ? load_m3(C_in, mu, site, g.V)
                    : staple_sum(make_rsrc(U, 576u * (uint32_t)g.V), site_coord(site, g), site, mu,
                                 wp, wr, g);
  const M3 u = load_m3(U, mu, site, g.V);
  const M3 m = m3_ta(m3_muld(c, u));
  const M3 gp = load_m3(gout, mu, site, g.V);
  // exp(M^+) = exp(-M) = E^+ (M is anti-Hermitian), and dL/dM = L(M^+, G' U^+)
  M3 ed, gm;
  m3_exp_frechet(m3_scale(m, -1.0), m3_muld(gp, u), &ed, &gm);
  const M3 go = m3_ta(gm);
  store_m3(gamma, mu, site, g.V, m3_mul(go, u));
  store_m3(direct, mu, site, g.V, m3_axpy(m3_mul(ed, gp), 1.0, m3_dmul(go, c)));
}

// Backward of one step, the staple part.  Link (y, d) receives w A^+ Gamma_nu(x) B^+ (its adjoint
// for a backward step) from every staple path of every link (x, nu) that runs through it, A and B
// the path's products before and after it.  Summed over the paths through (y, d), this equals the
// derivative of (y, d)'s own staple sum C_d(y) in the direction Gamma: every factor of each of its
// staple paths replaced in turn by the Gamma matrix of the same link, daggered like the factor
// (the staple sum is the gradient of the gauge action, whose second derivative is symmetric).  So
// each link walks its own 24 paths once, carrying the product X and its derivative T:
//   X <- X F,  T <- T F + X Gamma(F).
// out = direct + sum_paths w T: dL/dU of the step's input.  Grid (ceil(V / 256), 4).
// factor of path step (dir, sgn) at `pos` of U and the same link of Gamma (both daggered for a
// backward step); pos is advanced
__device__ __forceinline__ void path_factor2(rsrc_t U, rsrc_t Gm, const PlaneAddr &pa, int &a,
                                             int &b, int along, bool fwd, int mu, int nu, int V,
                                             M3 &f, M3 &gf) {
  const int dir = along == 0 ? mu : nu;
  int &z = along == 0 ? a : b;
  if (fwd) {
    const int site = plane_site(pa, a, b);
    f = load_m3r(U, dir, site, V);
    gf = load_m3r(Gm, dir, site, V);
    z += 1;
  } else {
    z -= 1;
    const int site = plane_site(pa, a, b);
    f = m3_dag(load_m3r(U, dir, site, V));
    gf = m3_dag(load_m3r(Gm, dir, site, V));
  }
}

__global__ void __launch_bounds__(256)
    stout_back_gather_kernel(const double2 *__restrict__ U, const double2 *__restrict__ gamma,
                             const double2 *__restrict__ direct, double2 *__restrict__ out,
                             double wp, double wr, Geom g) {
  const int site = blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y;
  if (site >= g.V) return;
  const SiteCoord y = site_coord(site, g);
  const rsrc_t ru = make_rsrc(U, 576u * (uint32_t)g.V);
  const rsrc_t rg = make_rsrc(gamma, 576u * (uint32_t)g.V);
  M3 acc = load_m3(direct, d, site, g.V);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == d) continue;
    const PlaneAddr pa = plane_addr(y, site, d, nu, g);
    for (int s = 1; s >= -1; s -= 2) {
      // shapes 0 and 1 share their first two factors (nu,s)(mu,+): the plaquette closes from
      // there, the rectangle goes on from the same (X, T) and position
      int a = 0, b = 0, along;
      bool fwd;
      M3 x, t, f, gf;
      path_move(0, 0, s, along, fwd);
      path_factor2(ru, rg, pa, a, b, along, fwd, d, nu, g.V, x, t);
      path_move(0, 1, s, along, fwd);
      path_factor2(ru, rg, pa, a, b, along, fwd, d, nu, g.V, f, gf);
      t = m3_axpy(m3_mul(t, f), 1.0, m3_mul(x, gf));
      x = m3_mul(x, f);
      if (wp != 0.0) {
        int a0 = a, b0 = b;
        path_move(0, 2, s, along, fwd);
        path_factor2(ru, rg, pa, a0, b0, along, fwd, d, nu, g.V, f, gf);
        acc = m3_axpy(acc, wp, m3_axpy(m3_mul(t, f), 1.0, m3_mul(x, gf)));
      }
      if (wr == 0.0) continue;
      for (int k = 2; k < path_len(1); ++k) {
        path_move(1, k, s, along, fwd);
        path_factor2(ru, rg, pa, a, b, along, fwd, d, nu, g.V, f, gf);
        t = m3_axpy(m3_mul(t, f), 1.0, m3_mul(x, gf));
        if (k + 1 < path_len(1)) x = m3_mul(x, f);
      }
      acc = m3_axpy(acc, wr, t);
      for (int shape = 2; shape < 4; ++shape) {
        a = b = 0;
        path_move(shape, 0, s, along, fwd);
        path_factor2(ru, rg, pa, a, b, along, fwd, d, nu, g.V, x, t);
        const int len = path_len(shape);
        for (int k = 1; k < len; ++k) {
          path_move(shape, k, s, along, fwd);
          path_factor2(ru, rg, pa, a, b, along, fwd, d, nu, g.V, f, gf);
          t = m3_axpy(m3_mul(t, f), 1.0, m3_mul(x, gf));
          if (k + 1 < len) x = m3_mul(x, f);
        }
        acc = m3_axpy(acc, wr, t);
      }
    }
  }
  store_m3(out, d, site, g.V, acc);
}

}  // namespace ovl
