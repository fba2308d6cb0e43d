// HIP kernels of the overlap-operator library (gfx950, wave64).
//
// One thread per lattice site (and right-hand side), site-fastest coalesced loads of spinors and
// links, half-spinor projection of every hop, and every per-step vector operation of the
// Chebyshev recurrence fused into the stencil kernel, so one K application of the recurrence is
// one pass over memory (the kernel merging the paper credits with its largest gain, Sec. 2).
#pragma once

#include "common.hpp"
#include "stencil.hpp"

namespace ovl {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)

// ---------------------------------------------------------------------------------------------
// block-wide FP64 sum of NV values per thread, result valid in thread 0 (fixed order: wave
// butterfly, then waves in index order -> deterministic)
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double *lds /* >= NV * 16 */) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nwave; ++w) s += lds[w * NV + k];
      v[k] = s;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Fused stencil step.  For every site and right-hand side r:
//   y   = kd v(x) + kh hop(v)(x)              (hop = the sum in eq. 2; v read with gamma5 if v_g5)
//   y   = gamma5 y                            (if y_g5)
//   res = y + a src(x) + t w(x)               (src read with gamma5 if src_g5; w may alias out)
// final modes add the deflation correction sum_i phi_i w_i c_i and combine into the overlap
// operator; they also emit FP64 block partials of ||res||^2 and ||src||^2.
enum : int { MODE_STEP = 0, MODE_SIGN = 1, MODE_OVERLAP = 2, MODE_OVERLAP_DAG = 3 };
// which vector of an item a step reads as v / w or writes as out
enum : int { ROLE_NONE = -1, ROLE_PSI = 0, ROLE_B0 = 1, ROLE_B1 = 2, ROLE_B2 = 3 };

// One lattice problem of a step launch.  A launch covers up to NI problems (different gauge
// fields, volumes and right-hand-side counts) that share the step's coefficients.
struct StepItem {
  const void *U;          // packed links, blocks of 64 sites: [V / 64][36][64] (link storage)
  const void *psi;        // source [nrhs][12][V]: the alpha_k term and the overlap combine
  void *buf[3];           // vectors addressed by role
  const void *phi;        // deflation basis [n_ev][12][V] (spinor storage), final modes
  const double2 *c;       // [nrhs][n_ev] projections
  const double *wdefl;    // [n_ev] weights
  double *norm_partial;   // [nblk * nrhs][2] or null
  Geom g;
  int lstride;            // elements between consecutive link components inside a block (64)
  int r12;                // the field allows two-row link reads (SU(3) within its tolerance)
  // Workgroup order.  ty > 0: the (x, y, z) volume is cut into tiles of Lx x ty x tz sites
  // (whole x lines); consecutive workgroups cover one t-slice of a tile, then the same tile at
  // t + 1, ... through all t, then the next tile.  The t-, z- and y-neighbours a workgroup reads
  // were then touched by workgroups that ran a tile-slice (well under 2 MB) earlier and are still
  // in the XCD's L2; halos arise only on the y and z faces of a tile.  ty = 0: memory order.
  int ty, tz;
  int n_ev, nrhs;
  int blk0;               // first global logical workgroup of this item
  // Twin recurrence (plain steps only, nrhs = 2): right-hand side 1 is a second, independent
  // vector set on the same field -- it reads twin_psi / twin_buf by role, without the
  // right-hand-side offset, and takes the coefficient twin_a instead of the launch's a -- so two
  // recurrences advance in one launch and share every link read.
  int twin;
  const void *twin_psi;
  void *twin_buf[3];
  double twin_a;
  // Right-hand-side groups of the workgroup order: right-hand-side blocks run fastest inside
  // groups of rgroup blocks, then the site blocks, then the groups (0: one group of all).
  int rgroup;
};

// item-local workgroup lb -> (right-hand-side block rb, site block b) for nrb right-hand-side
// blocks and nsb site blocks.  Inside a group the workgroups that read the same links run side by
// side (they share them through L2); with many right-hand sides, groups keep the spinor data
// between a site and its t neighbour within one XCD's L2.
__device__ __forceinline__ void item_block(const StepItem &I, int lb, int nrb, int nsb, int &rb,
                                           int &b) {
  const int gs = (I.rgroup > 0 && I.rgroup < nrb) ? I.rgroup : nrb;
  const int full = nrb / gs;      // groups of gs blocks; a last, smaller group follows
  const int span = gs * nsb;
  const int gi = min(lb / span, full);
  const int gl = gi < full ? gs : nrb - full * gs;
  const int within = lb - gi * span;
  rb = gi * gs + within % gl;
  b = within / gl;
}

// address of a role's vector for right-hand side r of an item
template <class SE>
__device__ __forceinline__ const SE *role_vec(const StepItem &I, int role, int r, int V) {
  if (I.twin && r == 1)
    return reinterpret_cast<const SE *>(role == ROLE_PSI ? I.twin_psi : I.twin_buf[role - 1]);
  const void *ptr = role == ROLE_PSI ? I.psi : I.buf[role - 1];
  return reinterpret_cast<const SE *>(ptr) + (int64_t)r * 12 * V;
}
__device__ __forceinline__ double role_a(const StepItem &I, double a, int r) {
  return (I.twin && r == 1) ? I.twin_a : a;
}

// Step coefficients plus the problems of one launch: a single problem travels in the kernel
// arguments (TABLE = false); a batch reads its item table from device memory (TABLE = true),
// written once per evaluation by write_item_kernel, so the arguments stay small.
template <bool TABLE>
struct StepArgs {
  double kd, kh, a, t, mu;
  int v_role, w_role, out_role;
  int v_g5, src_g5, y_g5, mode, remap, n_items;
  int r12;                // TABLE: every item allows two-row link reads
  int total_blocks;       // workgroups of the launch
  const StepItem *table;  // TABLE: n_items items in device memory
  StepItem item;          // !TABLE: the one problem
};

__global__ void write_item_kernel(StepItem it, StepItem *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = it;
}

// Both hops of direction MU (compile-time: kernels whose waves each take one direction) for one
// site, neighbours read raw with s5 = -1 applying gamma5; links read at lfw / lbw, or (PRE) taken
// from mfw / mbw read earlier.
template <int MU, bool PRE, class C, class SE, class LE>
__device__ __forceinline__ void site_hops_k(cx<C> acc[12], rsrc_t v, uint32_t cs, rsrc_t U,
                                            uint32_t ls, int fwd, int bwd, uint32_t lfw,
                                            uint32_t lbw, bool r12, C s5, const cx<C> mfw[3][3],
                                            const cx<C> mbw[3][3]) {
  cx<C> u[2][3], d[2][3];
  load_spinor<C, SE>(v, cs, fwd, false, u, d);
  if constexpr (PRE) {
    hop_apply_k<C, false, MU, 1>(acc, u, d, mfw, s5);
  } else {
    cx<C> m[3][3];
    load_link3<C, LE>(U, ls, lfw, r12, m);
    hop_apply_k<C, false, MU, 1>(acc, u, d, m, s5);
  }
  load_spinor<C, SE>(v, cs, bwd, false, u, d);
  if constexpr (PRE) {
    hop_apply_k<C, true, MU, -1>(acc, u, d, mbw, s5);
  } else {
    cx<C> m[3][3];
    load_link3<C, LE>(U, ls, lbw, r12, m);
    hop_apply_k<C, true, MU, -1>(acc, u, d, m, s5);
  }
}

// Fused stencil step.  For every site and right-hand side r of every item:
//   y   = kd v(x) + kh hop(v)(x)              (hop = the sum in eq. 2; v read with gamma5 if v_g5)
//   y   = gamma5 y                            (if y_g5)
//   res = y + a psi(x) + t w(x)               (psi read with gamma5 if src_g5; w may alias out)
// final modes add the deflation correction sum_i phi_i w_i c_i and combine into the overlap
// operator; they also emit FP64 block partials of ||res||^2 and ||psi||^2.
//
// NQ * SPB threads cover SPB sites.  NQ = 4: thread (q = threadIdx.x / SPB, sl = threadIdx.x %
// SPB) owns direction q (both hops) for the hopping sum and spin component q for everything after
// the LDS reduction.  NQ = 8 (small launches, bound by one wave's latency chain): threads q and
// q + 4 take the forward and the backward hop of direction q, which halves the loads and the
// arithmetic on each thread's path; threads q < 4 own the spin components afterwards.  Within
// an item the right-hand side is the fastest logical index inside each right-hand-side group
// (item_block), so the workgroups that read the same links run together and share them through
// L2.
//
// RB > 1 (right-hand-side block, NQ = 4): a workgroup takes RB consecutive right-hand sides of
// its sites; each thread reads its direction's two links once into registers and reuses them for
// the RB right-hand sides, one after the other (the LDS exchange is reused per right-hand side).
template <class C, class SE, class LE, int SPB, bool TABLE, int NQ = 4, bool R12 = false,
          int RB = 1>
__global__ void __launch_bounds__(NQ * SPB) step_kernel(StepArgs<TABLE> p) {
  static_assert(NQ == 4 || NQ == 8, "4 or 8 threads per site");
  static_assert(RB == 1 || NQ == 4, "right-hand-side blocks take four threads per site");
  __shared__ double lds[2 * 16];
  __shared__ cx<C> part[NQ][12][SPB];  // directional partial sums
  const int gb = xcd_block(blockIdx.x, gridDim.x, p.remap);
  int it = 0;
  if (TABLE)
    for (int i = 1; i < p.n_items; ++i)
      if (p.table[i].blk0 <= gb) it = i;
  const StepItem &I = TABLE ? p.table[it] : p.item;
  const Ext4 ex = ext_of(I.g);
  constexpr bool r12 = R12;  // two-row links (a launch-wide choice)
  const int nrhs = I.nrhs;
  const int nrb = (nrhs + RB - 1) / RB;  // right-hand-side blocks of the item
  const int lb = gb - I.blk0;
  int rbk, b;
  item_block(I, lb, nrb, (ex.V + SPB - 1) / SPB, rbk, b);
  const int r0 = rbk * RB;
  const int q = threadIdx.x / SPB;
  const int sl = threadIdx.x % SPB;
  const int dq = q & 3;       // direction of the thread's hop(s)
  const bool owner = q < 4;   // owns spin component q after the exchange
  Coord4 c4;
  int site;
  bool active;
  if (I.ty > 0) {
    const int slice = ex.lx * I.ty * I.tz;  // sites of one tile at one t
    const int nsub = slice / SPB;
    int tb = b;
    const int sub = tb % nsub;
    tb /= nsub;
    c4.t = tb % ex.lt;
    const int tile = tb / ex.lt;
    const int nty = ex.ly / I.ty;
    const int local = sub * SPB + sl;
    c4.x = local % ex.lx;
    const int rr = local / ex.lx;
    c4.y = (tile % nty) * I.ty + rr % I.ty;
    c4.z = (tile / nty) * I.tz + rr / I.ty;
    site = c4.x + ex.sy * c4.y + ex.sz * c4.z + ex.st * c4.t;
    active = true;
  } else {
    site = b * SPB + sl;
    active = site < ex.V;
    c4 = coords_of(ex, active ? site : 0);
  }
  const int V = ex.V;
  const uint32_t cs = (uint32_t)V * elem_traits<SE>::bytes;  // component stride (bytes)
  const uint32_t vb = 12u * cs;                               // one right-hand side (bytes)
  const uint32_t ls = (uint32_t)I.lstride * elem_traits<LE>::bytes;
  const bool lower = q >= 2;                                  // spin components 2, 3
  const bool vg5 = p.v_g5 != 0;
  int fwd = 0, bwd = 0;
  if (active) dir_neighbours(ex, c4, site, dq, fwd, bwd);
  const DirCoef<C> k = dir_coef<C>(dq);
  const uint32_t lane_links = (uint32_t)dq * 9u * (uint32_t)I.lstride;
  // with at least 64 sites per workgroup and four threads per site, a wave takes one direction
  constexpr bool kSpec = SPB % 64 == 0 && NQ == 4;
  // right-hand-side blocks: the thread's two links, read once for the RB right-hand sides
  cx<C> mfw[RB > 1 ? 3 : 1][3], mbw[RB > 1 ? 3 : 1][3];
  if constexpr (RB > 1) {
    if (active) {
      const rsrc_t U = make_rsrc(I.U, link_bytes(ex.V, ls));
      load_link3<C, LE>(U, ls, lane_links + link_lane(site), r12, mfw);
      load_link3<C, LE>(U, ls, lane_links + link_lane(bwd), r12, mbw);
    }
  }
  // After the LDS exchange the thread owns spin component q of its site.  Small launches
  // (SPB < 64: few waves per CU, bound by memory latency) load the operands of that component's
  // vector algebra before the stencil so the two latencies overlap; large launches load them
  // after the exchange and keep the registers for occupancy.
  constexpr bool kEarly = SPB < 64;
  const uint32_t e0 = (uint32_t)(3 * q) * (uint32_t)V + site;  // element of component 3q
#pragma unroll 1
  for (int rr = 0; rr < RB; ++rr) {
    const int r = r0 + rr;
    const bool ractive = r < nrhs;   // the last block of an item may be ragged
    const bool act = active && ractive;
    const int rv = ractive ? r : 0;
    auto vec = [&](int role) -> const SE * { return role_vec<SE>(I, role, rv, V); };
    const double pa = role_a(I, p.a, rv);
    const bool need_src = (pa != 0.0) || p.mode >= MODE_SIGN;
    double nrm[2] = {0.0, 0.0};
    const rsrc_t v = make_rsrc(vec(p.v_role), vb);
    cx<C> vx[3], srcx[3], wx[3];
    auto load_ops = [&]() {
#pragma unroll
      for (int c = 0; c < 3; ++c) vx[c] = srcx[c] = wx[c] = mk<C>(0, 0);
      if (!act || !owner) return;
#pragma unroll
      for (int c = 0; c < 3; ++c) vx[c] = bldv<C, SE>(v, e0 + c * V);
      if (need_src) {
        const rsrc_t sr = make_rsrc(vec(ROLE_PSI), vb);
#pragma unroll
        for (int c = 0; c < 3; ++c) srcx[c] = bldv<C, SE>(sr, e0 + c * V);
      }
      if (p.w_role != ROLE_NONE) {
        const rsrc_t w = make_rsrc(vec(p.w_role), vb);
#pragma unroll
        for (int c = 0; c < 3; ++c) wx[c] = bldv<C, SE>(w, e0 + c * V);
      }
    };
    if (kEarly) load_ops();
    {
      cx<C> acc[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) acc[i] = mk<C>(0, 0);
      if (act && kSpec) {
        // SPB >= 64: the wave's direction is uniform, one specialised path per direction
        const rsrc_t U = make_rsrc(I.U, link_bytes(ex.V, ls));
        const uint32_t lfw = lane_links + link_lane(site), lbw = lane_links + link_lane(bwd);
        const C s5 = vg5 ? C(-1) : C(1);
        switch (dq) {
          case 0: site_hops_k<0, (RB > 1), C, SE, LE>(acc, v, cs, U, ls, fwd, bwd, lfw, lbw, r12, s5, mfw, mbw); break;
          case 1: site_hops_k<1, (RB > 1), C, SE, LE>(acc, v, cs, U, ls, fwd, bwd, lfw, lbw, r12, s5, mfw, mbw); break;
          case 2: site_hops_k<2, (RB > 1), C, SE, LE>(acc, v, cs, U, ls, fwd, bwd, lfw, lbw, r12, s5, mfw, mbw); break;
          default: site_hops_k<3, (RB > 1), C, SE, LE>(acc, v, cs, U, ls, fwd, bwd, lfw, lbw, r12, s5, mfw, mbw); break;
        }
      } else if (act) {
        if constexpr (RB > 1) {
          cx<C> u[2][3], d[2][3];
          load_spinor<C, SE>(v, cs, fwd, vg5, u, d);
          hop_apply<C, false>(acc, u, d, mfw, k, C(1));
          load_spinor<C, SE>(v, cs, bwd, vg5, u, d);
          hop_apply<C, true>(acc, u, d, mbw, k, C(-1));
        } else {
          const rsrc_t U = make_rsrc(I.U, link_bytes(ex.V, ls));
          if (NQ == 4) {
            quad_hop<C, SE, LE, false>(acc, v, cs, U, ls, fwd, lane_links + link_lane(site), k,
                                       C(1), vg5, r12);
            quad_hop<C, SE, LE, true>(acc, v, cs, U, ls, bwd, lane_links + link_lane(bwd), k,
                                      C(-1), vg5, r12);
          } else {
            const bool bw = q >= 4;
            quad_hop_sel<C, SE, LE>(acc, v, cs, U, ls, bw ? bwd : fwd,
                                    lane_links + link_lane(bw ? bwd : site), k, bw, vg5, r12);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 12; ++i) part[q][i][sl] = acc[i];
    }
    __syncthreads();
    if (!kEarly) load_ops();
    if (act && owner) {
      cx<C> hop[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        hop[c] = part[0][3 * q + c][sl] + part[1][3 * q + c][sl] + part[2][3 * q + c][sl] +
                 part[3][3 * q + c][sl];
        if (NQ == 8)
          hop[c] = hop[c] + (part[4][3 * q + c][sl] + part[5][3 * q + c][sl] +
                             part[6][3 * q + c][sl] + part[7][3 * q + c][sl]);
      }
      const C kd = C(p.kd), kh = C(p.kh);
      cx<C> res[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<C> x = (vg5 && lower) ? -vx[c] : vx[c];
        cx<C> y = mk<C>(kd * x.re + kh * hop[c].re, kd * x.im + kh * hop[c].im);
        if (p.y_g5 && lower) y = -y;
        res[c] = y;
      }
      if (pa != 0.0) {
        const C a = (p.src_g5 && lower) ? C(-pa) : C(pa);
#pragma unroll
        for (int c = 0; c < 3; ++c) res[c] = res[c] + scale(srcx[c], a);
      }
      if (p.w_role != ROLE_NONE) {
        const C t = C(p.t);
#pragma unroll
        for (int c = 0; c < 3; ++c) res[c] = res[c] + scale(wx[c], t);
      }
      if (p.mode >= MODE_SIGN) {
        for (int e = 0; e < I.n_ev; ++e) {
          const rsrc_t ph = make_rsrc(reinterpret_cast<const SE *>(I.phi) + (int64_t)e * 12 * V, vb);
          const double2 ce = I.c[r * I.n_ev + e];
          const double we = I.wdefl[e];
          const cx<C> d = mk<C>(C(ce.x * we), C(ce.y * we));
#pragma unroll
          for (int c = 0; c < 3; ++c) res[c] = cmadd(res[c], bldv<C, SE>(ph, e0 + c * V), d);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          nrm[0] += double(res[c].re) * double(res[c].re) + double(res[c].im) * double(res[c].im);
          nrm[1] += double(srcx[c].re) * double(srcx[c].re) + double(srcx[c].im) * double(srcx[c].im);
        }
        if (p.mode == MODE_OVERLAP || p.mode == MODE_OVERLAP_DAG) {
          const C hp = C(0.5 * (1.0 + p.mu));
          const C hm = (p.mode == MODE_OVERLAP && lower) ? C(-0.5 * (1.0 - p.mu)) : C(0.5 * (1.0 - p.mu));
#pragma unroll
          for (int c = 0; c < 3; ++c) res[c] = scale(srcx[c], hp) + scale(res[c], hm);
        }
      }
      const rsrc_t o = make_rsrc(vec(p.out_role), vb);
#pragma unroll
      for (int c = 0; c < 3; ++c) bstv<C, SE>(o, e0 + c * V, res[c]);
    }
    if (I.norm_partial != nullptr && p.mode >= MODE_SIGN) {
      block_sum<2>(nrm, lds);
      if (threadIdx.x == 0 && ractive) {
        const int64_t pb = (int64_t)b * nrhs + r;  // partial of (site block b, right-hand side r)
        I.norm_partial[pb * 2 + 0] = nrm[0];
        I.norm_partial[pb * 2 + 1] = nrm[1];
      }
    }
    if constexpr (RB > 1) __syncthreads();  // part[] and lds[] are reused by the next one
  }
}

// ---------------------------------------------------------------------------------------------
// The same fused step with two x-adjacent sites (x even, x + 1) per lane, for FP32 spinors with
// FP32 or BF16 links and an even Lx.  Every spinor, link and output access of a pair is one
// 16-byte (links in BF16: 8-byte) lane access, which halves the vector-memory instructions per
// site; the x direction needs the own pair plus the single sites x + 2 and x - 1.  SPB pairs per
// workgroup, 4 * SPB threads; with SPB = 64 each wave works on one direction.
template <class SE>
__device__ __forceinline__ void load_spinor_pair(rsrc_t v, uint32_t cs, uint32_t s0, bool g5,
                                                 cx<float> u0[2][3], cx<float> d0[2][3],
                                                 cx<float> u1[2][3], cx<float> d1[2][3]) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bld2<SE>(v, (sp * 3 + c) * cs, s0, u0[sp][c], u1[sp][c]);
      cx<float> x0, x1;
      bld2<SE>(v, ((sp + 2) * 3 + c) * cs, s0, x0, x1);
      d0[sp][c] = g5 ? -x0 : x0;
      d1[sp][c] = g5 ? -x1 : x1;
    }
}

// the links of two x-adjacent sites (r12: two stored rows, the third completed)
template <class LE>
__device__ __forceinline__ void load_link_pair(rsrc_t U, uint32_t ls, uint32_t l0, bool r12,
                                               cx<float> m0[3][3], cx<float> m1[3][3]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) bld2<LE>(U, (a * 3 + b) * ls, l0, m0[a][b], m1[a][b]);
  if (r12) {
    su3_row2(m0);
    su3_row2(m1);
  } else {
#pragma unroll
    for (int b = 0; b < 3; ++b) bld2<LE>(U, (6 + b) * ls, l0, m0[2][b], m1[2][b]);
  }
}

// both hops of direction MU (a compile-time constant: every wave of the two-sites-per-lane kernel
// takes one direction) for the pair (s0, s0 + 1): accA / accB += the direction's part of the
// hopping sum at s0 / s0 + 1; the neighbours are read raw and s5 = -1 applies gamma5 to them
template <int MU, class LE, bool R12>
__device__ __forceinline__ void pair_hops_k(const StepItem &I, const Ext4 &ex, const Coord4 &c4,
                                            int s0, rsrc_t v, uint32_t cs, float s5,
                                            cx<float> accA[12], cx<float> accB[12]) {
  using C = float;
  using SE = float2;
  const uint32_t ls = (uint32_t)I.lstride * elem_traits<LE>::bytes;
  const rsrc_t U = make_rsrc(I.U, link_bytes(ex.V, ls));
  const uint32_t ll = (uint32_t)MU * 9u * (uint32_t)I.lstride;
  if constexpr (MU == 0) {
    const int xn = (c4.x + 2 == ex.lx) ? s0 + 2 - ex.lx : s0 + 2;  // site x + 2
    const int xp = (c4.x == 0) ? s0 + ex.lx - 1 : s0 - 1;          // site x - 1
    {
      cx<C> u0[2][3], d0[2][3], u1[2][3], d1[2][3], m0[3][3], m1[3][3];
      load_spinor_pair<SE>(v, cs, s0, false, u0, d0, u1, d1);
      load_link_pair<LE>(U, ls, ll + link_lane(s0), R12, m0, m1);
      hop_apply_k<C, false, 0, 1>(accA, u1, d1, m0, s5);  // x:     psi(x + 1), U(x)
      hop_apply_k<C, true, 0, -1>(accB, u0, d0, m0, s5);  // x + 1: psi(x), U(x)^+
      cx<C> un[2][3], dn[2][3];
      load_spinor<C, SE>(v, cs, xn, false, un, dn);
      hop_apply_k<C, false, 0, 1>(accB, un, dn, m1, s5);  // x + 1: psi(x + 2), U(x + 1)
    }
    {
      cx<C> up[2][3], dp[2][3], mp[3][3];
      load_spinor<C, SE>(v, cs, xp, false, up, dp);
      load_link3<C, LE>(U, ls, ll + link_lane(xp), R12, mp);
      hop_apply_k<C, true, 0, -1>(accA, up, dp, mp, s5);  // x: psi(x - 1), U(x - 1)^+
    }
  } else {
    int fwd, bwd;
    dir_neighbours(ex, c4, s0, MU, fwd, bwd);
    {
      cx<C> u0[2][3], d0[2][3], u1[2][3], d1[2][3], m0[3][3], m1[3][3];
      load_spinor_pair<SE>(v, cs, fwd, false, u0, d0, u1, d1);
      load_link_pair<LE>(U, ls, ll + link_lane(s0), R12, m0, m1);
      hop_apply_k<C, false, MU, 1>(accA, u0, d0, m0, s5);
      hop_apply_k<C, false, MU, 1>(accB, u1, d1, m1, s5);
    }
    {
      cx<C> u0[2][3], d0[2][3], u1[2][3], d1[2][3], m0[3][3], m1[3][3];
      load_spinor_pair<SE>(v, cs, bwd, false, u0, d0, u1, d1);
      load_link_pair<LE>(U, ls, ll + link_lane(bwd), R12, m0, m1);
      hop_apply_k<C, true, MU, -1>(accA, u0, d0, m0, s5);
      hop_apply_k<C, true, MU, -1>(accB, u1, d1, m1, s5);
    }
  }
}

template <class LE, int SPB, bool TABLE, bool R12 = false>
__global__ void __launch_bounds__(4 * SPB) step2_kernel(StepArgs<TABLE> p) {
  static_assert(SPB % 64 == 0, "one direction per wave");
  using C = float;
  using SE = float2;
  __shared__ double lds[2 * 16];
  __shared__ cx<C> part[4][12][2 * SPB];  // directional partial sums, two sites per pair
  const int gb = xcd_block(blockIdx.x, gridDim.x, p.remap);
  int it = 0;
  if (TABLE)
    for (int i = 1; i < p.n_items; ++i)
      if (p.table[i].blk0 <= gb) it = i;
  const StepItem &I = TABLE ? p.table[it] : p.item;
  const Ext4 ex = ext_of(I.g);
  const int nrhs = I.nrhs;
  const int lb = gb - I.blk0;
  int r, b;
  item_block(I, lb, nrhs, (ex.V + 2 * SPB - 1) / (2 * SPB), r, b);
  const int q = threadIdx.x / SPB;
  const int sl = threadIdx.x % SPB;
  Coord4 c4;
  int s0;  // first site of the pair (x even)
  bool active;
  if (I.ty > 0) {
    const int slice = ex.lx * I.ty * I.tz;
    const int nsub = slice / (2 * SPB);
    int tb = b;
    const int sub = tb % nsub;
    tb /= nsub;
    c4.t = tb % ex.lt;
    const int tile = tb / ex.lt;
    const int nty = ex.ly / I.ty;
    const int local = 2 * (sub * SPB + sl);
    c4.x = local % ex.lx;
    const int rr = local / ex.lx;
    c4.y = (tile % nty) * I.ty + rr % I.ty;
    c4.z = (tile / nty) * I.tz + rr / I.ty;
    s0 = c4.x + ex.sy * c4.y + ex.sz * c4.z + ex.st * c4.t;
    active = true;
  } else {
    s0 = 2 * (b * SPB + sl);
    active = s0 < ex.V;
    c4 = coords_of(ex, active ? s0 : 0);
  }
  const int V = ex.V;
  const uint32_t cs = (uint32_t)V * elem_traits<SE>::bytes;
  const uint32_t vb = 12u * cs;
  const bool lower = q >= 2;
  auto vec = [&](int role) -> const SE * { return role_vec<SE>(I, role, r, V); };
  const double pa = role_a(I, p.a, r);
  double nrm[2] = {0.0, 0.0};
  const rsrc_t v = make_rsrc(vec(p.v_role), vb);
  const bool vg5 = p.v_g5 != 0;
  {
    cx<C> accA[12], accB[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) accA[i] = accB[i] = mk<C>(0, 0);
    if (active) {
      // the wave's direction q is uniform: one specialised path per direction
      const C s5 = vg5 ? C(-1) : C(1);
      switch (q) {
        case 0: pair_hops_k<0, LE, R12>(I, ex, c4, s0, v, cs, s5, accA, accB); break;
        case 1: pair_hops_k<1, LE, R12>(I, ex, c4, s0, v, cs, s5, accA, accB); break;
        case 2: pair_hops_k<2, LE, R12>(I, ex, c4, s0, v, cs, s5, accA, accB); break;
        default: pair_hops_k<3, LE, R12>(I, ex, c4, s0, v, cs, s5, accA, accB); break;
      }
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      part[q][i][2 * sl] = accA[i];
      part[q][i][2 * sl + 1] = accB[i];
    }
  }
  __syncthreads();
  if (active) {
    cx<C> hop[2][3];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        hop[j][c] = part[0][3 * q + c][2 * sl + j] + part[1][3 * q + c][2 * sl + j] +
                    part[2][3 * q + c][2 * sl + j] + part[3][3 * q + c][2 * sl + j];
    const C kd = C(p.kd), kh = C(p.kh);
    const uint32_t e0 = (uint32_t)(3 * q) * (uint32_t)V + s0;  // even
    cx<C> res[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<C> vx[2];
      bldv2<SE>(v, e0 + c * V, vx[0], vx[1]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const cx<C> x = (vg5 && lower) ? -vx[j] : vx[j];
        cx<C> y = mk<C>(kd * x.re + kh * hop[j][c].re, kd * x.im + kh * hop[j][c].im);
        if (p.y_g5 && lower) y = -y;
        res[j][c] = y;
      }
    }
    cx<C> srcx[2][3];
    const bool need_src = (pa != 0.0) || p.mode >= MODE_SIGN;
    if (need_src) {
      const rsrc_t sr = make_rsrc(vec(ROLE_PSI), vb);
#pragma unroll
      for (int c = 0; c < 3; ++c) bldv2<SE>(sr, e0 + c * V, srcx[0][c], srcx[1][c]);
    }
    if (pa != 0.0) {
      const C a = (p.src_g5 && lower) ? C(-pa) : C(pa);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) res[j][c] = res[j][c] + scale(srcx[j][c], a);
    }
    if (p.w_role != ROLE_NONE) {
      const rsrc_t w = make_rsrc(vec(p.w_role), vb);
      const C t = C(p.t);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<C> w0, w1;
        bldv2<SE>(w, e0 + c * V, w0, w1);
        res[0][c] = res[0][c] + scale(w0, t);
        res[1][c] = res[1][c] + scale(w1, t);
      }
    }
    if (p.mode >= MODE_SIGN) {
      for (int e = 0; e < I.n_ev; ++e) {
        const rsrc_t ph = make_rsrc(reinterpret_cast<const SE *>(I.phi) + (int64_t)e * 12 * V, vb);
        const double2 ce = I.c[r * I.n_ev + e];
        const double we = I.wdefl[e];
        const cx<C> d = mk<C>(C(ce.x * we), C(ce.y * we));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cx<C> f0, f1;
          bldv2<SE>(ph, e0 + c * V, f0, f1);
          res[0][c] = cmadd(res[0][c], f0, d);
          res[1][c] = cmadd(res[1][c], f1, d);
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          nrm[0] += double(res[j][c].re) * double(res[j][c].re) +
                    double(res[j][c].im) * double(res[j][c].im);
          nrm[1] += double(srcx[j][c].re) * double(srcx[j][c].re) +
                    double(srcx[j][c].im) * double(srcx[j][c].im);
        }
      if (p.mode == MODE_OVERLAP || p.mode == MODE_OVERLAP_DAG) {
        const C hp = C(0.5 * (1.0 + p.mu));
        const C hm = (p.mode == MODE_OVERLAP && lower) ? C(-0.5 * (1.0 - p.mu)) : C(0.5 * (1.0 - p.mu));
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) res[j][c] = scale(srcx[j][c], hp) + scale(res[j][c], hm);
      }
    }
    const rsrc_t o = make_rsrc(vec(p.out_role), vb);
#pragma unroll
    for (int c = 0; c < 3; ++c) bstv2<SE>(o, e0 + c * V, res[0][c], res[1][c]);
  }
  if (I.norm_partial != nullptr && p.mode >= MODE_SIGN) {
    block_sum<2>(nrm, lds);
    if (threadIdx.x == 0) {
      const int64_t pb = (int64_t)b * nrhs + r;  // partial of (site block b, right-hand side r)
      I.norm_partial[pb * 2 + 0] = nrm[0];
      I.norm_partial[pb * 2 + 1] = nrm[1];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Slab form of the fused step for large lattices.  A workgroup covers the slab of whole x lines
// y0 .. y0 + ny - 1 at one (z, t), SPB = 64 NW = Lx ny sites, 4 SPB threads (NW waves per
// direction).  The slab's spinors and the two neighbouring rows y0 - 1 and y0 + ny (periodic)
// are staged in LDS once, so the x and y neighbours and the site's own value come from LDS
// instead of four separate global reads; the x links are shared through LDS for the backward x
// hop.  The z and t directions read global memory as in the one-site form.  The directional
// partial sums are combined in a fixed order, ((x + z) + (y + t)).  Dynamic LDS:
//   stage  [12][(ny + 2) Lx] complex,  slots [2][12][SPB] complex,  xlink [9][SPB] complex.
template <class C>
__host__ __device__ constexpr int slab_lds_bytes(int spb, int lx) {
  return (12 * (spb + 2 * lx) + 2 * 12 * spb + 9 * spb) * (int)sizeof(cx<C>);
}

template <class C, class SE, class LE, int NW, bool TABLE, bool R12 = false>
__global__ void __launch_bounds__(256 * NW) step_slab_kernel(StepArgs<TABLE> p) {
  constexpr int SPB = 64 * NW;
  extern __shared__ __align__(16) unsigned char slab_smem[];
  __shared__ double lds[2 * 16];
  const int gb = xcd_block(blockIdx.x, gridDim.x, p.remap);
  int it = 0;
  if (TABLE)
    for (int i = 1; i < p.n_items; ++i)
      if (p.table[i].blk0 <= gb) it = i;
  const StepItem &I = TABLE ? p.table[it] : p.item;
  const Ext4 ex = ext_of(I.g);
  constexpr bool r12 = R12;  // two-row links (a launch-wide choice)
  const int nrhs = I.nrhs;
  const int lb = gb - I.blk0;
  int r, b;
  item_block(I, lb, nrhs, ex.V / SPB, r, b);
  const int ny = SPB / ex.lx;
  const int nstage = SPB + 2 * ex.lx;
  cx<C> *stage = reinterpret_cast<cx<C> *>(slab_smem);  // [12][nstage]
  cx<C> *slots = stage + 12 * nstage;                     // [2][12][SPB]
  cx<C> *xlink = slots + 2 * 12 * SPB;                    // [9][SPB]
  // slab order: t fastest, then z, then the y block
  Coord4 c4;
  c4.t = b % ex.lt;
  b /= ex.lt;
  c4.z = b % ex.lz;
  const int y0 = (b / ex.lz) * ny;
  const int q = threadIdx.x / SPB;
  const int sl = threadIdx.x % SPB;
  const int row = sl / ex.lx;  // 0 .. ny - 1
  c4.x = sl % ex.lx;
  c4.y = y0 + row;
  const int site = c4.x + ex.sy * c4.y + ex.sz * c4.z + ex.st * c4.t;
  const int V = ex.V;
  const uint32_t cs = (uint32_t)V * elem_traits<SE>::bytes;
  const uint32_t vb = 12u * cs;
  const uint32_t ls = (uint32_t)I.lstride * elem_traits<LE>::bytes;
  const bool lower = q >= 2;
  auto vec = [&](int role) -> const SE * { return role_vec<SE>(I, role, r, V); };
  const double pa = role_a(I, p.a, r);
  double nrm[2] = {0.0, 0.0};
  const rsrc_t v = make_rsrc(vec(p.v_role), vb);
  const bool vg5 = p.v_g5 != 0;
  const rsrc_t U = make_rsrc(I.U, link_bytes(ex.V, ls));
  const DirCoef<C> k = dir_coef<C>(q);
  // 1. stage rows y0 - 1 .. y0 + ny of this (z, t), all 12 components (raw, gamma5 on use);
  //    consecutive threads read consecutive sites of a row
  {
    const int plane = ex.sz * c4.z + ex.st * c4.t;
    for (int e = threadIdx.x; e < 12 * nstage; e += 4 * SPB) {
      const int comp = e / nstage, j = e - comp * nstage;
      const int rr = j / ex.lx, xx = j - rr * ex.lx;
      int ys = y0 - 1 + rr;
      ys = ys < 0 ? ys + ex.ly : (ys >= ex.ly ? ys - ex.ly : ys);
      stage[comp * nstage + j] = bld<C, SE>(v, (uint32_t)comp * cs, (uint32_t)(xx + ex.sy * ys + plane));
    }
  }
  cx<C> mf[3][3];  // forward link of this thread's direction
  load_link3<C, LE>(U, ls, (uint32_t)q * 9u * (uint32_t)I.lstride + link_lane(site), r12, mf);
  if (q == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) xlink[(a * 3 + c) * SPB + sl] = mf[a][c];
  }
  __syncthreads();
  cx<C> acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<C>(0, 0);
  const uint32_t ll = (uint32_t)q * 9u * (uint32_t)I.lstride;
  if (q < 2) {
    // x or y: neighbours from the staged slab
    int jf, jb;  // staged indices of the forward and backward neighbour
    const int jc = (row + 1) * ex.lx + c4.x;
    if (q == 0) {
      jf = (row + 1) * ex.lx + (c4.x + 1 == ex.lx ? 0 : c4.x + 1);
      jb = (row + 1) * ex.lx + (c4.x == 0 ? ex.lx - 1 : c4.x - 1);
    } else {
      jf = jc + ex.lx;
      jb = jc - ex.lx;
    }
    cx<C> u[2][3], d[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u[sp][c] = stage[(sp * 3 + c) * nstage + jf];
        const cx<C> x = stage[((sp + 2) * 3 + c) * nstage + jf];
        d[sp][c] = vg5 ? -x : x;
      }
    hop_apply<C, false>(acc, u, d, mf, k, C(1));
    cx<C> mb[3][3];
    if (q == 0) {
      const int sb = row * ex.lx + (c4.x == 0 ? ex.lx - 1 : c4.x - 1);  // slab index of x - 1
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) mb[a][c] = xlink[(a * 3 + c) * SPB + sb];
    } else {
      const int bwd = c4.y == 0 ? site + (ex.ly - 1) * ex.sy : site - ex.sy;
      load_link3<C, LE>(U, ls, ll + link_lane(bwd), r12, mb);
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u[sp][c] = stage[(sp * 3 + c) * nstage + jb];
        const cx<C> x = stage[((sp + 2) * 3 + c) * nstage + jb];
        d[sp][c] = vg5 ? -x : x;
      }
    hop_apply<C, true>(acc, u, d, mb, k, C(-1));
  } else {
    int fwd, bwd;
    dir_neighbours(ex, c4, site, q, fwd, bwd);
    cx<C> u[2][3], d[2][3];
    load_spinor<C, SE>(v, cs, fwd, vg5, u, d);
    hop_apply<C, false>(acc, u, d, mf, k, C(1));
    cx<C> mb[3][3];
    load_link3<C, LE>(U, ls, ll + link_lane(bwd), r12, mb);
    load_spinor<C, SE>(v, cs, bwd, vg5, u, d);
    hop_apply<C, true>(acc, u, d, mb, k, C(-1));
  }
  // 2. ((x + z) + (y + t)) in a fixed order
  if (q < 2) {
#pragma unroll
    for (int i = 0; i < 12; ++i) slots[(q * 12 + i) * SPB + sl] = acc[i];
  }
  __syncthreads();
  if (q >= 2) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const int ix = ((q - 2) * 12 + i) * SPB + sl;
      slots[ix] = slots[ix] + acc[i];
    }
  }
  __syncthreads();
  {
    cx<C> hop[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      hop[c] = slots[(3 * q + c) * SPB + sl] + slots[(12 + 3 * q + c) * SPB + sl];
    const C kd = C(p.kd), kh = C(p.kh);
    const uint32_t e0 = (uint32_t)(3 * q) * (uint32_t)V + site;
    const int jc = (row + 1) * ex.lx + c4.x;
    cx<C> res[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<C> vx = stage[(3 * q + c) * nstage + jc];
      const cx<C> x = (vg5 && lower) ? -vx : vx;
      cx<C> y = mk<C>(kd * x.re + kh * hop[c].re, kd * x.im + kh * hop[c].im);
      if (p.y_g5 && lower) y = -y;
      res[c] = y;
    }
    cx<C> srcx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) srcx[c] = mk<C>(0, 0);
    const bool need_src = (pa != 0.0) || p.mode >= MODE_SIGN;
    if (need_src) {
      const rsrc_t sr = make_rsrc(vec(ROLE_PSI), vb);
#pragma unroll
      for (int c = 0; c < 3; ++c) srcx[c] = bldv<C, SE>(sr, e0 + c * V);
    }
    if (pa != 0.0) {
      const C a = (p.src_g5 && lower) ? C(-pa) : C(pa);
#pragma unroll
      for (int c = 0; c < 3; ++c) res[c] = res[c] + scale(srcx[c], a);
    }
    if (p.w_role != ROLE_NONE) {
      const rsrc_t w = make_rsrc(vec(p.w_role), vb);
      const C t = C(p.t);
#pragma unroll
      for (int c = 0; c < 3; ++c) res[c] = res[c] + scale(bldv<C, SE>(w, e0 + c * V), t);
    }
    if (p.mode >= MODE_SIGN) {
      for (int e = 0; e < I.n_ev; ++e) {
        const rsrc_t ph = make_rsrc(reinterpret_cast<const SE *>(I.phi) + (int64_t)e * 12 * V, vb);
        const double2 ce = I.c[r * I.n_ev + e];
        const double we = I.wdefl[e];
        const cx<C> d = mk<C>(C(ce.x * we), C(ce.y * we));
#pragma unroll
        for (int c = 0; c < 3; ++c) res[c] = cmadd(res[c], bldv<C, SE>(ph, e0 + c * V), d);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        nrm[0] += double(res[c].re) * double(res[c].re) + double(res[c].im) * double(res[c].im);
        nrm[1] += double(srcx[c].re) * double(srcx[c].re) + double(srcx[c].im) * double(srcx[c].im);
      }
      if (p.mode == MODE_OVERLAP || p.mode == MODE_OVERLAP_DAG) {
        const C hp = C(0.5 * (1.0 + p.mu));
        const C hm = (p.mode == MODE_OVERLAP && lower) ? C(-0.5 * (1.0 - p.mu)) : C(0.5 * (1.0 - p.mu));
#pragma unroll
        for (int c = 0; c < 3; ++c) res[c] = scale(srcx[c], hp) + scale(res[c], hm);
      }
    }
    const rsrc_t o = make_rsrc(vec(p.out_role), vb);
#pragma unroll
    for (int c = 0; c < 3; ++c) bstv<C, SE>(o, e0 + c * V, res[c]);
  }
  if (I.norm_partial != nullptr && p.mode >= MODE_SIGN) {
    block_sum<2>(nrm, lds);
    if (threadIdx.x == 0) {
      const int64_t pb = (int64_t)b * nrhs + r;  // partial of (site block b, right-hand side r)
      I.norm_partial[pb * 2 + 0] = nrm[0];
      I.norm_partial[pb * 2 + 1] = nrm[1];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// final check of the recurrence: ||res||^2 <= bound2 ||src||^2 and finite, per right-hand side.
// One workgroup per right-hand side sums the step kernel's block partials (fixed order).
__global__ void __launch_bounds__(kBlock)
    norm_check_kernel(const double *partial, int nblk, int nrhs, double bound2, uint32_t *flags,
                      double *norms_out) {
  __shared__ double lds[2 * 16];
  const int r = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
    v[0] += partial[((int64_t)b * nrhs + r) * 2 + 0];
    v[1] += partial[((int64_t)b * nrhs + r) * 2 + 1];
  }
  block_sum<2>(v, lds);
  if (threadIdx.x != 0) return;
  const double so = v[0], si = v[1];
  if (norms_out != nullptr) {
    norms_out[2 * r + 0] = so;
    norms_out[2 * r + 1] = si;
  }
  uint32_t f = 0;
  if (!isfinite(so)) f |= 1u;
  else if (so > bound2 * si * (1.0 + 1e-6) + 1e-300) f |= 2u;
  if (f) atomicOr(flags, f);
}

// ---------------------------------------------------------------------------------------------
// deflation projection, pass 1: partial[b][r][i] = sum over this block's sites of
// conj(phi_i) . psi_r (12 components), FP64 accumulation, CH eigenvectors per block row
template <class SE, int CH>
__global__ void __launch_bounds__(kBlock)
    project_partial_kernel(const SE *__restrict__ phi, int n_ev, const SE *__restrict__ psi,
                           int psi_g5, int V, double2 *__restrict__ partial) {
  __shared__ double lds[2 * CH * 16];
  const int i0 = blockIdx.y * CH;
  const int r = blockIdx.z;
  const int nblk = gridDim.x;
  const int nrhs = gridDim.z;
  double acc[2 * CH];
#pragma unroll
  for (int j = 0; j < 2 * CH; ++j) acc[j] = 0.0;
  const SE *__restrict__ ps = psi + (int64_t)r * 12 * V;
  for (int site = blockIdx.x * kBlock + threadIdx.x; site < V; site += nblk * kBlock) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cx<double> x = load_c<double>(ps, (int64_t)i * V + site);
      if (psi_g5 && i >= 6) x = -x;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        if (i0 + j < n_ev) {
          const cx<double> f = load_c<double>(phi, ((int64_t)(i0 + j) * 12 + i) * V + site);
          acc[2 * j] = fma(f.re, x.re, fma(f.im, x.im, acc[2 * j]));
          acc[2 * j + 1] = fma(f.re, x.im, fma(-f.im, x.re, acc[2 * j + 1]));
        }
      }
    }
  }
  block_sum<2 * CH>(acc, lds);
  if (threadIdx.x == 0) {
    for (int j = 0; j < CH && i0 + j < n_ev; ++j)
      partial[((int64_t)blockIdx.x * nrhs + r) * n_ev + i0 + j] = make_double2(acc[2 * j], acc[2 * j + 1]);
  }
}

// Deflation projection on the matrix cores (FP32 storage): c[r][e] = sum_k conj(phi_e[k]) psi_r[k]
// as a real product C = A B with K = 24 V reals (complex numbers stored as (re, im) pairs):
//   A[e][k] = raw phi_e data,  B[k][2r] = raw psi_r data,  B[k][2r+1] = psi_r pairs (re, im)
//   turned into (im, -re),  so C[e][2r] = Re c and C[e][2r+1] = Im c.
// One wave accumulates a 16 x 16 tile (16 eigenvectors x 8 right-hand sides) with
// v_mfma_f32_16x16x4f32 over its share of K (lane l holds A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16]; each lane reads MT consecutive reals per step); the four waves of a
// workgroup are added in FP64 in fixed order and pass 2 sums the workgroups in FP64.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaT = 4;  // reals per lane per step

__global__ void __launch_bounds__(256)
    project_mfma_kernel(const float *phi, int n_ev, const float *psi, int nrhs, int psi_g5, int V,
                        int chunk, double2 *__restrict__ partial) {
  __shared__ double tile[4][16][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int e = blockIdx.y * 16 + i;          // A row of this lane
  const int col = i;                          // B column of this lane
  const int r = blockIdx.z * 8 + (col >> 1);  // right-hand side of the column
  const bool imcol = (col & 1) != 0;
  const int64_t K = (int64_t)24 * V;          // reals per vector
  const uint32_t vecb = (uint32_t)K * 4u;     // bytes per vector
  const rsrc_t ra = make_rsrc(phi, vecb * (uint32_t)n_ev);
  const rsrc_t rb = make_rsrc(psi, vecb * (uint32_t)nrhs);
  const bool arow = e < n_ev, bcol = r < nrhs;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = k_begin + chunk < K ? k_begin + chunk : K;
  // the matrix core accumulates 16 products per lane group in FP32; the running sum is FP64
  double acc64[4] = {0.0, 0.0, 0.0, 0.0};
  // Each step covers 4 waves x 4 lane groups x MT reals.  The loop bound is uniform over the wave:
  // an MFMA reads its operands from every lane regardless of the execution mask, so no lane may
  // leave the loop early; positions past the chunk are masked to zero instead.
  for (int64_t kw = k_begin + (int64_t)wave * 4 * kMfmaT; kw < k_end; kw += 16 * kMfmaT) {
    const int64_t k0 = kw + (int64_t)g * kMfmaT;
    float a[kMfmaT], bv[kMfmaT];
    // row offsets differ per lane: they go in the VGPR offset (rows beyond the data read 0)
    const u32x4 wa = __builtin_amdgcn_raw_buffer_load_b128(ra, (uint32_t)e * vecb + (uint32_t)k0 * 4u, 0u, 0);
    const u32x4 wb = __builtin_amdgcn_raw_buffer_load_b128(rb, (uint32_t)r * vecb + (uint32_t)k0 * 4u, 0u, 0);
    a[0] = __uint_as_float(wa.x); a[1] = __uint_as_float(wa.y);
    a[2] = __uint_as_float(wa.z); a[3] = __uint_as_float(wa.w);
    float x0 = __uint_as_float(wb.x), y0 = __uint_as_float(wb.y);
    float x1 = __uint_as_float(wb.z), y1 = __uint_as_float(wb.w);
    if (psi_g5) {  // gamma5: spin components 2, 3 (complex index >= 6 V) change sign
      if ((k0 >> 1) >= 6 * (int64_t)V) { x0 = -x0; y0 = -y0; }
      if (((k0 + 2) >> 1) >= 6 * (int64_t)V) { x1 = -x1; y1 = -y1; }
    }
    if (imcol) { bv[0] = y0; bv[1] = -x0; bv[2] = y1; bv[3] = -x1; }
    else { bv[0] = x0; bv[1] = y0; bv[2] = x1; bv[3] = y1; }
    // the lane's A value belongs to row e and its B value to column col: separate masks
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kMfmaT; ++t) {
      const bool in = k0 + t < k_end;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32((in && arow) ? a[t] : 0.f,
                                                 (in && bcol) ? bv[t] : 0.f, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc64[q] += (double)acc[q];
  }
  // lane holds C[row = 4 g + q][col = i], q = 0..3
#pragma unroll
  for (int q = 0; q < 4; ++q) tile[wave][4 * g + q][i] = acc64[q];
  __syncthreads();
  if (threadIdx.x < 256) {
    const int row = threadIdx.x >> 4, c = threadIdx.x & 15;
    const double sum = tile[0][row][c] + tile[1][row][c] + tile[2][row][c] + tile[3][row][c];
    tile[0][row][c] = sum;
  }
  __syncthreads();
  if (threadIdx.x < 128) {
    const int row = threadIdx.x >> 3, rr = threadIdx.x & 7;
    const int ee = blockIdx.y * 16 + row, rhs = blockIdx.z * 8 + rr;
    if (ee < n_ev && rhs < nrhs)
      partial[((int64_t)blockIdx.x * nrhs + rhs) * n_ev + ee] =
          make_double2(tile[0][row][2 * rr], tile[0][row][2 * rr + 1]);
  }
}

// pass 2: c[r][i] = sum_b partial[b][r][i]; one wave per output, lane l sums blocks l, l + 64, ...
// and the wave adds the lanes in a fixed butterfly (deterministic)
__global__ void __launch_bounds__(64)
    project_reduce_kernel(const double2 *__restrict__ partial, int nblk, int count,
                          double2 *__restrict__ c) {
  const int k = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    const double2 v = partial[(int64_t)b * count + k];
    re += v.x;
    im += v.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (threadIdx.x == 0) c[k] = make_double2(re, im);
}

// inout_r += sum_i phi_i (wscale * w_i * c[r][i])   (w == null -> w_i = 1)
template <class C, class SE>
__global__ void __launch_bounds__(kBlock)
    correct_kernel(SE *inout, const SE *__restrict__ phi, int n_ev, const double2 *__restrict__ c,
                   const double *__restrict__ w, double wscale, int V) {
  const int site = blockIdx.x * kBlock + threadIdx.x;
  const int r = blockIdx.y;
  if (site >= V) return;
  SE *io = inout + (int64_t)r * 12 * V;
  cx<C> acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = load_c<C>(io, (int64_t)i * V + site);
  for (int e = 0; e < n_ev; ++e) {
    const double2 ce = c[r * n_ev + e];
    const double we = (w ? w[e] : 1.0) * wscale;
    const cx<C> d = mk<C>(C(ce.x * we), C(ce.y * we));
#pragma unroll
    for (int i = 0; i < 12; ++i)
      acc[i] = cmadd(acc[i], load_c<C>(phi, ((int64_t)e * 12 + i) * V + site), d);
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) store_c(io, (int64_t)i * V + site, acc[i]);
}

// inout_r += sum_{e0 <= i < e0 + ne} phi_i (w.v[i - e0] * c[r][i]) with the weights passed by value
// in the kernel arguments (the public correction entry point: nothing to stage on the device)
constexpr int kWChunk = 256;
struct WChunk {
  double v[kWChunk];
};
template <class C, class SE>
__global__ void __launch_bounds__(kBlock)
    correct_w_kernel(SE *inout, const SE *__restrict__ phi, int e0, int ne, int n_ev,
                     const double2 *__restrict__ c, WChunk w, int V) {
  const int site = blockIdx.x * kBlock + threadIdx.x;
  const int r = blockIdx.y;
  if (site >= V) return;
  SE *io = inout + (int64_t)r * 12 * V;
  cx<C> acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = load_c<C>(io, (int64_t)i * V + site);
  for (int k = 0; k < ne; ++k) {
    const int e = e0 + k;
    const double2 ce = c[r * n_ev + e];
    const double we = w.v[k];
    const cx<C> d = mk<C>(C(ce.x * we), C(ce.y * we));
#pragma unroll
    for (int i = 0; i < 12; ++i)
      acc[i] = cmadd(acc[i], load_c<C>(phi, ((int64_t)e * 12 + i) * V + site), d);
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) store_c(io, (int64_t)i * V + site, acc[i]);
}

// v *= 1 / sqrt(nrm2[0].x); records the norm before scaling into norms[slot]
__global__ void normalize_kernel(double2 *v, const double2 *nrm2, int64_t n, double *norms,
                                 int slot) {
  const double s = nrm2[0].x;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && norms != nullptr) norms[slot] = s;
  if (k >= n) return;
  const double inv = 1.0 / sqrt(s);
  double2 x = v[k];
  v[k] = make_double2(x.x * inv, x.y * inv);
}

// records nrm2[0].x into norms[slot]
__global__ void record_kernel(const double2 *nrm2, double *norms, int slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0) norms[slot] = nrm2[0].x;
}

// ---------------------------------------------------------------------------------------------
// element conversion between storage formats
__device__ __forceinline__ void cvt(double2 s, double2 &d) { d = s; }
__device__ __forceinline__ void cvt(float2 s, double2 &d) { d = make_double2(s.x, s.y); }
__device__ __forceinline__ void cvt(double2 s, float2 &d) { d = make_float2((float)s.x, (float)s.y); }
__device__ __forceinline__ void cvt(float2 s, float2 &d) { d = s; }
__device__ __forceinline__ void cvt(double2 s, bf16c &d) {
  d.bits = f32_to_bf16_bits((float)s.x) | (f32_to_bf16_bits((float)s.y) << 16);
}
__device__ __forceinline__ void cvt(float2 s, bf16c &d) {
  d.bits = f32_to_bf16_bits(s.x) | (f32_to_bf16_bits(s.y) << 16);
}

template <class S, class D>
__global__ void convert_kernel(const S *__restrict__ src, D *__restrict__ dst, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) cvt(src[k], dst[k]);
}

// vector algebra of the overlap solver, n complex elements:
//   out = a x + b y  (complex a, b; a null x or y drops its term; out may alias x or y)
template <class C, class SE>
__global__ void axpby_kernel(const SE *x, double2 a, const SE *y, double2 b, SE *out, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  cx<C> r = mk<C>(0, 0);
  if (x) r = cmadd(r, mk<C>(C(a.x), C(a.y)), load_c<C>(x, k));
  if (y) r = cmadd(r, mk<C>(C(b.x), C(b.y)), load_c<C>(y, k));
  store_c<C>(out, k, r);
}
//   dst = s src  (real s, converting between FP64 and FP32)
template <class S, class D>
__global__ void scale_convert_kernel(const S *__restrict__ src, D *__restrict__ dst, double s,
                                     int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const cx<double> v = load_c<double>(src, k);
  store_c<double>(dst, k, mk<double>(v.re * s, v.im * s));
}
//   x += s d  (x FP64, d FP64 or FP32)
template <class S>
__global__ void accumulate_kernel(double2 *__restrict__ x, const S *__restrict__ d, double s,
                                  int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const cx<double> v = load_c<double>(d, k);
  x[k] = make_double2(x[k].x + s * v.re, x[k].y + s * v.im);
}

// links [36][V] (caller layout) -> blocks [V / 64][36][64] in the storage format
template <class S, class D>
__global__ void pack_links_kernel(const S *__restrict__ src, D *__restrict__ dst, int V) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)36 * V) return;
  const int64_t comp = k / V, site = k - comp * V;
  cvt(src[k], dst[(int64_t)link_lane((uint32_t)site) + comp * 64]);
}

// Largest |stored third row - third row completed from the first two| (FP64, element-wise
// complex modulus) over the links of blockIdx.x's 256 (site, mu) pairs: partial[blockIdx.x].
template <class LE>
__global__ void __launch_bounds__(256) su3_row2_dev_kernel(const LE *U, int V, double *partial) {
  __shared__ double red[4];
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;  // k = 4 site + mu
  double dev = 0.0;
  if (k < (int64_t)4 * V) {
    const uint32_t site = (uint32_t)(k >> 2), mu = (uint32_t)(k & 3);
    const uint32_t ls = 64u * elem_traits<LE>::bytes;
    const rsrc_t r = make_rsrc(U, link_bytes(V, ls));
    cx<double> m[3][3], stored[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) m[a][b] = bld<double, LE>(r, (a * 3 + b) * ls, mu * 9u * 64u + link_lane(site));
#pragma unroll
    for (int b = 0; b < 3; ++b) stored[b] = m[2][b];
    su3_row2(m);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const cx<double> e = m[2][b] - stored[b];
      dev = fmax(dev, sqrt(e.re * e.re + e.im * e.im));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ---------------------------------------------------------------------------------------------
// Site of lane sl in workgroup gb of a VJP launch (64 sites per workgroup): memory order, or
// (ty > 0) the t-streaming tile order of the step kernels -- whole x lines, ty x tz in (y, z),
// consecutive workgroups walking t -- so the t neighbours a workgroup reads were loaded shortly
// before by the workgroup of the previous slice, and most y and z neighbours lie in its own
// tile (measured: 3% faster than memory order at 24^3 x 48).
__device__ __forceinline__ int vjp_site(int gb, int sl, const Ext4 &ex, int ty, int tz) {
  if (ty <= 0) return gb * 64 + sl;
  const int slice = ex.lx * ty * tz;
  const int nsub = slice / 64;
  int tb = gb;
  const int sub = tb % nsub;
  tb /= nsub;
  const int t = tb % ex.lt;
  const int tile = tb / ex.lt;
  const int nty = ex.ly / ty;
  const int local = sub * 64 + sl;
  const int x = local % ex.lx;
  const int rr = local / ex.lx;
  const int y = (tile % nty) * ty + rr % ty;
  const int z = (tile / nty) * tz + rr / ty;
  return x + ex.sy * y + ex.sz * z + ex.st * t;
}

// Link vector-Jacobian products of the hopping term, summed over a segment of vector pairs.
// For L = Re<a, D_W t> (a read with gamma5 when a_g5), with h^-(f) the half-spinor of
// (1 - gamma_mu) f and h^+(f) of (1 + gamma_mu) f:
//   G_mu(x)_ij (+)= -1/2 sum_pairs coef sum_{k<2} [ h^-(a(x))_{k,i} conj(h^-(t(x+mu))_{k,j})
//                                                 + h^+(t(x))_{k,i} conj(h^+(a(x+mu))_{k,j}) ]
// ((1 -+ gamma_mu)/2 are Hermitian projectors, so the 4-spin sums reduce to half-spinor sums.)
// Pair i < len0 uses a_i = a0 + i * a_step and t_i = t0 + i * t_step (elements), pair i >= len0
// the second run a1 + (i - len0) * a_step, t1 + (i - len0) * t_step; coef = coef_first for i = 0
// and coef_rest otherwise.  Thread (site, mu) owns link G_mu(x): the outer products of one pair
// are formed in the compute precision C and added into FP64 registers, so the sum over the
// segment's pairs (and, through the FP64 running buffer, over all segments) is FP64 whatever the
// storage precision; G is read and written once per launch (gather only, no atomics).
//   in_mode:  0 start from zero, 1 add the FP64 running sum G64, 2 add G (output dtype GE)
//   out_mode: 0 write the FP64 running sum G64, 1 write G
// The four direction waves of a workgroup share the 64 sites: a(x) and t(x) are read from HBM
// once per workgroup (wave mu loads spin-colour components 3 mu .. 3 mu + 2) and handed over in
// LDS, double-buffered so that one barrier per pair suffices; the forward neighbours a(x+mu),
// t(x+mu) are read per thread, issued before the barrier.  Sites follow vjp_site (ty, tz from
// the host; 0 = memory order).
template <class C, class SE, class GE>
__global__ void __launch_bounds__(256)
    link_vjp_kernel(GE *G, double2 *G64, const SE *a0, const SE *a1, int64_t a_step,
                    const SE *t0, const SE *t1, int64_t t_step, int len0, int len,
                    double coef_first, double coef_rest, Geom geo, int a_g5, int in_mode,
                    int out_mode, int ty, int tz) {
  const int mu = threadIdx.x >> 6, sl = threadIdx.x & 63;
  const Ext4 ex = ext_of(geo);
  const int site = vjp_site(blockIdx.x, sl, ex, ty, tz);
  // no early return: every thread reaches the barriers; inactive lanes load and store nothing
  const bool active = site < ex.V;
  const int s_site = active ? site : 0;
  const Coord4 c4 = coords_of(ex, s_site);
  int fwd, bwd;
  dir_neighbours(ex, c4, s_site, mu, fwd, bwd);
  const uint32_t cs = (uint32_t)ex.V * elem_traits<SE>::bytes;
  // own-site spinors of the 64 sites: [buffer][a, t][component][site]
  __shared__ cx<C> own[2][2][12][64];
  cx<double> acc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[i][j] = mk<double>(0, 0);
  for (int pi = 0; pi < len; ++pi) {
    const int b = pi & 1;
    const bool first_run = pi < len0;
    const rsrc_t ra = make_rsrc(first_run ? a0 + pi * a_step : a1 + (pi - len0) * a_step, 12u * cs);
    const rsrc_t rt = make_rsrc(first_run ? t0 + pi * t_step : t1 + (pi - len0) * t_step, 12u * cs);
    cx<C> hmt[2][3], hpa[2][3];
    if (active) {
      cx<C> u[2][3], d[2][3], xa[3], xt[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int comp = mu * 3 + c;
        xa[c] = bld<C, SE>(ra, comp * cs, site);
        xt[c] = bld<C, SE>(rt, comp * cs, site);
      }
      // mu is uniform per wave: the projections take the direction-specialised form
      load_spinor<C, SE>(rt, cs, fwd, false, u, d);
      dir_project_sw<C, 1>(mu, u, d, hmt);
      load_spinor<C, SE>(ra, cs, fwd, a_g5 != 0, u, d);
      dir_project_sw<C, -1>(mu, u, d, hpa);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int comp = mu * 3 + c;
        own[b][0][comp][sl] = (a_g5 != 0 && mu >= 2) ? -xa[c] : xa[c];
        own[b][1][comp][sl] = xt[c];
      }
    }
    __syncthreads();
    if (active) {
      cx<C> hma[2][3], hpt[2][3], ou[2][3], od[2][3];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ou[s2][c] = own[b][0][s2 * 3 + c][sl];
          od[s2][c] = own[b][0][(s2 + 2) * 3 + c][sl];
        }
      dir_project_sw<C, 1>(mu, ou, od, hma);
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ou[s2][c] = own[b][1][s2 * 3 + c][sl];
          od[s2][c] = own[b][1][(s2 + 2) * 3 + c][sl];
        }
      dir_project_sw<C, -1>(mu, ou, od, hpt);
      const double cf = pi == 0 ? coef_first : coef_rest;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          cx<C> s = mk<C>(0, 0);
#pragma unroll
          for (int kk = 0; kk < 2; ++kk) {
            s = cjmadd(s, hmt[kk][j], hma[kk][i]);
            s = cjmadd(s, hpa[kk][j], hpt[kk][i]);
          }
          acc[i][j].re = fma(cf, double(s.re), acc[i][j].re);
          acc[i][j].im = fma(cf, double(s.im), acc[i][j].im);
        }
    }
  }
  if (!active) return;
  const uint32_t gs = (uint32_t)ex.V * elem_traits<GE>::bytes;
  const uint32_t gs64 = (uint32_t)ex.V * 16u;
  const rsrc_t rg = make_rsrc(G, 36u * gs);
  const rsrc_t rg64 = make_rsrc(G64, 36u * gs64);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const uint32_t comp = (uint32_t)mu * 9u + (uint32_t)(i * 3 + j);
      cx<double> v = scale(acc[i][j], -0.5);
      if (in_mode == 1) v = v + bld<double, double2>(rg64, comp * gs64, site);
      else if (in_mode == 2) v = v + bld<double, GE>(rg, comp * gs, site);
      if (out_mode == 0) bst<double, double2>(rg64, comp * gs64, site, v);
      else bst<double, GE>(rg, comp * gs, site, v);
    }
}

// ---------------------------------------------------------------------------------------------
// Dense block algebra of the low-mode eigen-solve (FP64 complex, blocks of m vectors of n complex
// elements stored one vector after the other).
//
// Gram products  G[j][i] = sum_k conj(A_i[k]) B_j[k]  (the inner products <A_i, B_j>).  A
// workgroup of 256 threads owns a 32 x 32 tile of (i, j) and a slice of k; each thread keeps a
// 2 x 2 sub-tile in registers while the 32 A and 32 B vectors of the tile stream through LDS in
// chunks of kGramKC elements.  Slices are summed by gram_reduce_kernel in a fixed order.
constexpr int kGramT = 32;   // tile edge
constexpr int kGramKC = 32;  // k chunk staged in LDS
__global__ void __launch_bounds__(256)
    gram_partial_kernel(const double2 *__restrict__ A, int ma, const double2 *__restrict__ B,
                        int mb, int64_t n, int64_t slice, double2 *__restrict__ partial) {
  __shared__ double2 sa[kGramT][kGramKC + 1];
  __shared__ double2 sb[kGramT][kGramKC + 1];
  const int i0 = blockIdx.x * kGramT, j0 = blockIdx.y * kGramT;
  const int64_t kbeg = (int64_t)blockIdx.z * slice;
  const int64_t kend = kbeg + slice < n ? kbeg + slice : n;
  const int ti = (threadIdx.x & 15) * 2, tj = (threadIdx.x >> 4) * 2;
  double acc[2][2][2] = {};
  for (int64_t k0 = kbeg; k0 < kend; k0 += kGramKC) {
    // stage 32 x 32 elements of A and of B: 4 loads per thread each, consecutive k per lane
    for (int e = threadIdx.x; e < kGramT * kGramKC; e += 256) {
      const int r = e / kGramKC, c = e % kGramKC;
      const int64_t k = k0 + c;
      const bool kin = k < kend;
      sa[r][c] = (kin && i0 + r < ma) ? A[(int64_t)(i0 + r) * n + k] : make_double2(0.0, 0.0);
      sb[r][c] = (kin && j0 + r < mb) ? B[(int64_t)(j0 + r) * n + k] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < kGramKC; ++c) {
      const double2 a0 = sa[ti][c], a1 = sa[ti + 1][c];
      const double2 b0 = sb[tj][c], b1 = sb[tj + 1][c];
      const double2 av[2] = {a0, a1}, bv[2] = {b0, b1};
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          // conj(a) b
          acc[x][y][0] = fma(av[x].x, bv[y].x, fma(av[x].y, bv[y].y, acc[x][y][0]));
          acc[x][y][1] = fma(av[x].x, bv[y].y, fma(-av[x].y, bv[y].x, acc[x][y][1]));
        }
    }
    __syncthreads();
  }
  const int64_t tiles = (int64_t)gridDim.x * gridDim.y;
  const int64_t tile = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
      partial[((int64_t)blockIdx.z * tiles + tile) * (kGramT * kGramT) + (tj + y) * kGramT + ti + x] =
          make_double2(acc[x][y][0], acc[x][y][1]);
}

// G[j][i] (j < mb, i < ma) = sum over the slices of the partial tiles, in slice order
__global__ void __launch_bounds__(256)
    gram_reduce_kernel(const double2 *__restrict__ partial, int ma, int mb, int nslice,
                       double2 *__restrict__ G) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= ma * mb) return;
  const int j = idx / ma, i = idx % ma;
  const int gx = (ma + kGramT - 1) / kGramT, gy = (mb + kGramT - 1) / kGramT;
  const int64_t tiles = (int64_t)gx * gy;
  const int64_t tile = (int64_t)(j / kGramT) * gx + i / kGramT;
  const int off = (j % kGramT) * kGramT + i % kGramT;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < nslice; ++z) {
    const double2 v = partial[((int64_t)z * tiles + tile) * (kGramT * kGramT) + off];
    re += v.x;
    im += v.y;
  }
  G[(int64_t)j * ma + i] = make_double2(re, im);
}

// Block rotation  Out_j[k] = sum_i C[i][j] V_i[k]  (j < mo, i < mi; C complex, row-major mi x mo),
// Out must not overlap V.  A thread owns one k and kRotJ consecutive outputs j, C's column tile in
// LDS; every V_i[k] read feeds kRotJ multiply-adds.
constexpr int kRotJ = 32;
constexpr int kRotI = 64;  // rows of C staged per pass
__global__ void __launch_bounds__(256)
    rotate_kernel(const double2 *__restrict__ V, int mi, int64_t n, const double2 *__restrict__ C,
                  int mo, double2 *__restrict__ Out) {
  __shared__ double2 cs[kRotI][kRotJ];  // rows i0 .. i0 + kRotI - 1 of the tile's columns
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * kRotJ;
  double acc[kRotJ][2];
#pragma unroll
  for (int j = 0; j < kRotJ; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int i0 = 0; i0 < mi; i0 += kRotI) {
    __syncthreads();
    for (int e = threadIdx.x; e < kRotI * kRotJ; e += 256) {
      const int r = e / kRotJ, c = e % kRotJ;
      cs[r][c] = (i0 + r < mi && j0 + c < mo) ? C[(int64_t)(i0 + r) * mo + j0 + c]
                                              : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (k < n) {
      const int iend = mi - i0 < kRotI ? mi - i0 : kRotI;
      for (int r = 0; r < iend; ++r) {
        const double2 v = V[(int64_t)(i0 + r) * n + k];
#pragma unroll
        for (int j = 0; j < kRotJ; ++j) {
          const double2 c = cs[r][j];
          acc[j][0] = fma(c.x, v.x, fma(-c.y, v.y, acc[j][0]));
          acc[j][1] = fma(c.x, v.y, fma(c.y, v.x, acc[j][1]));
        }
      }
    }
  }
  if (k >= n) return;
#pragma unroll
  for (int j = 0; j < kRotJ; ++j)
    if (j0 + j < mo) Out[(int64_t)(j0 + j) * n + k] = make_double2(acc[j][0], acc[j][1]);
}

// partial[b][j] = sum over block b's elements of |W_j[k] - lam_j V_j[k]|^2 (lam null: |W_j|^2)
__global__ void __launch_bounds__(256)
    resid_partial_kernel(const double2 *__restrict__ W, const double2 *__restrict__ V,
                         const double *__restrict__ lam, int64_t n, double *__restrict__ partial) {
  __shared__ double lds[16];
  const int j = blockIdx.y;
  const double l = lam ? lam[j] : 0.0;
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    double2 w = W[(int64_t)j * n + k];
    if (lam) {
      const double2 v = V[(int64_t)j * n + k];
      w.x -= l * v.x;
      w.y -= l * v.y;
    }
    s += w.x * w.x + w.y * w.y;
  }
  double v1[1] = {s};
  block_sum<1>(v1, lds);
  if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = v1[0];
}

// Seeded complex Gaussian block (a + ib, a, b ~ N(0, 1)) from a counter-based generator:
// element e of the block draws two 64-bit words splitmix64(seed, 2e), splitmix64(seed, 2e + 1)
// (the SplitMix64 finaliser of Steele, Lea and Flood, 2014) turned into uniforms in (0, 1] and
// then into a normal pair by the Box-Muller transform.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
__global__ void gaussian_block_kernel(double2 *out, int64_t count, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const uint64_t base = splitmix64(seed);
  const uint64_t w0 = splitmix64(base ^ (uint64_t)(2 * e));
  const uint64_t w1 = splitmix64(base ^ (uint64_t)(2 * e + 1));
  const double u1 = ((w0 >> 11) + 1) * 0x1.0p-53;  // (0, 1]
  const double u2 = (w1 >> 11) * 0x1.0p-53;         // [0, 1)
  const double r = sqrt(-2.0 * log(u1));
  const double t = 2.0 * M_PI * u2;
  out[e] = make_double2(r * cos(t), r * sin(t));
}

// ---------------------------------------------------------------------------------------------
// Bandwidth ceilings of the device memory: plain streams of 16-byte elements, each element touched
// once, four loads in flight per thread (grid-stride).  Read: every element is loaded and folded
// into a per-thread value (stored once per thread so the loads stay live).  Copy: dst = src.
// Three-to-one: dst = x ^ y ^ z (three read streams, one write stream).
__global__ void __launch_bounds__(256) stream_read_kernel(const uint4 *__restrict__ src, int64_t n,
                                                          uint32_t *__restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    acc ^= (a.x ^ a.y ^ a.z ^ a.w) ^ (b.x ^ b.y ^ b.z ^ b.w) ^ (c.x ^ c.y ^ c.z ^ c.w) ^
           (d.x ^ d.y ^ d.z ^ d.w);
  }
  for (; i < n; i += stride) {
    const uint4 a = src[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(256) stream_copy_kernel(const uint4 *__restrict__ src, int64_t n,
                                                          uint4 *__restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(256) stream_3to1_kernel(const uint4 *__restrict__ src, int64_t n,
                                                          uint4 *__restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint4 *x = src, *y = src + n, *z = src + 2 * n;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + stride < n; i += 2 * stride) {
    const uint4 a0 = x[i], b0 = y[i], c0 = z[i];
    const uint4 a1 = x[i + stride], b1 = y[i + stride], c1 = z[i + stride];
    dst[i] = make_uint4(a0.x ^ b0.x ^ c0.x, a0.y ^ b0.y ^ c0.y, a0.z ^ b0.z ^ c0.z, a0.w ^ b0.w ^ c0.w);
    dst[i + stride] = make_uint4(a1.x ^ b1.x ^ c1.x, a1.y ^ b1.y ^ c1.y, a1.z ^ b1.z ^ c1.z,
                                 a1.w ^ b1.w ^ c1.w);
  }
  for (; i < n; i += stride) {
    const uint4 a = x[i], b = y[i], c = z[i];
    dst[i] = make_uint4(a.x ^ b.x ^ c.x, a.y ^ b.y ^ c.y, a.z ^ b.z ^ c.z, a.w ^ b.w ^ c.w);
  }
}

}  // namespace ovl
