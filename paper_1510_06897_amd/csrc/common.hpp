// Shared device-side building blocks: complex arithmetic, storage formats, lattice geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ovl {

// ---------------------------------------------------------------------------------------------
// complex numbers in the compute precision (float or double)
template <class T>
struct cx {
  T re, im;
};

template <class T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
  return cx<T>{r, i};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return cx<T>{a.re + b.re, a.im + b.im};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return cx<T>{a.re - b.re, a.im - b.im};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) {
  return cx<T>{-a.re, -a.im};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) {
  return cx<T>{a.re * s, a.im * s};
}
// acc + a * b
template <class T>
__host__ __device__ __forceinline__ cx<T> cmadd(cx<T> acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cx<T> cjmadd(cx<T> acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}

// Third row of an SU(3) matrix from the first two: unitarity and det = 1 give
// row2 = conj(row0 x row1).  Links kept with two rows are read as six elements and completed
// here (the stored third row is not read).
template <class T>
__host__ __device__ __forceinline__ void su3_row2(cx<T> m[3][3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int c = (b + 1) % 3, d = (b + 2) % 3;
    cx<T> x = cmadd(mk<T>(T(0), T(0)), m[0][c], m[1][d]);
    x = cmadd(x, -m[0][d], m[1][c]);
    m[2][b] = mk<T>(x.re, -x.im);
  }
}

// ---------------------------------------------------------------------------------------------
// storage formats of one complex element.  F64: double2, F32: float2, BF16: two bfloat16 in one
// 32-bit word (real part in the low half).
enum : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

struct bf16c {
  uint32_t bits;
};

template <int DT>
struct storage;
template <>
struct storage<DT_F64> {
  using elem = double2;
  using real = double;
  static constexpr int bytes = 16;
};
template <>
struct storage<DT_F32> {
  using elem = float2;
  using real = float;
  static constexpr int bytes = 8;
};
template <>
struct storage<DT_BF16> {
  using elem = bf16c;
  using real = float;
  static constexpr int bytes = 4;
};

__host__ __device__ __forceinline__ float bf16_lo(uint32_t w) {
  return __uint_as_float(w << 16);
}
__host__ __device__ __forceinline__ float bf16_hi(uint32_t w) {
  return __uint_as_float(w & 0xffff0000u);
}
// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__host__ __device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
  uint32_t b = __float_as_uint(f);
  uint32_t lsb = (b >> 16) & 1u;
  return (b + 0x7fffu + lsb) >> 16;
}

// Raw buffer resources: every array is addressed as (scalar base, scalar byte offset of the
// spin-colour component, 32-bit per-lane byte offset of the site).  Component offsets stay in
// SGPRs, one VGPR per neighbour site carries the lane part, and reads outside the declared range
// return zero instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  // dword3 0x00020000: raw (untyped) 32-bit data format on gfx9-class devices
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <class SE>
struct elem_traits;
template <>
struct elem_traits<double2> {
  static constexpr uint32_t bytes = 16;
};
template <>
struct elem_traits<float2> {
  static constexpr uint32_t bytes = 8;
};
template <>
struct elem_traits<bf16c> {
  static constexpr uint32_t bytes = 4;
};

template <class SE, class C>
struct bio;
template <class C>
struct bio<double2, C> {
  static __device__ __forceinline__ cx<C> ld(rsrc_t r, uint32_t voff, uint32_t soff) {
    u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    const double re = __hiloint2double((int)w.y, (int)w.x);
    const double im = __hiloint2double((int)w.w, (int)w.z);
    return cx<C>{C(re), C(im)};
  }
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t voff, uint32_t soff, cx<C> v) {
    const double re = double(v.re), im = double(v.im);
    u32x4 w;
    w.x = (unsigned)__double2loint(re);
    w.y = (unsigned)__double2hiint(re);
    w.z = (unsigned)__double2loint(im);
    w.w = (unsigned)__double2hiint(im);
    __builtin_amdgcn_raw_buffer_store_b128(w, r, voff, soff, 0);
  }
};
template <class C>
struct bio<float2, C> {
  static __device__ __forceinline__ cx<C> ld(rsrc_t r, uint32_t voff, uint32_t soff) {
    u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return cx<C>{C(__uint_as_float(w.x)), C(__uint_as_float(w.y))};
  }
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t voff, uint32_t soff, cx<C> v) {
    u32x2 w;
    w.x = __float_as_uint(float(v.re));
    w.y = __float_as_uint(float(v.im));
    __builtin_amdgcn_raw_buffer_store_b64(w, r, voff, soff, 0);
  }
};
template <class C>
struct bio<bf16c, C> {
  static __device__ __forceinline__ cx<C> ld(rsrc_t r, uint32_t voff, uint32_t soff) {
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    return cx<C>{C(bf16_lo(w)), C(bf16_hi(w))};
  }
};

// element `comp * V + site` of an array of SE described by resource r
template <class C, class SE>
__device__ __forceinline__ cx<C> bld(rsrc_t r, uint32_t comp_soff, uint32_t site) {
  return bio<SE, C>::ld(r, site * elem_traits<SE>::bytes, comp_soff);
}
template <class C, class SE>
__device__ __forceinline__ void bst(rsrc_t r, uint32_t comp_soff, uint32_t site, cx<C> v) {
  bio<SE, C>::st(r, site * elem_traits<SE>::bytes, comp_soff, v);
}

// element `index` (lane-dependent, any component) of an array of SE described by resource r
template <class C, class SE>
__device__ __forceinline__ cx<C> bldv(rsrc_t r, uint32_t index) {
  return bio<SE, C>::ld(r, index * elem_traits<SE>::bytes, 0u);
}
template <class C, class SE>
__device__ __forceinline__ void bstv(rsrc_t r, uint32_t index, cx<C> v) {
  bio<SE, C>::st(r, index * elem_traits<SE>::bytes, 0u, v);
}

// Two consecutive elements (an even site s and s + 1) in one lane: 16-byte loads and stores of
// FP32 data, 8-byte loads of BF16 links.  A vector-memory instruction costs the address unit
// roughly the same per lane at 8 and at 16 bytes, so pairs halve that cost per site.
template <class SE>
struct bio2;
template <>
struct bio2<float2> {
  static __device__ __forceinline__ void ld(rsrc_t r, uint32_t voff, uint32_t soff, cx<float> &a,
                                            cx<float> &b) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    a = cx<float>{__uint_as_float(w.x), __uint_as_float(w.y)};
    b = cx<float>{__uint_as_float(w.z), __uint_as_float(w.w)};
  }
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t voff, uint32_t soff, cx<float> a,
                                            cx<float> b) {
    u32x4 w;
    w.x = __float_as_uint(a.re);
    w.y = __float_as_uint(a.im);
    w.z = __float_as_uint(b.re);
    w.w = __float_as_uint(b.im);
    __builtin_amdgcn_raw_buffer_store_b128(w, r, voff, soff, 0);
  }
};
template <>
struct bio2<bf16c> {
  static __device__ __forceinline__ void ld(rsrc_t r, uint32_t voff, uint32_t soff, cx<float> &a,
                                            cx<float> &b) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    a = cx<float>{bf16_lo(w.x), bf16_hi(w.x)};
    b = cx<float>{bf16_lo(w.y), bf16_hi(w.y)};
  }
};

// elements `comp * V + s` and `comp * V + s + 1` (s even)
template <class SE>
__device__ __forceinline__ void bld2(rsrc_t r, uint32_t comp_soff, uint32_t s, cx<float> &a,
                                     cx<float> &b) {
  bio2<SE>::ld(r, s * elem_traits<SE>::bytes, comp_soff, a, b);
}
// elements `index` and `index + 1` (index even)
template <class SE>
__device__ __forceinline__ void bldv2(rsrc_t r, uint32_t index, cx<float> &a, cx<float> &b) {
  bio2<SE>::ld(r, index * elem_traits<SE>::bytes, 0u, a, b);
}
template <class SE>
__device__ __forceinline__ void bstv2(rsrc_t r, uint32_t index, cx<float> a, cx<float> b) {
  bio2<SE>::st(r, index * elem_traits<SE>::bytes, 0u, a, b);
}

// plain pointer access for the small set-up kernels
template <class C>
__device__ __forceinline__ cx<C> load_c(const double2 *p, int64_t i) {
  double2 v = p[i];
  return cx<C>{C(v.x), C(v.y)};
}
template <class C>
__device__ __forceinline__ cx<C> load_c(const float2 *p, int64_t i) {
  float2 v = p[i];
  return cx<C>{C(v.x), C(v.y)};
}
template <class C>
__device__ __forceinline__ void store_c(double2 *p, int64_t i, cx<C> v) {
  p[i] = make_double2(double(v.re), double(v.im));
}
template <class C>
__device__ __forceinline__ void store_c(float2 *p, int64_t i, cx<C> v) {
  p[i] = make_float2(float(v.re), float(v.im));
}

// ---------------------------------------------------------------------------------------------
// lattice geometry: extents, strides of the site index x + Lx (y + Ly (z + Lz t))
struct Geom {
  int L[4];
  int stride[4];
  int V;
};

// Link storage: blocks of 64 consecutive sites, [V / 64][36][64] (component = mu * 9 + a * 3 + b).
// A wave reads one component of 64 sites as one contiguous 64-element segment, and the links of
// a block form one contiguous stream instead of 36 separate component planes (DRAM serves the
// single stream about 15% faster).  Element of site s, component c: link_lane(s) + c * 64.
__host__ __device__ __forceinline__ uint32_t link_lane(uint32_t s) {
  return (s >> 6) * (36u * 64u) + (s & 63u);
}
// bytes of the link array of V sites, given the component stride ls (64 elements) in bytes
__host__ __device__ __forceinline__ uint32_t link_bytes(int V, uint32_t ls) {
  return (uint32_t)((V + 63) / 64) * 36u * ls;
}

// map a workgroup id so that each of the 8 XCDs (which receive workgroups round robin) works on
// a contiguous range of logical blocks, keeping stencil neighbours in the same L2
__device__ __forceinline__ int xcd_block(int b, int n, int remap) {
  if (!remap) return b;
  const int xcd = b & 7, local = b >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

}  // namespace ovl
