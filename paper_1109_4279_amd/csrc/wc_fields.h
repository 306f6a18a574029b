// Field storage accessors, batch descriptors and wavefront reductions.
#pragma once

#include "wc_common.h"

namespace wc {

constexpr int WG = 256;  // work-group size of every site-parallel kernel

// One lattice of a batch as seen by a kernel.  Spinor fields of a batch are
// concatenated lattice after lattice, each lattice holding nrhs consecutive
// fields in the storage layout of its precision.
struct LatDesc {
  Geom g;
  const void* gauge;   // links in the storage precision of the launch
  const float* gscale; // 16-bit link scales [V] (null otherwise)
  const void* clov;    // clover blocks in the storage precision of the launch
  const float* cscale; // 16-bit clover scales [V][2]
  long long foff;      // offset of rhs 0 of this lattice in a batched spinor field, in sites*rhs units
  int nrhs;
  int sys0;            // batch index of this lattice's first system
  int part0;           // offset of this lattice's first reduction partial
  int nchunks;         // ceil(V / WG): partials per system
  const int* tiles[2]; // tile indices of each chessboard colour (ntiles/2 each)
  // even/odd block solver (null unless it is in use)
  const void* clov_eo;    // A on even sites, A^-1 on odd sites, storage precision of the launch
  const float* cscale_eo; // its 16-bit scales [V][2]
  const short* eo_sites;  // [corner parity][site parity][(bvol+1)/2] tile-local site indices, -1 = none
  const short* eo_slot;   // [corner parity][bvol] slot of each tile-local site in the parity-sorted order
};

// A unit of work: WG consecutive sites (or one tile for the Schwarz kernels)
// of one lattice, for right-hand sides [rhs0, rhs0 + nr).
struct WorkItem {
  int lat;
  int chunk;
  int rhs0;
  int nr;
};

// Work items and lattice descriptors are read through the constant address space, word by
// word: with a uniform address the compiler then loads them with scalar loads into scalar
// registers once per item, instead of vector loads that it repeats at every use when
// registers run short (D_w: 12-rhs FP64 1.80 -> 1.67 ms, one 16-bit rhs per lane 0.77 ->
// 0.52 ms at 24^3 x 48; the even/odd block solver, short of scalar registers, got slower
// with it and keeps its vector loads).
template <class T> WC_D T load_uniform(const T* p, int i) {
  static_assert(sizeof(T) % 4 == 0, "whole words only");
  typedef const __attribute__((address_space(4))) uint32_t* cword_t;
  const cword_t src = (cword_t)(p + i);
  T out;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
  return out;
}

// Map a work index so that the items run by one XCD (work-groups are dealt to
// the 8 XCDs round-robin) form a contiguous range, keeping neighbouring sites
// in one L2.
WC_D int xcd_remap(int it, int n) {
  if (n & 7) return it;
  return (it & 7) * (n >> 3) + (it >> 3);
}

// ------------------------------------------------------------------ global loads

// The operator fields are reached through pointers read from the LatDesc array in device
// memory, which the compiler cannot prove to be global; loads through them would be flat
// loads, and a flat load also counts against the wait counter of LDS and scalar loads, so
// every LDS wait would drain the operator loads in flight.  These helpers load through
// address-space-1 pointers (global_load).
template <class T> using gptr_t = const __attribute__((address_space(1))) T*;
typedef float gf2v __attribute__((ext_vector_type(2)));
typedef float gf4v __attribute__((ext_vector_type(4)));
typedef double gd2v __attribute__((ext_vector_type(2)));
typedef unsigned gu4v __attribute__((ext_vector_type(4)));
WC_D float2 gld_f2(const void* p, size_t i) {
  const gf2v v = ((gptr_t<gf2v>)p)[i];
  return make_float2(v.x, v.y);
}
WC_D float4 gld_f4(const void* p, size_t i) {
  const gf4v v = ((gptr_t<gf4v>)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
WC_D double2 gld_d2(const void* p, size_t i) {
  const gd2v v = ((gptr_t<gd2v>)p)[i];
  return make_double2(v.x, v.y);
}
WC_D uint4 gld_u4(const void* p, size_t i) {
  const gu4v v = ((gptr_t<gu4v>)p)[i];
  return make_uint4(v.x, v.y, v.z, v.w);
}
WC_D uint32_t gld_u32(const void* p, size_t i) { return ((gptr_t<uint32_t>)p)[i]; }
WC_D int gld_i32(const void* p, size_t i) { return ((gptr_t<int>)p)[i]; }
WC_D short gld_s16(const void* p, size_t i) { return ((gptr_t<short>)p)[i]; }
WC_D float gld_f(const void* p, size_t i) { return ((gptr_t<float>)p)[i]; }
WC_D double gld_d(const void* p, size_t i) { return ((gptr_t<double>)p)[i]; }

// ------------------------------------------------------------------ spinors

// A spinor field view for one right-hand side: data + (16-bit) scales.
struct FieldRef {
  void* d;
  float* sc;
  int V;
};

template <int P> struct SpinorIO;

template <> struct SpinorIO<P_F64> {
  typedef double R;
  static WC_D Spinor<double> load(const FieldRef& f, int s) {
    Spinor<double> o;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 v = gld_d2(f.d, (size_t)k * f.V + s);
      o.c[k / 3][k % 3] = {v.x, v.y};
    }
    return o;
  }
  static WC_D void store(const FieldRef& f, int s, const Spinor<double>& o) {
    double2* p = (double2*)f.d + s;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[(size_t)k * f.V] = make_double2(o.c[k / 3][k % 3].re, o.c[k / 3][k % 3].im);
  }
  static constexpr int bytes_per_site = 192;
  static WC_D Spinor<double> load_raw(const FieldRef& f, int s) { return load(f, s); }
  static WC_D double scale(const FieldRef&, int) { return 1.0; }
};

template <> struct SpinorIO<P_F32> {
  typedef float R;
  static WC_D Spinor<float> load(const FieldRef& f, int s) {
    Spinor<float> o;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 v = gld_f4(f.d, (size_t)k * f.V + s);
      int c0 = 2 * k, c1 = 2 * k + 1;
      o.c[c0 / 3][c0 % 3] = {v.x, v.y};
      o.c[c1 / 3][c1 % 3] = {v.z, v.w};
    }
    return o;
  }
  static WC_D void store(const FieldRef& f, int s, const Spinor<float>& o) {
    float4* p = (float4*)f.d + s;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      int c0 = 2 * k, c1 = 2 * k + 1;
      p[(size_t)k * f.V] = make_float4(o.c[c0 / 3][c0 % 3].re, o.c[c0 / 3][c0 % 3].im,
                                       o.c[c1 / 3][c1 % 3].re, o.c[c1 / 3][c1 % 3].im);
    }
  }
  static constexpr int bytes_per_site = 96;
  static WC_D Spinor<float> load_raw(const FieldRef& f, int s) { return load(f, s); }
  static WC_D float scale(const FieldRef&, int) { return 1.f; }
};

template <int P> struct SpinorIO16 {
  typedef float R;
  // values without the site scale (multiply by scale() to get the field)
  static WC_D Spinor<float> load_raw(const FieldRef& f, int s) {
    Spinor<float> o;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 v = gld_u4(f.d, (size_t)k * f.V + s);
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int c = 4 * k + j;
        o.c[c / 3][c % 3] = {s16_to_f32<P>(uint16_t(w[j] & 0xFFFFu)), s16_to_f32<P>(uint16_t(w[j] >> 16))};
      }
    }
    return o;
  }
  static WC_D float scale(const FieldRef& f, int s) { return gld_f(f.sc, s); }
  static WC_D Spinor<float> load(const FieldRef& f, int s) {
    float sc = gld_f(f.sc, s);
    Spinor<float> o;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 v = gld_u4(f.d, (size_t)k * f.V + s);
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int c = 4 * k + j;
        o.c[c / 3][c % 3] = {sc * s16_to_f32<P>(uint16_t(w[j] & 0xFFFFu)), sc * s16_to_f32<P>(uint16_t(w[j] >> 16))};
      }
    }
    return o;
  }
  static WC_D void store(const FieldRef& f, int s, const Spinor<float>& o) {
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int a = 0; a < 3; ++a) m = fmaxf(m, fmaxf(fabsf(o.c[i][a].re), fabsf(o.c[i][a].im)));
    float sc = m > 0.f ? m : 1.f;
    float inv = 1.f / sc;
    uint4* p = (uint4*)f.d + s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int c = 4 * k + j;
        w[j] = f32x2_to_s16x2<P>(o.c[c / 3][c % 3].re * inv, o.c[c / 3][c % 3].im * inv);
      }
      p[(size_t)k * f.V] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    f.sc[s] = sc;
  }
  static constexpr int bytes_per_site = 52;
};
template <> struct SpinorIO<P_F16> : SpinorIO16<P_F16> {};
template <> struct SpinorIO<P_BF16> : SpinorIO16<P_BF16> {};

// element size of one site of one rhs in the data array (scales separate)
WC_HD int spinor_site_bytes(int P) { return P == P_F64 ? 192 : (P == P_F32 ? 96 : 48); }

// ------------------------------------------------------------------ links

template <int P> struct LinkIO;

template <> struct LinkIO<P_F64> {
  static WC_D double scale(const float*, int) { return 1.0; }
  static WC_D SU3<double> load_raw(const void* g, const float* sc, int V, int mu, int s) { return load(g, sc, V, mu, s); }
  static WC_D SU3<double> load(const void* g, const float*, int V, int mu, int s) {
    const size_t p = (size_t)mu * 9 * V + s;
    SU3<double> u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 v = gld_d2(g, p + (size_t)k * V);
      u.m[k / 3][k % 3] = {v.x, v.y};
    }
    return u;
  }
};
template <> struct LinkIO<P_F32> {
  static WC_D float scale(const float*, int) { return 1.f; }
  static WC_D SU3<float> load_raw(const void* g, const float* sc, int V, int mu, int s) { return load(g, sc, V, mu, s); }
  static WC_D SU3<float> load(const void* g, const float*, int V, int mu, int s) {
    const size_t p = (size_t)mu * 9 * V + s;
    SU3<float> u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 v = gld_f2(g, p + (size_t)k * V);
      u.m[k / 3][k % 3] = {v.x, v.y};
    }
    return u;
  }
};
template <int P> struct LinkIO16 {
  static WC_D float scale(const float* sc, int s) { return gld_f(sc, s); }
  // link without the site scale: 8 words in uint4 arrays 2 mu, 2 mu + 1, the ninth in the
  // word array after the eight uint4 arrays
  static WC_D SU3<float> load_raw(const void* g, const float*, int V, int mu, int s) {
    const size_t p = (size_t)mu * 2 * V + s;
    const size_t q = (size_t)8 * V * 4 + (size_t)mu * V + s;
    uint4 a = gld_u4(g, p), b = gld_u4(g, p + V);
    uint32_t w[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, gld_u32(g, q)};
    SU3<float> u;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      u.m[k / 3][k % 3] = {s16_to_f32<P>(uint16_t(w[k] & 0xFFFFu)), s16_to_f32<P>(uint16_t(w[k] >> 16))};
    return u;
  }
  static WC_D SU3<float> load(const void* g, const float* sc, int V, int mu, int s) {
    const size_t p = (size_t)mu * 2 * V + s;
    const size_t q = (size_t)8 * V * 4 + (size_t)mu * V + s;
    float f = gld_f(sc, s);
    uint4 a = gld_u4(g, p), b = gld_u4(g, p + V);
    uint32_t w[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, gld_u32(g, q)};
    SU3<float> u;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      u.m[k / 3][k % 3] = {f * s16_to_f32<P>(uint16_t(w[k] & 0xFFFFu)), f * s16_to_f32<P>(uint16_t(w[k] >> 16))};
    return u;
  }
};
template <> struct LinkIO<P_F16> : LinkIO16<P_F16> {};
template <> struct LinkIO<P_BF16> : LinkIO16<P_BF16> {};

// bytes of the link array per site (all four directions, scales excluded)
WC_HD int link_site_bytes(int P) { return P == P_F64 ? 576 : (P == P_F32 ? 288 : 144); }

// ------------------------------------------------------------------ clover

template <class R> struct Herm6 {
  R d[6];
  cplx<R> o[15];
};

template <int P> struct CloverIO;

template <> struct CloverIO<P_F64> {
  static WC_D double scale(const float*, int, int) { return 1.0; }
  static WC_D Herm6<double> load_raw(const void* c, const float* sc, int V, int s, int blk) { return load(c, sc, V, s, blk); }
  static WC_D Herm6<double> load(const void* c, const float*, int V, int s, int blk) {
    const size_t p = (size_t)(18 * blk) * V + s;
    Herm6<double> h;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double2 v = gld_d2(c, p + (size_t)k * V);
      h.d[2 * k] = v.x;
      h.d[2 * k + 1] = v.y;
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      double2 v = gld_d2(c, p + (size_t)(3 + k) * V);
      h.o[k] = {v.x, v.y};
    }
    return h;
  }
};
template <> struct CloverIO<P_F32> {
  static WC_D float scale(const float*, int, int) { return 1.f; }
  static WC_D Herm6<float> load_raw(const void* c, const float* sc, int V, int s, int blk) { return load(c, sc, V, s, blk); }
  static WC_D Herm6<float> load(const void* c, const float*, int V, int s, int blk) {
    const size_t p = (size_t)(9 * blk) * V + s;
    float r[36];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float4 v = gld_f4(c, p + (size_t)k * V);
      r[4 * k] = v.x; r[4 * k + 1] = v.y; r[4 * k + 2] = v.z; r[4 * k + 3] = v.w;
    }
    Herm6<float> h;
#pragma unroll
    for (int k = 0; k < 6; ++k) h.d[k] = r[k];
#pragma unroll
    for (int k = 0; k < 15; ++k) h.o[k] = {r[6 + 2 * k], r[7 + 2 * k]};
    return h;
  }
};
template <int P> struct CloverIO16 {
  static WC_D float scale(const float* sc, int s, int blk) { return gld_f(sc, 2 * (size_t)s + blk); }
  static WC_D Herm6<float> load_raw(const void* c, const float*, int V, int s, int blk) {
    return load_impl(c, 1.f, V, s, blk);
  }
  static WC_D Herm6<float> load(const void* c, const float* sc, int V, int s, int blk) {
    return load_impl(c, scale(sc, s, blk), V, s, blk);
  }
  // 72 halves per site in 9 uint4; reals 36*blk .. 36*blk+35 belong to block blk
  static WC_D Herm6<float> load_impl(const void* c, float f, int V, int s, int blk) {
    float r[36];
    // block 0 uses uint4 0..4 (reals 0..39), block 1 uses uint4 4..8 (reals 32..71)
    const int k0 = blk == 0 ? 0 : 4;
    const int off = blk == 0 ? 0 : 4;  // reals to skip at the start of uint4 k0
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      uint4 v = gld_u4(c, (size_t)(k0 + k) * V + s);
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int i0 = 8 * k + 2 * j - off, i1 = i0 + 1;
        if (i0 >= 0 && i0 < 36) r[i0] = f * s16_to_f32<P>(uint16_t(w[j] & 0xFFFFu));
        if (i1 >= 0 && i1 < 36) r[i1] = f * s16_to_f32<P>(uint16_t(w[j] >> 16));
      }
    }
    Herm6<float> h;
#pragma unroll
    for (int k = 0; k < 6; ++k) h.d[k] = r[k];
#pragma unroll
    for (int k = 0; k < 15; ++k) h.o[k] = {r[6 + 2 * k], r[7 + 2 * k]};
    return h;
  }
};
template <> struct CloverIO<P_F16> : CloverIO16<P_F16> {};
template <> struct CloverIO<P_BF16> : CloverIO16<P_BF16> {};

WC_HD int clover_site_bytes(int P) { return P == P_F64 ? 576 : (P == P_F32 ? 288 : 144); }

// out (6 complex) = H v for a Hermitian 6x6 stored as diagonal + upper triangle
template <class R> WC_D void herm6_apply(const Herm6<R>& h, const cplx<R>* v, cplx<R>* out) {
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = h.d[i] * v[i];
  int k = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j, ++k) {
      cmac(out[i], h.o[k], v[j]);
      cmac_conj(out[j], h.o[k], v[i]);
    }
}

// ------------------------------------------------------------------ reductions

template <class T> WC_D T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int CTRL> WC_D float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
WC_D float read_lane(float v, int lane) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane)); }

// FP32 wavefront sum without LDS-crossbar shuffles: within each 16-lane row by DPP (lane
// i plus lane i^1, then i^2 by quad permutes; then i plus 7-i within 8 lanes, i plus 15-i
// within 16), after which every lane of a row holds the row's sum; the four row sums are
// read as uniform values and added in a fixed order.  Needs all 64 lanes active.
template <> WC_D float wave_sum<float>(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum over the work-group of up to N values per thread; result valid in every thread.
// `lds` needs (blockDim/64) * N doubles.  GUARD = false drops the barrier that protects
// `lds` from the previous call's readers, for callers that pass a barrier in between.
template <int N, bool GUARD = true> WC_D void block_sum(double* v, double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  if (GUARD) __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wid * N + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[w * N + i];
    v[i] = s;
  }
}

// block_sum of N values held in precision T, result in `out` (every thread): the tree
// within each wavefront runs in T, so an FP32 kernel's partial sums cross lanes as single
// 32-bit words (half the shuffles of a double tree), and the sum over the wavefronts runs in
// double.  `lds` and GUARD as for block_sum.
template <int N, bool GUARD = true, class T> WC_D void block_sum_in(const T* v, double* out, double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = double(wave_sum(v[i]));
  if (GUARD) __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wid * N + i] = out[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[w * N + i];
    out[i] = s;
  }
}

}  // namespace wc
