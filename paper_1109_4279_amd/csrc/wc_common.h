// Shared device/host definitions of the Wilson-clover library for gfx950.
//
// Storage formats (all structure-of-arrays over sites so that consecutive lanes
// of a wavefront touch consecutive 16-byte words):
//   spinor  F64 : [rhs][12][V] double2            (one complex per chunk)
//           F32 : [rhs][6][V]  float4             (two complex per chunk)
//           16b : [rhs][3][V]  uint4 (8 halves) + [rhs][V] float scale
//   links   F64 : [4][9][V] double2, F32 : [4][9][V] float2,
//           16b : [4][2][V] uint4 + [4][V] uint (18 halves) + [V] float scale
//   clover  F64 : [36][V] double2, F32 : [18][V] float4,
//           16b : [9][V] uint4 + [V] float2 scales (one per chirality block)
// Clover blocks: per chirality, 6 real diagonal entries then the 15 complex
// entries above the diagonal in row-major order; row index = 3*spin + colour
// within the chirality (spins 0,1 for the + block, 2,3 for the - block).
//
// Sites are ordered tile-major: the lattice is cut into tiles of the Schwarz
// block shape, tiles are lexicographic (x3 fastest) and so are sites inside a
// tile.  Axis 0 is time.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#define WC_HD __host__ __device__ __forceinline__
#define WC_D __device__ __forceinline__

namespace wc {

enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

// ------------------------------------------------------------------ geometry

struct Geom {
  int L[4];       // lattice extents, axis 0 = time
  int B[4];       // tile (Schwarz block) extents
  int NB[4];      // tiles per axis
  int lstr[4];    // site stride of each axis inside a tile
  int tstr[4];    // tile-index stride of each axis
  int bvol;       // sites per tile
  int ntiles;
  int V;
  int bc_t;       // +1 periodic, -1 antiperiodic in time
};

// Neighbour of site s (tile t, local coords l[]) one step along mu.
// Returns the neighbour index; sets *phase to the time boundary sign and
// *same_tile to whether the neighbour lies in the same tile.
WC_HD int neighbour(const Geom& g, int s, int tile, const int* tc, const int* lc, int mu, int dir,
                    int* phase, bool* same_tile) {
  int ph = 1;
  int local = s - tile * g.bvol;
  int nl, nt;
  if (dir > 0) {
    if (lc[mu] + 1 < g.B[mu]) {
      *phase = 1;
      *same_tile = true;
      return s + g.lstr[mu];
    }
    nl = local - (g.B[mu] - 1) * g.lstr[mu];
    if (tc[mu] + 1 < g.NB[mu]) {
      nt = tile + g.tstr[mu];
    } else {
      nt = tile - (g.NB[mu] - 1) * g.tstr[mu];
      if (mu == 0) ph = g.bc_t;
    }
  } else {
    if (lc[mu] > 0) {
      *phase = 1;
      *same_tile = true;
      return s - g.lstr[mu];
    }
    nl = local + (g.B[mu] - 1) * g.lstr[mu];
    if (tc[mu] > 0) {
      nt = tile - g.tstr[mu];
    } else {
      nt = tile + (g.NB[mu] - 1) * g.tstr[mu];
      if (mu == 0) ph = g.bc_t;
    }
  }
  *phase = ph;
  *same_tile = (nt == tile);
  return nt * g.bvol + nl;
}

WC_HD void tile_coords(const Geom& g, int tile, int* tc) {
  int t = tile;
  tc[3] = t % g.NB[3]; t /= g.NB[3];
  tc[2] = t % g.NB[2]; t /= g.NB[2];
  tc[1] = t % g.NB[1]; t /= g.NB[1];
  tc[0] = t;
}

WC_HD void local_coords(const Geom& g, int local, int* lc) {
  int t = local;
  lc[3] = t % g.B[3]; t /= g.B[3];
  lc[2] = t % g.B[2]; t /= g.B[2];
  lc[1] = t % g.B[1]; t /= g.B[1];
  lc[0] = t;
}

WC_HD int tile_colour(const int* tc) { return (tc[0] + tc[1] + tc[2] + tc[3]) & 1; }

// lexicographic (canonical) index of a site from tile/local coordinates
WC_HD int lex_index(const Geom& g, const int* tc, const int* lc) {
  int x0 = tc[0] * g.B[0] + lc[0], x1 = tc[1] * g.B[1] + lc[1];
  int x2 = tc[2] * g.B[2] + lc[2], x3 = tc[3] * g.B[3] + lc[3];
  return ((x0 * g.L[1] + x1) * g.L[2] + x2) * g.L[3] + x3;
}

// ------------------------------------------------------------------ complex

template <class R>
struct cplx {
  R re, im;
};

template <class R> WC_HD cplx<R> mk(R a, R b) { return cplx<R>{a, b}; }
template <class R> WC_HD cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> WC_HD cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> WC_HD cplx<R> operator-(cplx<R> a) { return {-a.re, -a.im}; }
template <class R> WC_HD cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> WC_HD cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <class R> WC_HD cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
template <class R> WC_HD cplx<R> timesI(cplx<R> a) { return {-a.im, a.re}; }
template <class R> WC_HD cplx<R> timesMinusI(cplx<R> a) { return {a.im, -a.re}; }
// a += b * c
template <class R> WC_HD void cmac(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <class R> WC_HD void cmac_conj(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}

template <class R> struct Spinor { cplx<R> c[4][3]; };  // [spin][colour]
template <class R> struct Half { cplx<R> c[2][3]; };
template <class R> struct SU3 { cplx<R> m[3][3]; };

template <class R> WC_D void zero(Spinor<R>& s) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s.c[i][j] = {R(0), R(0)};
}

// h' = U h  and  h' = U^dag h on both spin components of a half spinor
template <class R> WC_D Half<R> mul_U(const SU3<R>& u, const Half<R>& h) {
  Half<R> o;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<R> acc = u.m[a][0] * h.c[s][0];
      cmac(acc, u.m[a][1], h.c[s][1]);
      cmac(acc, u.m[a][2], h.c[s][2]);
      o.c[s][a] = acc;
    }
  return o;
}
template <class R> WC_D Half<R> mul_Udag(const SU3<R>& u, const Half<R>& h) {
  Half<R> o;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<R> acc = {R(0), R(0)};
      cmac_conj(acc, u.m[0][a], h.c[s][0]);
      cmac_conj(acc, u.m[1][a], h.c[s][1]);
      cmac_conj(acc, u.m[2][a], h.c[s][2]);
      o.c[s][a] = acc;
    }
  return o;
}

// Spin projection with (1 + sgn * gamma_mu) in the chiral basis
//   gamma_0 = [[0,-1],[-1,0]],  gamma_k = [[0,-i sigma_k],[i sigma_k,0]].
// Writing psi = (u, l) in upper/lower spin pairs:
//   mu = 0 : h = u - sgn l,            lower part of the result = -sgn h
//   mu = k : h = u - sgn i sigma_k l,  lower part of the result =  sgn i sigma_k h
template <class R, int MU, int SGN> WC_D Half<R> project(const Spinor<R>& p) {
  Half<R> h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<R> u0 = p.c[0][a], u1 = p.c[1][a], l0 = p.c[2][a], l1 = p.c[3][a];
    if (MU == 0) {
      h.c[0][a] = SGN > 0 ? u0 - l0 : u0 + l0;
      h.c[1][a] = SGN > 0 ? u1 - l1 : u1 + l1;
    } else if (MU == 1) {  // i sigma_1 l = (i l1, i l0)
      h.c[0][a] = SGN > 0 ? u0 - timesI(l1) : u0 + timesI(l1);
      h.c[1][a] = SGN > 0 ? u1 - timesI(l0) : u1 + timesI(l0);
    } else if (MU == 2) {  // i sigma_2 l = (l1, -l0)
      h.c[0][a] = SGN > 0 ? u0 - l1 : u0 + l1;
      h.c[1][a] = SGN > 0 ? u1 + l0 : u1 - l0;
    } else {  // i sigma_3 l = (i l0, -i l1)
      h.c[0][a] = SGN > 0 ? u0 - timesI(l0) : u0 + timesI(l0);
      h.c[1][a] = SGN > 0 ? u1 + timesI(l1) : u1 - timesI(l1);
    }
  }
  return h;
}

// acc += w * (1 + sgn gamma_mu)-reconstruction of the transported half spinor h
template <class R, int MU, int SGN> WC_D void accum_recon(Spinor<R>& acc, const Half<R>& h, R w) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<R> h0 = w * h.c[0][a], h1 = w * h.c[1][a];
    acc.c[0][a] = acc.c[0][a] + h0;
    acc.c[1][a] = acc.c[1][a] + h1;
    cplx<R> lo0, lo1;
    if (MU == 0) {  // lower = -sgn h
      lo0 = SGN > 0 ? -h0 : h0;
      lo1 = SGN > 0 ? -h1 : h1;
    } else if (MU == 1) {  // i sigma_1 h = (i h1, i h0)
      lo0 = timesI(h1);
      lo1 = timesI(h0);
      if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
    } else if (MU == 2) {  // i sigma_2 h = (h1, -h0)
      lo0 = h1;
      lo1 = -h0;
      if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
    } else {  // i sigma_3 h = (i h0, -i h1)
      lo0 = timesI(h0);
      lo1 = timesMinusI(h1);
      if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
    }
    acc.c[2][a] = acc.c[2][a] + lo0;
    acc.c[3][a] = acc.c[3][a] + lo1;
  }
}

// ------------------------------------------------------------------ 16-bit storage

WC_HD float bf16_to_f32(uint16_t b) {
  union { uint32_t u; float f; } v;
  v.u = uint32_t(b) << 16;
  return v.f;
}
WC_HD uint16_t f32_to_bf16(float f) {  // round to nearest even; inputs are finite
  union { uint32_t u; float f; } v;
  v.f = f;
  uint32_t u = v.u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
WC_D float h16_to_f32(uint16_t b) { return __half2float(__ushort_as_half(b)); }
WC_D uint16_t f32_to_h16(float f) { return __half_as_ushort(__float2half_rn(f)); }

template <int P> WC_D float s16_to_f32(uint16_t b) {
  if (P == P_BF16) return bf16_to_f32(b);
  return h16_to_f32(b);
}
template <int P> WC_D uint16_t f32_to_s16(float f) {
  if (P == P_BF16) return f32_to_bf16(f);
  return f32_to_h16(f);
}
// Two values to packed 16-bit storage, a in the low half, rounded to nearest even: one
// v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32 on gfx950 (the same rounding as f32_to_s16).
template <int P> WC_D uint32_t f32x2_to_s16x2(float a, float b) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v v = {a, b};
  if constexpr (P == P_BF16) {
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2v));
  } else {
    typedef _Float16 h2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2v));
  }
}

// compute type per storage precision
template <int P> struct Real { typedef float T; };
template <> struct Real<P_F64> { typedef double T; };

}  // namespace wc
