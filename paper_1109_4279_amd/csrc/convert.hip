// Layout conversion between the canonical lexicographic complex128 arrays of the
// C interface and the tile-major structure-of-arrays storage, and the clover
// setup from the links.
#include "wc_kernels.h"

namespace wc {

// internal site s -> canonical lexicographic site index
WC_D int lex_of(const Geom& g, int s) {
  int tc[4], lc[4];
  const int tile = s / g.bvol;
  tile_coords(g, tile, tc);
  local_coords(g, s - tile * g.bvol, lc);
  return lex_index(g, tc, lc);
}

// canonical coordinates -> internal site index (periodic wrap of x)
WC_D int site_of(const Geom& g, const int* x) {
  int tc[4], lc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int v = x[m] % g.L[m];
    if (v < 0) v += g.L[m];
    tc[m] = v / g.B[m];
    lc[m] = v - tc[m] * g.B[m];
  }
  int tile = ((tc[0] * g.NB[1] + tc[1]) * g.NB[2] + tc[2]) * g.NB[3] + tc[3];
  int local = ((lc[0] * g.B[1] + lc[1]) * g.B[2] + lc[2]) * g.B[3] + lc[3];
  return tile * g.bvol + local;
}

WC_D void coords_of(const Geom& g, int s, int* x) {
  int tc[4], lc[4];
  const int tile = s / g.bvol;
  tile_coords(g, tile, tc);
  local_coords(g, s - tile * g.bvol, lc);
#pragma unroll
  for (int m = 0; m < 4; ++m) x[m] = tc[m] * g.B[m] + lc[m];
}

// ------------------------------------------------------------------ spinors

template <int P>
__global__ __launch_bounds__(WG) void k_pack_spinor(Geom g, int nrhs, const double2* canon, void* dst,
                                                    float* dst_sc) {
  typedef typename Real<P>::T R;
  const int s = blockIdx.x * WG + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.V || r >= nrhs) return;
  const int x = lex_of(g, s);
  const double2* src = canon + ((size_t)r * g.V + x) * 12;
  Spinor<R> p;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double2 v = src[k];
    p.c[k / 3][k % 3] = {R(v.x), R(v.y)};
  }
  const long long off = (long long)r * g.V;
  FieldRef f{(char*)dst + off * spinor_site_bytes(P), dst_sc ? dst_sc + off : nullptr, g.V};
  SpinorIO<P>::store(f, s, p);
}

template <int P>
__global__ __launch_bounds__(WG) void k_unpack_spinor(Geom g, int nrhs, const void* src, const float* src_sc,
                                                      double2* canon, int colour_only) {
  const int s = blockIdx.x * WG + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.V || r >= nrhs) return;
  int tc[4], lc[4];
  const int tile = s / g.bvol;
  tile_coords(g, tile, tc);
  local_coords(g, s - tile * g.bvol, lc);
  const int x = lex_index(g, tc, lc);
  double2* out = canon + ((size_t)r * g.V + x) * 12;
  if (colour_only >= 0 && tile_colour(tc) != colour_only) {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = make_double2(0.0, 0.0);
    return;
  }
  const long long off = (long long)r * g.V;
  FieldRef f{(char*)src + off * spinor_site_bytes(P), src_sc ? (float*)src_sc + off : nullptr, g.V};
  auto p = SpinorIO<P>::load(f, s);
#pragma unroll
  for (int k = 0; k < 12; ++k) out[k] = make_double2(double(p.c[k / 3][k % 3].re), double(p.c[k / 3][k % 3].im));
}

void launch_pack_spinor(int prec, const Geom& g, int nrhs, const void* canon, void* dst, float* dst_sc,
                        hipStream_t st) {
  dim3 grid((g.V + WG - 1) / WG, nrhs);
  const double2* c = (const double2*)canon;
  switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_pack_spinor<P_F64>, grid, dim3(WG), 0, st, g, nrhs, c, dst, dst_sc); break;
    case P_F32: hipLaunchKernelGGL(k_pack_spinor<P_F32>, grid, dim3(WG), 0, st, g, nrhs, c, dst, dst_sc); break;
    case P_F16: hipLaunchKernelGGL(k_pack_spinor<P_F16>, grid, dim3(WG), 0, st, g, nrhs, c, dst, dst_sc); break;
    default: hipLaunchKernelGGL(k_pack_spinor<P_BF16>, grid, dim3(WG), 0, st, g, nrhs, c, dst, dst_sc); break;
  }
}

void launch_unpack_spinor(int prec, const Geom& g, int nrhs, const void* src, const float* src_sc, void* canon,
                          int colour_only, hipStream_t st) {
  dim3 grid((g.V + WG - 1) / WG, nrhs);
  double2* c = (double2*)canon;
  switch (prec) {
    case P_F64:
      hipLaunchKernelGGL(k_unpack_spinor<P_F64>, grid, dim3(WG), 0, st, g, nrhs, src, src_sc, c, colour_only);
      break;
    case P_F32:
      hipLaunchKernelGGL(k_unpack_spinor<P_F32>, grid, dim3(WG), 0, st, g, nrhs, src, src_sc, c, colour_only);
      break;
    case P_F16:
      hipLaunchKernelGGL(k_unpack_spinor<P_F16>, grid, dim3(WG), 0, st, g, nrhs, src, src_sc, c, colour_only);
      break;
    default:
      hipLaunchKernelGGL(k_unpack_spinor<P_BF16>, grid, dim3(WG), 0, st, g, nrhs, src, src_sc, c, colour_only);
      break;
  }
}

// ------------------------------------------------------------------ links

template <int P>
__global__ __launch_bounds__(WG) void k_pack_links(Geom g, const double2* canon, void* dst, float* dst_sc) {
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= g.V) return;
  const int x = lex_of(g, s);
  const int V = g.V;
  if (P == P_F64) {
    double2* d = (double2*)dst;
    for (int mu = 0; mu < 4; ++mu)
      for (int k = 0; k < 9; ++k) d[((size_t)mu * 9 + k) * V + s] = canon[((size_t)mu * V + x) * 9 + k];
  } else if (P == P_F32) {
    float2* d = (float2*)dst;
    for (int mu = 0; mu < 4; ++mu)
      for (int k = 0; k < 9; ++k) {
        double2 v = canon[((size_t)mu * V + x) * 9 + k];
        d[((size_t)mu * 9 + k) * V + s] = make_float2(float(v.x), float(v.y));
      }
  } else {
    float m = 0.f;
    for (int mu = 0; mu < 4; ++mu)
      for (int k = 0; k < 9; ++k) {
        double2 v = canon[((size_t)mu * V + x) * 9 + k];
        m = fmaxf(m, fmaxf(fabsf(float(v.x)), fabsf(float(v.y))));
      }
    const float sc = m > 0.f ? m : 1.f, inv = 1.f / sc;
    uint4* d4 = (uint4*)dst;
    uint32_t* d1 = (uint32_t*)(d4 + (size_t)8 * V);
    for (int mu = 0; mu < 4; ++mu) {
      uint32_t w[9];
      for (int k = 0; k < 9; ++k) {
        double2 v = canon[((size_t)mu * V + x) * 9 + k];
        w[k] = f32x2_to_s16x2<P>(float(v.x) * inv, float(v.y) * inv);
      }
      d4[((size_t)mu * 2) * V + s] = make_uint4(w[0], w[1], w[2], w[3]);
      d4[((size_t)mu * 2 + 1) * V + s] = make_uint4(w[4], w[5], w[6], w[7]);
      d1[(size_t)mu * V + s] = w[8];
    }
    dst_sc[s] = sc;
  }
}

void launch_pack_links(int prec, const Geom& g, const void* canon, void* dst, float* dst_sc, hipStream_t st) {
  dim3 grid((g.V + WG - 1) / WG);
  const double2* c = (const double2*)canon;
  switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_pack_links<P_F64>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
    case P_F32: hipLaunchKernelGGL(k_pack_links<P_F32>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
    case P_F16: hipLaunchKernelGGL(k_pack_links<P_F16>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
    default: hipLaunchKernelGGL(k_pack_links<P_BF16>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
  }
}

// ------------------------------------------------------------------ clover

typedef SU3<double> M3;

WC_D M3 mload(const double2* links, const Geom& g, int mu, const int* x) {
  int s = site_of(g, x);
  return LinkIO<P_F64>::load(links, nullptr, g.V, mu, s);
}
WC_D M3 mmul(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<double> t = a.m[i][0] * b.m[0][j];
      cmac(t, a.m[i][1], b.m[1][j]);
      cmac(t, a.m[i][2], b.m[2][j]);
      c.m[i][j] = t;
    }
  return c;
}
WC_D M3 mdag(const M3& a) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[i][j] = conj(a.m[j][i]);
  return c;
}
WC_D void madd(M3& a, const M3& b) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) a.m[i][j] = a.m[i][j] + b.m[i][j];
}

// F_{mu nu}(x) = (Q - Q^dag)/8 with Q the four plaquettes at x oriented mu -> nu
WC_D M3 field_strength(const double2* links, const Geom& g, const int* x, int mu, int nu) {
  // link U_dir at x + dm * mu_hat + dn * nu_hat
  auto lk = [&](int dir, int dm, int dn) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] += dm;
    y[nu] += dn;
    return mload(links, g, dir, y);
  };
  M3 q, t;
  // x -> x+mu -> x+mu+nu -> x+nu -> x
  t = mmul(mmul(lk(mu, 0, 0), lk(nu, 1, 0)), mmul(mdag(lk(mu, 0, 1)), mdag(lk(nu, 0, 0))));
  q = t;
  // x -> x+nu -> x-mu+nu -> x-mu -> x
  t = mmul(mmul(lk(nu, 0, 0), mdag(lk(mu, -1, 1))), mmul(mdag(lk(nu, -1, 0)), lk(mu, -1, 0)));
  madd(q, t);
  // x -> x-mu -> x-mu-nu -> x-nu -> x
  t = mmul(mmul(mdag(lk(mu, -1, 0)), mdag(lk(nu, -1, -1))), mmul(lk(mu, -1, -1), lk(nu, 0, -1)));
  madd(q, t);
  // x -> x-nu -> x+mu-nu -> x+mu -> x
  t = mmul(mmul(mdag(lk(nu, 0, -1)), lk(mu, 0, -1)), mmul(lk(nu, 1, -1), mdag(lk(mu, 0, 0))));
  madd(q, t);
  M3 f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) f.m[i][j] = 0.125 * (q.m[i][j] - conj(q.m[j][i]));
  return f;
}

// A_pm = (4 + m0) + (i c_sw / 2) sum_l sigma_l (x) (pm F_{0l} - Ft_l), Ft = (F_23, F_31, F_12):
// the clover term in the chiral basis, where sigma_{0k} = diag(sigma_k, -sigma_k) and
// sigma_{jk} = -eps_jkl diag(sigma_l, sigma_l).  As a 6x6 matrix over (spin pair, colour):
//   [[E3, E1 - i E2], [E1 + i E2, -E3]],  E_l = (i c_sw / 2)(pm F_{0l} - Ft_l).
__global__ __launch_bounds__(WG) void k_clover_build(Geom g, const double2* links, double m0, double csw,
                                                     double2* clov) {
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= g.V) return;
  int x[4];
  coords_of(g, s, x);
  M3 F01 = field_strength(links, g, x, 0, 1), F02 = field_strength(links, g, x, 0, 2);
  M3 F03 = field_strength(links, g, x, 0, 3), F23 = field_strength(links, g, x, 2, 3);
  M3 F13 = field_strength(links, g, x, 1, 3), F12 = field_strength(links, g, x, 1, 2);
  for (int blk = 0; blk < 2; ++blk) {
    const double pm = blk == 0 ? 1.0 : -1.0;
    M3 E[3];
    // Ft_1 = F_23, Ft_2 = F_31 = -F_13, Ft_3 = F_12
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cplx<double> e1 = pm * F01.m[i][j] - F23.m[i][j];
        cplx<double> e2 = pm * F02.m[i][j] + F13.m[i][j];
        cplx<double> e3 = pm * F03.m[i][j] - F12.m[i][j];
        // times i c_sw / 2
        E[0].m[i][j] = (0.5 * csw) * timesI(e1);
        E[1].m[i][j] = (0.5 * csw) * timesI(e2);
        E[2].m[i][j] = (0.5 * csw) * timesI(e3);
      }
    cplx<double> A[6][6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        A[i][j] = E[2].m[i][j];
        A[3 + i][3 + j] = -E[2].m[i][j];
        A[i][3 + j] = E[0].m[i][j] - timesI(E[1].m[i][j]);
        A[3 + i][j] = E[0].m[i][j] + timesI(E[1].m[i][j]);
      }
    double2* p = clov + (size_t)(18 * blk) * g.V + s;
    double d[6];
    for (int i = 0; i < 6; ++i) d[i] = A[i][i].re + 4.0 + m0;
    for (int k = 0; k < 3; ++k) p[(size_t)k * g.V] = make_double2(d[2 * k], d[2 * k + 1]);
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j, ++k) p[(size_t)(3 + k) * g.V] = make_double2(A[i][j].re, A[i][j].im);
  }
}

void launch_clover_build(const Geom& g, const void* links64, double m0, double csw, void* clov64, hipStream_t st) {
  dim3 grid((g.V + WG - 1) / WG);
  hipLaunchKernelGGL(k_clover_build, grid, dim3(WG), 0, st, g, (const double2*)links64, m0, csw,
                     (double2*)clov64);
}

// Clover field of the even/odd block solver: A(x) on even sites, A(x)^-1 on odd sites
// (parity = sum of the global coordinates mod 2), FP64, same storage as the clover term.
// One thread per (site, chiral block).  A 6x6 Hermitian block is inverted in place by
// Gauss-Jordan elimination with partial pivoting: at step k the rows k..5 are compared and
// swapped into pivot order (selects, so every index is a compile-time constant, and a
// record of which original row each position holds), row k is scaled by the inverse
// pivot, whose column then holds the inverse's entries, and row k is eliminated from the
// others.  With P the accumulated row permutation the array then holds (P A)^-1 = A^-1 P^T,
// so column i of it is column prow[i] of A^-1; the stored upper triangle picks its entries
// through that record and is re-symmetrised.  The 36 complex entries fit the registers
// (an augmented [A | 1] of 72 did not, and spilled to scratch memory).
__global__ __launch_bounds__(WG) void k_clover_eo(Geom g, const double2* c64, double2* out) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= 2 * g.V) return;
  const int blk = i >= g.V ? 1 : 0;
  const int s = i - blk * g.V;
  const int tile = s / g.bvol;
  int tc[4], lc[4];
  tile_coords(g, tile, tc);
  local_coords(g, s - tile * g.bvol, lc);
  int par = 0;
  for (int m = 0; m < 4; ++m) par += tc[m] * g.B[m] + lc[m];
  const double2* src = c64 + (size_t)(18 * blk) * g.V + s;
  double2* dst = out + (size_t)(18 * blk) * g.V + s;
  if ((par & 1) == 0) {
#pragma unroll
    for (int k = 0; k < 18; ++k) dst[(size_t)k * g.V] = src[(size_t)k * g.V];
    return;
  }
  cplx<double> M[6][6];
  int prow[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double2 v = src[(size_t)k * g.V];
    M[2 * k][2 * k] = {v.x, 0.0};
    M[2 * k + 1][2 * k + 1] = {v.y, 0.0};
  }
  {
    int k = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = r + 1; c < 6; ++c, ++k) {
        double2 v = src[(size_t)(3 + k) * g.V];
        M[r][c] = {v.x, v.y};
        M[c][r] = {v.x, -v.y};
      }
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) prow[r] = r;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int r = k + 1; r < 6; ++r) {
      const double a = M[r][k].re * M[r][k].re + M[r][k].im * M[r][k].im;
      const double b = M[k][k].re * M[k][k].re + M[k][k].im * M[k][k].im;
      const bool sw = a > b;
      // (selects on the scalar parts: a select between two array elements would take their
      // addresses and keep the array out of registers)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double kr = M[k][c].re, ki = M[k][c].im, rr = M[r][c].re, ri = M[r][c].im;
        M[k][c] = {sw ? rr : kr, sw ? ri : ki};
        M[r][c] = {sw ? kr : rr, sw ? ki : ri};
      }
      const int t = prow[k];
      prow[k] = sw ? prow[r] : t;
      prow[r] = sw ? t : prow[r];
    }
    const cplx<double> p = M[k][k];
    const double den = p.re * p.re + p.im * p.im;
    const cplx<double> inv = {p.re / den, -p.im / den};
    M[k][k] = {1.0, 0.0};
#pragma unroll
    for (int c = 0; c < 6; ++c) M[k][c] = inv * M[k][c];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (r == k) continue;
      const cplx<double> f = M[r][k];
      M[r][k] = {0.0, 0.0};
#pragma unroll
      for (int c = 0; c < 6; ++c) M[r][c] = M[r][c] - f * M[k][c];
    }
  }
  // entry (r, j) of A^-1 is M[r][i] with prow[i] == j
  auto inv_at = [&](int r, int j) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const bool hit = prow[c] == j;
      re = hit ? M[r][c].re : re;
      im = hit ? M[r][c].im : im;
    }
    return cplx<double>{re, im};
  };
#pragma unroll
  for (int k = 0; k < 3; ++k) dst[(size_t)k * g.V] = make_double2(inv_at(2 * k, 2 * k).re, inv_at(2 * k + 1, 2 * k + 1).re);
  {
    int k = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = r + 1; c < 6; ++c, ++k) {
        const cplx<double> up = inv_at(r, c), lo = inv_at(c, r);
        dst[(size_t)(3 + k) * g.V] = make_double2(0.5 * (up.re + lo.re), 0.5 * (up.im - lo.im));
      }
  }
}

void launch_clover_eo(const Geom& g, const void* clov64, void* out64, hipStream_t st) {
  dim3 grid((2 * g.V + WG - 1) / WG);
  hipLaunchKernelGGL(k_clover_eo, grid, dim3(WG), 0, st, g, (const double2*)clov64, (double2*)out64);
}

// FP64 clover (36 double2 per site) -> storage precision
template <int P>
__global__ __launch_bounds__(WG) void k_clover_convert(Geom g, const double2* c64, void* dst, float* dst_sc) {
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= g.V) return;
  float r[72];
  for (int k = 0; k < 36; ++k) {
    double2 v = c64[(size_t)k * g.V + s];
    r[2 * k] = float(v.x);
    r[2 * k + 1] = float(v.y);
  }
  if (P == P_F32) {
    float4* d = (float4*)dst;
    for (int k = 0; k < 18; ++k) d[(size_t)k * g.V + s] = make_float4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
  } else {
    float sc[2];
    for (int b = 0; b < 2; ++b) {
      float m = 0.f;
      for (int i = 0; i < 36; ++i) m = fmaxf(m, fabsf(r[36 * b + i]));
      sc[b] = m > 0.f ? m : 1.f;
    }
    uint4* d = (uint4*)dst;
    for (int k = 0; k < 9; ++k) {
      uint32_t w[4];
      for (int j = 0; j < 4; ++j) {
        int i0 = 8 * k + 2 * j, i1 = i0 + 1;
        w[j] = f32x2_to_s16x2<P>(r[i0] / sc[i0 / 36], r[i1] / sc[i1 / 36]);
      }
      d[(size_t)k * g.V + s] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    dst_sc[2 * s] = sc[0];
    dst_sc[2 * s + 1] = sc[1];
  }
}

void launch_clover_convert(int prec, const Geom& g, const void* clov64, void* dst, float* dst_sc, hipStream_t st) {
  dim3 grid((g.V + WG - 1) / WG);
  const double2* c = (const double2*)clov64;
  switch (prec) {
    case P_F32: hipLaunchKernelGGL(k_clover_convert<P_F32>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
    case P_F16: hipLaunchKernelGGL(k_clover_convert<P_F16>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
    case P_BF16: hipLaunchKernelGGL(k_clover_convert<P_BF16>, grid, dim3(WG), 0, st, g, c, dst, dst_sc); break;
    default: break;
  }
}

}  // namespace wc

namespace wc {

// dst = gamma5 src on canonical complex128 spinors (spins 2, 3 change sign)
__global__ __launch_bounds__(WG) void k_gamma5_canon(long long nsite, const double2* src, double2* dst) {
  const long long s = (long long)blockIdx.x * WG + threadIdx.x;
  if (s >= nsite) return;
  for (int k = 0; k < 12; ++k) {
    double2 v = src[s * 12 + k];
    dst[s * 12 + k] = k < 6 ? v : make_double2(-v.x, -v.y);
  }
}

// gamma5 in place on nrhs FP64 fields of the library's layout ([12][V] double2 each): the
// components of the lower two spins (6..11) change sign
__global__ __launch_bounds__(WG) void k_gamma5_f64(double2* f, long long V, int nrhs) {
  const long long e = (long long)blockIdx.x * WG + threadIdx.x;
  if (e >= 6 * V * nrhs) return;
  const long long r = e / (6 * V), k = e - r * 6 * V;
  double2& v = f[r * 12 * V + 6 * V + k];
  v = make_double2(-v.x, -v.y);
}

void launch_gamma5_f64(void* f, long long V, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((6 * V * nrhs + WG - 1) / WG));
  hipLaunchKernelGGL(k_gamma5_f64, grid, dim3(WG), 0, st, (double2*)f, V, nrhs);
}

// out = coef * in on n canonical complex128 values
__global__ __launch_bounds__(WG) void k_scale_canon(long long n, double coef, const double2* in, double2* out) {
  const long long i = (long long)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const double2 v = in[i];
  out[i] = make_double2(coef * v.x, coef * v.y);
}

void launch_scale_canon(long long n, double coef, const void* in, void* out, hipStream_t st) {
  dim3 grid((unsigned)((n + WG - 1) / WG));
  hipLaunchKernelGGL(k_scale_canon, grid, dim3(WG), 0, st, n, coef, (const double2*)in, (double2*)out);
}

// |v|^2 of n canonical complex128 values, deterministically: each of `nblk` work-groups
// sums a strided share into partial[blk]; then one work-group adds the partials in order.
constexpr int NORM_BLOCKS = 1024;
__global__ __launch_bounds__(WG) void k_norm2_canon(long long n, const double2* v, double* partial) {
  __shared__ double lds[WG / 64];
  double t = 0.0;
  for (long long i = (long long)blockIdx.x * WG + threadIdx.x; i < n; i += (long long)gridDim.x * WG) {
    const double2 x = v[i];
    t += x.x * x.x + x.y * x.y;
  }
  double vals[1] = {t};
  block_sum<1>(vals, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = vals[0];
}
__global__ __launch_bounds__(WG) void k_sum_partials(const double* partial, int n, double* out) {
  __shared__ double lds[WG / 64];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) t += partial[i];
  double vals[1] = {t};
  block_sum<1>(vals, lds);
  if (threadIdx.x == 0) out[0] = vals[0];
}

// out[0] = |v|^2; `work` holds NORM_BLOCKS + 1 doubles
void launch_norm2_canon(long long n, const void* v, double* work, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2_canon, dim3(NORM_BLOCKS), dim3(WG), 0, st, n, (const double2*)v, work + 1);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(WG), 0, st, (const double*)(work + 1), NORM_BLOCKS, work);
}

void launch_gamma5_canon(long long nsite, const void* src, void* dst, hipStream_t st) {
  dim3 grid((unsigned)((nsite + WG - 1) / WG));
  hipLaunchKernelGGL(k_gamma5_canon, grid, dim3(WG), 0, st, nsite, (const double2*)src, (double2*)dst);
}

// FP64 clover blocks -> canonical A[V][2][6][6] complex128, Hermitian-completed
__global__ __launch_bounds__(WG) void k_clover_export(Geom g, const double2* c64, double2* out) {
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= g.V) return;
  const int x = lex_of(g, s);
  for (int blk = 0; blk < 2; ++blk) {
    Herm6<double> h = CloverIO<P_F64>::load(c64, nullptr, g.V, s, blk);
    double2* M = out + ((size_t)x * 2 + blk) * 36;
    for (int i = 0; i < 6; ++i) M[i * 6 + i] = make_double2(h.d[i], 0.0);
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j, ++k) {
        M[i * 6 + j] = make_double2(h.o[k].re, h.o[k].im);
        M[j * 6 + i] = make_double2(h.o[k].re, -h.o[k].im);
      }
  }
}

void launch_clover_export(const Geom& g, const void* c64, void* out, hipStream_t st) {
  dim3 grid((g.V + WG - 1) / WG);
  hipLaunchKernelGGL(k_clover_export, grid, dim3(WG), 0, st, g, (const double2*)c64, (double2*)out);
}

}  // namespace wc

namespace wc {

// deterministic pseudo-random canonical spinor (values in [-1, 1)), for autotuning sources
__global__ __launch_bounds__(WG) void k_fill_hash(long long n, unsigned seed, double2* out) {
  const long long i = (long long)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double a = double(z & 0xFFFFFFFFull) / 2147483648.0 - 1.0;
  const double b = double(z >> 32) / 2147483648.0 - 1.0;
  out[i] = make_double2(a, b);
}

void launch_fill_hash(long long n, unsigned seed, void* out, hipStream_t st) {
  dim3 grid((unsigned)((n + WG - 1) / WG));
  hipLaunchKernelGGL(k_fill_hash, grid, dim3(WG), 0, st, n, seed, (double2*)out);
}

}  // namespace wc
