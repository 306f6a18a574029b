// Schwarz block MR with one lane per (site, colour): an opt-in variant of k_sap_mr.
//
// Same arithmetic as k_sap_mr (arXiv:1109.4279, Sec. 4: MR steps on the Dirichlet block
// operator of every block of one chessboard colour, after the residual update from the
// other colour's latest block solutions), with the work of a site split over three lanes,
// one per colour component a.  Lane (x, a) owns the four spin components (s, a) of the
// residual, the solution and q = D_Lambda rho; it keeps in registers, for the whole
// half-sweep, row a of the forward links U_mu(x), column a of the backward links
// U_mu(x - mu) and the rows (3 s' + a) of both clover blocks.  Per MR step it reads the
// full spinors of its in-block neighbours from LDS, projects them, and forms its colour
// component of the transported half spinors.  The clover blocks of the block's sites are
// staged once in LDS (72 reals per site).  A 4^4 block is 768 lanes (12 wavefronts),
// three times the latency hiding of one lane per site, with a third of the registers.
// FP32 arithmetic only (FP32 or 16-bit storage); the FP64 preconditioner uses k_sap_mr.
#include "wc_kernels.h"

namespace wc {

constexpr int SAP3_MAX_WAVES = 12;

// ------------------------------------------------------------------ per-component access

template <int P> struct Comp;

template <> struct Comp<P_F64> {
  typedef double R;
  static WC_D cplx<R> spin(const FieldRef& f, int s, int c) {
    double2 v = gld_d2(f.d, (size_t)c * f.V + s);
    return {v.x, v.y};
  }
  static WC_D void spin_store(const FieldRef& f, int s, int c, cplx<R> v, float) {
    ((double2*)f.d)[(size_t)c * f.V + s] = make_double2(v.re, v.im);
  }
  static WC_D cplx<R> link(const void* g, const float*, int V, int mu, int s, int k) {
    double2 v = gld_d2(g, ((size_t)mu * 9 + k) * V + s);
    return {v.x, v.y};
  }
  static WC_D R clov(const void* c, const float*, int V, int s, int blk, int r) {
    const int g = 36 * blk + r;
    const double2 v = gld_d2(c, (size_t)(g >> 1) * V + s);
    return (g & 1) ? v.y : v.x;
  }
};

template <> struct Comp<P_F32> {
  typedef float R;
  static WC_D cplx<R> spin(const FieldRef& f, int s, int c) {
    float2 v = gld_f2(f.d, ((size_t)(c >> 1) * f.V + s) * 2 + (c & 1));
    return {v.x, v.y};
  }
  static WC_D void spin_store(const FieldRef& f, int s, int c, cplx<R> v, float) {
    ((float2*)f.d)[((size_t)(c >> 1) * f.V + s) * 2 + (c & 1)] = make_float2(v.re, v.im);
  }
  static WC_D cplx<R> link(const void* g, const float*, int V, int mu, int s, int k) {
    float2 v = gld_f2(g, ((size_t)mu * 9 + k) * V + s);
    return {v.x, v.y};
  }
  static WC_D R clov(const void* c, const float*, int V, int s, int blk, int r) {
    const int g = 36 * blk + r;
    return gld_f(c, ((size_t)(g >> 2) * V + s) * 4 + (g & 3));
  }
};

template <int P> struct Comp16 {
  typedef float R;
  static WC_D cplx<R> spin(const FieldRef& f, int s, int c) {
    const uint32_t w = gld_u32(f.d, ((size_t)(c >> 2) * f.V + s) * 4 + (c & 3));
    const float sc = gld_f(f.sc, s);
    return {sc * s16_to_f32<P>(uint16_t(w & 0xFFFFu)), sc * s16_to_f32<P>(uint16_t(w >> 16))};
  }
  // stores one component with the site scale `sc` agreed by the site's three lanes
  static WC_D void spin_store(const FieldRef& f, int s, int c, cplx<R> v, float sc) {
    const float inv = 1.f / sc;
    const uint32_t w = uint32_t(f32_to_s16<P>(v.re * inv)) | (uint32_t(f32_to_s16<P>(v.im * inv)) << 16);
    ((uint32_t*)f.d)[((size_t)(c >> 2) * f.V + s) * 4 + (c & 3)] = w;
  }
  static WC_D cplx<R> link(const void* g, const float* sc, int V, int mu, int s, int k) {
    uint32_t w;
    if (k < 8)
      w = gld_u32(g, (((size_t)mu * 2 + (k >> 2)) * V + s) * 4 + (k & 3));
    else
      w = gld_u32(g, (size_t)8 * V * 4 + (size_t)mu * V + s);
    const float f = gld_f(sc, s);
    return {f * s16_to_f32<P>(uint16_t(w & 0xFFFFu)), f * s16_to_f32<P>(uint16_t(w >> 16))};
  }
  static WC_D R clov(const void* c, const float* sc, int V, int s, int blk, int r) {
    const int g = 36 * blk + r;
    const uint32_t w = gld_u32(c, ((size_t)(g >> 3) * V + s) * 4 + ((g & 7) >> 1));
    const uint16_t h = (g & 1) ? uint16_t(w >> 16) : uint16_t(w & 0xFFFFu);
    return gld_f(sc, 2 * (size_t)s + blk) * s16_to_f32<P>(h);
  }
};
template <> struct Comp<P_F16> : Comp16<P_F16> {};
template <> struct Comp<P_BF16> : Comp16<P_BF16> {};

// index of the stored upper-triangle entry (i < j) of a 6x6 Hermitian block
WC_HD int tri(int i, int j) { return i * 6 - (i * (i + 1)) / 2 + (j - i - 1); }

// Colour component a of the hop term (1 + sgn gamma_mu) W h for a projected half spinor h
// (2 spins x 3 colours) transported by the 3-vector w (a row of U, or a column of U^dag),
// added with weight wt into acc[4] (the four spin components of colour a).
template <class R, int MU, int SGN>
WC_D void hop_component(cplx<R>* acc, const Half<R>& h, const cplx<R>* w, bool dag, R wt) {
  cplx<R> t[2];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    cplx<R> v = {R(0), R(0)};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (dag)
        cmac_conj(v, w[b], h.c[sp][b]);
      else
        cmac(v, w[b], h.c[sp][b]);
    }
    t[sp] = wt * v;
  }
  acc[0] = acc[0] + t[0];
  acc[1] = acc[1] + t[1];
  cplx<R> lo0, lo1;
  if (MU == 0) {
    lo0 = SGN > 0 ? -t[0] : t[0];
    lo1 = SGN > 0 ? -t[1] : t[1];
  } else if (MU == 1) {
    lo0 = timesI(t[1]);
    lo1 = timesI(t[0]);
    if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
  } else if (MU == 2) {
    lo0 = t[1];
    lo1 = -t[0];
    if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
  } else {
    lo0 = timesI(t[0]);
    lo1 = timesMinusI(t[1]);
    if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
  }
  acc[2] = acc[2] + lo0;
  acc[3] = acc[3] + lo1;
}

// projection (1 + sgn gamma_mu) of one colour component: (u0, u1, l0, l1) -> (h0, h1)
template <class R, int MU, int SGN>
WC_D void proj1(cplx<R> u0, cplx<R> u1, cplx<R> l0, cplx<R> l1, cplx<R>& h0, cplx<R>& h1) {
  if (MU == 0) {
    h0 = SGN > 0 ? u0 - l0 : u0 + l0;
    h1 = SGN > 0 ? u1 - l1 : u1 + l1;
  } else if (MU == 1) {
    h0 = SGN > 0 ? u0 - timesI(l1) : u0 + timesI(l1);
    h1 = SGN > 0 ? u1 - timesI(l0) : u1 + timesI(l0);
  } else if (MU == 2) {
    h0 = SGN > 0 ? u0 - l1 : u0 + l1;
    h1 = SGN > 0 ? u1 + l0 : u1 - l0;
  } else {
    h0 = SGN > 0 ? u0 - timesI(l0) : u0 + timesI(l0);
    h1 = SGN > 0 ? u1 + timesI(l1) : u1 - timesI(l1);
  }
}

// colour component of one hop, streaming the neighbour spinor colour by colour from `get`
// (get(k) returns component k = 3 spin + colour of the neighbour)
template <class R, int MU, int SGN, class G>
WC_D void hop_stream(cplx<R>* acc, const G& get, const cplx<R>* w, bool dag, R wt) {
  cplx<R> t0 = {R(0), R(0)}, t1 = {R(0), R(0)};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    cplx<R> h0, h1;
    proj1<R, MU, SGN>(get(b), get(3 + b), get(6 + b), get(9 + b), h0, h1);
    if (dag) {
      cmac_conj(t0, w[b], h0);
      cmac_conj(t1, w[b], h1);
    } else {
      cmac(t0, w[b], h0);
      cmac(t1, w[b], h1);
    }
  }
  t0 = wt * t0;
  t1 = wt * t1;
  acc[0] = acc[0] + t0;
  acc[1] = acc[1] + t1;
  cplx<R> lo0, lo1;
  if (MU == 0) {
    lo0 = SGN > 0 ? -t0 : t0;
    lo1 = SGN > 0 ? -t1 : t1;
  } else if (MU == 1) {
    lo0 = timesI(t1);
    lo1 = timesI(t0);
    if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
  } else if (MU == 2) {
    lo0 = t1;
    lo1 = -t0;
    if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
  } else {
    lo0 = timesI(t0);
    lo1 = timesMinusI(t1);
    if (SGN < 0) { lo0 = -lo0; lo1 = -lo1; }
  }
  acc[2] = acc[2] + lo0;
  acc[3] = acc[3] + lo1;
}

// q(2 blk + sp, COL) = sum_j A_blk[3 sp + COL][j] rho_blk[j] - q / 2 for both chirality blocks,
// with the clover reals of the site in LDS.  COL is a template parameter so that every LDS
// offset is a compile-time constant (no address registers survive across MR steps).
template <int COL, class R>
WC_D void clover_rows(cplx<R>* q, const float* cl, const cplx<R>* lds, int bvol, int l) {
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const float* c = cl + 36 * blk * bvol + l;
    cplx<R> v[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = lds[(6 * blk + j) * bvol + l];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      const int i = 3 * sp + COL;
      cplx<R> o = c[i * bvol] * v[i];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        if (j == i) continue;
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        const int k = 6 + 2 * tri(lo, hi);
        const cplx<R> aij = {c[k * bvol], i < j ? c[(k + 1) * bvol] : -c[(k + 1) * bvol]};
        cmac(o, aij, v[j]);
      }
      q[2 * blk + sp] = o - R(0.5) * q[2 * blk + sp];
    }
  }
}

// BV > 0 fixes the block volume at compile time (LDS offsets become immediates and no
// address registers are needed per neighbour component); BV = 0 reads it at run time.
template <int P, int BV>
__global__ __launch_bounds__(768) void k_sap_mr3(SapLaunch a) {
  typedef float R;
  extern __shared__ double smem_d[];
  double* red = smem_d;                                      // SAP3_MAX_WAVES * 3 doubles
  float* scx = (float*)(smem_d + SAP3_MAX_WAVES * 3);       // 3 * 256 floats: per-lane maxima
  cplx<R>* lds = (cplx<R>*)(smem_d + SAP3_MAX_WAVES * 3 + 384);  // residual [12][bvol]

  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    const WorkItem w = a.items[xcd_remap(it0, a.nitems)];
    const LatDesc& L = a.lats[w.lat];
    const Geom g = L.g;
    if (a.skip && a.skip[L.sys0 + w.rhs0]) continue;
    const int bvol = BV > 0 ? BV : g.bvol;
    float* cl = (float*)(lds + 12 * bvol);  // clover reals [72][bvol]
    const int tile = gld_i32(L.tiles[a.colour], w.chunk);
    const int tid = threadIdx.x;
    const bool active = tid < 3 * bvol;
    const int col = active ? tid / bvol : 0;   // colour component of this lane
    const int l = active ? tid - col * bvol : 0;
    const int s = tile * bvol + l;
    int tc[4], lc[4];
    tile_coords(g, tile, tc);
    local_coords(g, l, lc);

    const int sb = spinor_site_bytes(P);
    const long long off = L.foff + (long long)w.rhs0 * g.V;
    const FieldRef frho{(char*)a.rho + off * sb, a.rho_sc ? a.rho_sc + off : nullptr, g.V};
    const FieldRef fz{(char*)a.z + off * sb, a.z_sc ? a.z_sc + off : nullptr, g.V};
    const FieldRef fpsi{(char*)a.psi + off * sb, a.psi_sc ? a.psi_sc + off : nullptr, g.V};

    // in-block neighbours (local index, -1 outside) and time-boundary signs
    int lnb[8];
    unsigned neg = 0;
    cplx<R> wl[8][3];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      int phf, phb;
      bool sf, sbk;
      const int nf = neighbour(g, s, tile, tc, lc, mu, +1, &phf, &sf);
      const int nb = neighbour(g, s, tile, tc, lc, mu, -1, &phb, &sbk);
      lnb[2 * mu] = sf ? nf - tile * bvol : -1;
      lnb[2 * mu + 1] = sbk ? nb - tile * bvol : -1;
      if (phf < 0) neg |= 1u << (2 * mu);
      if (phb < 0) neg |= 1u << (2 * mu + 1);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        wl[2 * mu][b] = Comp<P>::link(L.gauge, L.gscale, g.V, mu, s, 3 * col + b);      // row col of U_mu(x)
        wl[2 * mu + 1][b] = Comp<P>::link(L.gauge, L.gscale, g.V, mu, nb, 3 * b + col);  // column col of U_mu(x-mu)
      }
    }
    // stage the clover reals of the block: lane (x, col) copies reals 24 col .. 24 col + 23
    if (active) {
#pragma unroll
      for (int k = 0; k < 24; ++k) {
        const int r = 24 * col + k;
        cl[r * bvol + l] = Comp<P>::clov(L.clov, L.cscale, g.V, s, r / 36, r % 36);
      }
    }

    cplx<R> rho[4], z[4], q[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      rho[sp] = Comp<P>::spin(frho, s, 3 * sp + col);
      z[sp] = {R(0), R(0)};
    }

    auto sign = [&](int d) { return (neg >> d) & 1u ? R(-1) : R(1); };

    // residual update from the other colour's block solutions: rho -= D z on this block
    if (a.border && active) {
      auto border = [&](auto MUc) {
        constexpr int MU = decltype(MUc)::value;
        int ph;
        bool same;
        if (lnb[2 * MU] < 0) {
          const int n = neighbour(g, s, tile, tc, lc, MU, +1, &ph, &same);
          hop_stream<R, MU, -1>(rho, [&](int k) { return Comp<P>::spin(fz, n, k); }, wl[2 * MU], false,
                                R(0.5) * sign(2 * MU));
        }
        if (lnb[2 * MU + 1] < 0) {
          const int n = neighbour(g, s, tile, tc, lc, MU, -1, &ph, &same);
          hop_stream<R, MU, +1>(rho, [&](int k) { return Comp<P>::spin(fz, n, k); }, wl[2 * MU + 1], true,
                                R(0.5) * sign(2 * MU + 1));
        }
      };
      border(std::integral_constant<int, 0>());
      border(std::integral_constant<int, 1>());
      border(std::integral_constant<int, 2>());
      border(std::integral_constant<int, 3>());
    }

    for (int it = 0; it < a.nmr; ++it) {
      if (active) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) lds[(3 * sp + col) * bvol + l] = rho[sp];
      }
      __syncthreads();
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) q[sp] = {R(0), R(0)};
      if (active) {
        // the scheduling barriers keep the compiler from hoisting all eight neighbour
        // loads ahead of the arithmetic (that would not fit the register budget)
        auto hop = [&](auto MUc) {
          constexpr int MU = decltype(MUc)::value;
          __builtin_amdgcn_sched_barrier(0);
          if (lnb[2 * MU] >= 0) {
            const cplx<R>* nb = lds + lnb[2 * MU];
            hop_stream<R, MU, -1>(q, [&](int k) { return nb[k * bvol]; }, wl[2 * MU], false, sign(2 * MU));
          }
          __builtin_amdgcn_sched_barrier(0);
          if (lnb[2 * MU + 1] >= 0) {
            const cplx<R>* nb = lds + lnb[2 * MU + 1];
            hop_stream<R, MU, +1>(q, [&](int k) { return nb[k * bvol]; }, wl[2 * MU + 1], true, sign(2 * MU + 1));
          }
        };
        hop(std::integral_constant<int, 0>());
        hop(std::integral_constant<int, 1>());
        hop(std::integral_constant<int, 2>());
        hop(std::integral_constant<int, 3>());
        // rows (3 sp + col) of both clover blocks, then q = A rho - 1/2 hops; col is uniform
        // across a wavefront whenever the block volume is a multiple of 64
        switch (col) {
          case 0: clover_rows<0>(q, cl, lds, bvol, l); break;
          case 1: clover_rows<1>(q, cl, lds, bvol, l); break;
          default: clover_rows<2>(q, cl, lds, bvol, l); break;
        }
      }
      double sums[3];
      {
        R qr_re = 0, qr_im = 0, qq = 0;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
          qr_re += q[sp].re * rho[sp].re + q[sp].im * rho[sp].im;
          qr_im += q[sp].re * rho[sp].im - q[sp].im * rho[sp].re;
          qq += q[sp].re * q[sp].re + q[sp].im * q[sp].im;
        }
        sums[0] = qr_re;
        sums[1] = qr_im;
        sums[2] = qq;
      }
      block_sum<3>(sums, red);
      const double are = sums[2] > 0.0 ? sums[0] / sums[2] : 0.0;
      const double aim = sums[2] > 0.0 ? sums[1] / sums[2] : 0.0;
      const cplx<R> alpha = {R(are), R(aim)};
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        cmac(z[sp], alpha, rho[sp]);
        rho[sp] = rho[sp] - alpha * q[sp];
      }
    }

    // stores; 16-bit storage needs the per-site scale agreed by the three lanes of a site
    auto site_scale = [&](const cplx<R>* v) {
      float m = 0.f;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) m = fmaxf(m, fmaxf(fabsf(v[sp].re), fabsf(v[sp].im)));
      __syncthreads();
      if (active) scx[col * bvol + l] = m;
      __syncthreads();
      float mm = 0.f;
      if (active) mm = fmaxf(scx[l], fmaxf(scx[bvol + l], scx[2 * bvol + l]));
      return mm > 0.f ? mm : 1.f;
    };
    auto store_field = [&](const FieldRef& f, const cplx<R>* v) {
      float sc = 1.f;
      if (P == P_F16 || P == P_BF16) sc = site_scale(v);
      if (active) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) Comp<P>::spin_store(f, s, 3 * sp + col, v[sp], sc);
        if ((P == P_F16 || P == P_BF16) && col == 0) f.sc[s] = sc;
      }
    };
    if (a.write_rho) store_field(frho, rho);
    if (a.write_z) store_field(fz, z);
    if (!a.first) {
      // psi += z; every lane reads the old values before any lane rewrites them
      cplx<R> p[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) p[sp] = active ? Comp<P>::spin(fpsi, s, 3 * sp + col) + z[sp] : z[sp];
      store_field(fpsi, p);
    } else {
      store_field(fpsi, z);
    }
    __syncthreads();
  }
}

size_t sap3_lds_bytes(int bvol) {
  return sizeof(double) * (SAP3_MAX_WAVES * 3 + 384) + (8 * 12 + 4 * 72) * (size_t)bvol;
}

template <int BV>
static void launch_bv(int prec, const SapLaunch& a, int grid, int threads, size_t lds, hipStream_t st) {
  switch (prec) {
    case P_F32: hipLaunchKernelGGL((k_sap_mr3<P_F32, BV>), dim3(grid), dim3(threads), lds, st, a); break;
    case P_F16: hipLaunchKernelGGL((k_sap_mr3<P_F16, BV>), dim3(grid), dim3(threads), lds, st, a); break;
    default: hipLaunchKernelGGL((k_sap_mr3<P_BF16, BV>), dim3(grid), dim3(threads), lds, st, a); break;
  }
}

// uniform_bvol: the block volume shared by every lattice of the launch, or 0 if they differ
void launch_sap_mr3(int prec, const SapLaunch& a, int grid, int threads, int max_bvol, int uniform_bvol,
                    hipStream_t st) {
  const size_t lds = sap3_lds_bytes(max_bvol);
  if (uniform_bvol == 256)
    launch_bv<256>(prec, a, grid, threads, lds, st);
  else
    launch_bv<0>(prec, a, grid, threads, lds, st);
}

}  // namespace wc
