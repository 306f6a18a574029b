// Schwarz block MR for batches of right-hand sides on 16-bit storage: the block operator
// (forward links and clover blocks of every site of the block, kept in their 16-bit
// form) is staged in LDS once per work-group and shared by NR right-hand sides and all
// MR steps.  Work-group = NR x 256 lanes, lane (site, rhs); 4^4 blocks only.
//
// Same arithmetic as k_sap_mr (arXiv:1109.4279, Sec. 4): residual update from the other
// colour's block solutions (a gather), then nmr MR steps on the Dirichlet block operator,
// FP32 arithmetic.  Each rhs has its own MR coefficients, reduced over its own 4 waves.
#include "wc_kernels.h"

namespace wc {

constexpr int SL_BV = 256;

template <int P> WC_D cplx<float> h2c(uint32_t w, float sc) {
  return {sc * s16_to_f32<P>(uint16_t(w & 0xFFFFu)), sc * s16_to_f32<P>(uint16_t(w >> 16))};
}

template <int P, int NR>
__global__ __launch_bounds__(NR * 256) void k_sap_mr_lds(SapLaunch a) {
  typedef float R;
  extern __shared__ double smem_d[];
  double* red = smem_d;                                         // 4 * NR waves x 3
  uint32_t* lk = (uint32_t*)(smem_d + 4 * NR * 3);              // links [36][256] (4 dirs x 9)
  uint32_t* cw = lk + 36 * SL_BV;                               // clover [36][256] half pairs
  float* lsc = (float*)(cw + 36 * SL_BV);                       // link scale [256]
  float* csc = lsc + SL_BV;                                     // clover scales [2][256]
  cplx<R>* ex = (cplx<R>*)(csc + 2 * SL_BV);                    // residual exchange [NR][12][256]

  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    const WorkItem w = a.items[xcd_remap(it0, a.nitems)];
    const LatDesc& L = a.lats[w.lat];
    const Geom g = L.g;
    bool any = false;
    for (int r = 0; r < w.nr; ++r) any |= !(a.skip && a.skip[L.sys0 + w.rhs0 + r]);
    if (!any) continue;
    const int tile = gld_i32(L.tiles[a.colour], w.chunk);
    const int tid = threadIdx.x;
    const int rr = tid >> 8;         // rhs of this lane within the group
    const int l = tid & 255;         // site of this lane within the block
    const bool live = rr < w.nr;
    const int s = tile * SL_BV + l;
    int tc[4], lc[4];
    tile_coords(g, tile, tc);
    local_coords(g, l, lc);

    // stage the block operator (16-bit words as stored)
    {
      const int V = g.V;
      for (int j = rr; j < 36; j += NR) {
        const int mu = j / 9, k = j % 9;
        uint32_t v;
        if (k < 8)
          v = gld_u32(L.gauge, (((size_t)mu * 2 + (k >> 2)) * V + s) * 4 + (k & 3));
        else
          v = gld_u32(L.gauge, (size_t)8 * V * 4 + (size_t)mu * V + s);
        lk[j * SL_BV + l] = v;
      }
      for (int j = rr; j < 36; j += NR) cw[j * SL_BV + l] = gld_u32(L.clov, ((size_t)(j >> 2) * V + s) * 4 + (j & 3));
      if (rr == 0) {
        lsc[l] = gld_f(L.gscale, s);
        csc[l] = gld_f(L.cscale, 2 * (size_t)s);
        csc[SL_BV + l] = gld_f(L.cscale, 2 * (size_t)s + 1);
      }
    }
    __syncthreads();

    const int sb = spinor_site_bytes(P);
    const long long off = L.foff + (long long)(w.rhs0 + (live ? rr : 0)) * g.V;
    const FieldRef frho{(char*)a.rho + off * sb, a.rho_sc + off, g.V};
    const FieldRef fz{(char*)a.z + off * sb, a.z_sc + off, g.V};
    const FieldRef fpsi{(char*)a.psi + off * sb, a.psi_sc + off, g.V};

    int lnb[8];
    unsigned neg = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      int phf, phb;
      bool sf, sbk;
      const int nf = neighbour(g, s, tile, tc, lc, mu, +1, &phf, &sf);
      const int nb = neighbour(g, s, tile, tc, lc, mu, -1, &phb, &sbk);
      lnb[2 * mu] = sf ? nf - tile * SL_BV : -1;
      lnb[2 * mu + 1] = sbk ? nb - tile * SL_BV : -1;
      if (phf < 0) neg |= 1u << (2 * mu);
      if (phb < 0) neg |= 1u << (2 * mu + 1);
    }
    auto sign = [&](int d) { return (neg >> d) & 1u ? R(-1) : R(1); };
    // link U_mu at block-local site j from LDS, without its site scale lsc[j] (the scale
    // joins the weight of the hop, so the halves feed mixed-precision FMAs directly)
    auto link_lds = [&](int mu, int j) {
      SU3<R> u;
#pragma unroll
      for (int k = 0; k < 9; ++k) u.m[k / 3][k % 3] = h2c<P>(lk[(mu * 9 + k) * SL_BV + j], 1.f);
      return u;
    };

    Spinor<R> rho = SpinorIO<P>::load(frho, s), z, q;
    zero(z);

    if (a.border && live) {
      auto border = [&](auto MUc) {
        constexpr int MU = decltype(MUc)::value;
        int ph;
        bool same;
        if (lnb[2 * MU] < 0) {
          const int n = neighbour(g, s, tile, tc, lc, MU, +1, &ph, &same);
          Spinor<R> p = SpinorIO<P>::load(fz, n);
          accum_recon<R, MU, -1>(rho, mul_U(link_lds(MU, l), project<R, MU, -1>(p)), R(0.5) * sign(2 * MU) * lsc[l]);
        }
        if (lnb[2 * MU + 1] < 0) {
          const int n = neighbour(g, s, tile, tc, lc, MU, -1, &ph, &same);
          Spinor<R> p = SpinorIO<P>::load(fz, n);
          SU3<R> u = LinkIO<P>::load(L.gauge, L.gscale, g.V, MU, n);
          accum_recon<R, MU, +1>(rho, mul_Udag(u, project<R, MU, +1>(p)), R(0.5) * sign(2 * MU + 1));
        }
      };
      border(std::integral_constant<int, 0>());
      border(std::integral_constant<int, 1>());
      border(std::integral_constant<int, 2>());
      border(std::integral_constant<int, 3>());
    }

    cplx<R>* myex = ex + rr * 12 * SL_BV;
    for (int it = 0; it < a.nmr; ++it) {
#pragma unroll
      for (int k = 0; k < 12; ++k) myex[k * SL_BV + l] = rho.c[k / 3][k % 3];
      __syncthreads();
      zero(q);
      auto hop = [&](auto MUc) {
        constexpr int MU = decltype(MUc)::value;
        if (lnb[2 * MU] >= 0) {
          const int ln = lnb[2 * MU];
          Spinor<R> p;
#pragma unroll
          for (int k = 0; k < 12; ++k) p.c[k / 3][k % 3] = myex[k * SL_BV + ln];
          accum_recon<R, MU, -1>(q, mul_U(link_lds(MU, l), project<R, MU, -1>(p)), R(-0.5) * sign(2 * MU) * lsc[l]);
        }
        if (lnb[2 * MU + 1] >= 0) {
          const int ln = lnb[2 * MU + 1];
          Spinor<R> p;
#pragma unroll
          for (int k = 0; k < 12; ++k) p.c[k / 3][k % 3] = myex[k * SL_BV + ln];
          accum_recon<R, MU, +1>(q, mul_Udag(link_lds(MU, ln), project<R, MU, +1>(p)),
                                 R(-0.5) * sign(2 * MU + 1) * lsc[ln]);
        }
      };
      hop(std::integral_constant<int, 0>());
      hop(std::integral_constant<int, 1>());
      hop(std::integral_constant<int, 2>());
      hop(std::integral_constant<int, 3>());
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        Herm6<R> hc;
        const float f = csc[blk * SL_BV + l];
        float rv[36];
#pragma unroll
        for (int j = 0; j < 18; ++j) {
          const uint32_t wv = cw[(18 * blk + j) * SL_BV + l];
          rv[2 * j] = s16_to_f32<P>(uint16_t(wv & 0xFFFFu));
          rv[2 * j + 1] = s16_to_f32<P>(uint16_t(wv >> 16));
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) hc.d[k] = rv[k];
#pragma unroll
        for (int k = 0; k < 15; ++k) hc.o[k] = {rv[6 + 2 * k], rv[7 + 2 * k]};
        cplx<R> v[6], o[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = rho.c[2 * blk + i / 3][i % 3];
        herm6_apply(hc, v, o);
        // q holds -1/2 of the hops already
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          cplx<R>& x = q.c[2 * blk + i / 3][i % 3];
          x = x + f * o[i];
        }
      }
      // per-rhs reductions over the rhs's four wavefronts
      R qr_re = 0, qr_im = 0, qq = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cplx<R> qv = q.c[i][c], rv = rho.c[i][c];
          qr_re += qv.re * rv.re + qv.im * rv.im;
          qr_im += qv.re * rv.im - qv.im * rv.re;
          qq += qv.re * qv.re + qv.im * qv.im;
        }
      double sv[3] = {double(wave_sum(qr_re)), double(wave_sum(qr_im)), double(wave_sum(qq))};
      const int wid = tid >> 6;
      if ((tid & 63) == 0) {
        red[wid * 3] = sv[0];
        red[wid * 3 + 1] = sv[1];
        red[wid * 3 + 2] = sv[2];
      }
      __syncthreads();
      double t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        t0 += red[(4 * rr + ww) * 3];
        t1 += red[(4 * rr + ww) * 3 + 1];
        t2 += red[(4 * rr + ww) * 3 + 2];
      }
      const cplx<R> alpha = {R(t2 > 0.0 ? t0 / t2 : 0.0), R(t2 > 0.0 ? t1 / t2 : 0.0)};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cmac(z.c[i][c], alpha, rho.c[i][c]);
          rho.c[i][c] = rho.c[i][c] - alpha * q.c[i][c];
        }
      __syncthreads();
    }

    const bool store = live && !(a.skip && a.skip[L.sys0 + w.rhs0 + rr]);
    if (store) {
      if (a.write_rho) SpinorIO<P>::store(frho, s, rho);
      if (a.write_z) SpinorIO<P>::store(fz, s, z);
      if (a.first) {
        SpinorIO<P>::store(fpsi, s, z);
      } else {
        Spinor<R> p = SpinorIO<P>::load(fpsi, s);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) p.c[i][c] = p.c[i][c] + z.c[i][c];
        SpinorIO<P>::store(fpsi, s, p);
      }
    }
    __syncthreads();
  }
}

size_t sap_lds_kernel_bytes(int nr) {
  return sizeof(double) * 4 * nr * 3 + sizeof(uint32_t) * 72 * SL_BV + sizeof(float) * 3 * SL_BV +
         sizeof(float) * 2 * 12 * (size_t)nr * SL_BV;
}

void launch_sap_mr_lds(int prec, int nr, const SapLaunch& a, int grid, hipStream_t st) {
  const size_t lds = sap_lds_kernel_bytes(nr);
  if (prec == P_F16) {
    if (nr == 2)
      hipLaunchKernelGGL((k_sap_mr_lds<P_F16, 2>), dim3(grid), dim3(512), lds, st, a);
    else
      hipLaunchKernelGGL((k_sap_mr_lds<P_F16, 1>), dim3(grid), dim3(256), lds, st, a);
  } else {
    if (nr == 2)
      hipLaunchKernelGGL((k_sap_mr_lds<P_BF16, 2>), dim3(grid), dim3(512), lds, st, a);
    else
      hipLaunchKernelGGL((k_sap_mr_lds<P_BF16, 1>), dim3(grid), dim3(256), lds, st, a);
  }
}

}  // namespace wc
