// Schwarz alternating procedure: minimal-residual relaxation of every block of one
// chessboard colour (arXiv:1109.4279, Sec. 4 and Sec. 5).
//
// One work-group per block (tile) and right-hand-side group, one lane per site.
// Before the MR steps the residual of the block is brought up to date with the hops
// out of the neighbouring blocks of the other colour, whose latest block solutions z
// are in memory: the paper's residual update on the border sites of the blocks, done as
// a gather so that no two work-groups write the same site.  Then nmr MR steps on the
// Dirichlet block operator run with the block residual exchanged through LDS:
//   q = D_Lambda rho,  alpha = <q, rho>/<q, q>,  z += alpha rho,  rho -= alpha q.
// The inner products are work-group reductions (wavefront shuffles + LDS).
#include "wc_kernels.h"

namespace wc {

constexpr int SAP_MAX_WAVES = 4;  // blocks of at most 256 sites

// BV > 0 fixes the block volume at compile time so that every LDS offset of the residual
// exchange is an immediate (no per-neighbour address registers); BV = 0 reads it at run time.
template <int P, int NR, bool CACHE, int BV>
__global__ __launch_bounds__(256) void k_sap_mr(SapLaunch a) {
  typedef typename Real<P>::T R;
  extern __shared__ double smem_d[];
  double* red = smem_d;                                   // SAP_MAX_WAVES * 3 * NR doubles
  cplx<R>* lds = (cplx<R>*)(smem_d + SAP_MAX_WAVES * 3 * NR);  // [NR][12][bvol]

  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    const WorkItem w = a.items[xcd_remap(it0, a.nitems)];
    const LatDesc& L = a.lats[w.lat];
    const Geom g = L.g;
    bool any = true;
    if (a.skip) {
      any = false;
      for (int r = 0; r < w.nr; ++r) any |= (a.skip[L.sys0 + w.rhs0 + r] == 0);
    }
    if (!any) continue;
    const int tile = gld_i32(L.tiles[a.colour], w.chunk);
    const int t = threadIdx.x;
    const bool active = t < g.bvol;
    const int s = tile * g.bvol + (active ? t : 0);
    int tc[4], lc[4];
    tile_coords(g, tile, tc);
    local_coords(g, active ? t : 0, lc);

    FieldRef frho[NR], fz[NR], fpsi[NR];
    const int sb = spinor_site_bytes(P);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int rr = w.rhs0 + (r < w.nr ? r : 0);
      const long long off = L.foff + (long long)rr * g.V;
      frho[r] = {(char*)a.rho + off * sb, a.rho_sc ? a.rho_sc + off : nullptr, g.V};
      fz[r] = {(char*)a.z + off * sb, a.z_sc ? a.z_sc + off : nullptr, g.V};
      fpsi[r] = {(char*)a.psi + off * sb, a.psi_sc ? a.psi_sc + off : nullptr, g.V};
    }

    Spinor<R> rho[NR], z[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      rho[r] = SpinorIO<P>::load(frho[r], s);
      zero(z[r]);
    }

    // residual update from the other colour's latest block solutions:
    // rho(y) -= (D z)(y) = +1/2 sum over hops from y into neighbouring blocks
    if (a.border && active) {
      auto border = [&](auto MUc) {
        constexpr int MU = decltype(MUc)::value;
        int ph;
        bool same;
        int nf = neighbour(g, s, tile, tc, lc, MU, +1, &ph, &same);
        if (!same) {
          SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, s);
          const R w = R(0.5) * R(ph) * LinkIO<P>::scale(L.gscale, s);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            Spinor<R> p = SpinorIO<P>::load_raw(fz[r], nf);
            accum_recon<R, MU, -1>(rho[r], mul_U(u, project<R, MU, -1>(p)), w * SpinorIO<P>::scale(fz[r], nf));
          }
        }
        int nb = neighbour(g, s, tile, tc, lc, MU, -1, &ph, &same);
        if (!same) {
          SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, nb);
          const R w = R(0.5) * R(ph) * LinkIO<P>::scale(L.gscale, nb);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            Spinor<R> p = SpinorIO<P>::load_raw(fz[r], nb);
            accum_recon<R, MU, +1>(rho[r], mul_Udag(u, project<R, MU, +1>(p)), w * SpinorIO<P>::scale(fz[r], nb));
          }
        }
      };
      border(std::integral_constant<int, 0>());
      border(std::integral_constant<int, 1>());
      border(std::integral_constant<int, 2>());
      border(std::integral_constant<int, 3>());
    }

    const int bvol = BV > 0 ? BV : g.bvol;
    // Operator data of this site for the in-block hops and the clover term.  With CACHE it
    // is loaded once per half-sweep and kept in registers across the MR steps (this needs
    // the whole register file of a SIMD, one wavefront each); otherwise it is reloaded
    // from the caches each step and two work-groups can share a CU.
    SU3<R> Uf[CACHE ? 4 : 1], Ub[CACHE ? 4 : 1];
    Herm6<R> Cl[CACHE ? 2 : 1];
    int nfw[4], nbw[4], phf[4], phb[4];
    bool inf[4], inb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      bool same;
      nfw[mu] = neighbour(g, s, tile, tc, lc, mu, +1, &phf[mu], &same);
      inf[mu] = same && active;
      nbw[mu] = neighbour(g, s, tile, tc, lc, mu, -1, &phb[mu], &same);
      inb[mu] = same && active;
    }
    if (CACHE) {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        Uf[CACHE ? mu : 0] = LinkIO<P>::load(L.gauge, L.gscale, g.V, mu, s);
        Ub[CACHE ? mu : 0] = LinkIO<P>::load(L.gauge, L.gscale, g.V, mu, inb[mu] ? nbw[mu] : s);
      }
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) Cl[CACHE ? blk : 0] = CloverIO<P>::load(L.clov, L.cscale, g.V, s, blk);
    }
    for (int it = 0; it < a.nmr; ++it) {
      if (active) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int k = 0; k < 12; ++k) lds[(r * 12 + k) * bvol + t] = rho[r].c[k / 3][k % 3];
      }
      __syncthreads();
      Spinor<R> q[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) zero(q[r]);
      if (active) {
        auto hop = [&](auto MUc) {
          constexpr int MU = decltype(MUc)::value;
          if (inf[MU]) {
            const int ln = nfw[MU] - tile * bvol;
            // uncached 16-bit links are used unscaled, the scale joins the hop weight
            SU3<R> u = CACHE ? Uf[CACHE ? MU : 0] : LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, s);
            const R w = R(-0.5) * (CACHE ? R(phf[MU]) : R(phf[MU]) * LinkIO<P>::scale(L.gscale, s));
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              Spinor<R> p;
#pragma unroll
              for (int k = 0; k < 12; ++k) p.c[k / 3][k % 3] = lds[(r * 12 + k) * bvol + ln];
              accum_recon<R, MU, -1>(q[r], mul_U(u, project<R, MU, -1>(p)), w);
            }
          }
          if (inb[MU]) {
            const int ln = nbw[MU] - tile * bvol;
            SU3<R> u = CACHE ? Ub[CACHE ? MU : 0] : LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, nbw[MU]);
            const R w = R(-0.5) * (CACHE ? R(phb[MU]) : R(phb[MU]) * LinkIO<P>::scale(L.gscale, nbw[MU]));
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              Spinor<R> p;
#pragma unroll
              for (int k = 0; k < 12; ++k) p.c[k / 3][k % 3] = lds[(r * 12 + k) * bvol + ln];
              accum_recon<R, MU, +1>(q[r], mul_Udag(u, project<R, MU, +1>(p)), w);
            }
          }
        };
        hop(std::integral_constant<int, 0>());
        hop(std::integral_constant<int, 1>());
        hop(std::integral_constant<int, 2>());
        hop(std::integral_constant<int, 3>());
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
          Herm6<R> hc = CACHE ? Cl[CACHE ? blk : 0] : CloverIO<P>::load_raw(L.clov, L.cscale, g.V, s, blk);
          const R cs = CACHE ? R(1) : CloverIO<P>::scale(L.cscale, s, blk);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            cplx<R> v[6], o[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) v[i] = rho[r].c[2 * blk + i / 3][i % 3];
            herm6_apply(hc, v, o);
#pragma unroll
            for (int i = 0; i < 6; ++i) {  // q holds -1/2 of the hops already
              cplx<R>& x = q[r].c[2 * blk + i / 3][i % 3];
              x = x + cs * o[i];
            }
          }
        }
      }
      R part[3 * NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        R qr_re = 0, qr_im = 0, qq = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            cplx<R> qv = q[r].c[i][c], rv = rho[r].c[i][c];
            qr_re += qv.re * rv.re + qv.im * rv.im;
            qr_im += qv.re * rv.im - qv.im * rv.re;
            qq += qv.re * qv.re + qv.im * qv.im;
          }
        part[3 * r] = qr_re;
        part[3 * r + 1] = qr_im;
        part[3 * r + 2] = qq;
      }
      // the LDS exchange of this step put a barrier after the previous reduction's reads
      double sums[3 * NR];
      block_sum_in<3 * NR, false>(part, sums, red);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double qq = sums[3 * r + 2];
        const double are = qq > 0.0 ? sums[3 * r] / qq : 0.0;
        const double aim = qq > 0.0 ? sums[3 * r + 1] / qq : 0.0;
        const cplx<R> alpha = {R(are), R(aim)};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            cmac(z[r].c[i][c], alpha, rho[r].c[i][c]);
            cplx<R> aq = alpha * q[r].c[i][c];
            rho[r].c[i][c] = rho[r].c[i][c] - aq;
          }
      }
    }

    if (active) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r >= w.nr || (a.skip && a.skip[L.sys0 + w.rhs0 + r])) continue;
        if (a.write_rho) SpinorIO<P>::store(frho[r], s, rho[r]);
        if (a.write_z) SpinorIO<P>::store(fz[r], s, z[r]);
        if (a.first) {
          SpinorIO<P>::store(fpsi[r], s, z[r]);
        } else {
          Spinor<R> p = SpinorIO<P>::load(fpsi[r], s);
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) p.c[i][c] = p.c[i][c] + z[r].c[i][c];
          SpinorIO<P>::store(fpsi[r], s, p);
        }
      }
    }
    __syncthreads();
  }
}

size_t sap_lds_bytes(int prec, int nr, int bvol) {
  const size_t cb = prec == P_F64 ? 16 : 8;
  return sizeof(double) * SAP_MAX_WAVES * 3 * nr + cb * 12 * (size_t)nr * bvol;
}

template <int P, bool C, int BV>
static void launch_pcb(const SapLaunch& a, int nr, int grid, int threads, size_t lds, hipStream_t st) {
  if (nr <= 1)
    hipLaunchKernelGGL((k_sap_mr<P, 1, C, BV>), dim3(grid), dim3(threads), lds, st, a);
  else
    hipLaunchKernelGGL((k_sap_mr<P, 2, C, BV>), dim3(grid), dim3(threads), lds, st, a);
}

template <int P, bool C>
static void launch_pc(const SapLaunch& a, int nr, int grid, int threads, size_t lds, hipStream_t st) {
  if (a.uniform_bvol == 256)
    launch_pcb<P, C, 256>(a, nr, grid, threads, lds, st);
  else
    launch_pcb<P, C, 0>(a, nr, grid, threads, lds, st);
}

template <int P>
static void launch_p(const SapLaunch& a, int nr, int grid, int threads, size_t lds, hipStream_t st) {
  if constexpr (P != P_F64) {
    if (a.cache) {
      launch_pc<P, true>(a, nr, grid, threads, lds, st);
      return;
    }
  }
  launch_pc<P, false>(a, nr, grid, threads, lds, st);
}

void launch_sap_mr(int prec, int nr, const SapLaunch& a, int grid, int threads, hipStream_t st) {
  const size_t lds = sap_lds_bytes(prec, nr, threads);
  switch (prec) {
    case P_F64: launch_p<P_F64>(a, nr, grid, threads, lds, st); break;
    case P_F32: launch_p<P_F32>(a, nr, grid, threads, lds, st); break;
    case P_F16: launch_p<P_F16>(a, nr, grid, threads, lds, st); break;
    default: launch_p<P_BF16>(a, nr, grid, threads, lds, st); break;
  }
}

}  // namespace wc
