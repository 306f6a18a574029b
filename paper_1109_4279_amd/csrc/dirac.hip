// D_w on the full lattice and its Dirichlet-block restriction, all storage precisions.
//
// The operator (Wilson-Dirac with clover term, arXiv:1109.4279 abstract and Sec. 4):
//   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// with A(x) the two 6x6 Hermitian chiral clover blocks (which include 4 + m0).
// Block mode drops every hop whose neighbour lies in another tile (Sec. 4: the
// blocks are solved with Dirichlet boundary conditions).
//
// One lane per site, NR right-hand sides per lane: each link and clover block is
// loaded once and applied to NR spinors.  The kernel is HBM-bound; neighbour
// spinors come mostly from L2 because tiles of one XCD are spatially contiguous.
#include "wc_kernels.h"

namespace wc {

template <class R> WC_D void g5(Spinor<R>& p) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    p.c[2][a] = -p.c[2][a];
    p.c[3][a] = -p.c[3][a];
  }
}

template <class R, class T> WC_D Spinor<R> to_real(const Spinor<T>& p) {
  Spinor<R> o;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.c[i][c] = {R(p.c[i][c].re), R(p.c[i][c].im)};
  return o;
}

// STAGE: every work item is one 256-site tile (Schwarz blocks of 256 sites); the tile's
// input spinors are decoded once into LDS and the in-tile neighbours are read from there,
// so each spinor leaves HBM/L2 once per tile instead of once per neighbour.
// PIN: storage precision of the input (FP64 and FP32 arithmetic may read an input of
// another storage, widened or rounded to the arithmetic's precision; the 16-bit launches
// read their own precision).
template <int P, int NR, bool STAGE, int PIN = P>
__global__ __launch_bounds__(WG) void k_dirac(DiracLaunch a) {
  typedef typename Real<P>::T R;
  __shared__ double red[(WG / 64) * NR];
  extern __shared__ double stage_d[];
  cplx<R>* st_sp = (cplx<R>*)stage_d;        // [NR][12][WG] input spinors of the tile (unscaled)
  R* st_sc = (R*)(st_sp + NR * 12 * WG);     // [NR][WG] their site scales
  if (cycle_dead(a.dead)) return;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    const WorkItem w = load_uniform(a.items, xcd_remap(it0, a.nitems));
    const LatDesc L = load_uniform(a.lats, w.lat);
    const Geom g = L.g;
    bool any = true;
    if (a.skip) {
      any = false;
      for (int r = 0; r < w.nr; ++r) any |= (a.skip[L.sys0 + w.rhs0 + r] == 0);
    }
    if (!any) continue;
    const int s_raw = w.chunk * WG + threadIdx.x;
    const bool valid = s_raw < g.V;
    const int s = valid ? s_raw : g.V - 1;
    const int tile = s / g.bvol;
    int tc[4], lc[4];
    tile_coords(g, tile, tc);
    local_coords(g, s - tile * g.bvol, lc);

    FieldRef fin[NR], fout[NR], fy[NR];
    const int sb = spinor_site_bytes(P), sbin = spinor_site_bytes(PIN);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int rr = w.rhs0 + (r < w.nr ? r : 0);
      const long long off = L.foff + (long long)rr * g.V;
      fin[r] = {(char*)a.in + off * sbin, a.in_sc ? (float*)a.in_sc + off : nullptr, g.V};
      fout[r] = {(char*)a.out + off * sb, a.out_sc ? a.out_sc + off : nullptr, g.V};
      fy[r] = {a.y ? (char*)a.y + off * sb : nullptr, a.y_sc ? (float*)a.y_sc + off : nullptr, g.V};
    }

    Spinor<R> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) zero(acc[r]);
    if (STAGE) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        Spinor<R> p = to_real<R>(SpinorIO<PIN>::load_raw(fin[r], s));
#pragma unroll
        for (int k = 0; k < 12; ++k) st_sp[(r * 12 + k) * WG + threadIdx.x] = p.c[k / 3][k % 3];
        st_sc[r * WG + threadIdx.x] = SpinorIO<PIN>::scale(fin[r], s);
      }
      __syncthreads();
    }
    // input spinor r at site n: from the staged tile when n is in it, else from memory
    auto in_raw = [&](int r, int n, bool in_tile, R& sc) {
      Spinor<R> p;
      if (STAGE && in_tile) {
        const int ln = n - tile * WG;
#pragma unroll
        for (int k = 0; k < 12; ++k) p.c[k / 3][k % 3] = st_sp[(r * 12 + k) * WG + ln];
        sc = st_sc[r * WG + ln];
      } else {
        p = to_real<R>(SpinorIO<PIN>::load_raw(fin[r], n));
        sc = SpinorIO<PIN>::scale(fin[r], n);
      }
      return p;
    };

    auto hop = [&](auto MUc) {
      constexpr int MU = decltype(MUc)::value;
      int ph;
      bool same;
      // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
      int nf = neighbour(g, s, tile, tc, lc, MU, +1, &ph, &same);
      // 16-bit storage: links and spinors are used unscaled and the site scales folded
      // into the one weight of the hop
      if (!a.block || same) {
        SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, s);
        const R w8 = R(ph) * LinkIO<P>::scale(L.gscale, s);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          R sc;
          Spinor<R> p = in_raw(r, nf, same, sc);
          if (a.dagger) g5(p);
          Half<R> h = mul_U(u, project<R, MU, -1>(p));
          accum_recon<R, MU, -1>(acc[r], h, w8 * sc);
        }
      }
      // backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
      int nb = neighbour(g, s, tile, tc, lc, MU, -1, &ph, &same);
      if (!a.block || same) {
        SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, nb);
        const R w8 = R(ph) * LinkIO<P>::scale(L.gscale, nb);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          R sc;
          Spinor<R> p = in_raw(r, nb, same, sc);
          if (a.dagger) g5(p);
          Half<R> h = mul_Udag(u, project<R, MU, +1>(p));
          accum_recon<R, MU, +1>(acc[r], h, w8 * sc);
        }
      }
    };
    hop(std::integral_constant<int, 0>());
    hop(std::integral_constant<int, 1>());
    hop(std::integral_constant<int, 2>());
    hop(std::integral_constant<int, 3>());

    // clover and the -1/2 of the hopping term; acc becomes the result
    Spinor<R> self[NR];
    R sself[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      self[r] = in_raw(r, s, true, sself[r]);
      if (a.dagger) g5(self[r]);
    }
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      Herm6<R> hc = CloverIO<P>::load_raw(L.clov, L.cscale, g.V, s, blk);
      const R cs = CloverIO<P>::scale(L.cscale, s, blk);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        cplx<R> v[6], o[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = self[r].c[2 * blk + i / 3][i % 3];
        herm6_apply(hc, v, o);
        const R w = cs * sself[r];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          cplx<R>& t = acc[r].c[2 * blk + i / 3][i % 3];
          t = w * o[i] - R(0.5) * t;
        }
      }
    }
    double nrm[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (a.dagger) g5(acc[r]);
      if (a.y) {  // residual form: out = y - D in
        Spinor<R> yv = SpinorIO<P>::load(fy[r], s);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r].c[i][c] = yv.c[i][c] - acc[r].c[i][c];
      }
      nrm[r] = 0.0;
      const bool skip_r = r >= w.nr || (a.skip && a.skip[L.sys0 + w.rhs0 + r]);
      if (valid && !skip_r) {
        SpinorIO<P>::store(fout[r], s, acc[r]);
        if (a.partials) {
          double t = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              t += double(acc[r].c[i][c].re) * double(acc[r].c[i][c].re) +
                   double(acc[r].c[i][c].im) * double(acc[r].c[i][c].im);
          nrm[r] = t;
        }
      }
    }
    if (a.partials) {
      block_sum<NR>(nrm, red);
      if (threadIdx.x == 0) {
        for (int r = 0; r < w.nr; ++r) a.partials[(size_t)(L.part0 + (w.rhs0 + r) * L.nchunks + w.chunk) * a.pw] = nrm[r];
      }
      __syncthreads();
    }
    if (STAGE) __syncthreads();  // the next item overwrites the staged tile
  }
}

// dynamic LDS of a staged launch: the tile's input spinors (12 complex) and site scale per
// rhs of the lane's tile (nr clamped to the 1..4 the launch switch instantiates)
size_t dirac_stage_lds_bytes(int prec, int nr) {
  const size_t real = prec == P_F64 ? 8 : 4;
  return (2 * real * 12 + real) * (size_t)std::min(std::max(nr, 1), 4) * WG;
}

template <int P, bool S, int PIN>
static void launch_ps(const DiracLaunch& a, int nr, int grid, hipStream_t st) {
  auto lds = [&](int n) { return S ? dirac_stage_lds_bytes(P, n) : size_t(0); };
  switch (nr) {
    case 1: hipLaunchKernelGGL((k_dirac<P, 1, S, PIN>), dim3(grid), dim3(WG), lds(1), st, a); break;
    case 2: hipLaunchKernelGGL((k_dirac<P, 2, S, PIN>), dim3(grid), dim3(WG), lds(2), st, a); break;
    case 3: hipLaunchKernelGGL((k_dirac<P, 3, S, PIN>), dim3(grid), dim3(WG), lds(3), st, a); break;
    default: hipLaunchKernelGGL((k_dirac<P, 4, S, PIN>), dim3(grid), dim3(WG), lds(4), st, a); break;
  }
}

template <int P, int PIN>
static void launch_p(const DiracLaunch& a, int nr, int grid, hipStream_t st) {
  if (a.stage)
    launch_ps<P, true, PIN>(a, nr, grid, st);
  else
    launch_ps<P, false, PIN>(a, nr, grid, st);
}

void launch_dirac(int prec, int nr, const DiracLaunch& a, int grid, hipStream_t st) {
  if (prec == P_F64) {
    switch (a.in_prec) {
      case P_F64: launch_p<P_F64, P_F64>(a, nr, grid, st); break;
      case P_F32: launch_p<P_F64, P_F32>(a, nr, grid, st); break;
      case P_F16: launch_p<P_F64, P_F16>(a, nr, grid, st); break;
      default: launch_p<P_F64, P_BF16>(a, nr, grid, st); break;
    }
    return;
  }
  if (prec == P_F32) {
    switch (a.in_prec) {
      case P_F64: launch_p<P_F32, P_F64>(a, nr, grid, st); break;
      case P_F32: launch_p<P_F32, P_F32>(a, nr, grid, st); break;
      case P_F16: launch_p<P_F32, P_F16>(a, nr, grid, st); break;
      default: launch_p<P_F32, P_BF16>(a, nr, grid, st); break;
    }
    return;
  }
  switch (prec) {
    case P_F16: launch_p<P_F16, P_F16>(a, nr, grid, st); break;
    default: launch_p<P_BF16, P_BF16>(a, nr, grid, st); break;
  }
}

}  // namespace wc
