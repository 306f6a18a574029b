// Even/odd-preconditioned block solver of the Schwarz alternating procedure
// (arXiv:1109.4279, Sec. 4, Table 1: even/odd preconditioning inside the block solver).
//
// On a block the sites split by parity (sum of the global coordinates mod 2) and the
// Dirichlet block operator is [[A_ee, H_eo], [H_oe, A_oo]], H its in-block hops.  With the
// odd half eliminated, MR runs on the Schur complement on the even sites,
//   S = A_ee - H_eo A_oo^-1 H_oe,    S z_e = eta_e - H_eo A_oo^-1 eta_o,
// from z_e = 0 for nmr steps (alpha per block), and the odd half follows exactly,
//   z_o = A_oo^-1 (eta_o - H_oe z_e).
// The MR residual of S is the block residual on the even sites; on the odd sites the block
// residual is zero, and that is what is stored.
//
// Work mapping: one work-group per (block, rhs group); the block's sites are paired (one
// even, one odd site per pair) and every pair is served by two adjacent lanes, s = 0, 1:
//  * vectors: lane s holds chirality block s (spins 2s, 2s+1) of each site of its pair and
//    applies clover block s (A on even sites, A^-1 on odd ones);
//  * hops: lane s computes the hops along mu = 2s and 2s+1 at both sites of its pair, so
//    both lanes work in both phases of an application of S.  In the chiral basis the two
//    direction pairs (0, 2) and (1, 3) differ only in which lower spin enters the
//    projection and with which sign, so one instruction stream serves both lanes with a
//    few selects.  One shuffle of six complex numbers per phase then gives each lane its
//    chirality block of the pair's hop sum;
//  * with `cache` the eight links and two clover blocks a lane uses are loaded once per
//    half-sweep and held in registers across the MR steps.
// An application of S is two phases through one LDS buffer of the block (rows of slots:
// even sites first, then odd ones, each in pair order): the even-site
// vector is written to the even slots, the odd sites form w_o = A_oo^-1 H_oe v into the
// odd slots, then the even sites form A_ee v - H_eo w_o.  The set-up (residual update from
// the other colour's latest block solutions) and the final stores are split by site
// instead: lane 0 works on the even site, lane 1 on the odd one.
#include "sap_eo.h"

namespace wc {

constexpr int EO_MAX_WAVES = 4;  // blocks of at most 256 sites: 128 pairs, 256 lanes

// acc += w * (1 + SGN gamma_mu)-hop of a transported neighbour spinor, for mu = 2s + J.
// J = 0: mu = 0 or 2;  J = 1: mu = 1 or 3.  In the chiral basis the projection is
//   J = 0: mu = 0: h = u - SGN (l0, l1);        mu = 2: h = u - SGN (l1, -l0)
//   J = 1: mu = 1: h = u - SGN i (l1, l0);      mu = 3: h = u - SGN i (l0, -l1)
// so with lA, lB the lower spins in the lane's order (J = 0: lA = l_{2+s}, lB = l_{3-s};
// J = 1: lA = l_{3-s}, lB = l_{2+s}; read from LDS at lane-dependent rows) and the lane sign
// sg = +1 (s = 0), -1 (s = 1), h0 = u0 - SGN phase lA and h1 = u1 - SGN phase sg lB, phase 1
// or i.  The reconstruction adds t = w U h to the upper spins and, to the lower pair kept in
// the lane's order (L0, L1) = (acc2, acc3) for s = 0 and (acc3, acc2) for s = 1,
//   J = 0: L0 += -SGN t0,      L1 += -SGN sg t1
//   J = 1: L0 += SGN sg i t1,  L1 += SGN i t0.
// The lane sign enters as a per-lane coefficient of a fused multiply-add: no selects.
template <class R, int J, int SGN, bool DAG>
WC_D void hop_dir(const SU3<R>& U, const cplx<R>* u0, const cplx<R>* u1, const cplx<R>* lA, const cplx<R>* lB,
                  R sg, R w, Spinor<R>& acc) {
  constexpr R S = R(SGN);
  const R c1 = -S * sg;  // J = 0: h1 = u1 + c1 lB;  J = 1: h1 = u1 - c1 i lB
  Half<R> h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (J == 0) {
      h.c[0][a] = {u0[a].re - S * lA[a].re, u0[a].im - S * lA[a].im};
      h.c[1][a] = {fma(c1, lB[a].re, u1[a].re), fma(c1, lB[a].im, u1[a].im)};
    } else {
      h.c[0][a] = {u0[a].re + S * lA[a].im, u0[a].im - S * lA[a].re};
      h.c[1][a] = {fma(-c1, lB[a].im, u1[a].re), fma(c1, lB[a].re, u1[a].im)};
    }
  }
  const Half<R> t = DAG ? mul_Udag(U, h) : mul_U(U, h);
  // J = 0: L0 += wl0 t0, L1 += wl1 t1;  J = 1: L0 += -wl0 i t1, L1 += wl1 i t0
  const R wl0 = J == 0 ? -S * w : -S * sg * w;
  const R wl1 = J == 0 ? -S * sg * w : S * w;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<R> t0 = t.c[0][a], t1 = t.c[1][a];
    acc.c[0][a] = {fma(w, t0.re, acc.c[0][a].re), fma(w, t0.im, acc.c[0][a].im)};
    acc.c[1][a] = {fma(w, t1.re, acc.c[1][a].re), fma(w, t1.im, acc.c[1][a].im)};
    if (J == 0) {
      acc.c[2][a] = {fma(wl0, t0.re, acc.c[2][a].re), fma(wl0, t0.im, acc.c[2][a].im)};
      acc.c[3][a] = {fma(wl1, t1.re, acc.c[3][a].re), fma(wl1, t1.im, acc.c[3][a].im)};
    } else {
      // L0 += S sg w i t1 = (-S sg w t1.im, S sg w t1.re);  L1 += S w i t0 = (-S w t0.im, S w t0.re)
      acc.c[2][a] = {fma(wl0, t1.im, acc.c[2][a].re), fma(-wl0, t1.re, acc.c[2][a].im)};
      acc.c[3][a] = {fma(-wl1, t0.im, acc.c[3][a].re), fma(wl1, t0.re, acc.c[3][a].im)};
    }
  }
}

// Geometry and operator of one site for this lane's two directions.
template <class R, bool CACHE> struct LaneSite {
  int site;        // site index
  int local;       // its index inside the tile
  int lnf[2];      // tile-local index of the forward / backward neighbour along mu = 2s + j
  int lnb[2];
  int snf[2], snb[2];  // their LDS slots (even sites first, then odd, each in pair order)
  bool f[2], b[2]; // neighbour inside the block
  SU3<R> Uf[CACHE ? 2 : 1], Ub[CACHE ? 2 : 1];
  Herm6<R> C[CACHE ? 1 : 1];  // clover block s (scaled) when cached
};

// the geometry part of LaneSite (lane_links adds the cached links)
template <int P, class R, bool CACHE>
WC_D void lane_site(const LatDesc& L, const Geom& g, int site, int local, const int* lc, int s, const short* slot,
                    LaneSite<R, CACHE>& x) {
  x.site = site;
  x.local = local;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int m = s ? lc[2 + j] : lc[j];
    const int bm = s ? g.B[2 + j] : g.B[j];
    const int st = s ? g.lstr[2 + j] : g.lstr[j];
    x.f[j] = m + 1 < bm;
    x.b[j] = m > 0;
    x.lnf[j] = local + (x.f[j] ? st : 0);
    x.lnb[j] = local - (x.b[j] ? st : 0);
    x.snf[j] = gld_s16(slot, x.lnf[j]);
    x.snb[j] = gld_s16(slot, x.lnb[j]);
  }
}

// the cached operator's links of lane_site's site (CACHE only)
template <int P, class R, bool CACHE>
WC_D void lane_links(const LatDesc& L, const Geom& g, int s, LaneSite<R, CACHE>& x) {
  if (CACHE) {
    const int base = x.site - x.local;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      x.Uf[CACHE ? j : 0] = LinkIO<P>::load(L.gauge, L.gscale, g.V, 2 * s + j, x.site);
      x.Ub[CACHE ? j : 0] = LinkIO<P>::load(L.gauge, L.gscale, g.V, 2 * s + j, base + x.lnb[j]);
    }
  }
}

template <int NR, class R>
WC_D void lds_spinor(const cplx<R>* lds, int ls, int r, int slot, Spinor<R>& p) {
#pragma unroll
  for (int k = 0; k < 12; ++k) p.c[k / 3][k % 3] = lds[(r * 12 + k) * ls + slot];
}

// out[r] = chirality block s of wt * (sum of this pair's in-block hops at site x), read from
// LDS.  Every lane of the wavefront must call this (it shuffles).  The lower spins of the
// accumulator are kept in the lane's order (hop_dir), resolved once in the final exchange.
template <int P, int NR, bool CACHE, class R>
WC_D void pair_hops(const LatDesc& L, const Geom& g, const LaneSite<R, CACHE>& x, bool act, const cplx<R>* lds,
                    int ls, int s, R wt, cplx<R> (*out)[6]) {
  Spinor<R> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) zero(acc[r]);
  const R sg = s ? R(-1) : R(1);
  if (act) {
    const int base = x.site - x.local;
    auto dir = [&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      const int mu = 2 * s + J;
      // rows of the lower spins in the lane's order
      const int rowA = 3 * (J == 0 ? 2 + s : 3 - s), rowB = 3 * (J == 0 ? 3 - s : 2 + s);
      auto read = [&](int r, int slot, cplx<R>* u0, cplx<R>* u1, cplx<R>* lA, cplx<R>* lB) {
        const cplx<R>* q = lds + (size_t)(r * 12) * ls + slot;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          u0[a] = q[a * ls];
          u1[a] = q[(3 + a) * ls];
          lA[a] = q[(rowA + a) * ls];
          lB[a] = q[(rowB + a) * ls];
        }
      };
      if (x.f[J]) {
        const SU3<R> U = CACHE ? x.Uf[CACHE ? J : 0] : LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, mu, x.site);
        const R w = CACHE ? wt : wt * LinkIO<P>::scale(L.gscale, x.site);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          cplx<R> u0[3], u1[3], lA[3], lB[3];
          read(r, x.snf[J], u0, u1, lA, lB);
          hop_dir<R, J, -1, false>(U, u0, u1, lA, lB, sg, w, acc[r]);
        }
      }
      if (x.b[J]) {
        const int nb = base + x.lnb[J];
        const SU3<R> U = CACHE ? x.Ub[CACHE ? J : 0] : LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, mu, nb);
        const R w = CACHE ? wt : wt * LinkIO<P>::scale(L.gscale, nb);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          cplx<R> u0[3], u1[3], lA[3], lB[3];
          read(r, x.snb[J], u0, u1, lA, lB);
          hop_dir<R, J, +1, true>(U, u0, u1, lA, lB, sg, w, acc[r]);
        }
      }
    };
    dir(std::integral_constant<int, 0>());
    dir(std::integral_constant<int, 1>());
  }
  // lane 0 keeps the upper spins and sends its lower pair (acc2, acc3); lane 1 keeps its
  // lower pair, stored as (acc3, acc2), and sends its upper spins
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const cplx<R> up = acc[r].c[i / 3][i % 3];
      const cplx<R> low = acc[r].c[2 + i / 3][i % 3];
      const cplx<R> low_sw = acc[r].c[2 + (1 - i / 3)][i % 3];
      const cplx<R> mine = s ? low_sw : up;
      const cplx<R> send = s ? up : low;
      out[r][i] = mine + shfl1(send);
    }
}

// out[r] (+)= C_s(x) in[r] on chirality block s (a 16-bit block's scale multiplies the
// product, six complex numbers, rather than the block's 36 entries)
template <int P, int NR, bool CACHE, bool ACC, class R>
WC_D void clover_half(const LatDesc& L, const Geom& g, const LaneSite<R, CACHE>& x, int s, const cplx<R> (*in)[6],
                      cplx<R> (*out)[6]) {
  const Herm6<R> h = CACHE ? x.C[0] : clover_block<P, R>(L, g.V, x.site, s);
  const R cs = CACHE ? R(1) : clover_scale<P, R>(L, x.site, s);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    cplx<R> o[6];
    herm6_apply(h, in[r], o);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (!CACHE && (P == P_F16 || P == P_BF16)) o[i] = cs * o[i];
      out[r][i] = ACC ? out[r][i] + o[i] : o[i];
    }
  }
}

template <int NR, class R>
WC_D void half_to_lds(cplx<R>* lds, int ls, int slot, int s, const cplx<R> (*v)[6]) {
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 6; ++i) lds[(r * 12 + 6 * s + i) * ls + slot] = v[r][i];
}

// rho(site) -= (D z)(site) for the hops from site into neighbouring blocks (the other
// colour's latest z): full spinor, all directions, +1/2 weight
template <int P, int NR, class R>
WC_D void border_update(const LatDesc& L, const Geom& g, int site, int tile, const int* tc, const int* lc,
                        const FieldRef* fz, Spinor<R>* rho) {
  auto one = [&](auto MUc) {
    constexpr int MU = decltype(MUc)::value;
    int ph;
    bool inside;
    const int nf = neighbour(g, site, tile, tc, lc, MU, +1, &ph, &inside);
    if (!inside) {
      const SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, site);
      const R w = R(0.5) * R(ph) * LinkIO<P>::scale(L.gscale, site);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const Spinor<R> p = SpinorIO<P>::load_raw(fz[r], nf);
        accum_recon<R, MU, -1>(rho[r], mul_U(u, project<R, MU, -1>(p)), w * SpinorIO<P>::scale(fz[r], nf));
      }
    }
    const int nb = neighbour(g, site, tile, tc, lc, MU, -1, &ph, &inside);
    if (!inside) {
      const SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, nb);
      const R w = R(0.5) * R(ph) * LinkIO<P>::scale(L.gscale, nb);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const Spinor<R> p = SpinorIO<P>::load_raw(fz[r], nb);
        accum_recon<R, MU, +1>(rho[r], mul_Udag(u, project<R, MU, +1>(p)), w * SpinorIO<P>::scale(fz[r], nb));
      }
    }
  };
  one(std::integral_constant<int, 0>());
  one(std::integral_constant<int, 1>());
  one(std::integral_constant<int, 2>());
  one(std::integral_constant<int, 3>());
}

// The border update as entries: every hop out of the block (direction mu, forward or
// backward face, face site f) is one entry, ordered by direction, forward face before
// backward, face sites lexicographic in the other three coordinates (x3 fastest).  The
// entries of one face share the direction, so a wavefront of them runs one code path; each
// writes the hop's contribution to rho (+1/2 (1 -+ gamma_mu) U z of the neighbouring block)
// to its own LDS slot, and the sites then add their entries (none inside the block, up to
// one per face they lie on).
WC_HD int face_size(const Geom& g, int mu) { return g.bvol / g.B[mu]; }

WC_D int face_index(const Geom& g, const int* lc, int mu) {
  int f = 0;
#pragma unroll
  for (int nu = 0; nu < 4; ++nu)
    if (nu != mu) f = f * g.B[nu] + lc[nu];
  return f;
}

template <int P, int NR, int MU, class R>
WC_D void border_entry(const LatDesc& L, const Geom& g, int tile, const int* tc, int base, int f, bool fwd,
                       const FieldRef* fz, cplx<R>* bord, int ne, int e) {
  int lc[4];
  int q = f;
#pragma unroll
  for (int nu = 3; nu >= 0; --nu) {
    if (nu == MU) continue;
    lc[nu] = q % g.B[nu];
    q /= g.B[nu];
  }
  lc[MU] = fwd ? g.B[MU] - 1 : 0;
  const int local = lc[0] * g.lstr[0] + lc[1] * g.lstr[1] + lc[2] * g.lstr[2] + lc[3] * g.lstr[3];
  const int site = base + local;
  Spinor<R> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) zero(acc[r]);
  int ph;
  bool inside;
  if (fwd) {
    const int nf = neighbour(g, site, tile, tc, lc, MU, +1, &ph, &inside);
    const SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, site);
    const R w = R(0.5) * R(ph) * LinkIO<P>::scale(L.gscale, site);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const Spinor<R> p = SpinorIO<P>::load_raw(fz[r], nf);
      accum_recon<R, MU, -1>(acc[r], mul_U(u, project<R, MU, -1>(p)), w * SpinorIO<P>::scale(fz[r], nf));
    }
  } else {
    const int nb = neighbour(g, site, tile, tc, lc, MU, -1, &ph, &inside);
    const SU3<R> u = LinkIO<P>::load_raw(L.gauge, L.gscale, g.V, MU, nb);
    const R w = R(0.5) * R(ph) * LinkIO<P>::scale(L.gscale, nb);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const Spinor<R> p = SpinorIO<P>::load_raw(fz[r], nb);
      accum_recon<R, MU, +1>(acc[r], mul_Udag(u, project<R, MU, +1>(p)), w * SpinorIO<P>::scale(fz[r], nb));
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) bord[(r * 12 + k) * ne + e] = acc[r].c[k / 3][k % 3];
}

// all entries of the block into LDS; the caller puts a barrier after it
template <int P, int NR, class R>
WC_D void border_entries(const LatDesc& L, const Geom& g, int tile, const int* tc, int base, const FieldRef* fz,
                         cplx<R>* bord, int ne) {
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    int off = 0, mu = 3, f = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int n2 = 2 * face_size(g, m);
      if (e - off < n2) {
        mu = m;
        break;
      }
      off += n2;
    }
    f = e - off;
    const int F = face_size(g, mu);
    const bool fwd = f < F;
    if (!fwd) f -= F;
    switch (mu) {
      case 0: border_entry<P, NR, 0>(L, g, tile, tc, base, f, fwd, fz, bord, ne, e); break;
      case 1: border_entry<P, NR, 1>(L, g, tile, tc, base, f, fwd, fz, bord, ne, e); break;
      case 2: border_entry<P, NR, 2>(L, g, tile, tc, base, f, fwd, fz, bord, ne, e); break;
      default: border_entry<P, NR, 3>(L, g, tile, tc, base, f, fwd, fz, bord, ne, e); break;
    }
  }
}

// rho(site) += its border entries (site with tile-local coordinates lc)
template <int NR, class R>
WC_D void border_gather(const Geom& g, const int* lc, const cplx<R>* bord, int ne, Spinor<R>* rho) {
  int off = 0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int F = face_size(g, mu);
    const int f = face_index(g, lc, mu);
    if (lc[mu] == g.B[mu] - 1) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) rho[r].c[k / 3][k % 3] = rho[r].c[k / 3][k % 3] + bord[(r * 12 + k) * ne + off + f];
    }
    if (lc[mu] == 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k)
          rho[r].c[k / 3][k % 3] = rho[r].c[k / 3][k % 3] + bord[(r * 12 + k) * ne + off + F + f];
    }
    off += 2 * F;
  }
}

template <int P, int NR, bool CACHE>
__global__ __launch_bounds__(64 * EO_MAX_WAVES) void k_sap_eo(SapLaunch a) {
  typedef typename Real<P>::T R;
  extern __shared__ double smem_d[];
  double* red = smem_d;                                        // EO_MAX_WAVES * 3 * NR doubles
  cplx<R>* lds = (cplx<R>*)(smem_d + EO_MAX_WAVES * 3 * NR);  // [NR][12][bvol]
  cplx<R>* bord = lds + (size_t)NR * 12 * a.eo_rows;           // [NR][12][border entries]

  const int s = threadIdx.x & 1;
  const int pr = threadIdx.x >> 1;
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
    const int base = tile * g.bvol;
    const int nh = (g.bvol + 1) >> 1;
    int tc[4];
    tile_coords(g, tile, tc);
    const int cp = (tc[0] * g.B[0] + tc[1] * g.B[1] + tc[2] * g.B[2] + tc[3] * g.B[3]) & 1;
    const int le = pr < nh ? gld_s16(L.eo_sites, (2 * cp) * nh + pr) : -1;
    const int lo = pr < nh ? gld_s16(L.eo_sites, (2 * cp + 1) * nh + pr) : -1;
    const bool he = le >= 0, ho = lo >= 0;
    const int lel = he ? le : 0, lol = ho ? lo : 0;
    int lce[4], lco[4];
    local_coords(g, lel, lce);
    local_coords(g, lol, lco);
    LaneSite<R, CACHE> xe, xo;
    const short* slot = L.eo_slot + cp * g.bvol;
    const int ls = 2 * nh;  // LDS row: slots 0..nh-1 even sites, nh..2nh-1 odd sites, in pair order
    lane_site<P, R, CACHE>(L, g, base + lel, lel, lce, s, slot, xe);
    lane_site<P, R, CACHE>(L, g, base + lol, lol, lco, s, slot, xo);

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

    // Block residual at this lane's site (lane 0: even, lane 1: odd), brought up to date
    // with the other colour's latest block solutions; then each lane takes chirality block
    // s of both sites.
    const int own = s ? xo.site : xe.site;
    const bool own_act = s ? ho : he;
    cplx<R> re[NR][6], eo[NR][6];
    {
      Spinor<R> v[NR];
      const bool implicit_zero = s == 1 && a.odd_rho == 2;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (implicit_zero)
          zero(v[r]);
        else
          v[r] = SpinorIO<P>::load(frho[r], own);
      }
      if (a.border && a.border_entries) {
        const int ne = border_entry_count(g.B);
        border_entries<P, NR>(L, g, tile, tc, base, fz, bord, ne);
        __syncthreads();
        if (own_act) border_gather<NR>(g, s ? lco : lce, bord, ne, v);
      } else if (a.border && own_act) {
        border_update<P, NR>(L, g, own, tile, tc, s ? lco : lce, fz, v);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          // lane 0 keeps block 0 of the even site and sends block 1; lane 1 keeps block 1
          // of the odd site and sends block 0
          const cplx<R> lo_blk = v[r].c[i / 3][i % 3], hi_blk = v[r].c[2 + i / 3][i % 3];
          const cplx<R> got = shfl1(s ? lo_blk : hi_blk);  // lane 0: odd block 0; lane 1: even block 1
          re[r][i] = s ? got : lo_blk;
          eo[r][i] = s ? hi_blk : got;
        }
    }

    // the cached operator is loaded after the residual and the border update, whose loads
    // the first arithmetic waits for
    lane_links<P, R, CACHE>(L, g, s, xe);
    lane_links<P, R, CACHE>(L, g, s, xo);
    if (CACHE) {
      xe.C[0] = clover_block_scaled<P, R>(L, g.V, xe.site, s);
      xo.C[0] = clover_block_scaled<P, R>(L, g.V, xo.site, s);
    }
    // t_o = A_oo^-1 eta_o ; source of the Schur system: eta_e - H_eo t_o
    cplx<R> to[NR][6];
    clover_half<P, NR, CACHE, false>(L, g, xo, s, eo, to);
    if (ho) half_to_lds<NR>(lds, ls, nh + pr, s, to);
    __syncthreads();
    {
      cplx<R> d[NR][6];
      pair_hops<P, NR, CACHE>(L, g, xe, he, lds, ls, s, R(0.5), d);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 6; ++i) re[r][i] = re[r][i] + d[r][i];
    }

    cplx<R> ze[NR][6];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < 6; ++i) ze[r][i] = {R(0), R(0)};
    for (int it = 0; it < a.nmr; ++it) {
      // q = S rho_e = A_ee rho_e - H_eo A_oo^-1 H_oe rho_e   (H = -1/2 sum of hops)
      if (he) half_to_lds<NR>(lds, ls, pr, s, re);
      __syncthreads();
      {
        cplx<R> t[NR][6], wo[NR][6];
        pair_hops<P, NR, CACHE>(L, g, xo, ho, lds, ls, s, R(-0.5), t);
        clover_half<P, NR, CACHE, false>(L, g, xo, s, t, wo);
        if (ho) half_to_lds<NR>(lds, ls, nh + pr, s, wo);
      }
      __syncthreads();
      cplx<R> q[NR][6];
      pair_hops<P, NR, CACHE>(L, g, xe, he, lds, ls, s, R(0.5), q);
      clover_half<P, NR, CACHE, true>(L, g, xe, s, re, q);
      R part[3 * NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        R qr_re = 0, qr_im = 0, qq = 0;
        if (he) {
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const cplx<R> qv = q[r][i], rv = re[r][i];
            qr_re += qv.re * rv.re + qv.im * rv.im;
            qr_im += qv.re * rv.im - qv.im * rv.re;
            qq += qv.re * qv.re + qv.im * qv.im;
          }
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
        for (int i = 0; i < 6; ++i) {
          cmac(ze[r][i], alpha, re[r][i]);
          re[r][i] = re[r][i] - alpha * q[r][i];
        }
      }
    }

    // z_o = t_o - A_oo^-1 H_oe z_e
    if (he) half_to_lds<NR>(lds, ls, pr, s, ze);
    __syncthreads();
    cplx<R> zo[NR][6];
    {
      cplx<R> t[NR][6];
      pair_hops<P, NR, CACHE>(L, g, xo, ho, lds, ls, s, R(0.5), t);
      clover_half<P, NR, CACHE, false>(L, g, xo, s, t, zo);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 6; ++i) zo[r][i] = zo[r][i] + to[r][i];
    }

    // Lane 0 of a pair stores the even site, lane 1 the odd one; each first collects the
    // other chirality block of what it stores from its partner.
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      Spinor<R> Z, RH;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const cplx<R> x = shfl1(s ? re[r][i] : zo[r][i]);  // lane 0 gets rho_e block 1, lane 1 z_o block 0
        const cplx<R> y = shfl1(ze[r][i]);                 // lane 0 gets z_e block 1
        const cplx<R> zero_c = {R(0), R(0)};
        Z.c[i / 3][i % 3] = s ? x : ze[r][i];
        Z.c[2 + i / 3][i % 3] = s ? zo[r][i] : y;
        RH.c[i / 3][i % 3] = s ? zero_c : re[r][i];
        RH.c[2 + i / 3][i % 3] = s ? zero_c : x;
      }
      if (!own_act || r >= w.nr || (a.skip && a.skip[L.sys0 + w.rhs0 + r])) continue;
      if (a.write_rho && !(s == 1 && a.odd_rho != 0)) SpinorIO<P>::store(frho[r], own, RH);
      if (a.write_z) SpinorIO<P>::store(fz[r], own, Z);
      if (!a.first) {
        const Spinor<R> p = SpinorIO<P>::load(fpsi[r], own);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) Z.c[i][c] = Z.c[i][c] + p.c[i][c];
      }
      SpinorIO<P>::store(fpsi[r], own, Z);
    }
    __syncthreads();
  }
}

static int eo_threads(int max_bvol) { return (2 * ((max_bvol + 1) / 2) + 63) / 64 * 64; }

size_t sap_eo_lds_bytes(int prec, int nr, int max_bvol, int border_entries) {
  const size_t cb = prec == P_F64 ? 16 : 8;
  return sizeof(double) * EO_MAX_WAVES * 3 * nr + cb * 12 * (size_t)nr * (2 * ((max_bvol + 1) / 2)) +
         cb * 12 * (size_t)nr * border_entries;
}

template <int P>
static void launch_p(const SapLaunch& a, int nr, int grid, int threads, size_t lds, hipStream_t st) {
  if (nr <= 1) {
    if constexpr (P != P_F64) {
      if (a.cache) {
        hipLaunchKernelGGL((k_sap_eo<P, 1, true>), dim3(grid), dim3(threads), lds, st, a);
        return;
      }
    }
    hipLaunchKernelGGL((k_sap_eo<P, 1, false>), dim3(grid), dim3(threads), lds, st, a);
  } else {
    hipLaunchKernelGGL((k_sap_eo<P, 2, false>), dim3(grid), dim3(threads), lds, st, a);
  }
}

void launch_sap_eo(int prec, int nr, const SapLaunch& a, int grid, int max_bvol, hipStream_t st) {
  const size_t lds = sap_eo_lds_bytes(prec, nr, max_bvol, a.border_entries);
  const int threads = eo_threads(max_bvol);
  switch (prec) {
    case P_F64: launch_p<P_F64>(a, nr, grid, threads, lds, st); break;
    case P_F32: launch_p<P_F32>(a, nr, grid, threads, lds, st); break;
    case P_F16: launch_p<P_F16>(a, nr, grid, threads, lds, st); break;
    default: launch_p<P_BF16>(a, nr, grid, threads, lds, st); break;
  }
}

}  // namespace wc
