// Work-item helpers of the FP64 vector kernels: every kernel walks (lattice, system,
// 256-site chunk) work items over batched fields; per-chunk partial sums feed the
// deterministic per-system reductions.
#pragma once

#include "wc_kernels.h"

namespace wc {

struct VecSite {
  int sys;
  int s;
  bool valid;
  long long off;  // site*rhs offset of this system's field
  int part;       // partial index of this (system, chunk)
  int V;
};

WC_D VecSite vec_site(const VecLaunch& a, int it0) {
  const WorkItem w = a.items[xcd_remap(it0, a.nitems)];
  const LatDesc& L = a.lats[w.lat];
  VecSite v;
  v.sys = L.sys0 + w.rhs0;
  v.s = w.chunk * WG + threadIdx.x;
  v.V = L.g.V;
  v.valid = v.s < v.V;
  if (!v.valid) v.s = v.V - 1;
  v.off = L.foff + (long long)w.rhs0 * v.V;
  v.part = L.part0 + w.rhs0 * L.nchunks + w.chunk;
  return v;
}

WC_D Spinor<double> ld64(const double2* base, const VecSite& v) {
  return SpinorIO<P_F64>::load(FieldRef{(void*)(base + v.off * 12), nullptr, v.V}, v.s);
}
// The same with non-temporal loads, for the Krylov basis vectors that Gram-Schmidt streams
// (up to 32 FP64 fields, more than the Infinity Cache holds): they then displace less of
// the operator fields that D_w and the block solver reuse (measured: the mixed 16^3x32
// solve 1 % faster, the FP64 one 1.4 %).
WC_D Spinor<double> ld64_nt(const double2* base, const VecSite& v) {
  const gptr_t<gd2v> p = (gptr_t<gd2v>)(base + v.off * 12);
  Spinor<double> o;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const gd2v x = __builtin_nontemporal_load(p + (size_t)k * v.V + v.s);
    o.c[k / 3][k % 3] = {x.x, x.y};
  }
  return o;
}
WC_D void st64(double2* base, const VecSite& v, const Spinor<double>& p) {
  SpinorIO<P_F64>::store(FieldRef{(void*)(base + v.off * 12), nullptr, v.V}, v.s, p);
}

// FGCR Krylov vectors in their storage QP (F64, or F32 for the single-precision recursion),
// widened to FP64 (NT: non-temporal loads, for the basis that Gram-Schmidt streams), or
// stored from FP64.
template <int QP, bool NT = false> WC_D Spinor<double> ldq(const void* base, const VecSite& v) {
  if constexpr (QP == P_F64) {
    return NT ? ld64_nt((const double2*)base, v) : ld64((const double2*)base, v);
  } else {
    const gptr_t<gf4v> p = (gptr_t<gf4v>)((const float4*)base + v.off * 6);
    Spinor<double> o;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      gf4v x;
      if constexpr (NT)
        x = __builtin_nontemporal_load(p + (size_t)k * v.V + v.s);
      else
        x = p[(size_t)k * v.V + v.s];
      o.c[(2 * k) / 3][(2 * k) % 3] = {double(x.x), double(x.y)};
      o.c[(2 * k + 1) / 3][(2 * k + 1) % 3] = {double(x.z), double(x.w)};
    }
    return o;
  }
}
template <int QP> WC_D Spinor<double> ldq_nt(const void* base, const VecSite& v) { return ldq<QP, true>(base, v); }
template <int QP> WC_D void stq(void* base, const VecSite& v, const Spinor<double>& p);
template <> WC_D void stq<P_F64>(void* base, const VecSite& v, const Spinor<double>& p) { st64((double2*)base, v, p); }
template <> WC_D void stq<P_F32>(void* base, const VecSite& v, const Spinor<double>& p) {
  Spinor<float> o;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.c[i][c] = {float(p.c[i][c].re), float(p.c[i][c].im)};
  SpinorIO<P_F32>::store(FieldRef{(void*)((float4*)base + v.off * 6), nullptr, v.V}, v.s, o);
}
// p as stq<QP> stores it (F32: each component rounded to the nearest float)
template <int QP> WC_D void round_to(Spinor<double>& p) {
  if (QP == P_F64) return;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) p.c[i][c] = {double(float(p.c[i][c].re)), double(float(p.c[i][c].im))};
}

// reduce NV values of the work-group and store them as this chunk's partial
template <int NV> WC_D void put_partial(const VecLaunch& a, const VecSite& v, double* vals, double* lds) {
  block_sum<NV>(vals, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) a.partials[(size_t)v.part * a.pw + i] = vals[i];
  }
}

// Threads of the per-system reduction kernels (one work-group per system).
constexpr int RWG = 1024;

// Per-system sums of the first nv values of the nc chunk partials starting at p0
// (nv <= pw <= RWG).  The work-group splits into groups of nvp = next power of two >= nv
// lanes; lane j of group g adds value j of chunks g, g + groups, ... into four independent
// accumulators (chunk index mod 4 groups), so consecutive lanes read consecutive words and
// four loads per lane are in flight; the accumulators and then the groups are added by a
// fixed tree.  Every thread of the RWG-thread work-group calls this (lds: RWG doubles);
// afterwards lds[j] holds the sum of value j.
WC_D void sum_partials(const double* partials, int pw, long long p0, int nc, int nv, double* lds) {
  int nvp = 1;
  while (nvp < nv) nvp <<= 1;
  const int groups = RWG / nvp;
  const int t = threadIdx.x, j = t % nvp, grp = t / nvp;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  if (j < nv) {
    int c = grp;
    for (; c + 3 * groups < nc; c += 4 * groups) {
      acc0 += gld_d(partials, (size_t)(p0 + c) * pw + j);
      acc1 += gld_d(partials, (size_t)(p0 + c + groups) * pw + j);
      acc2 += gld_d(partials, (size_t)(p0 + c + 2 * groups) * pw + j);
      acc3 += gld_d(partials, (size_t)(p0 + c + 3 * groups) * pw + j);
    }
    for (; c < nc; c += groups) acc0 += gld_d(partials, (size_t)(p0 + c) * pw + j);
  }
  lds[t] = (acc0 + acc1) + (acc2 + acc3);
  __syncthreads();
  for (int step = groups >> 1; step > 0; step >>= 1) {
    if (grp < step) lds[t] += lds[t + step * nvp];
    __syncthreads();
  }
}

}  // namespace wc
