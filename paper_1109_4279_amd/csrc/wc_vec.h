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
WC_D void st64(double2* base, const VecSite& v, const Spinor<double>& p) {
  SpinorIO<P_F64>::store(FieldRef{(void*)(base + v.off * 12), nullptr, v.V}, v.s, p);
}

// reduce NV values of the work-group and store them as this chunk's partial
template <int NV> WC_D void put_partial(const VecLaunch& a, const VecSite& v, double* vals, double* lds) {
  block_sum<NV>(vals, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) a.partials[(size_t)v.part * a.pw + i] = vals[i];
  }
}

}  // namespace wc
