// Vector kernels of the restarted FGCR outer solver (arXiv:1109.4279, Sec. 4), in FP64
// arithmetic over an FP64 or F32-stored Krylov basis:
// Gram-Schmidt against the previous directions, residual update, solution update,
// and the conversions to and from the Schwarz preconditioner's precision.
//
// Every kernel walks (lattice, system, 256-site chunk) work items; per-system scalars
// live in device memory (SysState) so a whole restart cycle runs without the host.
// Reductions are deterministic: per-chunk partial sums, then one work-group per
// system adds them in a fixed order.
#include "wc_vec.h"

namespace wc {

// ------------------------------------------------------------------ conversions

template <int P, int QP>
__global__ __launch_bounds__(WG) void k_to_sap(VecLaunch a) {
  typedef typename Real<P>::T R;
  // a new cycle: its launches run again
  if (a.dead && blockIdx.x == 0 && threadIdx.x == 0) a.dead[0] = 0;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys] || !v.valid) continue;
    const double inv = 1.0 / sqrt(a.sys[v.sys].rnorm2);
    Spinor<double> r = ld64(a.r, v);
    if (QP != P_F64) stq<QP>(a.rq, v, r);
    Spinor<R> o;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) o.c[i][c] = {R(r.c[i][c].re * inv), R(r.c[i][c].im * inv)};
    SpinorIO<P>::store(FieldRef{(char*)a.sp + v.off * spinor_site_bytes(P), a.sp_sc ? a.sp_sc + v.off : nullptr, v.V},
                       v.s, o);
  }
}

// the next preconditioner input eta = r / |r_k| at one site, written by the residual
// update (|r_k|^2 is still the system's rnorm2 there: the reduction after the update
// replaces it); any positive scale would do, the preconditioner's storage only needs r
// brought to a modest range
template <int P>
WC_D void store_sap_input(const VecLaunch& a, const VecSite& v, const Spinor<double>& r) {
  typedef typename Real<P>::T R;
  const double n2 = a.sys[v.sys].rnorm2;
  const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 1.0;
  Spinor<R> o;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.c[i][c] = {R(r.c[i][c].re * inv), R(r.c[i][c].im * inv)};
  SpinorIO<P>::store(FieldRef{(char*)a.sp + v.off * spinor_site_bytes(P), a.sp_sc ? a.sp_sc + v.off : nullptr, v.V},
                     v.s, o);
}

// ------------------------------------------------------------------ Gram-Schmidt

// One pass over chi_k, r and chi_0..chi_{k-1}: partial sums of
//   a_l = <chi_l, chi_k>, e_l = <chi_l, r> (l < k), |chi_k|^2 and <chi_k, r>.
// With them the reduction gets the classical Gram-Schmidt coefficients a_lk, the squared
// norm |chi_k|^2 - sum |a_lk|^2 of chi_k - sum a_lk chi_l (the chi_l being orthonormal)
// and c_k = <chi_k - sum a_lk chi_l, r> / b_k without another pass over the vectors.  The
// subtraction is exact enough only while it keeps a fair share of |chi_k|^2; below half of
// it (the criterion of Daniel, Gragg, Kaufman and Stewart, Math. Comp. 30 (1976) 772) the
// reduction asks for a second classical pass instead (k_gs_update, RED_GS2, k_gs_update2).
// Partial layout per chunk: [2k a][2k e][|chi_k|^2][2 <chi_k, r>].
// Before its Gram-Schmidt chi_k is the direction w = D phi_k; w and the earlier chi_l are
// read from the basis storage QP (F32 for the single-precision recursion of Sec. 4).
template <int QP>
__global__ __launch_bounds__(WG) void k_gs_dots(VecLaunch a) {
  __shared__ double lds[(WG / 64) * (4 * NKV_MAX + 4)];
  if (cycle_dead(a.dead)) return;
  const int k = a.k;
  const int nv = 4 * k + 3;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys]) continue;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Spinor<double> ck = ldq<QP>(a.w, v);
    Spinor<double> r = ldq<QP>(a.rq, v);
    if (!v.valid) {
      zero(ck);
      zero(r);
    }
    auto put = [&](int j, double x) {
      x = wave_sum(x);
      if (lane == 0) lds[wid * (4 * NKV_MAX + 4) + j] = x;
    };
    for (int l = 0; l < k; ++l) {
      Spinor<double> cl = ldq_nt<QP>(a.q[l], v);
      double are = 0.0, aim = 0.0, ere = 0.0, eim = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cplx<double> x = cl.c[i][c];
          are += x.re * ck.c[i][c].re + x.im * ck.c[i][c].im;
          aim += x.re * ck.c[i][c].im - x.im * ck.c[i][c].re;
          ere += x.re * r.c[i][c].re + x.im * r.c[i][c].im;
          eim += x.re * r.c[i][c].im - x.im * r.c[i][c].re;
        }
      put(2 * l, are);
      put(2 * l + 1, aim);
      put(2 * k + 2 * l, ere);
      put(2 * k + 2 * l + 1, eim);
    }
    double n2 = 0.0, cre = 0.0, cim = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cplx<double> x = ck.c[i][c];
        n2 += x.re * x.re + x.im * x.im;
        cre += x.re * r.c[i][c].re + x.im * r.c[i][c].im;
        cim += x.re * r.c[i][c].im - x.im * r.c[i][c].re;
      }
    put(4 * k, n2);
    put(4 * k + 1, cre);
    put(4 * k + 2, cim);
    __syncthreads();
    for (int j = threadIdx.x; j < nv; j += WG) {
      double t = 0.0;
      for (int w = 0; w < WG / 64; ++w) t += lds[w * (4 * NKV_MAX + 4) + j];
      a.partials[(size_t)v.part * a.pw + j] = t;
    }
    __syncthreads();
  }
}

// chi_k <- (w - sum_l a_lk chi_l) / b_k, stored in QP;  r <- r - c_k chi_k with chi_k as
// stored (so that r stays the residual of the stored basis), r held in QP too (the FP64 r
// with an FP64 basis, its F32 copy rq with an F32 one);  partial |r|^2 of r as stored; with
// fuse_sap also the next preconditioner input r / |r_k| (storage P).
// A system flagged by the reduction for a second pass (S.reorth) instead stores
// chi_k' = w - sum_l a_lk chi_l in w (storage QP) and the partial sums of the second pass,
//   a2_l = <chi_l, chi_k'> (l < k), |chi_k'|^2 and <chi_k', r>,
// as [2k a2][|chi_k'|^2][2 <chi_k', r>]; r is left for k_gs_update2.
template <int P, int QP>
__global__ __launch_bounds__(WG) void k_gs_update(VecLaunch a) {
  __shared__ double lds[(WG / 64) * (2 * NKV_MAX + 4)];
  if (cycle_dead(a.dead)) return;
  const int k = a.k;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys]) continue;
    const SysState& S = a.sys[v.sys];
    Spinor<double> ck = ldq<QP>(a.w, v);
    for (int l = 0; l < k; ++l) {
      const double2 al = S.a[l * NKV_MAX + k];
      const cplx<double> m = {-al.x, -al.y};
      Spinor<double> cl = ldq_nt<QP>(a.q[l], v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(ck.c[i][c], m, cl.c[i][c]);
    }
    if (S.reorth) {
      const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
      constexpr int LD = 2 * NKV_MAX + 4;
      if (v.valid)
        stq<QP>(a.w, v, ck);
      else
        zero(ck);
      Spinor<double> r = ldq<QP>(a.rq, v);
      if (!v.valid) zero(r);
      auto put = [&](int j, double x) {
        x = wave_sum(x);
        if (lane == 0) lds[wid * LD + j] = x;
      };
      for (int l = 0; l < k; ++l) {
        const Spinor<double> cl = ldq_nt<QP>(a.q[l], v);
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const cplx<double> x = cl.c[i][c];
            re += x.re * ck.c[i][c].re + x.im * ck.c[i][c].im;
            im += x.re * ck.c[i][c].im - x.im * ck.c[i][c].re;
          }
        put(2 * l, re);
        put(2 * l + 1, im);
      }
      double n2 = 0.0, cre = 0.0, cim = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cplx<double> x = ck.c[i][c];
          n2 += x.re * x.re + x.im * x.im;
          cre += x.re * r.c[i][c].re + x.im * r.c[i][c].im;
          cim += x.re * r.c[i][c].im - x.im * r.c[i][c].re;
        }
      put(2 * k, n2);
      put(2 * k + 1, cre);
      put(2 * k + 2, cim);
      __syncthreads();
      for (int j = threadIdx.x; j < 2 * k + 3; j += WG) {
        double t = 0.0;
        for (int w = 0; w < WG / 64; ++w) t += lds[w * LD + j];
        a.partials[(size_t)v.part * a.pw + j] = t;
      }
      __syncthreads();
      continue;
    }
    const double ib = 1.0 / S.bk[k];
    const cplx<double> mc = {-S.ck[k].x, -S.ck[k].y};
    double vals[1] = {0.0};
    if (v.valid) {
      Spinor<double> r = ldq<QP>(a.rq, v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) ck.c[i][c] = ib * ck.c[i][c];
      round_to<QP>(ck);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(r.c[i][c], mc, ck.c[i][c]);
      round_to<QP>(r);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) vals[0] += r.c[i][c].re * r.c[i][c].re + r.c[i][c].im * r.c[i][c].im;
      stq<QP>(a.q[k], v, ck);
      stq<QP>(a.rq, v, r);
      if (a.fuse_sap) store_sap_input<P>(a, v, r);
    }
    put_partial<1>(a, v, vals, lds);
    __syncthreads();
  }
}

// Second Gram-Schmidt pass of the flagged systems: chi_k <- (chi_k' - sum_l a2_l chi_l) / b_k
// (chi_k' from w), stored in QP; r <- r - c_k chi_k as stored; partial |r|^2.  Other
// systems were finished by k_gs_update.
template <int P, int QP>
__global__ __launch_bounds__(WG) void k_gs_update2(VecLaunch a) {
  __shared__ double lds[(WG / 64)];
  if (cycle_dead(a.dead)) return;
  const int k = a.k;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys]) continue;
    const SysState& S = a.sys[v.sys];
    if (!S.reorth) continue;
    Spinor<double> ck = ldq<QP>(a.w, v);
    for (int l = 0; l < k; ++l) {
      const cplx<double> m = {-S.a2[l].x, -S.a2[l].y};
      Spinor<double> cl = ldq_nt<QP>(a.q[l], v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(ck.c[i][c], m, cl.c[i][c]);
    }
    const double ib = 1.0 / S.bk[k];
    const cplx<double> mc = {-S.ck[k].x, -S.ck[k].y};
    double vals[1] = {0.0};
    if (v.valid) {
      Spinor<double> r = ldq<QP>(a.rq, v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) ck.c[i][c] = ib * ck.c[i][c];
      round_to<QP>(ck);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(r.c[i][c], mc, ck.c[i][c]);
      round_to<QP>(r);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) vals[0] += r.c[i][c].re * r.c[i][c].re + r.c[i][c].im * r.c[i][c].im;
      stq<QP>(a.q[k], v, ck);
      stq<QP>(a.rq, v, r);
      if (a.fuse_sap) store_sap_input<P>(a, v, r);
    }
    put_partial<1>(a, v, vals, lds);
    __syncthreads();
  }
}

// x += sum_{l < k_done} alpha_l phi_l
__global__ __launch_bounds__(WG) void k_x_update(VecLaunch a) {
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    const SysState& S = a.sys[v.sys];
    if (S.converged || !v.valid) continue;
    Spinor<double> x = ld64(a.x, v);
    for (int l = 0; l < S.k_done; ++l) {
      const cplx<double> al = {S.alpha[l].x, S.alpha[l].y};
      Spinor<double> p = ld64(a.phi[l], v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(x.c[i][c], al, p.c[i][c]);
    }
    st64(a.x, v, x);
  }
}

// x += sum_{l < k_done} alpha_l phi_l with phi_l the preconditioner's output in its storage
template <int P>
__global__ __launch_bounds__(WG) void k_x_update_dir(VecLaunch a) {
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    const SysState& S = a.sys[v.sys];
    if (S.converged || !v.valid) continue;
    Spinor<double> x = ld64(a.x, v);
    for (int l = 0; l < S.k_done; ++l) {
      const cplx<double> al = {S.alpha[l].x, S.alpha[l].y};
      const FieldRef f{(char*)a.dir[l] + v.off * spinor_site_bytes(P), a.dir_sc[l] ? a.dir_sc[l] + v.off : nullptr,
                       v.V};
      // the direction as FP64 D used it: stored value times site scale, formed in double
      const auto p = SpinorIO<P>::load_raw(f, v.s);
      const double sc = double(SpinorIO<P>::scale(f, v.s));
      const cplx<double> as = {al.re * sc, al.im * sc};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(x.c[i][c], as, cplx<double>{double(p.c[i][c].re), double(p.c[i][c].im)});
    }
    st64(a.x, v, x);
  }
}

__global__ __launch_bounds__(WG) void k_norm2(VecLaunch a, const double2* f) {
  __shared__ double lds[(WG / 64)];
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    double vals[1] = {0.0};
    if (v.valid) {
      Spinor<double> p = ld64(f, v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) vals[0] += p.c[i][c].re * p.c[i][c].re + p.c[i][c].im * p.c[i][c].im;
    }
    put_partial<1>(a, v, vals, lds);
    __syncthreads();
  }
}

__global__ __launch_bounds__(WG) void k_copy(VecLaunch a, double2* dst, const double2* src) {
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (!v.valid) continue;
    st64(dst, v, ld64(src, v));
  }
}

// x = 0 on the systems whose source is zero (|b|^2 from the preceding reduction): their
// only solution, reached before any iteration whatever initial guess was given.
__global__ __launch_bounds__(WG) void k_zero_if_b0(VecLaunch a, double2* x) {
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (!v.valid || a.sys[v.sys].bnorm2 != 0.0) continue;
    Spinor<double> z;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) z.c[i][c] = {0.0, 0.0};
    st64(x, v, z);
  }
}

// ------------------------------------------------------------------ per-system reductions

// a vanishing or non-finite direction ends the system's solve with a breakdown
WC_D void gs_breakdown(SysState& S, int* skip, int sys, int k) {
  S.breakdown = 1;
  S.cycle_done = 1;
  S.reorth = 0;
  S.bk[k] = 1.0;
  S.ck[k] = make_double2(0.0, 0.0);
  skip[sys] = 1;
}

WC_D void reduce_sys(int op, const VecLaunch& a, const int* sys_part, const int* sys_nchunks, double* lds) {
  const int sys = blockIdx.x;
  SysState& S = a.sys[sys];
  const int nv = op == RED_GS ? 4 * a.k + 3 : (op == RED_GS2 ? 2 * a.k + 3 : 1);
  const bool global_op = (op == RED_TRUE || op == RED_BNORM || op == RED_INITR);
  if (!global_op && (a.skip[sys] != 0)) return;
  if (op == RED_GS2 && !S.reorth) return;
  if ((op == RED_TRUE || op == RED_INITR) && S.converged) return;
  if (nv == 0) return;
  sum_partials(a.partials, a.pw, sys_part[sys], sys_nchunks[sys], nv, lds);
  if (threadIdx.x != 0) return;
  const double* sum = lds;
  const int k = a.k;
  switch (op) {
    case RED_GS: {
      // a_lk, s = |chi_k|^2 - sum |a_lk|^2, c_k = (<chi_k, r> - sum conj(a_lk) <chi_l, r>) / b_k
      const double n2 = sum[4 * k];
      double b2 = n2, cre = sum[4 * k + 1], cim = sum[4 * k + 2];
      for (int l = 0; l < k; ++l) {
        const double are = sum[2 * l], aim = sum[2 * l + 1];
        const double ere = sum[2 * k + 2 * l], eim = sum[2 * k + 2 * l + 1];
        S.a[l * NKV_MAX + k] = make_double2(are, aim);
        S.e[l] = make_double2(ere, eim);
        b2 -= are * are + aim * aim;
        cre -= are * ere + aim * eim;
        cim -= are * eim - aim * ere;
      }
      S.n2_first = n2;
      S.a[k * NKV_MAX + k] = make_double2(0.0, 0.0);
      if (!(n2 > 0.0) || !isfinite(n2) || !isfinite(b2)) {
        gs_breakdown(S, a.skip, sys, k);
        break;
      }
      // one pass kept more than half of |chi_k|^2: b_k from the subtraction
      S.reorth = !(b2 > 0.5 * n2);
      if (S.reorth) {
        S.reorths += 1;
        break;
      }
      const double b = sqrt(b2);
      S.bk[k] = b;
      S.ck[k] = make_double2(cre / b, cim / b);
      break;
    }
    case RED_GS2: {
      // second pass: a_lk += a2_l, b_k^2 = |chi_k'|^2 - sum |a2_l|^2,
      // c_k = (<chi_k', r> - sum conj(a2_l) <chi_l, r>) / b_k
      if (!S.reorth) break;
      double b2 = sum[2 * k], cre = sum[2 * k + 1], cim = sum[2 * k + 2];
      for (int l = 0; l < k; ++l) {
        const double are = sum[2 * l], aim = sum[2 * l + 1];
        const double ere = S.e[l].x, eim = S.e[l].y;
        S.a2[l] = make_double2(are, aim);
        const double2 a1 = S.a[l * NKV_MAX + k];
        S.a[l * NKV_MAX + k] = make_double2(a1.x + are, a1.y + aim);
        b2 -= are * are + aim * aim;
        cre -= are * ere + aim * eim;
        cim -= are * eim - aim * ere;
      }
      const double b = sqrt(b2);
      // a direction that keeps less than 1e-14 of |chi_k| after two passes is rounding noise
      if (!(b2 > 1e-28 * S.n2_first) || !isfinite(b)) {
        gs_breakdown(S, a.skip, sys, k);
        break;
      }
      S.bk[k] = b;
      S.ck[k] = make_double2(cre / b, cim / b);
      break;
    }
    case RED_RNORM:
      S.rnorm2 = sum[0];
      S.k_done = k + 1;
      S.iters += 1;
      if (!(sum[0] > S.thr2) || !(sum[0] > S.cyc2) || S.iters >= a.maxit) {
        S.cycle_done = 1;
        a.skip[sys] = 1;
      }
      break;
    case RED_BNORM:
      S.bnorm2 = sum[0];
      S.rnorm2 = sum[0];
      S.tol2 = a.tol * a.tol * sum[0];
      S.thr2 = 0.25 * S.tol2;
      S.cyc2 = a.drop2 * sum[0];
      S.cycle_done = 0;
      S.converged = (sum[0] == 0.0);
      S.k_done = 0;
      S.iters = 0;
      S.restarts = 0;
      S.reorth = 0;
      S.reorths = 0;
      S.stall = 0;
      S.stagnated = 0;
      S.prev_true2 = sum[0];
      S.breakdown = !isfinite(sum[0]);
      if (S.breakdown) S.converged = 1;
      a.skip[sys] = S.converged;
      break;
    case RED_INITR:  // residual of a given initial guess
      S.rnorm2 = sum[0];
      S.cyc2 = a.drop2 * sum[0];
      S.prev_true2 = sum[0];
      if (!isfinite(sum[0])) S.breakdown = 1;
      S.converged = (sum[0] <= S.tol2) || S.breakdown;
      S.cycle_done = S.converged;
      a.skip[sys] = S.converged;
      break;
    case RED_TRUE: {
      S.rnorm2 = sum[0];
      S.cyc2 = a.drop2 * sum[0];
      S.restarts += 1;
      if (!isfinite(sum[0])) S.breakdown = 1;
      if (a.hist && S.restarts <= a.hist_max)
        a.hist[(size_t)sys * a.hist_max + S.restarts - 1] = S.bnorm2 > 0.0 ? sqrt(sum[0] / S.bnorm2) : 0.0;
      // stagnation: the true residual of a restart is no smaller than the previous one
      const bool done = (sum[0] <= S.tol2) || S.breakdown || S.iters >= a.maxit;
      S.stall = (S.restarts > 1 && !(sum[0] < S.prev_true2)) ? S.stall + 1 : 0;
      S.prev_true2 = sum[0];
      if (!done && a.stag > 0 && S.stall >= a.stag) S.stagnated = 1;
      S.converged = done || S.stagnated;
      S.cycle_done = S.converged;
      S.k_done = 0;
      a.skip[sys] = S.converged;
      break;
    }
  }
}

// One work-group per system.  After the residual-norm reduction of an FGCR cycle (a.dead
// set) every work-group adds whether its system has ended the cycle; the last one to arrive
// raises a.dead[0] when all have (the cycle's remaining launches then return at once) and
// clears the two counts for the next launch.
__global__ __launch_bounds__(RWG) void k_reduce(int op, VecLaunch a, const int* sys_part, const int* sys_nchunks) {
  __shared__ double lds[RWG];
  reduce_sys(op, a, sys_part, sys_nchunks, lds);
  if (op != RED_RNORM || !a.dead || threadIdx.x != 0) return;
  __threadfence();
  atomicAdd(&a.dead[2], a.skip[blockIdx.x] != 0 ? 1 : 0);
  __threadfence();
  if (atomicAdd(&a.dead[1], 1) == (int)gridDim.x - 1) {
    const int ended = atomicAdd(&a.dead[2], 0);
    atomicExch(&a.dead[2], 0);
    atomicExch(&a.dead[1], 0);
    atomicExch(&a.dead[0], ended == (int)gridDim.x ? 1 : 0);
  }
}

// alpha from the upper-triangular system b_k alpha_k + sum_{l>k} a_kl alpha_l = c_k
__global__ void k_backsub(VecLaunch a, int nsys) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= nsys) return;
  SysState& S = a.sys[sys];
  if (S.converged) return;
  const int n = S.k_done;
  for (int k = n - 1; k >= 0; --k) {
    double re = S.ck[k].x, im = S.ck[k].y;
    for (int l = k + 1; l < n; ++l) {
      const double2 akl = S.a[k * NKV_MAX + l], al = S.alpha[l];
      re -= akl.x * al.x - akl.y * al.y;
      im -= akl.x * al.y + akl.y * al.x;
    }
    S.alpha[k] = make_double2(re / S.bk[k], im / S.bk[k]);
  }
}

// ------------------------------------------------------------------ launchers

template <class F> static void launch_vec(F kern, const VecLaunch& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), 0, st, a);
}

template <int QP> static void to_sap_q(int prec, const VecLaunch& a, int grid, hipStream_t st) {
  switch (prec) {
    case P_F64: launch_vec(k_to_sap<P_F64, QP>, a, grid, st); break;
    case P_F32: launch_vec(k_to_sap<P_F32, QP>, a, grid, st); break;
    case P_F16: launch_vec(k_to_sap<P_F16, QP>, a, grid, st); break;
    default: launch_vec(k_to_sap<P_BF16, QP>, a, grid, st); break;
  }
}
void launch_to_sap(int prec, int basis_prec, const VecLaunch& a, int grid, hipStream_t st) {
  if (basis_prec == P_F32)
    to_sap_q<P_F32>(prec, a, grid, st);
  else
    to_sap_q<P_F64>(prec, a, grid, st);
}
void launch_gs_dots(int basis_prec, const VecLaunch& a, int grid, hipStream_t st) {
  if (basis_prec == P_F32)
    launch_vec(k_gs_dots<P_F32>, a, grid, st);
  else
    launch_vec(k_gs_dots<P_F64>, a, grid, st);
}
template <int QP> static void gs_update_q(int sap_prec, const VecLaunch& a, int grid, hipStream_t st) {
  switch (sap_prec) {
    case P_F64: launch_vec(k_gs_update<P_F64, QP>, a, grid, st); break;
    case P_F32: launch_vec(k_gs_update<P_F32, QP>, a, grid, st); break;
    case P_F16: launch_vec(k_gs_update<P_F16, QP>, a, grid, st); break;
    default: launch_vec(k_gs_update<P_BF16, QP>, a, grid, st); break;
  }
}
template <int QP> static void gs_update2_q(int sap_prec, const VecLaunch& a, int grid, hipStream_t st) {
  switch (sap_prec) {
    case P_F64: launch_vec(k_gs_update2<P_F64, QP>, a, grid, st); break;
    case P_F32: launch_vec(k_gs_update2<P_F32, QP>, a, grid, st); break;
    case P_F16: launch_vec(k_gs_update2<P_F16, QP>, a, grid, st); break;
    default: launch_vec(k_gs_update2<P_BF16, QP>, a, grid, st); break;
  }
}
void launch_gs_update(int sap_prec, int basis_prec, const VecLaunch& a, int grid, hipStream_t st) {
  if (basis_prec == P_F32)
    gs_update_q<P_F32>(sap_prec, a, grid, st);
  else
    gs_update_q<P_F64>(sap_prec, a, grid, st);
}
void launch_gs_update2(int sap_prec, int basis_prec, const VecLaunch& a, int grid, hipStream_t st) {
  if (basis_prec == P_F32)
    gs_update2_q<P_F32>(sap_prec, a, grid, st);
  else
    gs_update2_q<P_F64>(sap_prec, a, grid, st);
}
void launch_x_update(const VecLaunch& a, int grid, hipStream_t st) { launch_vec(k_x_update, a, grid, st); }
void launch_x_update_dir(const VecLaunch& a, int grid, hipStream_t st) {
  switch (a.dir_prec) {
    case P_F64: launch_vec(k_x_update_dir<P_F64>, a, grid, st); break;
    case P_F32: launch_vec(k_x_update_dir<P_F32>, a, grid, st); break;
    case P_F16: launch_vec(k_x_update_dir<P_F16>, a, grid, st); break;
    default: launch_vec(k_x_update_dir<P_BF16>, a, grid, st); break;
  }
}
void launch_norm2(const VecLaunch& a, const double2* v, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(grid), dim3(WG), 0, st, a, v);
}
void launch_copy_f64(const VecLaunch& a, double2* dst, const double2* src, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(WG), 0, st, a, dst, src);
}
void launch_zero_if_b0(const VecLaunch& a, double2* x, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_if_b0, dim3(grid), dim3(WG), 0, st, a, x);
}
void launch_reduce(int op, const VecLaunch& a, int nsys, const int* sys_part, const int* sys_nchunks,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(nsys), dim3(RWG), 0, st, op, a, sys_part, sys_nchunks);
}
void launch_backsub(const VecLaunch& a, int nsys, hipStream_t st) {
  hipLaunchKernelGGL(k_backsub, dim3((nsys + 63) / 64), dim3(64), 0, st, a, nsys);
}

}  // namespace wc
