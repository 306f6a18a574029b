// FP64 kernels of the FGMRES-DR outer solver (arXiv:1109.4279, Sec. 4): the flexible
// Arnoldi step (z_j = M(v_j), w = D z_j, classical Gram-Schmidt of w against v_0..v_j
// applied twice, v_{j+1} = w / h_{j+1,j}), the least-squares residual estimate by Givens
// rotations on the device, and the in-place recombination of the bases V and Z at a
// deflated restart.  The basis is carried from cycle to cycle (V <- V P), so its loss of
// orthogonality would accumulate over restarts; the second Gram-Schmidt pass keeps V
// orthonormal to working precision.
//
// The cycle's matrix Hbar lives in device memory (ArnState) so that a whole cycle runs as
// one captured graph; the host reads Hbar at the restart, solves the small dense problems
// (least squares, harmonic Ritz pairs, deflation basis P) and writes back P and the new
// cycle's Hbar, rotations and residual coefficients.
#include "wc_vec.h"

namespace wc {

// V_0 = r / |r|  (the start of a cycle without deflation)
__global__ __launch_bounds__(WG) void k_arn_init(VecLaunch a) {
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys] || !v.valid) continue;
    const double inv = 1.0 / sqrt(a.sys[v.sys].rnorm2);
    Spinor<double> r = ld64(a.r, v);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) r.c[i][c] = inv * r.c[i][c];
    st64(a.chi[0], v, r);
  }
}

// eta(P) = V_j (a unit vector: no scaling) ; Z_j = psi(P)
template <int P>
__global__ __launch_bounds__(WG) void k_arn_to_sap(VecLaunch a) {
  typedef typename Real<P>::T R;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys] || !v.valid) continue;
    const Spinor<double> p = ld64(a.chi[a.k], v);
    Spinor<R> o;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) o.c[i][c] = {R(p.c[i][c].re), R(p.c[i][c].im)};
    SpinorIO<P>::store(FieldRef{(char*)a.sp + v.off * spinor_site_bytes(P), a.sp_sc ? a.sp_sc + v.off : nullptr, v.V},
                       v.s, o);
  }
}

template <int P>
__global__ __launch_bounds__(WG) void k_arn_from_sap(VecLaunch a) {
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys] || !v.valid) continue;
    const auto p = SpinorIO<P>::load(
        FieldRef{(char*)a.sp + v.off * spinor_site_bytes(P), a.sp_sc ? a.sp_sc + v.off : nullptr, v.V}, v.s);
    Spinor<double> o;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) o.c[i][c] = {double(p.c[i][c].re), double(p.c[i][c].im)};
    st64(a.phi[a.k], v, o);
  }
}

// Partials of h_i = <V_i, w> (i <= j) and |w|^2 for w = V_{j+1} (which holds D z_j).
// Layout per chunk: [2 (j+1) reals of h][|w|^2].
__global__ __launch_bounds__(WG) void k_arn_dots(VecLaunch a) {
  constexpr int LD = 2 * ARN_LD + 2;
  __shared__ double lds[(WG / 64) * LD];
  const int j = a.k;
  const int nv = 2 * (j + 1) + 1;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys]) continue;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Spinor<double> w = ld64(a.chi[j + 1], v);
    if (!v.valid) zero(w);
    auto put = [&](int idx, double x) {
      x = wave_sum(x);
      if (lane == 0) lds[wid * LD + idx] = x;
    };
    for (int i = 0; i <= j; ++i) {
      const Spinor<double> q = ld64(a.chi[i], v);
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cplx<double> x = q.c[s][c], y = w.c[s][c];
          re += x.re * y.re + x.im * y.im;
          im += x.re * y.im - x.im * y.re;
        }
      put(2 * i, v.valid ? re : 0.0);
      put(2 * i + 1, v.valid ? im : 0.0);
    }
    double n2 = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) n2 += w.c[s][c].re * w.c[s][c].re + w.c[s][c].im * w.c[s][c].im;
    put(2 * (j + 1), n2);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nv; idx += WG) {
      double t = 0.0;
      for (int q = 0; q < WG / 64; ++q) t += lds[q * LD + idx];
      a.partials[(size_t)v.part * a.pw + idx] = t;
    }
    __syncthreads();
  }
}

// First pass of the update: w <- w - sum_{i <= j} h1_i V_i, fused with the partials of the
// second pass (<V_i, w>, |w|^2 of the updated w; layout as k_arn_dots).
__global__ __launch_bounds__(WG) void k_arn_update1(VecLaunch a) {
  constexpr int LD = 2 * ARN_LD + 2;
  __shared__ double lds[(WG / 64) * LD];
  const int j = a.k;
  const int nv = 2 * (j + 1) + 1;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.skip[v.sys]) continue;
    const ArnState& A = a.arn[v.sys];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Spinor<double> w = ld64(a.chi[j + 1], v);
    for (int i = 0; i <= j; ++i) {
      const cplx<double> m = {-A.h1[i].x, -A.h1[i].y};
      const Spinor<double> q = ld64(a.chi[i], v);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(w.c[s][c], m, q.c[s][c]);
    }
    if (v.valid)
      st64(a.chi[j + 1], v, w);
    else
      zero(w);
    auto put = [&](int idx, double x) {
      x = wave_sum(x);
      if (lane == 0) lds[wid * LD + idx] = x;
    };
    for (int i = 0; i <= j; ++i) {
      const Spinor<double> q = ld64(a.chi[i], v);
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cplx<double> x = q.c[s][c], y = w.c[s][c];
          re += x.re * y.re + x.im * y.im;
          im += x.re * y.im - x.im * y.re;
        }
      put(2 * i, re);
      put(2 * i + 1, im);
    }
    double n2 = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) n2 += w.c[s][c].re * w.c[s][c].re + w.c[s][c].im * w.c[s][c].im;
    put(2 * (j + 1), n2);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nv; idx += WG) {
      double t = 0.0;
      for (int q = 0; q < WG / 64; ++q) t += lds[q * LD + idx];
      a.partials[(size_t)v.part * a.pw + idx] = t;
    }
    __syncthreads();
  }
}

// One work-group per system: add the partials in a fixed order, then (thread 0) form column
// j of Hbar.  Pass 1 keeps the first coefficients h1 and |w|^2.  Pass 2: column j = h1 + h2,
// h_{j+1,j} = (|w|^2 - sum |h2_i|^2)^(1/2) for the once-orthogonalised w (the V_i
// orthonormal), the column rotated by the stored Givens rotations, the rotation that
// removes h_{j+1,j}, and the residual estimate |g[j+1]|.  The cycle ends at m columns, at
// the tolerance, at maxit or on a breakdown.
__global__ __launch_bounds__(RWG) void k_arn_reduce(int pass, VecLaunch a, const int* sys_part, const int* sys_nchunks,
                                                    int m) {
  __shared__ double lds[RWG];
  // the stored rotations and the new column, for the serial work of thread 0
  __shared__ double rot_c[ARN_ROT_MAX];
  __shared__ double2 rot_s[ARN_ROT_MAX];
  __shared__ int rot_p[ARN_ROT_MAX];
  __shared__ double2 cc[ARN_LD];
  const int sys = blockIdx.x;
  if (a.skip[sys]) return;
  SysState& S = a.sys[sys];
  ArnState& A = a.arn[sys];
  const int j = a.k;
  const int nv = 2 * (j + 1) + 1;
  sum_partials(a.partials, a.pw, sys_part[sys], sys_nchunks[sys], nv, lds);
  if (pass != 1) {
    for (int q = threadIdx.x; q < A.nrot; q += RWG) {
      rot_c[q] = A.rc[q];
      rot_s[q] = A.rs[q];
      rot_p[q] = A.rp[q];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double* sum = lds;
  if (pass == 1) {
    for (int i = 0; i <= j; ++i) A.h1[i] = make_double2(sum[2 * i], sum[2 * i + 1]);
    A.w2 = sum[2 * (j + 1)];
    return;
  }
  double2* col = A.H + (size_t)j * ARN_LD;
  const double w2 = A.w2;
  double hh = sum[2 * (j + 1)];
  for (int i = 0; i <= j; ++i) {
    A.h2[i] = make_double2(sum[2 * i], sum[2 * i + 1]);
    col[i] = make_double2(A.h1[i].x + sum[2 * i], A.h1[i].y + sum[2 * i + 1]);
    hh -= sum[2 * i] * sum[2 * i] + sum[2 * i + 1] * sum[2 * i + 1];
  }
  S.iters += 1;
  S.k_done = j + 1;
  if (!isfinite(w2) || !isfinite(hh)) {
    S.breakdown = 1;
    S.cycle_done = 1;
    a.skip[sys] = 1;
    return;
  }
  // an (almost) invariant subspace: the new direction is rounding noise
  const bool lucky = !(hh > 1e-24 * w2);
  const double h = lucky ? 0.0 : sqrt(hh);
  col[j + 1] = make_double2(h, 0.0);
  A.lucky = lucky;
  // rotate a copy of the new column by the stored rotations (Hbar itself stays unrotated
  // for the host's least squares), then add the rotation that removes h_{j+1,j}
  for (int i = 0; i <= j + 1; ++i) cc[i] = col[i];
  for (int q = 0; q < A.nrot; ++q) {
    const int p = rot_p[q];
    const double c = rot_c[q];
    const double2 s = rot_s[q];
    const double2 x = cc[p], y = cc[p + 1];
    // x' = c x + s y ; y' = -conj(s) x + c y
    cc[p] = make_double2(c * x.x + s.x * y.x - s.y * y.y, c * x.y + s.x * y.y + s.y * y.x);
    cc[p + 1] = make_double2(-(s.x * x.x + s.y * x.y) + c * y.x, -(s.x * x.y - s.y * x.x) + c * y.y);
  }
  const double2 a0 = cc[j], b0 = cc[j + 1];
  const double na = hypot(a0.x, a0.y), nb = hypot(b0.x, b0.y);
  double c;
  double2 s;
  if (nb == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
  } else if (na == 0.0) {
    c = 0.0;
    s = make_double2(b0.x / nb, -b0.y / nb);
  } else {
    const double rho = hypot(na, nb);
    c = na / rho;
    // s = (a / |a|) conj(b) / rho
    const double ux = a0.x / na, uy = a0.y / na;
    s = make_double2((ux * b0.x + uy * b0.y) / rho, (uy * b0.x - ux * b0.y) / rho);
  }
  const int q = A.nrot;
  A.rp[q] = j;
  A.rc[q] = c;
  A.rs[q] = s;
  A.nrot = q + 1;
  const double2 gx = A.g[j];
  A.g[j] = make_double2(c * gx.x, c * gx.y);
  // g[j+1] = -conj(s) g[j]
  A.g[j + 1] = make_double2(-(s.x * gx.x + s.y * gx.y), -(s.x * gx.y - s.y * gx.x));
  const double res2 = A.g[j + 1].x * A.g[j + 1].x + A.g[j + 1].y * A.g[j + 1].y;
  S.rnorm2 = res2;
  if (lucky || !(res2 > S.thr2) || S.iters >= a.maxit || j + 1 >= m) {
    S.cycle_done = 1;
    a.skip[sys] = 1;
  }
}

// V_{j+1} = (w - sum_{i <= j} h2_i V_i) / h_{j+1,j}  (w already once orthogonalised)
__global__ __launch_bounds__(WG) void k_arn_update(VecLaunch a) {
  const int j = a.k;
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    const ArnState& A = a.arn[v.sys];
    // skip flags are set by the reduction when this column ended the cycle; the last
    // column's basis vector is still needed (Hbar has j+2 rows), so update unless the
    // system was already idle before this column
    if (a.sys[v.sys].k_done != j + 1 || A.lucky || !v.valid || a.sys[v.sys].breakdown) continue;
    const double2* col = A.H + (size_t)j * ARN_LD;
    Spinor<double> w = ld64(a.chi[j + 1], v);
    for (int i = 0; i <= j; ++i) {
      const cplx<double> m = {-A.h2[i].x, -A.h2[i].y};
      const Spinor<double> q = ld64(a.chi[i], v);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(w.c[s][c], m, q.c[s][c]);
    }
    const double ih = 1.0 / col[j + 1].x;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) w.c[s][c] = ih * w.c[s][c];
    st64(a.chi[j + 1], v, w);
  }
}

// In-place recombination at a deflated restart: every element of the new vectors needs the
// same element of all old ones, so each thread loads its element of the old basis into
// registers before writing the new one over it.
template <int NMAX>
__global__ __launch_bounds__(WG) void k_arn_recombine(VecLaunch a, int which) {
  __shared__ double2 Ps[ARN_LD * ARN_LD];
  for (int it0 = blockIdx.x; it0 < a.nitems; it0 += gridDim.x) {
    VecSite v = vec_site(a, it0);
    if (a.sys[v.sys].converged) continue;  // uniform over the work-group
    const ArnState& A = a.arn[v.sys];
    for (int i = threadIdx.x; i < ARN_LD * ARN_LD; i += WG) Ps[i] = A.P[i];
    __syncthreads();
    const int nin = which ? A.pin - 1 : A.pin;
    const int nout = which ? A.pout - 1 : A.pout;
    double2* const* tab = which ? a.phi : a.chi;
    const long long base = v.off * 12;
    if (v.valid) {
      for (int k = 0; k < 12; ++k) {
        const size_t e = base + (size_t)k * v.V + v.s;
        double2 in[NMAX];
#pragma unroll
        for (int i = 0; i < NMAX; ++i) in[i] = i < nin ? gld_d2(tab[i], e) : make_double2(0.0, 0.0);
        for (int l = 0; l < nout; ++l) {
          double re = 0.0, im = 0.0;
#pragma unroll
          for (int i = 0; i < NMAX; ++i) {
            const double2 p = Ps[l * ARN_LD + i];
            re += p.x * in[i].x - p.y * in[i].y;
            im += p.x * in[i].y + p.y * in[i].x;
          }
          tab[l][e] = make_double2(re, im);
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launchers

template <class F> static void launch_vec(F kern, const VecLaunch& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), 0, st, a);
}

void launch_arn_init(const VecLaunch& a, int grid, hipStream_t st) { launch_vec(k_arn_init, a, grid, st); }
void launch_arn_to_sap(int prec, const VecLaunch& a, int grid, hipStream_t st) {
  switch (prec) {
    case P_F64: launch_vec(k_arn_to_sap<P_F64>, a, grid, st); break;
    case P_F32: launch_vec(k_arn_to_sap<P_F32>, a, grid, st); break;
    case P_F16: launch_vec(k_arn_to_sap<P_F16>, a, grid, st); break;
    default: launch_vec(k_arn_to_sap<P_BF16>, a, grid, st); break;
  }
}
void launch_arn_from_sap(int prec, const VecLaunch& a, int grid, hipStream_t st) {
  switch (prec) {
    case P_F64: launch_vec(k_arn_from_sap<P_F64>, a, grid, st); break;
    case P_F32: launch_vec(k_arn_from_sap<P_F32>, a, grid, st); break;
    case P_F16: launch_vec(k_arn_from_sap<P_F16>, a, grid, st); break;
    default: launch_vec(k_arn_from_sap<P_BF16>, a, grid, st); break;
  }
}
void launch_arn_dots(const VecLaunch& a, int grid, hipStream_t st) { launch_vec(k_arn_dots, a, grid, st); }
void launch_arn_reduce(int pass, const VecLaunch& a, int nsys, const int* sys_part, const int* sys_nchunks, int m,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_arn_reduce, dim3(nsys), dim3(RWG), 0, st, pass, a, sys_part, sys_nchunks, m);
}
void launch_arn_update1(const VecLaunch& a, int grid, hipStream_t st) { launch_vec(k_arn_update1, a, grid, st); }
void launch_arn_update(const VecLaunch& a, int grid, hipStream_t st) { launch_vec(k_arn_update, a, grid, st); }
void launch_arn_recombine(const VecLaunch& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_arn_recombine<ARN_LD>, dim3(grid), dim3(WG), 0, st, a, 0);
  hipLaunchKernelGGL(k_arn_recombine<ARN_LD>, dim3(grid), dim3(WG), 0, st, a, 1);
}

}  // namespace wc
