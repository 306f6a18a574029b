// Gauge-link derivative of Re<Y, D X> and the pseudofermion force.
//
// The solves of arXiv:1109.4279 feed the HMC force from the fermion determinant
// (Sec. 1).  For S = phi^dag (D^dag D)^-1 phi, Y = D^-dag phi and X = D^-1 Y,
// dS = -2 Re<Y, dD X>.  This file computes, per link, the matrix K_mu(x) with
//   d Re<Y, D X> = Re tr(dU_mu(x) K_mu(x))        for any complex dU,
// from two parts:
//   hopping: K += -1/2 ph sum_t [ X(x+mu)_t ((1-g_mu) Y(x))_t^dag + ((1+g_mu) Y(x+mu))_t X(x)_t^dag ]
//   clover : with Xi_{rs}(y) = (i c_sw/16)(G + G^dag), G_{rs}(y) = sum_{st} (sigma_rs)_{st} X_t(y) Y_s(y)^dag,
//            every plaquette leaf W1 W2 W3 W4 at y that contains the link at position i adds
//            W_{i+1}..W_4 Xi(y) W_1..W_{i-1} (or its dagger when the leaf runs the link backwards).
// Work runs in the canonical lexicographic layout: one lane per link, gathering the
// leaves that contain it, so that no two lanes write the same output.
#include "wc_kernels.h"

namespace wc {

typedef cplx<double> zc;
struct Mat { zc m[3][3]; };

WC_D Mat mz() {
  Mat a;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a.m[i][j] = {0.0, 0.0};
  return a;
}
WC_D Mat mmul(const Mat& a, const Mat& b) {
  Mat c;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      zc t = a.m[i][0] * b.m[0][j];
      cmac(t, a.m[i][1], b.m[1][j]);
      cmac(t, a.m[i][2], b.m[2][j]);
      c.m[i][j] = t;
    }
  return c;
}
WC_D Mat mdag(const Mat& a) {
  Mat c;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c.m[i][j] = conj(a.m[j][i]);
  return c;
}

struct Lat {
  int L[4];
  int V;
  int bc_t;
};

WC_D int lex(const Lat& g, const int* x) {
  int y[4];
  for (int m = 0; m < 4; ++m) {
    int v = x[m] % g.L[m];
    y[m] = v < 0 ? v + g.L[m] : v;
  }
  return ((y[0] * g.L[1] + y[1]) * g.L[2] + y[2]) * g.L[3] + y[3];
}
WC_D void coords(const Lat& g, int s, int* x) {
  x[3] = s % g.L[3]; s /= g.L[3];
  x[2] = s % g.L[2]; s /= g.L[2];
  x[1] = s % g.L[1]; s /= g.L[1];
  x[0] = s;
}
WC_D Mat link(const double2* U, const Lat& g, int mu, int s) {
  Mat a;
  const double2* p = U + ((size_t)mu * g.V + s) * 9;
  for (int k = 0; k < 9; ++k) a.m[k / 3][k % 3] = {p[k].x, p[k].y};
  return a;
}
WC_D void spin(const double2* F, const Lat& g, int r, int s, zc (*v)[3]) {
  const double2* p = F + ((size_t)r * g.V + s) * 12;
  for (int k = 0; k < 12; ++k) v[k / 3][k % 3] = {p[k].x, p[k].y};
}

// (sigma_{rs})_{st} in the chiral basis: sigma_{0k} = diag(sigma_k, -sigma_k),
// sigma_{jk} = -eps_{jkl} diag(sigma_l, sigma_l)
WC_D void sigma_munu(int r, int s, zc (*sg)[4]) {
  const zc Z = {0, 0}, O = {1, 0}, I = {0, 1};
  zc pauli[3][2][2] = {{{Z, O}, {O, Z}}, {{Z, -I}, {I, Z}}, {{O, Z}, {Z, -O}}};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) sg[i][j] = Z;
  int l;
  double up, lo;
  if (r == 0) {
    l = s - 1;
    up = 1.0;
    lo = -1.0;
  } else {
    // (j,k) with j<k among 1..3: (1,2)->l=3 (eps=+1), (1,3)->l=2 (eps=-1), (2,3)->l=1 (eps=+1)
    int j = r, k = s;
    l = 6 - j - k;
    double eps = (j == 1 && k == 3) ? -1.0 : 1.0;
    up = lo = -eps;
    l = l - 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      sg[i][j] = up * pauli[l][i][j];
      sg[2 + i][2 + j] = lo * pauli[l][i][j];
    }
}

constexpr int PLANE_R[6] = {0, 0, 0, 1, 1, 2};
constexpr int PLANE_S[6] = {1, 2, 3, 2, 3, 3};

// pass 1: Xi_{rs}(y) for the six planes, summed over right-hand sides
__global__ __launch_bounds__(WG) void k_force_xi(Lat g, const double2* Y, const double2* X, int nrhs, double csw,
                                                 double2* xi) {
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= g.V) return;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    zc sg[4][4];
    sigma_munu(PLANE_R[p], PLANE_S[p], sg);
    Mat G = mz();
    for (int r = 0; r < nrhs; ++r) {
      zc x[4][3], y[4][3];
      spin(X, g, r, s, x);
      spin(Y, g, r, s, y);
#pragma unroll
      for (int si = 0; si < 4; ++si)
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) {
          if (sg[si][ti].re == 0.0 && sg[si][ti].im == 0.0) continue;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              zc t = sg[si][ti] * x[ti][a];
              cmac(G.m[a][b], t, conj(y[si][b]));
            }
        }
    }
    double2* o = xi + ((size_t)p * g.V + s) * 9;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        zc h = G.m[a][b] + conj(G.m[b][a]);
        zc v = (csw / 16.0) * timesI(h);
        o[a * 3 + b] = make_double2(v.re, v.im);
      }
  }
}

// the four leaves at y in the (r, s) plane, oriented r -> s, as (axis: 0 = r, 1 = s; step);
// compile-time tables, so that the unrolled loops below index every array with constants
// and the arrays stay in registers
constexpr int LEAF_AX[4][4] = {{0, 1, 0, 1}, {1, 0, 1, 0}, {0, 1, 0, 1}, {1, 0, 1, 0}};
constexpr int LEAF_SG[4][4] = {{1, 1, -1, -1}, {1, -1, -1, 1}, {-1, -1, 1, 1}, {-1, 1, 1, -1}};

// pass 2: K_mu(x) (hopping + clover), then the requested output
__global__ __launch_bounds__(WG) void k_force_link(Lat g, const double2* U, const double2* Y, const double2* X,
                                                   int nrhs, double csw, const double2* xi, double coef,
                                                   int out_kind, double2* out) {
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= g.V) return;
  int x[4];
  coords(g, s, x);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Mat K = mz();
    int xp[4] = {x[0], x[1], x[2], x[3]};
    xp[mu] += 1;
    const int sp = lex(g, xp);
    const double ph = (mu == 0 && x[0] == g.L[0] - 1) ? double(g.bc_t) : 1.0;
    // hopping part
    for (int r = 0; r < nrhs; ++r) {
      zc Xs[4][3], Xp[4][3], Ys[4][3], Yp[4][3];
      spin(X, g, r, s, Xs);
      spin(X, g, r, sp, Xp);
      spin(Y, g, r, s, Ys);
      spin(Y, g, r, sp, Yp);
      // (1 - g_mu) Y(x) and (1 + g_mu) Y(x + mu) in the chiral basis
      zc Pm[4][3], Pp[4][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        zc u0 = Ys[0][a], u1 = Ys[1][a], l0 = Ys[2][a], l1 = Ys[3][a];
        zc v0 = Yp[0][a], v1 = Yp[1][a], w0 = Yp[2][a], w1 = Yp[3][a];
        // gamma_mu psi: g0 (u,l) = (-l,-u); g1 = (-i s1 l, i s1 u); g2 = (-i s2 l, i s2 u); g3 = (-i s3 l, i s3 u)
        zc gm[4], gp[4];
        auto gam = [&](zc a0, zc a1, zc b0, zc b1, zc* o) {
          if (mu == 0) { o[0] = -b0; o[1] = -b1; o[2] = -a0; o[3] = -a1; }
          else if (mu == 1) { o[0] = timesMinusI(b1); o[1] = timesMinusI(b0); o[2] = timesI(a1); o[3] = timesI(a0); }
          else if (mu == 2) { o[0] = -b1; o[1] = b0; o[2] = a1; o[3] = -a0; }
          else { o[0] = timesMinusI(b0); o[1] = timesI(b1); o[2] = timesI(a0); o[3] = timesMinusI(a1); }
        };
        gam(u0, u1, l0, l1, gm);
        gam(v0, v1, w0, w1, gp);
        zc ys[4] = {u0, u1, l0, l1}, yp[4] = {v0, v1, w0, w1};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          Pm[t][a] = ys[t] - gm[t];
          Pp[t][a] = yp[t] + gp[t];
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          zc acc = {0.0, 0.0};
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            cmac(acc, Xp[t][a], conj(Pm[t][b]));
            cmac(acc, Pp[t][a], conj(Xs[t][b]));
          }
          K.m[a][b] = K.m[a][b] + (-0.5 * ph) * acc;
        }
    }
    // clover part: the planes that contain mu, every leaf position holding U_mu(x)
    if (csw != 0.0) {
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int pr = PLANE_R[p], ps = PLANE_S[p];
        if (pr != mu && ps != mu) continue;
        const int ax_mu = (pr == mu) ? 0 : 1;
#pragma unroll
        for (int lf = 0; lf < 4; ++lf) {
          // offsets of each step's link from the leaf origin y
          int off[4][4], pos[4] = {0, 0, 0, 0}, dir[4];
          bool dg[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int d = LEAF_AX[lf][j] == 0 ? pr : ps;
            dir[j] = d;
            if (LEAF_SG[lf][j] > 0) {
#pragma unroll
              for (int m = 0; m < 4; ++m) off[j][m] = pos[m];
              pos[d] += 1;
              dg[j] = false;
            } else {
              pos[d] -= 1;
#pragma unroll
              for (int m = 0; m < 4; ++m) off[j][m] = pos[m];
              dg[j] = true;
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (LEAF_AX[lf][i] != ax_mu) continue;
            int y[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) y[m] = x[m] - off[i][m];
            Mat W[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              int z[4];
#pragma unroll
              for (int m = 0; m < 4; ++m) z[m] = y[m] + off[j][m];
              Mat l = link(U, g, dir[j], lex(g, z));
              W[j] = dg[j] ? mdag(l) : l;
            }
            Mat Xi;
            const double2* xp2 = xi + ((size_t)p * g.V + lex(g, y)) * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k) Xi.m[k / 3][k % 3] = {xp2[k].x, xp2[k].y};
            Mat R;
            bool have = false;
#pragma unroll
            for (int j = i + 1; j < 4; ++j) { R = have ? mmul(R, W[j]) : W[j]; have = true; }
            R = have ? mmul(R, Xi) : Xi;
#pragma unroll
            for (int j = 0; j < i; ++j) R = mmul(R, W[j]);
            if (dg[i]) R = mdag(R);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int b = 0; b < 3; ++b) K.m[a][b] = K.m[a][b] + R.m[a][b];
          }
        }
      }
    }
    double2* o = out + ((size_t)mu * g.V + s) * 9;
    if (out_kind == 0) {  // torch-convention gradient G = coef * K^dag
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          zc v = coef * conj(K.m[b][a]);
          o[a * 3 + b] = make_double2(v.re, v.im);
        }
    } else {  // Lie-algebra force TA(U K) * coef
      Mat UK = mmul(link(U, g, mu, s), K);
      Mat A;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) A.m[a][b] = 0.5 * (UK.m[a][b] - conj(UK.m[b][a]));
      zc tr = A.m[0][0] + A.m[1][1] + A.m[2][2];
#pragma unroll
      for (int a = 0; a < 3; ++a) A.m[a][a] = A.m[a][a] - (1.0 / 3.0) * tr;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          zc v = coef * A.m[a][b];
          o[a * 3 + b] = make_double2(v.re, v.im);
        }
    }
  }
}

void launch_force(const int* L, int bc_t, const void* Ucanon, const void* Y, const void* X, int nrhs, double csw,
                  double coef, int out_kind, void* xi_work, void* out, hipStream_t st) {
  Lat g;
  for (int m = 0; m < 4; ++m) g.L[m] = L[m];
  g.V = L[0] * L[1] * L[2] * L[3];
  g.bc_t = bc_t;
  dim3 grid((g.V + WG - 1) / WG);
  if (csw != 0.0)
    hipLaunchKernelGGL(k_force_xi, grid, dim3(WG), 0, st, g, (const double2*)Y, (const double2*)X, nrhs, csw,
                       (double2*)xi_work);
  hipLaunchKernelGGL(k_force_link, grid, dim3(WG), 0, st, g, (const double2*)Ucanon, (const double2*)Y,
                     (const double2*)X, nrhs, csw, (const double2*)xi_work, coef, out_kind, (double2*)out);
}

}  // namespace wc
