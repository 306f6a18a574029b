// Small dense complex linear algebra on the host (FP64) for the deflated restarts of
// FGMRES-DR; see dense_host.h.  Textbook algorithms: Givens QR, Householder reduction
// to Hessenberg form, the shifted QR iteration (Wilkinson shift) for the complex Schur
// form, triangular back-substitution for the eigenvectors.
#include "dense_host.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace wc {
namespace dense {

Rot make_rot(cd a, cd b, int p) {
  Rot g;
  g.p = p;
  const double na = std::abs(a), nb = std::abs(b);
  if (nb == 0.0) {
    g.c = 1.0;
    g.s = 0.0;
  } else if (na == 0.0) {
    g.c = 0.0;
    g.s = std::conj(b) / nb;
  } else {
    const double rho = std::hypot(na, nb);
    g.c = na / rho;
    g.s = (a / na) * std::conj(b) / rho;
  }
  return g;
}

void givens_qr(int rows, int cols, cd* H, int ld, cd* g, std::vector<Rot>& rots) {
  for (int l = 0; l < cols; ++l) {
    for (int i = rows - 1; i > l; --i) {
      cd& top = H[(i - 1) + l * ld];
      cd& bot = H[i + l * ld];
      if (bot == cd(0.0)) continue;
      const Rot r = make_rot(top, bot, i - 1);
      for (int j = l; j < cols; ++j) apply_rot(r, H[(i - 1) + j * ld], H[i + j * ld]);
      bot = 0.0;
      if (g) apply_rot(r, g[i - 1], g[i]);
      rots.push_back(r);
    }
  }
}

bool lstsq(int rows, int cols, const cd* H, int ld, const cd* c, cd* d) {
  std::vector<cd> R(H, H + (size_t)ld * cols), g(c, c + rows);
  std::vector<Rot> rots;
  givens_qr(rows, cols, R.data(), ld, g.data(), rots);
  for (int i = cols - 1; i >= 0; --i) {
    cd t = g[i];
    for (int j = i + 1; j < cols; ++j) t -= R[i + j * ld] * d[j];
    const cd piv = R[i + i * ld];
    if (std::abs(piv) == 0.0) return false;
    d[i] = t / piv;
  }
  return true;
}

namespace {

// A = Q H Q^H with H upper Hessenberg (in place in A), Q accumulated into Z (n x n)
void hessenberg(int n, cd* A, int lda, cd* Z, int ldz) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Z[i + j * ldz] = (i == j) ? 1.0 : 0.0;
  std::vector<cd> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double nx = 0.0;
    for (int i = k + 1; i < n; ++i) nx += std::norm(A[i + k * lda]);
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const cd x0 = A[(k + 1) + k * lda];
    const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0);
    const cd alpha = -ph * nx;
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = A[i + k * lda];
    v[k + 1] -= alpha;
    double nv = 0.0;
    for (int i = k + 1; i < n; ++i) nv += std::norm(v[i]);
    nv = std::sqrt(nv);
    if (nv == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= nv;
    // A <- (1 - 2 v v^H) A (1 - 2 v v^H);  Z <- Z (1 - 2 v v^H)
    for (int j = 0; j < n; ++j) {
      cd t = 0.0;
      for (int i = k + 1; i < n; ++i) t += std::conj(v[i]) * A[i + j * lda];
      for (int i = k + 1; i < n; ++i) A[i + j * lda] -= 2.0 * v[i] * t;
    }
    for (int i = 0; i < n; ++i) {
      cd t = 0.0;
      for (int j = k + 1; j < n; ++j) t += A[i + j * lda] * v[j];
      for (int j = k + 1; j < n; ++j) A[i + j * lda] -= 2.0 * t * std::conj(v[j]);
    }
    for (int i = 0; i < n; ++i) {
      cd t = 0.0;
      for (int j = k + 1; j < n; ++j) t += Z[i + j * ldz] * v[j];
      for (int j = k + 1; j < n; ++j) Z[i + j * ldz] -= 2.0 * t * std::conj(v[j]);
    }
    for (int i = k + 2; i < n; ++i) A[i + k * lda] = 0.0;
  }
}

// eigenvalue of the 2x2 block [a b; c d] closest to d
cd wilkinson(cd a, cd b, cd c, cd d) {
  const cd tr = a + d, det = a * d - b * c;
  const cd disc = std::sqrt(tr * tr / 4.0 - det);
  const cd l1 = tr / 2.0 + disc, l2 = tr / 2.0 - disc;
  return std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
}

}  // namespace

bool eig(int n, const cd* Ain, int lda, cd* w, cd* V, int ldv) {
  std::vector<cd> T((size_t)n * n), Z((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) T[i + j * n] = Ain[i + j * lda];
  double anorm = 0.0;
  for (const cd& x : T) anorm = std::max(anorm, std::abs(x));
  if (anorm == 0.0) anorm = 1.0;
  hessenberg(n, T.data(), n, Z.data(), n);
  const double eps = 2.2e-16;
  int hi = n - 1, iter = 0, total = 0;
  std::vector<Rot> rs;
  while (hi > 0) {
    // deflate at a negligible subdiagonal entry
    int lo = hi;
    while (lo > 0) {
      const double s = std::abs(T[(lo - 1) + (lo - 1) * n]) + std::abs(T[lo + lo * n]);
      if (std::abs(T[lo + (lo - 1) * n]) <= eps * (s > 0.0 ? s : anorm)) {
        T[lo + (lo - 1) * n] = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 60 * n) return false;
    ++iter;
    cd mu = wilkinson(T[(hi - 1) + (hi - 1) * n], T[(hi - 1) + hi * n], T[hi + (hi - 1) * n], T[hi + hi * n]);
    if (iter % 11 == 10) mu = T[hi + hi * n] + std::abs(T[hi + (hi - 1) * n]);  // exceptional shift
    // one explicit shifted QR step on the active window [lo, hi]
    for (int i = lo; i <= hi; ++i) T[i + i * n] -= mu;
    rs.clear();
    for (int i = lo; i < hi; ++i) {
      const Rot r = make_rot(T[i + i * n], T[(i + 1) + i * n], i);
      for (int j = i; j < n; ++j) apply_rot(r, T[i + j * n], T[(i + 1) + j * n]);
      T[(i + 1) + i * n] = 0.0;
      rs.push_back(r);
    }
    for (const Rot& r : rs) {
      // columns (p, p+1) times the rotation's conjugate transpose, rows 0..min(p+2, hi)
      const int p = r.p, top = std::min(p + 2, hi);
      for (int i = 0; i <= top; ++i) {
        cd& x = T[i + p * n];
        cd& y = T[i + (p + 1) * n];
        const cd a = x, b = y;
        x = r.c * a + std::conj(r.s) * b;
        y = -r.s * a + r.c * b;
      }
      for (int i = 0; i < n; ++i) {
        cd& x = Z[i + p * n];
        cd& y = Z[i + (p + 1) * n];
        const cd a = x, b = y;
        x = r.c * a + std::conj(r.s) * b;
        y = -r.s * a + r.c * b;
      }
    }
    for (int i = lo; i <= hi; ++i) T[i + i * n] += mu;
  }
  for (int i = 0; i < n; ++i) w[i] = T[i + i * n];
  // eigenvectors of the triangular T, then back to the original basis
  std::vector<cd> y(n);
  for (int k = 0; k < n; ++k) {
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    y[k] = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      cd t = 0.0;
      for (int l = i + 1; l <= k; ++l) t += T[i + l * n] * y[l];
      cd den = T[i + i * n] - w[k];
      if (std::abs(den) < eps * anorm) den = eps * anorm;
      y[i] = -t / den;
    }
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
      cd t = 0.0;
      for (int l = 0; l <= k; ++l) t += Z[i + l * n] * y[l];
      V[i + k * ldv] = t;
      nrm += std::norm(t);
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) V[i + k * ldv] /= nrm;
  }
  return true;
}

bool harmonic_ritz(int m, const cd* Hbar, int ld, cd* theta, cd* G, int ldg) {
  // f = H^-H e_m by Gaussian elimination with partial pivoting on H^H
  std::vector<cd> A((size_t)m * m), f(m, cd(0.0));
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) A[i + j * m] = std::conj(Hbar[j + i * ld]);
  f[m - 1] = 1.0;
  for (int k = 0; k < m; ++k) {
    int piv = k;
    for (int i = k + 1; i < m; ++i)
      if (std::abs(A[i + k * m]) > std::abs(A[piv + k * m])) piv = i;
    if (std::abs(A[piv + k * m]) == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < m; ++j) std::swap(A[k + j * m], A[piv + j * m]);
      std::swap(f[k], f[piv]);
    }
    for (int i = k + 1; i < m; ++i) {
      const cd l = A[i + k * m] / A[k + k * m];
      for (int j = k; j < m; ++j) A[i + j * m] -= l * A[k + j * m];
      f[i] -= l * f[k];
    }
  }
  for (int i = m - 1; i >= 0; --i) {
    cd t = f[i];
    for (int j = i + 1; j < m; ++j) t -= A[i + j * m] * f[j];
    f[i] = t / A[i + i * m];
  }
  const double h2 = std::norm(Hbar[m + (m - 1) * ld]);
  std::vector<cd> Hh((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Hh[i + j * m] = Hbar[i + j * ld];
  for (int i = 0; i < m; ++i) Hh[i + (m - 1) * m] += h2 * f[i];
  std::vector<cd> w(m), Vv((size_t)m * m);
  if (!eig(m, Hh.data(), m, w.data(), Vv.data(), m)) return false;
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::abs(w[a]) < std::abs(w[b]); });
  for (int k = 0; k < m; ++k) {
    theta[k] = w[order[k]];
    for (int i = 0; i < m; ++i) G[i + k * ldg] = Vv[i + order[k] * m];
  }
  return true;
}

bool orthonormalise(int len, int n, cd* Q, int ld) {
  for (int j = 0; j < n; ++j) {
    cd* q = Q + (size_t)j * ld;
    double n0 = 0.0;
    for (int i = 0; i < len; ++i) n0 += std::norm(q[i]);
    for (int l = 0; l < j; ++l) {
      const cd* p = Q + (size_t)l * ld;
      cd t = 0.0;
      for (int i = 0; i < len; ++i) t += std::conj(p[i]) * q[i];
      for (int i = 0; i < len; ++i) q[i] -= t * p[i];
    }
    double nq = 0.0;
    for (int i = 0; i < len; ++i) nq += std::norm(q[i]);
    if (!(nq > 1e-28 * n0) || nq == 0.0) return false;
    nq = std::sqrt(nq);
    for (int i = 0; i < len; ++i) q[i] /= nq;
  }
  return true;
}

}  // namespace dense
}  // namespace wc
