// Small dense complex linear algebra on the host, FP64, for the restarts of FGMRES-DR
// (arXiv:1109.4279, Sec. 4): least squares with the Hessenberg-like matrix of a cycle,
// harmonic Ritz pairs, Gram-Schmidt of the deflation basis.  Matrices are column-major,
// element (i, j) at a[i + j * ld].  Sizes are at most a few dozen.
#pragma once

#include <complex>
#include <vector>

namespace wc {
namespace dense {

typedef std::complex<double> cd;

// Givens rotation on rows (p, p+1): [c s; -conj(s) c] [a; b] = [r; 0], c real.
struct Rot {
  double c;
  cd s;
  int p;
};
Rot make_rot(cd a, cd b, int p);
inline void apply_rot(const Rot& g, cd& a, cd& b) {
  const cd x = a, y = b;
  a = g.c * x + g.s * y;
  b = -std::conj(g.s) * x + g.c * y;
}

// Triangularise the rows x cols matrix H (rows >= cols) in place by Givens rotations,
// column by column from the bottom up, appending them to `rots`; the same rotations are
// applied to the vector g (length rows).  Afterwards |g[cols..rows)| is the least-squares
// residual norm and H's top cols x cols block is upper triangular.
void givens_qr(int rows, int cols, cd* H, int ld, cd* g, std::vector<Rot>& rots);

// d = argmin |c - H d| for the rows x cols matrix H (rows >= cols).  Returns false if the
// triangular factor is singular.
bool lstsq(int rows, int cols, const cd* H, int ld, const cd* c, cd* d);

// Eigenvalues w and unit eigenvectors (columns of V) of the general n x n matrix A:
// Householder reduction to Hessenberg form, shifted QR iteration to the complex Schur
// form, back-substitution on the triangular factor.  Returns false if the iteration did
// not converge.
bool eig(int n, const cd* A, int lda, cd* w, cd* V, int ldv);

// Harmonic Ritz pairs of an Arnoldi cycle from its (m+1) x m matrix Hbar: eigenpairs of
// H + |h_{m+1,m}|^2 H^-H e_m e_m^T, H the top m x m block, sorted by increasing |theta|.
bool harmonic_ritz(int m, const cd* Hbar, int ld, cd* theta, cd* G, int ldg);

// Modified Gram-Schmidt: the n columns of length len of Q (leading dimension ld) are
// orthonormalised in place, in order.  Returns false on a (numerically) dependent column.
bool orthonormalise(int len, int n, cd* Q, int ld);

}  // namespace dense
}  // namespace wc
