// Eigenvalues and right eigenvectors of a small dense complex matrix (host).
//
// Used for the projected (subspace) matrix of the EOM-EE Davidson solver,
// n of order 10-200.  Householder reduction to upper Hessenberg form, complex
// QR iteration with Wilkinson shifts (Givens rotations, deflation on small
// subdiagonals) to the Schur form T = Q^H A Q, then eigenvectors of T by
// back substitution, mapped back with Q.  Textbook algorithms (Golub and
// Van Loan, "Matrix Computations", ch. 7); plain C++, no device code.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace eigsmall {

typedef std::complex<double> zc;

// A: n x n row-major (overwritten by nothing; copied).  On return w[k] are the
// eigenvalues and V (n x n row-major) holds the unit-norm eigenvector of w[k]
// in column k.  Returns false if the QR iteration did not converge.
inline bool eig(int n, const std::vector<zc>& A, std::vector<zc>& w, std::vector<zc>& V) {
  std::vector<zc> H(A), Q((size_t)n * n, 0.0);
  auto h = [&](int i, int j) -> zc& { return H[(size_t)i * n + j]; };
  auto q = [&](int i, int j) -> zc& { return Q[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i) q(i, i) = 1.0;
  // ---- Householder reduction to Hessenberg form: H <- P H P, Q <- Q P
  std::vector<zc> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(h(i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const zc x0 = h(k + 1, k);
    const zc ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : zc(1.0);
    const zc alpha = -ph * xn;
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = h(i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // H <- (I - 2 v v^H) H
    for (int j = 0; j < n; ++j) {
      zc s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * h(i, j);
      for (int i = k + 1; i < n; ++i) h(i, j) -= 2.0 * v[i] * s;
    }
    // H <- H (I - 2 v v^H), Q <- Q (I - 2 v v^H)
    for (int i = 0; i < n; ++i) {
      zc s = 0.0, t = 0.0;
      for (int j = k + 1; j < n; ++j) s += h(i, j) * v[j], t += q(i, j) * v[j];
      for (int j = k + 1; j < n; ++j) h(i, j) -= 2.0 * s * std::conj(v[j]), q(i, j) -= 2.0 * t * std::conj(v[j]);
    }
    for (int i = k + 2; i < n; ++i) h(i, k) = 0.0;
  }
  // ---- shifted QR on the Hessenberg matrix
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double s = std::abs(h(l - 1, l - 1)) + std::abs(h(l, l));
      if (std::abs(h(l, l - 1)) <= eps * (s > 0.0 ? s : 1.0)) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {  // one eigenvalue converged
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) return false;
    ++iter;
    // Wilkinson shift from the trailing 2x2 block of the active window
    const zc a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    const zc tr = a + d, det = a * d - b * c;
    const zc disc = std::sqrt(tr * tr * 0.25 - det);
    zc mu1 = tr * 0.5 + disc, mu2 = tr * 0.5 - disc;
    zc mu = std::abs(mu1 - d) < std::abs(mu2 - d) ? mu1 : mu2;
    if (iter % 11 == 10) mu = d + zc(std::abs(h(hi, hi - 1)), 0.0);  // exceptional shift
    // QR step on rows/columns l..hi of H - mu I with Givens rotations
    std::vector<zc> cs(hi - l), sn(hi - l);
    for (int k = l; k <= hi; ++k) h(k, k) -= mu;
    for (int k = l; k < hi; ++k) {
      const zc x = h(k, k), y = h(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      zc cc = 1.0, ss = 0.0;
      if (r > 0.0) cc = x / r, ss = y / r;
      cs[k - l] = cc, sn[k - l] = ss;
      // rows k, k+1 <- G^H rows  (G = [[cc, -conj(ss)], [ss, conj(cc)]])
      for (int j = k; j < n; ++j) {
        const zc u = h(k, j), t = h(k + 1, j);
        h(k, j) = std::conj(cc) * u + std::conj(ss) * t;
        h(k + 1, j) = -ss * u + cc * t;
      }
    }
    for (int k = l; k < hi; ++k) {
      const zc cc = cs[k - l], ss = sn[k - l];
      const int imax = std::min(hi, k + 2);
      for (int i = 0; i <= imax; ++i) {
        const zc u = h(i, k), t = h(i, k + 1);
        h(i, k) = u * cc + t * ss;
        h(i, k + 1) = -u * std::conj(ss) + t * std::conj(cc);
      }
      for (int i = 0; i < n; ++i) {
        const zc u = q(i, k), t = q(i, k + 1);
        q(i, k) = u * cc + t * ss;
        q(i, k + 1) = -u * std::conj(ss) + t * std::conj(cc);
      }
    }
    for (int k = l; k <= hi; ++k) h(k, k) += mu;
  }
  // ---- eigenvectors of the triangular T by back substitution
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) w[k] = h(k, k);
  std::vector<zc> Z((size_t)n * n, 0.0);
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) tnorm = std::max(tnorm, std::abs(h(i, j)));
  const double small = eps * (tnorm > 0.0 ? tnorm : 1.0);
  for (int k = 0; k < n; ++k) {
    Z[(size_t)k * n + k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      zc s = 0.0;
      for (int m = j + 1; m <= k; ++m) s += h(j, m) * Z[(size_t)m * n + k];
      zc den = h(j, j) - w[k];
      if (std::abs(den) < small) den = small;
      Z[(size_t)j * n + k] = -s / den;
    }
  }
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      zc s = 0.0;
      for (int m = 0; m <= k; ++m) s += q(i, m) * Z[(size_t)m * n + k];
      V[(size_t)i * n + k] = s;
    }
  for (int k = 0; k < n; ++k) {
    double nr = 0.0;
    for (int i = 0; i < n; ++i) nr += std::norm(V[(size_t)i * n + k]);
    nr = std::sqrt(nr);
    if (nr > 0.0)
      for (int i = 0; i < n; ++i) V[(size_t)i * n + k] /= nr;
  }
  return true;
}

}  // namespace eigsmall
