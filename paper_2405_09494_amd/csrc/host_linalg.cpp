// Small dense host linear algebra for the symmetry setup and the transform matrices:
// complex Jacobi eigen-decomposition, Householder least squares, Gauss-Legendre nodes and
// real spherical harmonics.  Sizes here are at most a few hundred.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.hpp"

namespace gw {

CMat matmul(const CMat& A, const CMat& B) {
  CMat C(A.rows, B.cols);
  for (int i = 0; i < A.rows; ++i)
    for (int k = 0; k < A.cols; ++k) {
      const cplx a = A(i, k);
      if (a == cplx(0.0)) continue;
      const cplx* b = &B.a[size_t(k) * B.cols];
      cplx* c = &C.a[size_t(i) * C.cols];
      for (int j = 0; j < B.cols; ++j) c[j] += a * b[j];
    }
  return C;
}

CMat adjoint(const CMat& A) {
  CMat B(A.cols, A.rows);
  for (int i = 0; i < A.rows; ++i)
    for (int j = 0; j < A.cols; ++j) B(j, i) = std::conj(A(i, j));
  return B;
}

// Cyclic Jacobi for a Hermitian matrix.  Each rotation first removes the phase of the
// pivot A_pq with diag(1, e^{-i phi}), then applies the real rotation that zeroes it.
bool herm_eig(const CMat& H, std::vector<double>& w, CMat& V, int max_sweeps) {
  const int n = H.rows;
  CMat A = H;
  V = CMat::eye(n);
  double total = 0;
  for (auto& x : A.a) total += std::norm(x);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(A(p, q));
    if (off <= 1e-34 * std::max(total, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cplx b = A(p, q);
        const double ab = std::abs(b);
        if (ab < 1e-300) continue;
        const cplx ph = b / ab;  // e^{i phi}
        const double a = A(p, p).real(), d = A(q, q).real();
        const double th = (d - a) / (2.0 * ab);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(1.0 + th * th));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        const cplx emp = std::conj(ph);  // e^{-i phi}
        // A <- A J, V <- V J with J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
        for (int k = 0; k < n; ++k) {
          const cplx akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * emp * akq;
          A(k, q) = s * akp + c * emp * akq;
          const cplx vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * emp * vkq;
          V(k, q) = s * vkp + c * emp * vkq;
        }
        // A <- J^H A
        for (int k = 0; k < n; ++k) {
          const cplx apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * ph * aqk;
          A(q, k) = s * apk + c * ph * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        A(p, p) = A(p, p).real();
        A(q, q) = A(q, q).real();
      }
  }
  double off = 0;
  for (int p = 0; p < n; ++p)
    for (int q = p + 1; q < n; ++q) off += std::norm(A(p, q));
  if (off > 1e-26 * std::max(total, 1e-300)) return false;
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return A(i, i).real() < A(j, j).real(); });
  w.resize(n);
  CMat Vs(n, n);
  for (int j = 0; j < n; ++j) {
    w[j] = A(idx[j], idx[j]).real();
    for (int i = 0; i < n; ++i) Vs(i, j) = V(i, idx[j]);
  }
  V = Vs;
  return true;
}

// Householder QR least squares.
bool lstsq(const CMat& Ain, const CMat& Bin, CMat& X) {
  CMat A = Ain, B = Bin;
  const int m = A.rows, n = A.cols, nr = B.cols;
  if (m < n || B.rows != m) return false;
  std::vector<cplx> v(m);
  for (int j = 0; j < n; ++j) {
    double nx = 0;
    for (int i = j; i < m; ++i) nx += std::norm(A(i, j));
    nx = std::sqrt(nx);
    if (nx == 0) return false;
    const cplx x0 = A(j, j);
    const cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1.0);
    const cplx alpha = -ph * nx;
    for (int i = j; i < m; ++i) v[i] = A(i, j);
    v[j] -= alpha;
    double nv = 0;
    for (int i = j; i < m; ++i) nv += std::norm(v[i]);
    nv = std::sqrt(nv);
    for (int i = j; i < m; ++i) v[i] /= nv;
    // apply I - 2 v v^H to A[j:, j:] and B[j:, :]
    for (int col = j; col < n; ++col) {
      cplx s = 0;
      for (int i = j; i < m; ++i) s += std::conj(v[i]) * A(i, col);
      for (int i = j; i < m; ++i) A(i, col) -= 2.0 * v[i] * s;
    }
    for (int col = 0; col < nr; ++col) {
      cplx s = 0;
      for (int i = j; i < m; ++i) s += std::conj(v[i]) * B(i, col);
      for (int i = j; i < m; ++i) B(i, col) -= 2.0 * v[i] * s;
    }
  }
  X = CMat(n, nr);
  for (int col = 0; col < nr; ++col)
    for (int i = n - 1; i >= 0; --i) {
      cplx s = B(i, col);
      for (int k = i + 1; k < n; ++k) s -= A(i, k) * X(k, col);
      X(i, col) = s / A(i, i);
    }
  return true;
}

// Newton iteration on the Legendre polynomial from the asymptotic initial guesses.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
  x.assign(n, 0.0);
  wt.assign(n, 0.0);
  const int half = (n + 1) / 2;
  for (int i = 0; i < half; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pp = 0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) {
        // one more derivative at the converged node
        p1 = 1.0; p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double p3 = p2;
          p2 = p1;
          p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1.0);
        break;
      }
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    wt[i] = wt[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Real harmonics: Y_{l,0} = N_l0 P_l(z); Y_{l,+-m} = sqrt(2) N_lm P_l^m(z) {cos, sin}(m phi),
// N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m without the Condon-Shortley phase,
// order m = -l..l.  P_l^m(z) (cos, sin)(m phi) is evaluated as Q_l^m(z) (Re, Im)(x + i y)^m.
void real_ylm(int l, const double p[3], double* out) {
  const double x = p[0], y = p[1], z = p[2];
  cplx wm(1.0, 0.0);
  for (int m = 0; m <= l; ++m) {
    double qmm = 1.0;
    for (int k = 1; k < 2 * m; k += 2) qmm *= k;
    double qprev = 0.0, q = qmm;
    for (int j = m + 1; j <= l; ++j) {
      double qn;
      if (j == m + 1) qn = z * (2 * m + 1) * q;
      else qn = ((2.0 * j - 1.0) * z * q - (j + m - 1.0) * qprev) / (j - m);
      qprev = q;
      q = qn;
    }
    double ratio = 1.0;  // (l-m)!/(l+m)!
    for (int k = l - m + 1; k <= l + m; ++k) ratio /= k;
    const double nrm = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
    if (m == 0) out[l] = nrm * q;
    else {
      out[l + m] = std::sqrt(2.0) * nrm * q * wm.real();
      out[l - m] = std::sqrt(2.0) * nrm * q * wm.imag();
    }
    wm *= cplx(x, y);
  }
}

}  // namespace gw
