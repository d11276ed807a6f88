// Sparse-sampling grids on the intermediate-representation (IR) basis (Sec. 5.1: the tau and
// Matsubara grids of the paper's calculations are IR grids).
//
// The basis is the singular value expansion K(x, y) = sum_l s_l u_l(x) v_l(y) of the logistic
// kernel K(x, y) = exp(-L y (x + 1)/2) / (1 + exp(-L y)), x = 2 tau/beta - 1, y = omega/wmax,
// L = beta wmax; its tau functions serve fermionic and bosonic quantities alike.  The kernel is
// discretised with composite Gauss-Legendre rules on panels that halve towards x = -1, 1 and
// towards y = 0 down to a width of about 1/L, and the singular vectors of
// sqrt(w_x) K sqrt(w_y) (one-sided Jacobi rotations, which orthogonalise the columns) give
// u_l at the nodes; inside a panel u_l is the Legendre series through its nodes.  Functions
// with s_l > eps s_0 are kept (L of them) and one more, u_L, whose zeros are the tau sampling
// points; the tau grid is 0, those points and beta.  The Matsubara sampling points are the
// n >= 0 at which hat u_L(i nu_n) changes sign (the bosonic n = 0 always), computed separately
// for the two statistics; both lists are filled to a common length nw with 2 nw - 1 >= L,
// each added index in the widest gap of its list.  The transforms fit the tau samples with u_0 .. u_{L-1} (least squares) and
// evaluate the Fourier integrals of the basis at the sampled frequencies; the inverse is the
// least-squares fit of the sampled frequencies and their negatives, as for the Chebyshev grid.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "internal.hpp"

namespace gw {

namespace {

constexpr int IR_ORDER = 16;   // Gauss-Legendre nodes per panel

std::vector<double> ir_breaks(double lam, bool toward_ends) {
  const int k = int(std::ceil(std::log2(lam))) + 2;
  std::vector<double> b = {-1.0, 0.0, 1.0};
  for (int j = 1; j < k; ++j) {
    const double h = std::ldexp(1.0, -j);
    b.push_back(toward_ends ? 1.0 - h : h);
    b.push_back(toward_ends ? -(1.0 - h) : -h);
  }
  std::sort(b.begin(), b.end());
  b.erase(std::unique(b.begin(), b.end()), b.end());
  return b;
}

double logistic(double lam, double x, double y) {
  const double e = y >= 0 ? -lam * y * (x + 1) / 2 : lam * y * (1 - x) / 2;
  return std::exp(e) / (1.0 + std::exp(-lam * std::fabs(y)));
}

// Legendre polynomials P_0..P_{n-1} at t
void legendre(int n, double t, double* p) {
  p[0] = 1.0;
  if (n > 1) p[1] = t;
  for (int k = 2; k < n; ++k) p[k] = ((2 * k - 1) * t * p[k - 1] - (k - 1) * p[k - 2]) / k;
}

// One-sided Jacobi: the columns of A (m x n, column-major as cols[c][r]) are rotated pairwise
// until orthogonal; returns the column norms (singular values) and leaves the normalised
// columns (left singular vectors) in place, sorted by decreasing norm.
void jacobi_columns(std::vector<std::vector<double>>& cols, std::vector<double>& s) {
  const int n = int(cols.size()), m = int(cols[0].size());
  for (int sweep = 0; sweep < 60; ++sweep) {
    double worst = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0, b = 0, c = 0;
        const double* cp = cols[p].data();
        const double* cq = cols[q].data();
        for (int r = 0; r < m; ++r) {
          a += cp[r] * cp[r];
          b += cq[r] * cq[r];
          c += cp[r] * cq[r];
        }
        if (a == 0.0 || b == 0.0) continue;
        const double rel = std::fabs(c) / std::sqrt(a * b);
        if (rel <= 1e-16) continue;
        worst = std::max(worst, rel);
        const double z = (b - a) / (2.0 * c);
        const double t = (z >= 0 ? 1.0 : -1.0) / (std::fabs(z) + std::sqrt(1.0 + z * z));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        double* xp = cols[p].data();
        double* xq = cols[q].data();
        for (int r = 0; r < m; ++r) {
          const double u = xp[r], v = xq[r];
          xp[r] = cs * u - sn * v;
          xq[r] = sn * u + cs * v;
        }
      }
    if (worst < 1e-15) break;
  }
  s.resize(n);
  for (int c = 0; c < n; ++c) {
    double nn = 0;
    for (double v : cols[c]) nn += v * v;
    s[c] = std::sqrt(nn);
  }
  std::vector<int> o(n);
  for (int i = 0; i < n; ++i) o[i] = i;
  std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return s[a] > s[b]; });
  std::vector<std::vector<double>> sorted(n);
  std::vector<double> ss(n);
  for (int i = 0; i < n; ++i) {
    sorted[i] = std::move(cols[o[i]]);
    ss[i] = s[o[i]];
    if (ss[i] > 0)
      for (double& v : sorted[i]) v /= ss[i];
  }
  cols = std::move(sorted);
  s = std::move(ss);
}

struct IrBasis {
  std::vector<double> xb;                 // panel breaks
  int L = 0;                              // functions kept; u_L is one more
  std::vector<double> coef;               // [panel][degree][l], l = 0..L
  double eval(int l, double x) const {
    const int np = int(xb.size()) - 1;
    int p = int(std::upper_bound(xb.begin(), xb.end(), x) - xb.begin()) - 1;
    p = std::min(std::max(p, 0), np - 1);
    const double t = (2 * x - xb[p] - xb[p + 1]) / (xb[p + 1] - xb[p]);
    double P[IR_ORDER];
    legendre(IR_ORDER, t, P);
    double v = 0;
    for (int d = 0; d < IR_ORDER; ++d) v += coef[(size_t(p) * IR_ORDER + d) * (L + 1) + l] * P[d];
    return v;
  }
};

IrBasis ir_basis(double lam, double eps) {
  IrBasis B;
  B.xb = ir_breaks(lam, true);
  const std::vector<double> yb = ir_breaks(lam, false);
  std::vector<double> xg, wg;
  gauss_legendre(IR_ORDER, xg, wg);
  auto nodes = [&](const std::vector<double>& br, std::vector<double>& x, std::vector<double>& w) {
    for (size_t p = 0; p + 1 < br.size(); ++p) {
      const double h = 0.5 * (br[p + 1] - br[p]), m = 0.5 * (br[p + 1] + br[p]);
      for (int i = 0; i < IR_ORDER; ++i) {
        x.push_back(m + h * xg[i]);
        w.push_back(h * wg[i]);
      }
    }
  };
  std::vector<double> x, wx, y, wy;
  nodes(B.xb, x, wx);
  nodes(yb, y, wy);
  const int m = int(x.size()), n = int(y.size());
  std::vector<std::vector<double>> cols(n, std::vector<double>(m));
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < m; ++r) cols[c][r] = std::sqrt(wx[r]) * logistic(lam, x[r], y[c]) * std::sqrt(wy[c]);
  std::vector<double> s;
  jacobi_columns(cols, s);
  int L = 0;
  while (L < n && s[L] > eps * s[0]) ++L;
  if (L + 1 > std::min(m, n)) throw std::runtime_error("IR basis: eps below the discretisation");
  B.L = L;
  const int np = int(B.xb.size()) - 1;
  B.coef.assign(size_t(np) * IR_ORDER * (L + 1), 0.0);
  std::vector<double> P(IR_ORDER);
  for (int l = 0; l <= L; ++l)
    for (int p = 0; p < np; ++p)
      for (int i = 0; i < IR_ORDER; ++i) {
        const int r = p * IR_ORDER + i;
        const double u = cols[l][r] / std::sqrt(wx[r]);
        legendre(IR_ORDER, xg[i], P.data());
        for (int d = 0; d < IR_ORDER; ++d)
          B.coef[(size_t(p) * IR_ORDER + d) * (L + 1) + l] += (2 * d + 1) / 2.0 * wg[i] * P[d] * u;
      }
  // sign: u_l(1) > 0
  for (int l = 0; l <= L; ++l)
    if (B.eval(l, 1.0) < 0)
      for (int p = 0; p < np; ++p)
        for (int d = 0; d < IR_ORDER; ++d) B.coef[(size_t(p) * IR_ORDER + d) * (L + 1) + l] *= -1.0;
  return B;
}

// zeros of u_l on (-1, 1): sign changes on 64 points per panel, then bisection
std::vector<double> ir_roots(const IrBasis& B, int l) {
  std::vector<double> xs;
  for (size_t p = 0; p + 1 < B.xb.size(); ++p)
    for (int i = 0; i < 64; ++i) xs.push_back(B.xb[p] + (B.xb[p + 1] - B.xb[p]) * i / 64.0);
  xs.push_back(1.0);
  std::vector<double> f(xs.size());
  for (size_t i = 0; i < xs.size(); ++i) f[i] = B.eval(l, xs[i]);
  std::vector<double> out;
  for (size_t i = 0; i + 1 < xs.size(); ++i) {
    if (!((f[i] < 0 && f[i + 1] > 0) || (f[i] > 0 && f[i + 1] < 0))) continue;
    double lo = xs[i], hi = xs[i + 1], flo = f[i];
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (lo + hi), fm = B.eval(l, mid);
      if ((fm < 0) == (flo < 0)) {
        lo = mid;
        flo = fm;
      } else {
        hi = mid;
      }
    }
    out.push_back(0.5 * (lo + hi));
  }
  return out;
}

// hat u_l(i nu) = int_0^beta sqrt(2/beta) u_l(2 tau/beta - 1) exp(i nu tau) d tau for l < nl and
// every nu, by Gauss-Legendre rules on sub-panels short enough that the phase nu tau turns by
// at most about 4 radians across each
CMat ir_fourier(const IrBasis& B, double beta, const std::vector<double>& nu, int nl) {
  double numax = 0;
  for (double v : nu) numax = std::max(numax, std::fabs(v));
  std::vector<double> xg, wg;
  gauss_legendre(2 * IR_ORDER, xg, wg);
  CMat F(int(nu.size()), nl);
  for (size_t p = 0; p + 1 < B.xb.size(); ++p) {
    const double a = B.xb[p], b = B.xb[p + 1];
    const int sub = std::max(1, int(std::ceil(numax * beta * (b - a) / 2.0 / 4.0)));
    for (int s = 0; s < sub; ++s) {
      const double sa = a + (b - a) * s / sub, sb = a + (b - a) * (s + 1) / sub;
      const double h = 0.5 * (sb - sa), m = 0.5 * (sb + sa);
      for (size_t i = 0; i < xg.size(); ++i) {
        const double x = m + h * xg[i], tau = beta * (x + 1) / 2, w = h * wg[i] * beta / 2 * std::sqrt(2.0 / beta);
        std::vector<double> u(nl);
        for (int l = 0; l < nl; ++l) u[l] = B.eval(l, x);
        for (size_t k = 0; k < nu.size(); ++k) {
          const cplx e = std::polar(w, nu[k] * tau);
          for (int l = 0; l < nl; ++l) F(int(k), l) += e * u[l];
        }
      }
    }
  }
  return F;
}

std::vector<int> sign_changes(const IrBasis& B, double beta, bool boson, int nmax) {
  std::vector<double> nu(nmax);
  for (int n = 0; n < nmax; ++n) nu[n] = (2.0 * n + (boson ? 0 : 1)) * M_PI / beta;
  const CMat F = ir_fourier(B, beta, nu, B.L + 1);
  double mre = 0, mim = 0;
  for (int n = 0; n < nmax; ++n) {
    mre = std::max(mre, std::fabs(F(n, B.L).real()));
    mim = std::max(mim, std::fabs(F(n, B.L).imag()));
  }
  auto part = [&](int n) { return mre > mim ? F(n, B.L).real() : F(n, B.L).imag(); };
  std::vector<int> out;
  if (boson) out.push_back(0);
  for (int n = 0; n + 1 < nmax; ++n) {
    const double a = part(n), b = part(n + 1);
    if ((a < 0 && b > 0) || (a > 0 && b < 0))
      if (!(boson && n == 0)) out.push_back(n);
  }
  return out;
}

}  // namespace

void build_ir_grids(Ctx& c) {
  const double beta = c.prm.beta, lam = beta * c.prm.ir_wmax;
  const IrBasis B = ir_basis(lam, c.prm.ir_eps);
  const int L = B.L;
  std::vector<double> r = ir_roots(B, L);
  const int nr = int(r.size());
  if (nr != L) throw std::runtime_error("IR basis: u_L has " + std::to_string(nr) + " zeros, expected " + std::to_string(L));
  std::vector<double> rs(nr);
  for (int i = 0; i < nr; ++i) rs[i] = 0.5 * (r[i] - r[nr - 1 - i]);   // exact mirror symmetry
  c.tau.assign(1, 0.0);
  for (double x : rs) c.tau.push_back(beta * (x + 1) / 2);
  c.tau.push_back(beta);
  const int nt = int(c.tau.size());
  const int nmax = int(4.0 * lam / M_PI) + 64;
  std::vector<int> nf = sign_changes(B, beta, false, nmax), nb = sign_changes(B, beta, true, nmax);
  // both lists hold nw entries, enough that the bosonic stacked system (n = 0 once) has at
  // least L rows
  const size_t nw = std::max({nf.size(), nb.size(), size_t((L + 2) / 2)});
  // filled where the list is sparsest: between the neighbours with the largest ratio
  // (n_{i+1} + 1) / (n_i + 1), at the integer geometric mean of n + 1 (minus one)
  for (auto* v : {&nf, &nb})
    while (v->size() < nw) {
      size_t best = 0;
      for (size_t i = 1; i + 1 < v->size(); ++i)
        if (double((*v)[i + 1] + 1) / ((*v)[i] + 1) > double((*v)[best + 1] + 1) / ((*v)[best] + 1)) best = i;
      const int m = int(std::lround(std::sqrt(double((*v)[best] + 1) * ((*v)[best + 1] + 1)))) - 1;
      if (m <= (*v)[best] || m >= (*v)[best + 1]) v->push_back(v->back() + 1);
      else v->insert(v->begin() + best + 1, m);
    }
  c.ntau = nt;
  c.nw = int(nw);
  c.nfreq_f = nf;
  c.nfreq_b = nb;
  // tau samples of u_0 .. u_{L-1} and the least-squares fit from them
  CMat Ut(nt, L);
  for (int j = 0; j < nt; ++j)
    for (int l = 0; l < L; ++l) Ut(j, l) = std::sqrt(2.0 / beta) * B.eval(l, 2 * c.tau[j] / beta - 1);
  CMat fit;
  if (!lstsq(Ut, CMat::eye(nt), fit)) throw std::runtime_error("IR grid: tau sampling matrix without full rank");
  for (int boson = 0; boson < 2; ++boson) {
    const std::vector<int>& ns = boson ? nb : nf;
    std::vector<double> nu(nw);
    for (size_t n = 0; n < nw; ++n) nu[n] = (2.0 * ns[n] + (boson ? 0 : 1)) * M_PI / beta;
    const CMat Fm = ir_fourier(B, beta, nu, L);
    const CMat Tfwd = matmul(Fm, fit);    // nw x nt
    // inverse: least squares on [Fm; conj rows]; the bosonic n = 0 row is not repeated
    std::vector<int> conj_rows;
    for (size_t n = 0; n < nw; ++n)
      if (!(boson && ns[n] == 0)) conj_rows.push_back(int(n));
    const int nrow = int(nw + conj_rows.size());
    CMat S(nrow, L);
    for (size_t n = 0; n < nw; ++n)
      for (int l = 0; l < L; ++l) S(int(n), l) = Fm(int(n), l);
    for (size_t q = 0; q < conj_rows.size(); ++q)
      for (int l = 0; l < L; ++l) S(int(nw + q), l) = std::conj(Fm(conj_rows[q], l));
    CMat Pinv;
    if (!lstsq(S, CMat::eye(nrow), Pinv))   // L x nrow
      throw std::runtime_error("IR grid: " + std::to_string(nrow) + " frequency rows for " + std::to_string(L) +
                               " basis functions");
    std::vector<cplx> Bm(size_t(nt) * nw), Tv(Tfwd.a.begin(), Tfwd.a.end());
    for (int j = 0; j < nt; ++j)
      for (size_t n = 0; n < nw; ++n) {
        cplx s = 0;
        for (int l = 0; l < L; ++l) s += Ut(j, l) * Pinv(l, int(n));
        if (boson && ns[n] == 0) s *= 0.5;
        Bm[size_t(j) * nw + n] = s;
      }
    if (boson) {
      c.Tb = Tv;
      c.Bb = Bm;
    } else {
      c.Tf = Tv;
      c.Bf = Bm;
    }
  }
}

}  // namespace gw
