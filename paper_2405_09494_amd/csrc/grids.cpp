// Imaginary-time grid and the fixed Matsubara transform matrices (Sec. 4.1:
// X(i nu_n) = int_0^beta X(tau) exp(i nu_n tau) d tau; eq. P02P for bosons).
//
// tau_j = (beta/2) (1 - cos(pi j / (ntau-1))) are Chebyshev-Gauss-Lobatto nodes.  A
// function sampled there is represented by its interpolating Chebyshev series; the
// forward transform integrates that series exactly (Gauss-Legendre quadrature), and the
// inverse is the least-squares inverse over the frequencies n >= 0 together with their
// conjugate rows X(-i nu_n) = X(i nu_n)^H, which keeps X(tau) Hermitian.
#include <cmath>

#include "internal.hpp"

namespace gw {

void build_grids(Ctx& c) {
  if (c.prm.grid == GWSYM_GRID_IR) {
    build_ir_grids(c);
    return;
  }
  const int nt = c.prm.ntau, nw = c.prm.nw, N1 = nt - 1;
  c.nfreq_f.resize(nw);
  c.nfreq_b.resize(nw);
  for (int n = 0; n < nw; ++n) c.nfreq_f[n] = c.nfreq_b[n] = n;
  const double beta = c.prm.beta;
  c.ntau = nt;
  c.nw = nw;
  c.tau.resize(nt);
  for (int j = 0; j < nt; ++j) c.tau[j] = 0.5 * beta * (1.0 - std::cos(M_PI * j / N1));
  // Vm[j][l] = T_l(x_j) with x_j = -cos(pi j / N1):  T_l(x_j) = cos(pi l (N1 - j) / N1)
  auto Tl_node = [&](int l, int j) {
    const long r = (long(l) * (N1 - j)) % (2L * N1);
    return std::cos(M_PI * double(r) / N1);
  };
  // discrete orthogonality at the Lobatto nodes gives the inverse in closed form
  std::vector<double> Vinv(size_t(nt) * nt);
  for (int l = 0; l < nt; ++l)
    for (int j = 0; j < nt; ++j) {
      const double cl = (l == 0 || l == N1) ? 2.0 : 1.0;
      const double wj = (j == 0 || j == N1) ? 0.5 : 1.0;
      Vinv[size_t(l) * nt + j] = 2.0 / (N1 * cl) * wj * Tl_node(l, j);
    }
  for (int boson = 0; boson < 2; ++boson) {
    std::vector<double> nu(nw);
    for (int n = 0; n < nw; ++n) nu[n] = (2.0 * n + (boson ? 0 : 1)) * M_PI / beta;
    const int nq = int(2.0 * (nt + nu[nw - 1] * beta / 2.0)) + 100;
    std::vector<double> xq, wq;
    gauss_legendre(nq, xq, wq);
    // Fm[n][l] = int_0^beta T_l(2 tau/beta - 1) exp(i nu_n tau) d tau
    CMat Fm(nw, nt);
    std::vector<double> T(nt);
    for (int q = 0; q < nq; ++q) {
      const double x = xq[q], tq = 0.5 * beta * (x + 1.0), wgt = 0.5 * beta * wq[q];
      T[0] = 1.0;
      if (nt > 1) T[1] = x;
      for (int l = 2; l < nt; ++l) T[l] = 2.0 * x * T[l - 1] - T[l - 2];
      for (int n = 0; n < nw; ++n) {
        const cplx e = std::polar(wgt, nu[n] * tq);
        for (int l = 0; l < nt; ++l) Fm(n, l) += e * T[l];
      }
    }
    // forward: Tfwd = Fm Vinv
    std::vector<cplx> Tfwd(size_t(nw) * nt);
    for (int n = 0; n < nw; ++n)
      for (int j = 0; j < nt; ++j) {
        cplx s = 0;
        for (int l = 0; l < nt; ++l) s += Fm(n, l) * Vinv[size_t(l) * nt + j];
        Tfwd[size_t(n) * nt + j] = s;
      }
    // inverse: least squares on [Fm; conj(Fm) rows]; the n = 0 boson row is not repeated
    const int n0 = boson ? 1 : 0;
    const int nrow = nw + (nw - n0);
    CMat S(nrow, nt);
    for (int n = 0; n < nw; ++n)
      for (int l = 0; l < nt; ++l) S(n, l) = Fm(n, l);
    for (int n = n0; n < nw; ++n)
      for (int l = 0; l < nt; ++l) S(nw + n - n0, l) = std::conj(Fm(n, l));
    CMat Pinv;
    lstsq(S, CMat::eye(nrow), Pinv);   // nt x nrow
    // B[j][n] = sum_l T_l(x_j) Pinv[l][n] for n < nw; X(tau) = Y + Y^H with Y = B X(i nu)
    std::vector<cplx> B(size_t(nt) * nw);
    for (int j = 0; j < nt; ++j)
      for (int n = 0; n < nw; ++n) {
        cplx s = 0;
        for (int l = 0; l < nt; ++l) s += Tl_node(l, j) * Pinv(l, n);
        if (boson && n == 0) s *= 0.5;
        B[size_t(j) * nw + n] = s;
      }
    if (boson) {
      c.Tb = Tfwd;
      c.Bb = B;
    } else {
      c.Tf = Tfwd;
      c.Bf = B;
    }
  }
}

}  // namespace gw
