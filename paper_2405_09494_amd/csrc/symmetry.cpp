// Alg. 1 of the paper on the host: operation tables, stars of the k mesh, the orbital
// representation O^k(alpha) (eq. basis_rot), projective representations and Dirac
// characters of the little co-groups (eq. projrep, eq. factor, eq. dirac) and the
// unitary U^k from their simultaneous diagonalisation (Sec. 3.4).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>

#include "internal.hpp"

namespace gw {

namespace {

void inv3(const double* a, double* r) {
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  r[0] = (a[4] * a[8] - a[5] * a[7]) / det;
  r[1] = (a[2] * a[7] - a[1] * a[8]) / det;
  r[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  r[3] = (a[5] * a[6] - a[3] * a[8]) / det;
  r[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  r[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  r[6] = (a[3] * a[7] - a[4] * a[6]) / det;
  r[7] = (a[1] * a[6] - a[0] * a[7]) / det;
  r[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}

void mul3(const double* a, const double* b, double* r) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      r[3 * i + j] = s;
    }
}

int mesh_index(const int m[3], int n) {
  int a = ((m[0] % n) + n) % n, b = ((m[1] % n) + n) % n, c = ((m[2] % n) + n) % n;
  return (a * n + b) * n + c;
}

void mesh_point(int k, int n, int m[3]) {
  m[0] = k / (n * n);
  m[1] = (k / n) % n;
  m[2] = k % n;
}

// D^l(R) with Y_m(R^{-1} r) = sum_m' Y_m'(r) D[m', m], fitted at points of a Fibonacci
// sphere (the fit is exact: the rotated harmonics lie in the span of the originals).
CMat wigner_real(int l, const double* R) {
  const int d = 2 * l + 1, np = 48;
  CMat A(np, d), B(np, d);
  std::vector<double> y(d);
  const double golden = M_PI * (3.0 - std::sqrt(5.0));
  for (int s = 0; s < np; ++s) {
    const double z = 1.0 - (s + 0.5) * 2.0 / np;
    const double r = std::sqrt(1.0 - z * z);
    const double p[3] = {r * std::cos(golden * s), r * std::sin(golden * s), z};
    // R^{-1} p = R^T p for an orthogonal R
    const double q[3] = {R[0] * p[0] + R[3] * p[1] + R[6] * p[2], R[1] * p[0] + R[4] * p[1] + R[7] * p[2],
                         R[2] * p[0] + R[5] * p[1] + R[8] * p[2]};
    real_ylm(l, p, y.data());
    for (int m = 0; m < d; ++m) A(s, m) = y[m];
    real_ylm(l, q, y.data());
    for (int m = 0; m < d; ++m) B(s, m) = y[m];
  }
  CMat D;
  lstsq(A, B, D);
  for (auto& x : D.a) x = x.real();
  return D;
}

}  // namespace

// O^k(alpha): maps the Bloch orbitals at k to those at alpha k (reduced to the mesh):
// element [(x', m'), (x, m)] = exp(-i k~ . v_x^alpha) D^l[m', m] delta_{x', perm(x)}, with
// alpha r_x + v(alpha) = r_{x'} + v_x^alpha and k~ = alpha k on the mesh (eq. basis_rot).
CMat orbital_rep(const Ctx& c, bool aux, int a, int k) {
  const std::vector<int>& atom = aux ? c.aux_atom : c.ao_atom;
  const std::vector<int>& L = aux ? c.aux_l : c.ao_l;
  const int nb = aux ? c.naux : c.nao;
  const int ns = int(atom.size());
  std::vector<int> off(ns), local(ns);
  std::map<std::pair<int, int>, int> lookup;
  std::vector<int> cnt(c.natom, 0);
  int o = 0;
  for (int s = 0; s < ns; ++s) {
    off[s] = o;
    o += 2 * L[s] + 1;
    local[s] = cnt[atom[s]]++;
    lookup[{atom[s], local[s]}] = s;
  }
  int kt[3];
  mesh_point(c.kmap[size_t(a) * c.nk + k], c.n, kt);
  const auto& D = c.wigner[a];
  CMat O(nb, nb);
  for (int s = 0; s < ns; ++s) {
    const int x = atom[s];
    const int xp = c.perm[size_t(a) * c.natom + x];
    const int sp = lookup.at({xp, local[s]});
    const int* sh = &c.shift[(size_t(a) * c.natom + x) * 3];
    const double arg = -2.0 * M_PI * double(kt[0] * sh[0] + kt[1] * sh[1] + kt[2] * sh[2]) / c.n;
    const cplx ph(std::cos(arg), std::sin(arg));
    const int d = 2 * L[s] + 1;
    const CMat& Dl = D[L[s]];
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) O(off[sp] + i, off[s] + j) = ph * Dl(i, j);
  }
  return O;
}

namespace {

// Partner functions (Sec. 3.4).  On the isotypic block of an irrep of dimension d and
// multiplicity m the little group acts as I_m (x) D(alpha), so a generic Hermitian element of
// its span, A + A^H with A = sum_alpha w_alpha D(alpha), acts as I_m (x) h with h a d x d
// Hermitian matrix of d distinct eigenvalues.  Its eigenspaces are d subspaces of dimension m
// (one partner index each), and every operator that commutes with the little group, being
// X (x) I_d on the block, maps each of them into itself: the block splits into d blocks of size
// m.  A block whose eigenvalues do not fall into equal clusters is left whole.  Check: the
// group average of a fixed generic matrix is block diagonal in the split basis.
template <class Rnd>
bool partner_split(Ctx& c, const std::vector<CMat>& Dk, Rnd& rnd, CMat& U, Blocks& B) {
  const int nb = U.rows, h = int(Dk.size());
  CMat A(nb, nb);
  for (int i = 0; i < h; ++i) {
    const cplx w(rnd() - 1.0, rnd() - 1.0);
    for (size_t e = 0; e < A.a.size(); ++e) A.a[e] += w * Dk[i].a[e];
  }
  CMat H2(nb, nb);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) H2(i, j) = A(i, j) + std::conj(A(j, i));
  const CMat HB = matmul(adjoint(U), matmul(H2, U));
  Blocks out;
  CMat Un = U;
  for (size_t r = 0; r < B.size.size(); ++r) {
    const int s = B.size[r], o = B.off[r];
    CMat Hs(s, s);
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) Hs(i, j) = HB(o + i, o + j);
    std::vector<double> ev;
    CMat Vs;
    if (!herm_eig(Hs, ev, Vs)) return c.fail("Jacobi eigen-decomposition did not converge");
    double emax = 1.0;
    for (double x : ev) emax = std::max(emax, std::fabs(x));
    std::vector<int> cl{1};
    for (int j = 1; j < s; ++j) {
      if (ev[j] - ev[j - 1] > 1e-7 * emax) cl.push_back(1);
      else ++cl.back();
    }
    const bool equal = std::all_of(cl.begin(), cl.end(), [&](int x) { return x == cl[0]; });
    if (cl.size() < 2 || !equal) {
      out.size.push_back(s);
      out.off.push_back(o);
      out.lead.push_back(int(out.size.size()) - 1);
      continue;
    }
    // U_r <- U_r V, the partner subspaces one after another
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < s; ++j) {
        cplx x = 0;
        for (int q = 0; q < s; ++q) x += U(i, o + q) * Vs(q, j);
        Un(i, o + j) = x;
      }
    // align partners p > 1 to partner 1: in coordinates where the block is (multiplicity) x
    // (partner), E_p = A_p R_p with R_p unitary, and for a generic element B of the group's
    // span E_p^H B E_1 = c_p R_p^H R_1 with a scalar c_p; E_p <- E_p F_p / |c_p| makes every
    // commuting operator's partner blocks equal
    const int m = cl[0], d = int(cl.size()), lead = int(out.size.size());
    for (int p = 0; p < d; ++p) {
      out.size.push_back(m);
      out.off.push_back(o + p * m);
      out.lead.push_back(lead);
    }
    CMat Bg(nb, nb);
    for (int i = 0; i < h; ++i) {
      const cplx w(rnd() - 1.0, rnd() - 1.0);
      for (size_t e = 0; e < Bg.a.size(); ++e) Bg.a[e] += w * Dk[i].a[e];
    }
    CMat E1(nb, m);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < m; ++j) E1(i, j) = Un(i, o + j);
    const CMat BE1 = matmul(Bg, E1);
    bool aligned = true;
    std::vector<CMat> Ep(d);
    for (int p = 1; p < d && aligned; ++p) {
      CMat E(nb, m);
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < m; ++j) E(i, j) = Un(i, o + p * m + j);
      const CMat F = matmul(adjoint(E), BE1);
      const CMat FF = matmul(adjoint(F), F);
      double c2 = 0, dev = 0;
      for (int j = 0; j < m; ++j) c2 += FF(j, j).real() / m;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) dev = std::max(dev, std::abs(FF(i, j) - (i == j ? c2 : 0.0)));
      if (!(c2 > 1e-12) || dev > 1e-8 * c2) {
        aligned = false;
        break;
      }
      Ep[p] = matmul(E, F);
      for (auto& x : Ep[p].a) x /= std::sqrt(c2);
    }
    if (!aligned) {
      for (int p = 0; p < d; ++p) out.lead[lead + p] = lead + p;
      continue;
    }
    for (int p = 1; p < d; ++p)
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < m; ++j) Un(i, o + p * m + j) = Ep[p](i, j);
  }
  // group average of a fixed generic matrix: commutes with the little group
  CMat R(nb, nb), X(nb, nb);
  for (auto& x : R.a) x = cplx(rnd() - 1.0, rnd() - 1.0);
  for (int i = 0; i < h; ++i) {
    const CMat t = matmul(matmul(Dk[i], R), adjoint(Dk[i]));
    for (size_t e = 0; e < X.a.size(); ++e) X.a[e] += t.a[e];
  }
  const CMat XB = matmul(adjoint(Un), matmul(X, Un));
  std::vector<int> blk_of(nb);
  for (size_t r = 0; r < out.size.size(); ++r)
    for (int j = 0; j < out.size[r]; ++j) blk_of[out.off[r] + j] = int(r);
  double xmax = 0;
  for (const auto& x : XB.a) xmax = std::max(xmax, std::abs(x));
  for (int p = 0; p < nb; ++p)
    for (int q = 0; q < nb; ++q)
      if (blk_of[p] != blk_of[q] && std::abs(XB(p, q)) > 1e-9 * xmax)
        return c.fail("partner-function blocks do not block-diagonalise a symmetric operator");
  // and its aligned partner blocks are equal
  for (size_t r = 0; r < out.size.size(); ++r) {
    const int l = out.lead[r];
    if (l == int(r)) continue;
    for (int i = 0; i < out.size[r]; ++i)
      for (int j = 0; j < out.size[r]; ++j)
        if (std::abs(XB(out.off[r] + i, out.off[r] + j) - XB(out.off[l] + i, out.off[l] + j)) > 1e-9 * xmax)
          return c.fail("aligned partner blocks of a symmetric operator differ");
  }
  U = Un;
  B = out;
  return true;
}

// Simultaneous eigenbasis of the Dirac characters of the little co-group of mesh point k0.
bool block_basis(Ctx& c, bool aux, int k0, CMat& U, Blocks& B) {
  const int nb = aux ? c.naux : c.nao;
  int m0[3];
  mesh_point(k0, c.n, m0);
  std::vector<int> little;
  for (int a = 0; a < c.nop; ++a)
    if (c.kmap[size_t(a) * c.nk + k0] == k0) little.push_back(a);
  const int h = int(little.size());
  // D^k(alpha) = exp(i k . v(alpha)) O^k(alpha)   (eq. projrep)
  std::vector<CMat> Dk(h), DkH(h);
  for (int i = 0; i < h; ++i) {
    const int a = little[i];
    const double arg = 2.0 * M_PI * (m0[0] * c.w[3 * a] + m0[1] * c.w[3 * a + 1] + m0[2] * c.w[3 * a + 2]) / c.n;
    Dk[i] = orbital_rep(c, aux, a, k0);
    for (auto& x : Dk[i].a) x *= cplx(std::cos(arg), std::sin(arg));
    DkH[i] = adjoint(Dk[i]);
  }
  // conjugacy classes of the little co-group (on rotation parts)
  auto op_of_rot = [&](const int* R) {
    for (int a = 0; a < c.nop; ++a)
      if (std::equal(R, R + 9, &c.W[9 * a])) return a;
    return -1;
  };
  std::vector<int> cls(h, -1);
  std::vector<std::pair<int, int>> classes;  // (representative index, size)
  for (int g = 0; g < h; ++g) {
    if (cls[g] >= 0) continue;
    const int id = int(classes.size());
    int size = 0;
    for (int b = 0; b < h; ++b) {
      double Wb[9], Wg[9], Wbi[9], t[9], r[9];
      for (int j = 0; j < 9; ++j) {
        Wb[j] = c.W[9 * little[b] + j];
        Wg[j] = c.W[9 * little[g] + j];
      }
      inv3(Wb, Wbi);
      mul3(Wb, Wg, t);
      mul3(t, Wbi, r);
      int Ri[9];
      for (int j = 0; j < 9; ++j) Ri[j] = int(std::lround(r[j]));
      const int a = op_of_rot(Ri);
      const int idx = int(std::find(little.begin(), little.end(), a) - little.begin());
      if (idx >= h) return c.fail("conjugate of a little-group element is not in the little group");
      if (cls[idx] < 0) {
        cls[idx] = id;
        ++size;
      }
    }
    classes.push_back({g, size});
  }
  // Dirac characters Omega_c = (n_c / h) sum_beta D(beta) D(gamma) D(beta)^{-1}  (eq. dirac)
  // and one generic Hermitian combination of their Hermitian components.
  CMat H(nb, nb);
  uint64_t lcg = 0x9E3779B97F4A7C15ull;
  auto rnd = [&]() {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return 0.5 + double(lcg >> 11) / double(1ull << 53);
  };
  for (const auto& cl : classes) {
    CMat Om(nb, nb);
    for (int b = 0; b < h; ++b) {
      const CMat t = matmul(matmul(Dk[b], Dk[cl.first]), DkH[b]);
      for (size_t j = 0; j < Om.a.size(); ++j) Om.a[j] += t.a[j];
    }
    const double sc = double(cl.second) / h;
    for (auto& x : Om.a) x *= sc;
    const double ca = rnd(), cb = rnd();
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        const cplx o = Om(i, j), oh = std::conj(Om(j, i));
        H(i, j) += ca * (o + oh) + cb * cplx(0.0, 1.0) * (o - oh);
      }
  }
  // Invariant subspaces: shells related by the little co-group (same l, same position in
  // the shell list of their atoms).  H is block diagonal over them.
  const std::vector<int>& atom = aux ? c.aux_atom : c.ao_atom;
  const std::vector<int>& L = aux ? c.aux_l : c.ao_l;
  const int ns = int(atom.size());
  std::vector<int> off(ns), local(ns), cnt(c.natom, 0);
  std::map<std::pair<int, int>, int> lookup;
  int o = 0;
  for (int s = 0; s < ns; ++s) {
    off[s] = o;
    o += 2 * L[s] + 1;
    local[s] = cnt[atom[s]]++;
    lookup[{atom[s], local[s]}] = s;
  }
  std::vector<int> orbit(ns, -1);
  int norb = 0;
  for (int s = 0; s < ns; ++s) {
    if (orbit[s] >= 0) continue;
    std::vector<int> stack{s};
    orbit[s] = norb;
    while (!stack.empty()) {
      const int u = stack.back();
      stack.pop_back();
      for (int a : little) {
        const int v = lookup.at({c.perm[size_t(a) * c.natom + atom[u]], local[u]});
        if (orbit[v] < 0) {
          orbit[v] = norb;
          stack.push_back(v);
        }
      }
    }
    ++norb;
  }
  struct Vec {
    double lam;
    int order;
    std::vector<cplx> v;
  };
  std::vector<Vec> vecs;
  double lmax = 0;
  for (int ob = 0; ob < norb; ++ob) {
    std::vector<int> idx;
    for (int s = 0; s < ns; ++s)
      if (orbit[s] == ob)
        for (int m = 0; m < 2 * L[s] + 1; ++m) idx.push_back(off[s] + m);
    const int d = int(idx.size());
    CMat Hs(d, d);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) Hs(i, j) = H(idx[i], idx[j]);
    std::vector<double> ev;
    CMat Vs;
    if (!herm_eig(Hs, ev, Vs)) return c.fail("Jacobi eigen-decomposition did not converge");
    for (int j = 0; j < d; ++j) {
      Vec x{ev[j], int(vecs.size()), std::vector<cplx>(nb)};
      for (int i = 0; i < d; ++i) x.v[idx[i]] = Vs(i, j);
      lmax = std::max(lmax, std::fabs(ev[j]));
      vecs.push_back(std::move(x));
    }
  }
  std::stable_sort(vecs.begin(), vecs.end(), [](const Vec& a, const Vec& b) { return a.lam < b.lam; });
  const double tol = 1e-8 * std::max(1.0, lmax);
  B = Blocks();
  U = CMat(nb, nb);
  int start = 0;
  for (int j = 0; j < nb; ++j) {
    for (int i = 0; i < nb; ++i) U(i, j) = vecs[j].v[i];
    if (j + 1 == nb || vecs[j + 1].lam - vecs[j].lam > tol) {
      B.size.push_back(j + 1 - start);
      B.off.push_back(start);
      start = j + 1;
    }
  }
  // checks: U unitary, U^H D(alpha) U block diagonal for every alpha of the little group
  CMat UH = adjoint(U);
  CMat I = matmul(UH, U);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j)
      if (std::abs(I(i, j) - (i == j ? 1.0 : 0.0)) > 1e-10) return c.fail("block basis is not unitary");
  std::vector<int> blk_of(nb);
  for (size_t r = 0; r < B.size.size(); ++r)
    for (int j = 0; j < B.size[r]; ++j) blk_of[B.off[r] + j] = int(r);
  for (int i = 0; i < h; ++i) {
    const CMat Db = matmul(UH, matmul(Dk[i], U));
    for (int p = 0; p < nb; ++p)
      for (int q = 0; q < nb; ++q)
        if (blk_of[p] != blk_of[q] && std::abs(Db(p, q)) > 1e-9)
          return c.fail("Dirac-character basis does not block-diagonalise the little group");
  }
  if (c.prm.blocks == GWSYM_BLOCKS_PARTNER) return partner_split(c, Dk, rnd, U, B);
  return true;
}

void single_block(int nb, Blocks& B) {
  B = Blocks();
  B.size = {nb};
  B.off = {0};
}

}  // namespace

int build_symmetry(Ctx& c, const gwsym_crystal* cr) {
  if (!cr || cr->natom <= 0 || !cr->positions || cr->nop <= 0 || !cr->rot || !cr->trans || cr->kmesh <= 0 ||
      cr->nshell_ao <= 0 || cr->nshell_aux <= 0 || !cr->ao_atom || !cr->ao_l || !cr->aux_atom || !cr->aux_l) {
    c.err = "invalid crystal description";
    return GWSYM_EINVAL;
  }
  std::memcpy(c.A, cr->lattice, sizeof(c.A));
  inv3(c.A, c.Ainv);
  c.natom = cr->natom;
  c.pos.assign(cr->positions, cr->positions + 3 * c.natom);
  c.nop = cr->nop;
  c.W.assign(cr->rot, cr->rot + 9 * c.nop);
  c.w.assign(cr->trans, cr->trans + 3 * c.nop);
  c.n = cr->kmesh;
  c.nk = c.n * c.n * c.n;
  c.ao_atom.assign(cr->ao_atom, cr->ao_atom + cr->nshell_ao);
  c.ao_l.assign(cr->ao_l, cr->ao_l + cr->nshell_ao);
  c.aux_atom.assign(cr->aux_atom, cr->aux_atom + cr->nshell_aux);
  c.aux_l.assign(cr->aux_l, cr->aux_l + cr->nshell_aux);
  c.nao = c.naux = 0;
  int lmax = 0;
  for (int s = 0; s < cr->nshell_ao; ++s) {
    if (c.ao_l[s] < 0 || c.ao_l[s] > 4 || c.ao_atom[s] < 0 || c.ao_atom[s] >= c.natom) {
      c.err = "orbital shell with l outside 0..4 or bad atom";
      return GWSYM_EINVAL;
    }
    c.nao += 2 * c.ao_l[s] + 1;
    lmax = std::max(lmax, c.ao_l[s]);
  }
  for (int s = 0; s < cr->nshell_aux; ++s) {
    if (c.aux_l[s] < 0 || c.aux_l[s] > 4 || c.aux_atom[s] < 0 || c.aux_atom[s] >= c.natom) {
      c.err = "auxiliary shell with l outside 0..4 or bad atom";
      return GWSYM_EINVAL;
    }
    c.naux += 2 * c.aux_l[s] + 1;
    lmax = std::max(lmax, c.aux_l[s]);
  }
  // op 0 must be the identity
  for (int j = 0; j < 9; ++j)
    if (c.W[j] != (j % 4 == 0 ? 1 : 0)) {
      c.err = "operation 0 is not the identity";
      return GWSYM_EINVAL;
    }
  // Cartesian rotations; atom permutations and lattice shifts
  c.Rcart.resize(9 * c.nop);
  c.perm.assign(size_t(c.nop) * c.natom, -1);
  c.shift.assign(size_t(c.nop) * c.natom * 3, 0);
  for (int a = 0; a < c.nop; ++a) {
    double Wd[9], t[9];
    for (int j = 0; j < 9; ++j) Wd[j] = c.W[9 * a + j];
    mul3(c.A, Wd, t);
    mul3(t, c.Ainv, &c.Rcart[9 * a]);
    const double* R = &c.Rcart[9 * a];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += R[3 * i + k] * R[3 * j + k];
        if (std::fabs(s - (i == j)) > 1e-9) {
          c.err = "operation " + std::to_string(a) + " is not orthogonal in Cartesian coordinates";
          return GWSYM_EINVAL;
        }
      }
    for (int x = 0; x < c.natom; ++x) {
      double img[3];
      for (int i = 0; i < 3; ++i)
        img[i] = c.W[9 * a + 3 * i] * c.pos[3 * x] + c.W[9 * a + 3 * i + 1] * c.pos[3 * x + 1] +
                 c.W[9 * a + 3 * i + 2] * c.pos[3 * x + 2] + c.w[3 * a + i];
      for (int y = 0; y < c.natom; ++y) {
        double d[3];
        bool ok = true;
        for (int i = 0; i < 3; ++i) {
          d[i] = img[i] - c.pos[3 * y + i];
          if (std::fabs(d[i] - std::nearbyint(d[i])) > 1e-9) ok = false;
        }
        if (ok) {
          c.perm[size_t(a) * c.natom + x] = y;
          for (int i = 0; i < 3; ++i) c.shift[(size_t(a) * c.natom + x) * 3 + i] = int(std::lround(d[i]));
          break;
        }
      }
      if (c.perm[size_t(a) * c.natom + x] < 0) {
        c.err = "operation " + std::to_string(a) + " does not map the crystal onto itself";
        return GWSYM_EINVAL;
      }
    }
  }
  // atoms related by an operation must carry the same shell sequence
  for (int which = 0; which < 2; ++which) {
    const std::vector<int>& atom = which ? c.aux_atom : c.ao_atom;
    const std::vector<int>& L = which ? c.aux_l : c.ao_l;
    std::vector<std::vector<int>> per(c.natom);
    for (size_t s = 0; s < atom.size(); ++s) per[atom[s]].push_back(L[s]);
    for (int a = 0; a < c.nop; ++a)
      for (int x = 0; x < c.natom; ++x)
        if (per[x] != per[c.perm[size_t(a) * c.natom + x]]) {
          c.err = std::string(which ? "auxiliary" : "orbital") +
                  " shells differ between symmetry-equivalent atoms";
          return GWSYM_EINVAL;
        }
  }
  // Wigner matrices per op and l
  c.wigner.assign(c.nop, {});
  for (int a = 0; a < c.nop; ++a)
    for (int l = 0; l <= lmax; ++l) c.wigner[a].push_back(wigner_real(l, &c.Rcart[9 * a]));
  // action on the mesh: k -> W^{-T} k
  c.kmap.assign(size_t(c.nop) * c.nk, 0);
  for (int a = 0; a < c.nop; ++a) {
    double Wd[9], Wi[9];
    for (int j = 0; j < 9; ++j) Wd[j] = c.W[9 * a + j];
    inv3(Wd, Wi);
    for (int k = 0; k < c.nk; ++k) {
      int m[3], mp[3];
      mesh_point(k, c.n, m);
      for (int i = 0; i < 3; ++i)
        mp[i] = int(std::lround(Wi[i] * m[0] + Wi[3 + i] * m[1] + Wi[6 + i] * m[2]));
      c.kmap[size_t(a) * c.nk + k] = mesh_index(mp, c.n);
    }
  }
  // stars: representative = smallest mesh index; alpha_k = first op mapping rep to k
  c.ibz.clear();
  c.rep.assign(c.nk, -1);
  c.alpha.assign(c.nk, -1);
  c.ibz_of_mesh.assign(c.nk, -1);
  const bool full = c.prm.mode == GWSYM_MODE_FULL;
  for (int k = 0; k < c.nk; ++k) {
    if (c.rep[k] >= 0) continue;
    const int i = int(c.ibz.size());
    c.ibz.push_back(k);
    c.ibz_of_mesh[k] = i;
    if (full) {
      c.rep[k] = i;
      c.alpha[k] = 0;
      continue;
    }
    for (int a = 0; a < c.nop; ++a) {
      const int kp = c.kmap[size_t(a) * c.nk + k];
      if (c.rep[kp] < 0) {
        c.rep[kp] = i;
        c.alpha[kp] = a;
      }
    }
  }
  c.nibz = int(c.ibz.size());
  // block bases at the representatives
  c.bao.assign(c.nibz, {});
  c.baux.assign(c.nibz, {});
  std::vector<CMat> Uao_ibz(c.nibz), Uaux_ibz(c.nibz);
  for (int i = 0; i < c.nibz; ++i) {
    if (c.prm.mode == GWSYM_MODE_BLOCK) {
      if (!block_basis(c, false, c.ibz[i], Uao_ibz[i], c.bao[i])) return GWSYM_ENOCONV;
      if (!block_basis(c, true, c.ibz[i], Uaux_ibz[i], c.baux[i])) return GWSYM_ENOCONV;
    } else {
      Uao_ibz[i] = CMat::eye(c.nao);
      Uaux_ibz[i] = CMat::eye(c.naux);
      single_block(c.nao, c.bao[i]);
      single_block(c.naux, c.baux[i]);
    }
  }
  // U^k = O^{rep}(alpha_k) U^{rep} for every mesh point
  c.U_ao.assign(c.nk, {});
  c.U_aux.assign(c.nk, {});
  for (int k = 0; k < c.nk; ++k) {
    const int i = c.rep[k];
    if (c.ibz[i] == k) {
      c.U_ao[k] = Uao_ibz[i];
      c.U_aux[k] = Uaux_ibz[i];
    } else {
      c.U_ao[k] = matmul(orbital_rep(c, false, c.alpha[k], c.ibz[i]), Uao_ibz[i]);
      c.U_aux[k] = matmul(orbital_rep(c, true, c.alpha[k], c.ibz[i]), Uaux_ibz[i]);
    }
  }
  // packed layouts
  c.f_off.assign(c.nibz + 1, 0);
  c.g_off.assign(c.nibz + 1, 0);
  c.p_off.assign(c.nibz + 1, 0);
  for (int i = 0; i < c.nibz; ++i) {
    for (Blocks* B : {&c.bao[i], &c.baux[i]}) {
      B->poff.clear();
      B->packed = 0;
      if (B->lead.size() != B->size.size()) {   // no aligned partners: every block leads itself
        B->lead.resize(B->size.size());
        std::iota(B->lead.begin(), B->lead.end(), 0);
      }
      for (int s : B->size) {
        B->poff.push_back(B->packed);
        B->packed += i64(s) * s;
      }
    }
    c.f_off[i + 1] = c.f_off[i] + c.bao[i].packed;
    c.g_off[i + 1] = c.g_off[i] + i64(c.ntau) * c.bao[i].packed;
    c.p_off[i + 1] = c.p_off[i] + i64(c.ntau) * c.baux[i].packed;
  }
  return GWSYM_OK;
}

}  // namespace gw
