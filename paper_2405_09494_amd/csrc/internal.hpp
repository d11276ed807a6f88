// Internal declarations shared by the host and device translation units of libgwsym.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gwsym.h"

namespace gw {

using cplx = std::complex<double>;
using i64 = int64_t;

// Dense row-major complex matrix.
struct CMat {
  int rows = 0, cols = 0;
  std::vector<cplx> a;
  CMat() = default;
  CMat(int r, int c) : rows(r), cols(c), a(size_t(r) * c) {}
  cplx& operator()(int i, int j) { return a[size_t(i) * cols + j]; }
  const cplx& operator()(int i, int j) const { return a[size_t(i) * cols + j]; }
  static CMat eye(int n) {
    CMat m(n, n);
    for (int i = 0; i < n; ++i) m(i, i) = 1.0;
    return m;
  }
};

CMat matmul(const CMat& A, const CMat& B);
CMat adjoint(const CMat& A);
// Eigen-decomposition of a Hermitian matrix by cyclic complex Jacobi rotations.
// Returns eigenvalues (ascending) and eigenvectors as columns of V.
bool herm_eig(const CMat& H, std::vector<double>& w, CMat& V, int max_sweeps = 60);
// Least-squares solution X of A X = B (A m x n, m >= n, full column rank) by Householder QR.
bool lstsq(const CMat& A, const CMat& B, CMat& X);
// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// Real spherical harmonics of degree l at the unit vector p (convention in symmetry.cpp).
void real_ylm(int l, const double p[3], double* out);

// Block structure of one basis (orbital or auxiliary) at one irreducible point.
struct Blocks {
  std::vector<int> size;    // n_r
  std::vector<int> off;     // first basis function of block r (in the block basis)
  std::vector<i64> poff;    // offset of block r in the packed layout
  i64 packed = 0;           // sum n_r^2
  // lead[r]: the block whose values block r repeats for every operator that commutes with the
  // group (aligned partner blocks of one irrep), r itself when it has none
  std::vector<int> lead;
};

// One problem of the grouped batch-reduce complex GEMM:
//   C_b (M x N) = alpha * sum_{t<T} opA(A_{b,t}) (M x K) * opB(B_{b,t}) (K x N) + beta * C_b
// with A_{b,t} = base[abuf] + aoff + b*sAb + t*sAt (complex elements), element (m, k) of
// opA at m*lda + k (N), k*lda + m (T), conj of that (C: no transpose, H: transpose).
enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2, OP_H = 3 };

struct GemmProblem {
  int M, N, K, T, batch;
  int abuf, bbuf, cbuf;
  int opA, opB;
  i64 aoff, lda, sAt, sAb;
  i64 boff, ldb, sBt, sBb;
  i64 coff, ldc, sCb;
  double alpha_re, alpha_im;
  int beta;                 // 0: overwrite, 1: accumulate
  // Optional right multiply of A by a block-diagonal K x K matrix that depends on the
  // outer index: opA(A_t) <- opA(A_t) * G_(t / gdiv).  Entry t / gdiv of the int64 table at
  // bases[B_GT] + gtab holds (offset of the packed blocks in bases[gbuf], offset of their
  // block list in the block table bases[B_BT]).  Requires K <= 32 and opA = N.
  int gfuse;
  int gbuf, gdiv, pad_;
  i64 gtab;
  // Row and column batches (wave-tile kernel): row r of A and C is row r % rdiv of batch
  // r / rdiv, whose A and C start sArb and sCrb elements further on; column n of B and C is
  // column n % cdiv of batch n / cdiv, offset by sBcb and sCcb.  rdiv = M, cdiv = N: none.
  int rdiv, cdiv;
  i64 sArb, sCrb, sBcb, sCcb;
  // K-segment list (the polarization and self-energy orbital contractions, which skip the
  // vanishing tiles of V): nkseg entries at bases[B_KL] + kseg replace the outer range; entry
  // {t0, np, kb, ke} sums the outer indices [t0, t0 + np) over k in [kb, ke) only.
  i64 kseg;
  int nkseg, pad2_;
};

// One entry of a K-segment list (see GemmProblem::kseg): 0 <= kb < ke <= K, np >= 1.
struct KSeg {
  int t0, np, kb, ke;
};

// An output tile of one problem over the outer range [t0, t1), in units of 16: rows
// [16 tm, 16 (tm + mh)) with mh = 1 or 2, columns [16 tn, 16 (tn + nn)) walked in chunks of
// 32.  slot < 0: the tile writes C directly; otherwise (nn <= 2) it writes its raw sum to
// the 32 x 32 partial slot `slot` and a reduction item combines the slots in order.
struct GemmTile {
  int prob, batch, tm, tn, t0, t1, slot, mh, nn;
  int nsub;   // with a K-segment list: [t0, t1) are entries and nsub their k sub-steps (of 4)
};

struct GemmReduce {
  int prob, batch, tm, tn, slot0, nslot, mh, nh;   // tm, tn, mh, nh in units of 16
};

struct GemmPlan {
  std::vector<GemmProblem> probs;
  std::vector<GemmTile> tiles;
  std::vector<GemmReduce> reds;
  int nslots = 0;
  double macs = 0;          // complex MACs actually requested (no padding)
  // device copies
  void* d_probs = nullptr;
  void* d_tiles = nullptr;
  void* d_reds = nullptr;
};

// Buffer ids used in GemmProblem::abuf/bbuf/cbuf; the launch passes the base pointers.
enum Buf : int {
  B_VP = 0, B_VS, B_G, B_P, B_W1, B_W2, B_OUT, B_TR, B_IN, B_U, B_WT, B_F, B_SCR, B_GT, B_BT, B_KL, NBUF
};

struct Ctx {
  gwsym_params prm{};
  gwsym_tuning tune{};                     // contraction launch plan (device_init, autotune)
  std::string err;
  bool built = false, dev = false, vloaded = false;

  // crystal
  double A[9]{}, Ainv[9]{};
  int natom = 0;
  std::vector<double> pos;                 // natom x 3
  int nop = 0;
  std::vector<int> W;                      // nop x 9
  std::vector<double> w;                   // nop x 3
  std::vector<double> Rcart;               // nop x 9
  std::vector<int> perm;                   // nop x natom
  std::vector<int> shift;                  // nop x natom x 3
  int n = 0, nk = 0, nibz = 0, nao = 0, naux = 0, ntau = 0, nw = 0;
  std::vector<int> ao_atom, ao_l, aux_atom, aux_l;
  std::vector<std::vector<CMat>> wigner;   // [op][l]: D^l of the Cartesian rotation

  // k mesh and stars
  std::vector<int> kmap;                   // nop x nk
  std::vector<int> ibz;                    // mesh index of representative i
  std::vector<int> rep;                    // nk -> i
  std::vector<int> alpha;                  // nk -> op with alpha rep = k
  std::vector<int> ibz_of_mesh;            // mesh index -> i or -1

  // blocks and bases
  std::vector<Blocks> bao, baux;           // per i
  std::vector<CMat> U_ao, U_aux;           // per k (all mesh points)
  std::vector<i64> g_off, p_off, f_off;    // packed offsets per i (nibz + 1)

  // grids
  std::vector<double> tau;
  std::vector<cplx> Tf, Tb, Bf, Bb;        // [nw][ntau], [ntau][nw]
  std::vector<int> nfreq_f, nfreq_b;       // Matsubara index n of each stored frequency (>= 0)

  // vanishing tiles of V in the block bases (Sec. 4.3), from the last load_V: per pair
  // p = i nk + k of each copy (0: self-energy, indexed (k0 in IBZ, k'); 1: polarization,
  // (q0 in IBZ, k)) a flag per (auxiliary block s, orbital block r, orbital block r'), 1 for a
  // tile that is kept, at vt_off[copy][p] + (s nr + r) nr' + r'
  std::vector<uint8_t> vt_nz[2];
  std::vector<i64> vt_off[2];
  // tiles and kept tiles of the self-energy copy, the same for the polarization copy; per
  // iteration the complex MACs of the P0 GEMM over all tiles and over the kept ones, the same
  // for the Sigma orbital GEMM; the P0 and Sigma orbital GEMM launches that walk K-segment
  // lists, and the launches of the two stages
  double vt_stats[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

  // device state (device.hip)
  void* dev_state = nullptr;
  double last_macs[2] = {0, 0};

  bool fail(const std::string& m) {
    err = m;
    return false;
  }
};

// symmetry.cpp
CMat orbital_rep(const Ctx& c, bool aux, int op, int k);
int build_symmetry(Ctx& c, const gwsym_crystal* cr);
// grids.cpp
void build_grids(Ctx& c);
// grids_ir.cpp: tau and Matsubara sampling on the IR basis (sets ntau, nw and the matrices)
void build_ir_grids(Ctx& c);
// device.hip
int device_init(Ctx& c, void* stream);
void device_free(Ctx& c);
int device_load_V(Ctx& c, const void* V, void* stream);
int device_to_block(Ctx& c, int kind, const void* full, void* blk, void* stream);
int device_from_block(Ctx& c, int kind, const void* blk, void* full, void* stream);
int device_g0(Ctx& c, const void* F, double mu, void* G, double* nfree, void* stream);
int device_polarization(Ctx& c, const void* G, void* P0, void* stream);
int device_screened(Ctx& c, const void* P0, void* P, void* stream);
int device_exchange(Ctx& c, const void* G, void* K, void* stream);
int device_hartree(Ctx& c, const void* G, void* J, const void* add, int accumulate, void* stream);
int device_fock(Ctx& c, const void* H0, const void* G, void* F, void* stream);
int device_self_energy(Ctx& c, const void* G, const void* P, void* S, void* stream);
int device_find_mu(Ctx& c, const void* F, const void* S, double ntarget, double* mu, void* stream);
int device_check(Ctx& c, void* stream);
int device_dyson(Ctx& c, const void* F, const void* S, const double* mu, void* G, void* stream);
int device_dyson_noalloc(Ctx& c, const void* F, const void* S, const double* mu, void* G, void* stream);
int device_iteration(Ctx& c, const void* H0, const void* F, void* G, void* P0, void* P, void* S, double* mu,
                     double ntarget, int use_graph, void* stream);
int device_profile(Ctx& c, int enable);
int device_replan(Ctx& c, void* stream);
int device_autotune(Ctx& c, void* stream);
int device_profile_read(Ctx& c, double* ms, int64_t* launches, double* macs, double* bytes);

}  // namespace gw
