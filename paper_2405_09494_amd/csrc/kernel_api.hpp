// Work-item structures shared by the kernels (kernels.hip) and their host-side planner
// (pipeline.hip).  Every offset counts complex elements from the base pointer of the
// buffer id it names; the launch passes the current base pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace gw {

struct Bases {
  void* p[NBUF];
};

struct GemmPlanDev {
  void* probs = nullptr;
  void* tiles = nullptr;
  void* reds = nullptr;
  int ntiles = 0, nreds = 0, nslots = 0;
  int shape[4] = {0, 0, 0, 0};   // wave-tile lists: tiles per shape (16x16, 16x32, 32x16, 32x32), in order
  int kdepth = 32;               // split-bfloat16 forms: k values per MFMA (32, or 16 for short sums)
  int prefetch = 2;              // FP64 / FP32 forms: K sub-steps per group (2 or 4)
  int lists = 0;                 // the tiles walk K-segment lists (ranges of list entries)
};

// One slab for a block-diagonal multiply (bdiag.hip).  Right multiply: nrows rows of n
// columns, each row times the block-diagonal matrix at g_off (and, with out_off2 >= 0, also
// times the one at g_off2 with the same blocks, into out_off2).  Both-sided multiply: n rows of
// nrows columns made of nrows / n square n x n matrices side by side, each X -> Gl^H X Gr^H
// with Gl at (g_off, blk) and Gr at (g_off2, blk2).
struct RowSeg {
  int inbuf, outbuf, gbuf, blk;  // blk: offset of the block table entry in btab
  int64_t in_off, out_off, g_off;
  int nrows, blk2;
  int64_t g_off2;
  int64_t out_off2;   // right multiply: >= 0 writes a second product, by the matrix at g_off2
  // Sub-ranges of a slab (0: the whole slab).  Both-sided multiply: ld = row stride of the
  // slab when nrows (the width taken) is less.  Right multiply: logical row r is the physical
  // row (r / rw) ld + r % rw (groups of rw rows ld apart).
  int ld, rw;
};

struct RowSegList {
  void* segs = nullptr;
  int nseg = 0, maxrows = 0;
};

struct CopySeg {
  int inbuf, outbuf, n;
  int flags;   // k_herm_fill: 1 = the source block is only read (a copy of a leading partner block)
  int64_t in_off, out_off, len;
};

enum { INV_P = 0, INV_G = 1, INV_TRACE = 2 };

// One (pair, auxiliary block) of the tile-norm pass over V: auxiliary functions
// [q0, q0 + nq), strides of Q, a and b from v_off, block tables of a (bta) and b (btb) in
// btab, and where the nr(a) x nr(b) squared tile norms go.
struct TileNormItem {
  int64_t v_off, out_off;
  int64_t sQ;
  int sa, sb, q0, nq, bta, btb;
};
constexpr int TN_MAXN = 64;   // orbitals per basis the tile-norm pass takes
constexpr int TN_MAXB = 64;   // orbital blocks per basis

// One diagonal orbital block of one irreducible point for the Hartree term: the block's
// first function and size in the block basis, the block of G(beta) it pairs with, the
// diagonal pair V_S^{k0,k0} it reads and where the block of J goes in the F layout.
struct HartreeItem {
  int off, n;
  int64_t g_off, v_off, f_off;
};

struct InvItem {
  int n, xbuf, fbuf, outbuf;
  int64_t x_off, f_off, out_off;
  double w;
};

struct MuItem {
  int n, pad_;
  double weight;
};

struct EigItem {
  int n, fbuf, gbuf, pad_;
  int64_t f_off, g_off, g_stride;
};

// tag: 0 generic, 1 polarization contraction, 2 self-energy auxiliary contraction,
// 3 self-energy orbital contraction (separate kernel names in profiles)
// fp32: operands are float2 and the FP32 MFMA is used; f32mask bit b: buffer b holds float2
void launch_brgemm(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag = 0,
                   bool fp32 = false, unsigned f32mask = 0);
void launch_to_f32(const void* in, void* out, int64_t n, hipStream_t s);
// block-diagonal multiplies on the matrix cores (bdiag.hip); ncol = n <= 64
void launch_rowblock_right(const RowSegList& l, const Bases& b, const int* btab, int ncol, hipStream_t s,
                           bool fp32 = false);
void launch_rowblock_both(const RowSegList& l, const Bases& b, const int* btab, int n, hipStream_t s,
                          bool fp32);
// Wave-tile complex GEMM over the same problem and tile lists (tiles of at most 32 x 32).
// arith: 0 FP64 operands and MFMA; on float2 operands 1 FP32 MFMA, 2 three-piece and
// 3 two-piece bfloat16 splits on the bfloat16 MFMA with FP32 accumulation
void launch_wgemm(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag, int arith,
                  unsigned f32mask);
void launch_herm(const void* segs, int nseg, const Bases& b, hipStream_t s);
void launch_tile_norm(const void* items, int nitems, const void* V, const int* btab, double* out, int no,
                      hipStream_t s);
void launch_copy(const void* segs, int nseg, const Bases& b, hipStream_t s);
// upper triangle of each n x n block from its lower one (and a copy to out_off when >= 0)
void launch_herm_fill(const void* segs, int nseg, const Bases& b, hipStream_t s);
void launch_pack(const void* segs, int nseg, const Bases& b, hipStream_t s);
void launch_hartree(const void* items, const int* first, int nib, int nitems, const double* w, const void* proj,
                    int naux, int nao, void* rpart, void* rho, const void* add, int accumulate, const Bases& b,
                    hipStream_t s);
// nmax: largest matrix among the items
void launch_inverse(const void* items, int nitems, int nmax, const Bases& b, int mode, const double* mu,
                    double* trace, int* status, hipStream_t s);
void launch_mu_init(const double* eps_range, double* state, double* mu, hipStream_t s);
// probe 0: one bisection step; 1: residual check of the result (status bit 2)
void launch_mu_update(const void* items, int nitems, const double* trace, const void* Blast, double scale,
                      double ntarget, double* state, double* mu, int probe, int* status, hipStream_t s);
// largest orbital block for the free G0 (the Jacobi matrix stays under 64 KB of LDS)
constexpr int JAC_N = 60;
void launch_jacobi_g0(const void* items, int nitems, const Bases& b, const double* tau, int ntau, double beta,
                      double mu, double* occ, double* erange, void* vwork, hipStream_t s);
void launch_g0_reduce(const double* occ, const double* w, const double* erange, int nitems, double scale,
                      double* nfree, double* eps, hipStream_t s);

}  // namespace gw
