// HIP kernels of libgwsym for gfx950 (MI355X).
//
//  k_wgemm        grouped batch-reduce complex GEMM for the P0 and Sigma contractions: one
//                 wave per tile of up to 32 x 32, MFMA operands loaded straight from HBM.
//  k_brgemm       the same problem lists with 32 x 32 workgroup tiles staged through LDS
//                 (transforms, block changes of basis): C_b = alpha sum_t opA(A_{b,t})
//                 opB(B_{b,t}) + beta C_b with uneven sizes, one launch per tile list.
//  k_reduce       ordered sum of split-K partial tiles (deterministic, no atomics).
//  k_inverse      batched Gauss-Jordan inverses for the two Dyson equations.
//  k_jacobi_g0    batched Hermitian Jacobi eigen-decomposition and the free G0(tau).
//  k_herm, k_copy packed-block helpers; k_mu_* the chemical-potential bisection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "kernel_api.hpp"

namespace gw {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// s += x g and s += x conj(g), four fused multiply-adds each
template <typename V2>
__device__ __forceinline__ void cfma(V2& s, const V2 x, const V2 g) {
  s.x = fma(x.x, g.x, s.x);
  s.x = fma(-x.y, g.y, s.x);
  s.y = fma(x.x, g.y, s.y);
  s.y = fma(x.y, g.x, s.y);
}
template <typename V2>
__device__ __forceinline__ void cfma_conj(V2& s, const V2 x, const V2 g) {
  s.x = fma(x.x, g.x, s.x);
  s.x = fma(x.y, g.y, s.x);
  s.y = fma(x.y, g.x, s.y);
  s.y = fma(-x.x, g.y, s.y);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// ----------------------------------------------------------------------------
// grouped batch-reduce complex GEMM on FP64 (or FP32) MFMA.  A workgroup of four waves owns
// an output tile of 16 or 32 rows and walks its columns in chunks of 16 or 32; each 16 x 16
// quarter of a chunk belongs to one wave, and when a chunk has fewer than four quarters the
// waves of a quarter share out its K steps and add their sums through LDS at the end.  A
// complex K step of 4 is four real MFMAs.  The next step's A and B elements are fetched into
// registers while the current step computes.

constexpr int TM = 32, TN = 32, BK = 32;
constexpr int LD = TM + 1;     // LDS row length (padding against bank conflicts)
constexpr int PF = TM * BK / 256;  // elements of A (and of B) fetched per thread per step

// Element type of the operands: FP64 (double2, FP64 MFMA) or FP32 (float2, FP32 MFMA).
template <typename R> struct Cx;
template <> struct Cx<double> { using V2 = double2; using A4 = d4; };
template <> struct Cx<float> { using V2 = float2; using A4 = f4; };

template <typename V2>
__device__ __forceinline__ V2 load_op(const V2* __restrict__ p, int op, int64_t r, int64_t c, int64_t ld) {
  // element (r, c) of op(X): N -> X[r][c], T -> X[c][r], C -> conj X[r][c], H -> conj X[c][r]
  V2 v = (op & 1) ? p[c * ld + r] : p[r * ld + c];
  if (op & 2) v.y = -v.y;
  return v;
}

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row held by register j of lane l in the 16 x 16 result (column l % 16): the FP64 MFMA
// interleaves rows (l/16 + 4 j), the FP32 one keeps them consecutive (4 (l/16) + j).
__device__ __forceinline__ int mrow(double, int lane, int j) { return (lane >> 4) + 4 * j; }
__device__ __forceinline__ int mrow(float, int lane, int j) { return 4 * (lane >> 4) + j; }

// Position (row or column index within the tile, k index within the chunk) of fetch slot
// idx of an operand whose tile dimension is 16 << lg16: the contiguous index of the source
// runs fastest across threads.
__device__ __forceinline__ void slot_pos(int idx, bool kfast, int lg16, int& x, int& k) {
  if (kfast) { x = idx >> 5; k = idx & (BK - 1); }
  else { k = idx >> (4 + lg16); x = idx & ((16 << lg16) - 1); }
}

// offset of element (row, col) of C within one batch, row and column batches included
__device__ __forceinline__ int64_t c_offset(const GemmProblem& P, int row, int col) {
  const int rb = row / P.rdiv, cb = col / P.cdiv;
  return rb * P.sCrb + int64_t(row - rb * P.rdiv) * P.ldc + cb * P.sCcb + (col - cb * P.cdiv);
}

// TAG only separates the stages in profiles (P0, Sigma aux / orbital contractions, others).
// f32mask: bit b set when buffer b holds float2 (then C is stored as float2).
// The steps of all column chunks of a tile form one sequence, so the fetch of the next
// step (possibly the first of the next chunk) overlaps the current step's arithmetic.
template <typename R, int TAG>
__global__ __launch_bounds__(256, 3) void k_brgemm(const GemmProblem* __restrict__ probs,
                                                   const GemmTile* __restrict__ tiles, Bases bases,
                                                   double2* __restrict__ partials, unsigned f32mask) {
  using V2 = typename Cx<R>::V2;
  using A4 = typename Cx<R>::A4;
  __shared__ R lds_ab[4][BK][LD];   // A re, A im, B re, B im; also the cross-wave sums
  __shared__ R Gs_re[BK][BK + 1], Gs_im[BK][BK + 1];
  __shared__ int gcol_off[BK], gcol_sz[BK];
  R(*As_re)[LD] = lds_ab[0];
  R(*As_im)[LD] = lds_ab[1];
  R(*Bs_re)[LD] = lds_ab[2];
  R(*Bs_im)[LD] = lds_ab[3];
  const GemmTile tl = tiles[blockIdx.x];
  if (tl.prob < 0) return;   // padding entry of the XCD-ordered tile list
  const GemmProblem P = probs[tl.prob];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = tl.tm * 16, lgm = tl.mh - 1, tmv = tl.mh * 16;
  const V2* Ab = reinterpret_cast<const V2*>(bases.p[P.abuf]) + P.aoff + int64_t(tl.batch) * P.sAb;
  const V2* Bb = reinterpret_cast<const V2*>(bases.p[P.bbuf]) + P.boff + int64_t(tl.batch) * P.sBb;
  const bool a_kfast = (P.opA & 1) == 0;  // N, C: k is the contiguous index of A
  const bool b_nfast = (P.opB & 1) == 0;  // N, C: n is the contiguous index of B
  const int nkc = (P.K + BK - 1) / BK;
  const int spc = (tl.t1 - tl.t0) * nkc;   // steps per column chunk
  const int nchunk = (tl.nn + 1) >> 1;
  const int total = spc * nchunk;
  V2 ra[PF], rb[PF];
  auto fetch = [&](int st) {
    const int ch = st / spc, sc = st - ch * spc;
    const int cu = tl.tn + 2 * ch, nc = min(2, tl.tn + tl.nn - cu), n0 = cu * 16, lgn = nc - 1;
    const int tt = sc / nkc, t = tl.t0 + tt, k0 = (sc - tt * nkc) * BK, kv = min(BK, P.K - k0);
    const V2* A = Ab + int64_t(t) * P.sAt;
    const V2* B = Bb + int64_t(t) * P.sBt;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int idx = tid + 256 * q;
      int x, kk;
      V2 v = {0, 0};
      if (idx < (tmv << 5)) {
        slot_pos(idx, a_kfast, lgm, x, kk);
        if (m0 + x < P.M && kk < kv) v = load_op(A, P.opA, m0 + x, k0 + kk, P.lda);
      }
      ra[q] = v;
      V2 w = {0, 0};
      if (idx < (nc << 9)) {
        slot_pos(idx, !b_nfast, lgn, x, kk);
        if (n0 + x < P.N && kk < kv) w = load_op(B, P.opB, k0 + kk, n0 + x, P.ldb);
      }
      rb[q] = w;
    }
  };
  int gcur = -1;
  int nc = 0, n0 = 0, wpq = 1, quarter = 0, phase = 0, qm = 0, qn = 0;
  A4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
  if (total > 0) fetch(0);
  for (int st = 0; st < total; ++st) {
    const int ch = st / spc, sc = st - ch * spc;
    if (sc == 0) {
      // a new column chunk: its quarters and the waves that share one
      const int cu = tl.tn + 2 * ch;
      nc = min(2, tl.tn + tl.nn - cu);
      n0 = cu * 16;
      const int nq = tl.mh * nc;
      wpq = 4 / nq;
      quarter = wave / wpq;
      phase = wave % wpq;
      qm = (tl.mh == 2) ? (nc == 2 ? quarter >> 1 : quarter) : 0;
      qn = (tl.mh == 2) ? (nc == 2 ? (quarter & 1) : 0) : quarter;
      cre = A4{0, 0, 0, 0};
      cim = A4{0, 0, 0, 0};
    }
    const int tnv = nc * 16, lgn = nc - 1;
    const int tt = sc / nkc, t = tl.t0 + tt, kv = min(BK, P.K - (sc - tt * nkc) * BK);
    if (P.gfuse) {
      // block-diagonal right factor of A for this outer index (uniform over the group)
      const int gi = t / P.gdiv;
      if (gi != gcur) {
        gcur = gi;
        const int64_t* gt = reinterpret_cast<const int64_t*>(bases.p[B_GT]) + P.gtab + 2 * int64_t(gi);
        const V2* G = reinterpret_cast<const V2*>(bases.p[P.gbuf]) + gt[0];
        const int* bt = reinterpret_cast<const int*>(bases.p[B_BT]) + gt[1];
        __syncthreads();
        for (int e = tid; e < BK * BK; e += 256) {
          Gs_re[e / BK][e % BK] = 0.0;
          Gs_im[e / BK][e % BK] = 0.0;
        }
        __syncthreads();
        const int nb = bt[0];
        for (int b = 0; b < nb; ++b) {
          const int off = bt[1 + 3 * b], sz = bt[2 + 3 * b], po = bt[3 + 3 * b];
          for (int e = tid; e < sz * sz; e += 256) {
            const V2 g = G[po + e];
            Gs_re[off + e / sz][off + e % sz] = g.x;
            Gs_im[off + e / sz][off + e % sz] = g.y;
          }
          for (int cc = tid; cc < sz; cc += 256) {
            gcol_off[off + cc] = off;
            gcol_sz[off + cc] = sz;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int idx = tid + 256 * q;
      int x, kk;
      if (idx < (tmv << 5)) {
        slot_pos(idx, a_kfast, lgm, x, kk);
        As_re[kk][x] = ra[q].x;
        As_im[kk][x] = ra[q].y;
      }
      if (idx < (tnv << 5)) {
        slot_pos(idx, !b_nfast, lgn, x, kk);
        Bs_re[kk][x] = rb[q].x;
        Bs_im[kk][x] = rb[q].y;
      }
    }
    __syncthreads();
    if (st + 1 < total) fetch(st + 1);
    if (P.gfuse) {
      // A <- A G within each block of G (K = kv <= BK, a single chunk)
      V2 res[PF];
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int idx = tid + 256 * q, mm = idx & (tmv - 1), kc = idx >> (4 + lgm);
        V2 s = {0, 0};
        if (idx < (tmv << 5) && kc < kv) {
          const int off = gcol_off[kc], sz = gcol_sz[kc];
          for (int kk = off; kk < off + sz; ++kk) {
            const R ar = As_re[kk][mm], ai = As_im[kk][mm], gr = Gs_re[kk][kc], gim = Gs_im[kk][kc];
            s.x += ar * gr - ai * gim;
            s.y += ar * gim + ai * gr;
          }
        }
        res[q] = s;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int idx = tid + 256 * q, mm = idx & (tmv - 1), kc = idx >> (4 + lgm);
        if (idx < (tmv << 5)) {
          As_re[kc][mm] = res[q].x;
          As_im[kc][mm] = res[q].y;
        }
      }
      __syncthreads();
    }
    {
      const int r = qm * 16 + (lane & 15), cix = qn * 16 + (lane & 15), kq = lane >> 4;
      for (int kk = 4 * phase; kk < kv; kk += 4 * wpq) {
        const R are = As_re[kk + kq][r], aim = As_im[kk + kq][r];
        const R bre = Bs_re[kk + kq][cix], bim = Bs_im[kk + kq][cix];
        cre = mfma16(are, bre, cre);
        cim = mfma16(are, bim, cim);
        cre = mfma16(-aim, bim, cre);
        cim = mfma16(aim, bre, cim);
      }
    }
    __syncthreads();
    if (sc != spc - 1) continue;
    // ---- end of a column chunk ----
    if (wpq > 1) {
      // waves that shared a quarter's K steps add their sums in LDS (the tile buffers are free)
      R* red = &lds_ab[0][0][0];
      if (phase > 0) {
        R* dst = red + ((quarter * 3 + phase - 1) * 64 + lane) * 8;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          dst[j] = cre[j];
          dst[4 + j] = cim[j];
        }
      }
      __syncthreads();
      if (phase == 0)
        for (int p2 = 1; p2 < wpq; ++p2) {
          const R* src = red + ((quarter * 3 + p2 - 1) * 64 + lane) * 8;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cre[j] += src[j];
            cim[j] += src[4 + j];
          }
        }
      __syncthreads();
      if (phase > 0) continue;
    }
    const int col = qn * 16 + (lane & 15);
    if (tl.slot >= 0) {
      double2* out = partials + int64_t(tl.slot) * TM * TN;
      for (int j = 0; j < 4; ++j) {
        const int row = qm * 16 + mrow(R(0), lane, j);
        out[row * TN + col] = make_double2(double(cre[j]), double(cim[j]));
      }
      continue;
    }
    const double2 al = make_double2(P.alpha_re, P.alpha_im);
    const bool cf32 = (f32mask >> P.cbuf) & 1u;
    for (int j = 0; j < 4; ++j) {
      const int row = m0 + qm * 16 + mrow(R(0), lane, j), cc = n0 + col;
      if (row < P.M && cc < P.N) {
        double2 v = cmul(al, make_double2(double(cre[j]), double(cim[j])));
        const int64_t at = P.coff + int64_t(tl.batch) * P.sCb + int64_t(row) * P.ldc + cc;
        if (cf32) {
          float2* C = reinterpret_cast<float2*>(bases.p[P.cbuf]);
          if (P.beta) v = cadd(v, make_double2(C[at].x, C[at].y));
          C[at] = make_float2(float(v.x), float(v.y));
        } else {
          double2* C = reinterpret_cast<double2*>(bases.p[P.cbuf]);
          if (P.beta) v = cadd(v, C[at]);
          C[at] = v;
        }
      }
    }
  }
}

// Ordered sum of the split-K partial slots of one output tile; a workgroup takes a quarter
// of the tile (one element per thread) and keeps eight running sums over the slots, combined
// in a fixed order at the end (deterministic).
template <int TAG>
__global__ __launch_bounds__(256) void k_reduce(const GemmProblem* __restrict__ probs,
                                                const GemmReduce* __restrict__ reds, Bases bases,
                                                const double2* __restrict__ partials, unsigned f32mask) {
  const GemmReduce rd = reds[blockIdx.x];
  const GemmProblem P = probs[rd.prob];
  const bool cf32 = (f32mask >> P.cbuf) & 1u;
  const double2 al = make_double2(P.alpha_re, P.alpha_im);
  const int e = blockIdx.y * 256 + threadIdx.x;
  const int er = e / TN, ec = e % TN;
  const int row = rd.tm * 16 + er, cc = rd.tn * 16 + ec;
  if (er >= rd.mh * 16 || ec >= rd.nh * 16 || row >= P.M || cc >= P.N) return;
  const double2* src = partials + int64_t(rd.slot0) * TM * TN + e;
  double2 acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = make_double2(0.0, 0.0);
  int q = 0;
  for (; q + 8 <= rd.nslot; q += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = cadd(acc[u], src[int64_t(q + u) * TM * TN]);
  }
  for (int u = 0; q + u < rd.nslot; ++u) acc[u] = cadd(acc[u], src[int64_t(q + u) * TM * TN]);
  const double2 s = cadd(cadd(cadd(acc[0], acc[1]), cadd(acc[2], acc[3])), cadd(cadd(acc[4], acc[5]), cadd(acc[6], acc[7])));
  double2 v = cmul(al, s);
  const int64_t at = P.coff + int64_t(rd.batch) * P.sCb + c_offset(P, row, cc);
  if (cf32) {
    float2* C = reinterpret_cast<float2*>(bases.p[P.cbuf]);
    if (P.beta) v = cadd(v, make_double2(C[at].x, C[at].y));
    C[at] = make_float2(float(v.x), float(v.y));
  } else {
    double2* C = reinterpret_cast<double2*>(bases.p[P.cbuf]);
    if (P.beta) v = cadd(v, C[at]);
    C[at] = v;
  }
}

template <int TAG>
void launch_reduce(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, unsigned mask) {
  if (p.nreds > 0)
    hipLaunchKernelGGL(k_reduce<TAG>, dim3(p.nreds, TM * TN / 256), dim3(256), 0, s, (const GemmProblem*)p.probs,
                       (const GemmReduce*)p.reds, b, (const double2*)partials, mask);
}

void launch_reduce_tag(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag, unsigned mask) {
  switch (tag) {
    case 1: launch_reduce<1>(p, b, partials, s, mask); break;
    case 2: launch_reduce<2>(p, b, partials, s, mask); break;
    case 3: launch_reduce<3>(p, b, partials, s, mask); break;
    default: launch_reduce<0>(p, b, partials, s, mask); break;
  }
}

// ----------------------------------------------------------------------------
// Wave-tile grouped complex GEMM for the contractions: one wave per workgroup owns an output
// tile of 16 or 32 rows by 16 or 32 columns (M2, N2) over its outer range.  The MFMA operands
// come straight from global memory: in a sub-step over four k values lane l holds row (column)
// l % 16 of each 16-row quarter at k = 4 s + l / 16, so four lanes read 64 contiguous bytes of
// a row.  The sub-steps of all outer indices of the tile form one sequence, taken GS at a time
// with the next group in flight; the loop body has no branches (sub-steps past the end of the
// sequence and k values beyond K are zeroed through the B operand).  Rows and columns beyond
// the problem read clamped, in-range addresses and are never stored.  No LDS, no barriers.
//
// Arithmetic (AR): 0 FP64 MFMA, 1 FP32 MFMA, and the split-bfloat16 forms on FP32 operands:
// 2 splits each FP32 value into three bfloat16 pieces (hi + mid + lo, each rounded to nearest
// even from the remainder of the previous ones) and sums the six piece products whose piece
// indices add to at most 2; 3 splits into two pieces and sums three products.  Both accumulate
// in FP32 on the 16 x 16 x 32 bfloat16 MFMA.  A group of eight sub-steps feeds one such MFMA:
// lane l passes its eight values of the group as its eight k slots, for A and B alike, so
// the slot-to-k assignment is the same on both sides and the sum over k is unchanged.  Where
// the sub-step sequences are short (a small K and one outer index), groups of four on the
// 16 x 16 x 16 bfloat16 MFMA waste less on padding (AR 4 and 5, the same splits).

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));

template <int AR> struct WArith;
template <> struct WArith<0> { using R = double; static constexpr int GS = 2, NS = 0; };
template <> struct WArith<1> { using R = float; static constexpr int GS = 2, NS = 0; };
template <> struct WArith<2> { using R = float; static constexpr int GS = 8, NS = 3; };
template <> struct WArith<3> { using R = float; static constexpr int GS = 8, NS = 2; };
template <> struct WArith<4> { using R = float; static constexpr int GS = 4, NS = 3; };
template <> struct WArith<5> { using R = float; static constexpr int GS = 4, NS = 2; };
// FP64 and FP32 with four sub-steps per group: twice the operand bytes in flight per wave
template <> struct WArith<6> { using R = double; static constexpr int GS = 4, NS = 0; };
template <> struct WArith<7> { using R = float; static constexpr int GS = 4, NS = 0; };
template <int GS> struct BfV;
template <> struct BfV<8> { using T = bf8; };
template <> struct BfV<4> { using T = bf4; };

// x = p[0] + p[1] + ... + rest: each piece is the bfloat16 nearest to what the pieces before
// it leave over
template <int NS, int GS, typename V>
__device__ __forceinline__ void bf_split(const float (&x)[GS], V (&p)[NS]) {
  float r[GS];
#pragma unroll
  for (int i = 0; i < GS; ++i) r[i] = x[i];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int i = 0; i < GS; ++i) p[s][i] = __bf16(r[i]);
    if (s + 1 < NS) {
#pragma unroll
      for (int i = 0; i < GS; ++i) r[i] -= float(p[s][i]);
    }
  }
}
__device__ __forceinline__ bf8 bf_neg(bf8 v) {
  u4 u = __builtin_bit_cast(u4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf8, u);
}
__device__ __forceinline__ bf4 bf_neg(bf4 v) {
  u2 u = __builtin_bit_cast(u2, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf4, u);
}
__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf(bf4 a, bf4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0, 0);
}
// c_re += a b_re-part sums and c_im likewise for one 16 x 16 quarter pair, from the pieces of
// a = ar + i ai (with an = -ai) and b = br + i bi; the smaller piece products go first
template <int NS, typename V>
__device__ __forceinline__ void bf_cmac(const V (&ar)[NS], const V (&ai)[NS], const V (&an)[NS],
                                        const V (&br)[NS], const V (&bi)[NS], f4& cr, f4& ci) {
#pragma unroll
  for (int d = NS - 1; d >= 0; --d)
#pragma unroll
    for (int i = 0; i <= d; ++i) {
      const int j = d - i;
      cr = mfma_bf(ar[i], br[j], cr);
      cr = mfma_bf(an[i], bi[j], cr);
      ci = mfma_bf(ar[i], bi[j], ci);
      ci = mfma_bf(ai[i], br[j], ci);
    }
}

template <int AR, int TAG, bool M2, bool N2, bool KL>
__global__ __launch_bounds__(64) void k_wgemm(const GemmProblem* __restrict__ probs,
                                              const GemmTile* __restrict__ tiles, Bases bases,
                                              double2* __restrict__ partials, unsigned f32mask) {
  using R = typename WArith<AR>::R;
  constexpr int GS = WArith<AR>::GS, NS = WArith<AR>::NS;
  using V2 = typename Cx<R>::V2;
  using A4 = typename Cx<R>::A4;
  const GemmTile tl = tiles[blockIdx.x];
  if (tl.prob < 0) return;   // padding entry of the XCD-ordered tile list
  const GemmProblem P = probs[tl.prob];
  const int lane = threadIdx.x, li = lane & 15, kq = lane >> 4;
  const int m0 = tl.tm * 16, n0 = tl.tn * 16;
  const V2* Ab = reinterpret_cast<const V2*>(bases.p[P.abuf]) + P.aoff + int64_t(tl.batch) * P.sAb;
  const V2* Bb = reinterpret_cast<const V2*>(bases.p[P.bbuf]) + P.boff + int64_t(tl.batch) * P.sBb;
  const int K = P.K, nk4 = (K + 3) >> 2;
  const bool aT = P.opA & 1, bT = P.opB & 1;
  const R sA = (P.opA & 2) ? R(-1) : R(1), sB = (P.opB & 2) ? R(-1) : R(1);
  // element offset of (row or column x, k): x * ldx + k (k contiguous) or k * ldx + x, plus
  // the offset of the row (column) batch that x falls in
  auto arow = [&](int r) -> int64_t {
    const int rb = r / P.rdiv, rl = r - rb * P.rdiv;
    return rb * P.sArb + (aT ? int64_t(rl) : int64_t(rl) * P.lda);
  };
  auto bcol = [&](int c) -> int64_t {
    const int cb = c / P.cdiv, cl = c - cb * P.cdiv;
    return cb * P.sBcb + (bT ? int64_t(cl) * P.ldb : int64_t(cl));
  };
  const int64_t ax0 = arow(min(m0 + li, P.M - 1)), ax1 = arow(min(m0 + 16 + li, P.M - 1));
  const int64_t ak = aT ? P.lda : 1;
  const int64_t bk = bT ? 1 : P.ldb;
  // a tile of an N2 class covers nn / 2 consecutive 32-column chunks, walked in one sequence of
  // sub-step groups so that the first loads of a chunk overlap the last MFMAs of the one before
  const int nchunk = N2 ? (tl.nn >> 1) : 1;
  // KL: the tiles walk their problems' K-segment lists: entries [t0, t1) of {first outer index,
  // count, k range}, the k outside a range being zero tiles of V
  const KSeg* kl = reinterpret_cast<const KSeg*>(bases.p[B_KL]) + (KL ? P.kseg : 0);
  const int nsub = KL ? tl.nsub : (tl.t1 - tl.t0) * nk4, ngrp = (nsub + GS - 1) / GS, total = ngrp * nchunk;
  A4 c00r = {0, 0, 0, 0}, c00i = c00r, c01r = c00r, c01i = c00r, c10r = c00r, c10i = c00r, c11r = c00r, c11i = c00r;
  // FP64 and FP32 forms take three real products per complex one (3M): the r, i and x
  // accumulators hold sum a_r b_r, sum a_i b_i and sum (a_r + a_i)(b_r + b_i), and the complex
  // sum is (r - i) + i (x - r - i); the split-bfloat16 forms keep real and imaginary parts
  constexpr bool M3 = NS == 0;
  A4 c00x = c00r, c01x = c00r, c10x = c00r, c11x = c00r;
  // FP32 forms: the FP32 accumulators are added into FP64 sums every 256 k values of the
  // sequence, so the rounding of a tile's sum does not grow with the length of its outer range
  constexpr bool F32 = !std::is_same<R, double>::value;
  constexpr int FLUSH = 256 / (4 * GS);   // groups per FP32 partial sum
  d4 s00r = {0, 0, 0, 0}, s00i = s00r, s01r = s00r, s01i = s00r, s10r = s00r, s10i = s00r, s11r = s00r, s11i = s00r;
  int since = 0;
  // complex value of a tile's accumulators (in FP64 for the sums of the FP32 forms)
  auto re_of = [&](const A4& r, const A4& i) __attribute__((always_inline)) {
    const d4 dr = __builtin_convertvector(r, d4), di = __builtin_convertvector(i, d4);
    return M3 ? dr - di : dr;
  };
  auto im_of = [&](const A4& r, const A4& i, const A4& x) __attribute__((always_inline)) {
    const d4 dr = __builtin_convertvector(r, d4), di = __builtin_convertvector(i, d4);
    return M3 ? __builtin_convertvector(x, d4) - dr - di : di;
  };
  auto flush = [&]() __attribute__((always_inline)) {
    if constexpr (F32) {
      const A4 z = {0, 0, 0, 0};
      s00r += re_of(c00r, c00i);
      s00i += im_of(c00r, c00i, c00x);
      c00r = z;
      c00i = z;
      c00x = z;
      if (N2) {
        s01r += re_of(c01r, c01i);
        s01i += im_of(c01r, c01i, c01x);
        c01r = z;
        c01i = z;
        c01x = z;
      }
      if (M2) {
        s10r += re_of(c10r, c10i);
        s10i += im_of(c10r, c10i, c10x);
        c10r = z;
        c10i = z;
        c10x = z;
      }
      if (M2 && N2) {
        s11r += re_of(c11r, c11i);
        s11i += im_of(c11r, c11i, c11x);
        c11r = z;
        c11i = z;
        c11x = z;
      }
    }
  };
  // fetch position: chunk, outer index t and k step j of the next sub-step; the mask zeroes
  // k >= K and the sub-steps past the end of a chunk's sequence
  int fc = 0, ft = tl.t0, fj = 0, fs = 0;
  // list state: entry fe (its values E, the next entry's En loaded one entry ahead), outer
  // index fp within it and its k sub-steps enj; an empty tile reads no entry
  int fe = tl.t0, fp = 0;
  KSeg E{0, 1, 0, 1}, En = E;
  auto enter = [&]() __attribute__((always_inline)) {
    fe = tl.t0;
    fp = 0;
    if (tl.t1 > tl.t0) {
      E = kl[fe];
      En = kl[min(fe + 1, tl.t1 - 1)];
    }
  };
  if (KL) enter();
  int enj = (E.ke - E.kb + 3) >> 2;
  int64_t fbx0 = bcol(min(n0 + li, P.N - 1)), fbx1 = bcol(min(n0 + 16 + li, P.N - 1));
  V2 fa[GS][2], fb[GS][2];
  R fm[GS];
  auto fetch1 = [&](int h) __attribute__((always_inline)) {
    const bool live = fs < nsub;
    int t, k;
    int64_t kc;
    if constexpr (KL) {
      // past the end the state stays on the last live position: in-range addresses
      t = E.t0 + fp;
      k = E.kb + 4 * fj + kq;
      kc = min(k, E.ke - 1);
    } else {
      t = live ? ft : tl.t1 - 1;
      k = 4 * fj + kq;
      kc = min(k, K - 1);
    }
    const V2* A = Ab + int64_t(t) * P.sAt;
    const V2* B = Bb + int64_t(t) * P.sBt;
    fa[h][0] = A[ax0 + kc * ak];
    if (M2) fa[h][1] = A[ax1 + kc * ak];
    fb[h][0] = B[fbx0 + kc * bk];
    if (N2) fb[h][1] = B[fbx1 + kc * bk];
    if constexpr (KL) fm[h] = (live && k < E.ke) ? R(1) : R(0);
    else fm[h] = (live && k < K) ? R(1) : R(0);
    ++fs;
    if constexpr (KL) {
      if (live && ++fj == enj) {
        fj = 0;
        if (++fp == E.np) {
          fp = 0;
          if (fe + 1 < tl.t1) {
            ++fe;
            E = En;
            En = kl[min(fe + 1, tl.t1 - 1)];
            enj = (E.ke - E.kb + 3) >> 2;
          }
        }
      }
    } else if (++fj == nk4) {
      fj = 0;
      ++ft;
    }
    if (fs == GS * ngrp && fc + 1 < nchunk) {   // on to the next chunk
      ++fc;
      fs = 0;
      fj = 0;
      ft = tl.t0;
      if (KL) {
        enter();
        enj = (E.ke - E.kb + 3) >> 2;
      }
      const int nc = n0 + 32 * fc;
      fbx0 = bcol(min(nc + li, P.N - 1));
      fbx1 = bcol(min(nc + 16 + li, P.N - 1));
    }
  };
  auto fetch = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < GS; ++h) fetch1(h);
  };
  const double2 al = make_double2(P.alpha_re, P.alpha_im);
  const bool cf32 = (f32mask >> P.cbuf) & 1u;
  const int64_t cbase = P.coff + int64_t(tl.batch) * P.sCb;
  int64_t roffs[2][4];
#pragma unroll
  for (int qm = 0; qm < 2; ++qm)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gr = m0 + qm * 16 + mrow(R(0), lane, j), rb = gr / P.rdiv;
      roffs[qm][j] = cbase + rb * P.sCrb + int64_t(gr - rb * P.rdiv) * P.ldc;
    }
  auto store = [&](int cn0, int qm, int qn, const d4& cr, const d4& ci) {
    const int gc = cn0 + qn * 16 + li, cb = gc / P.cdiv;
    const int64_t coff = cb * P.sCcb + (gc - cb * P.cdiv);
    for (int j = 0; j < 4; ++j) {
      const int row = qm * 16 + mrow(R(0), lane, j), col = qn * 16 + li;
      if (tl.slot >= 0) {
        partials[int64_t(tl.slot) * TM * TN + row * TN + col] = make_double2(cr[j], ci[j]);
        continue;
      }
      if (m0 + row >= P.M || gc >= P.N) continue;
      double2 v = cmul(al, make_double2(cr[j], ci[j]));
      const int64_t at = roffs[qm][j] + coff;
      if (cf32) {
        float2* C = reinterpret_cast<float2*>(bases.p[P.cbuf]);
        if (P.beta) v = cadd(v, make_double2(C[at].x, C[at].y));
        C[at] = make_float2(float(v.x), float(v.y));
      } else {
        double2* C = reinterpret_cast<double2*>(bases.p[P.cbuf]);
        if (P.beta) v = cadd(v, C[at]);
        C[at] = v;
      }
    }
  };
  if (total > 0) fetch();
  int cc = 0, cp = 0;   // chunk and group being computed
  for (int st = 0; st < total; ++st) {
    V2 a[GS][2], b[GS][2];
    R m[GS];
#pragma unroll
    for (int h = 0; h < GS; ++h) {
      a[h][0] = fa[h][0];
      a[h][1] = M2 ? fa[h][1] : fa[h][0];
      b[h][0] = fb[h][0];
      b[h][1] = N2 ? fb[h][1] : fb[h][0];
      m[h] = fm[h];
    }
    if (st + 1 < total) fetch();
    if constexpr (NS == 0) {
#pragma unroll
      for (int h = 0; h < GS; ++h) {
        const R a0r = R(a[h][0].x), a0i = R(a[h][0].y) * sA, a1r = R(a[h][1].x), a1i = R(a[h][1].y) * sA;
        const R b0r = R(b[h][0].x) * m[h], b0i = R(b[h][0].y) * (sB * m[h]);
        const R b1r = R(b[h][1].x) * m[h], b1i = R(b[h][1].y) * (sB * m[h]);
        const R a0s = a0r + a0i, a1s = a1r + a1i, b0s = b0r + b0i, b1s = b1r + b1i;
        c00r = mfma16(a0r, b0r, c00r);
        c00i = mfma16(a0i, b0i, c00i);
        c00x = mfma16(a0s, b0s, c00x);
        if (N2) {
          c01r = mfma16(a0r, b1r, c01r);
          c01i = mfma16(a0i, b1i, c01i);
          c01x = mfma16(a0s, b1s, c01x);
        }
        if (M2) {
          c10r = mfma16(a1r, b0r, c10r);
          c10i = mfma16(a1i, b0i, c10i);
          c10x = mfma16(a1s, b0s, c10x);
        }
        if (M2 && N2) {
          c11r = mfma16(a1r, b1r, c11r);
          c11i = mfma16(a1i, b1i, c11i);
          c11x = mfma16(a1s, b1s, c11x);
        }
      }
    } else {
      // pieces of the B quarters (mask and conjugation applied first), then of each A quarter
      using BV = typename BfV<GS>::T;
      BV br[2][NS], bi[2][NS];
#pragma unroll
      for (int q = 0; q < (N2 ? 2 : 1); ++q) {
        float xr[GS], xi[GS];
#pragma unroll
        for (int h = 0; h < GS; ++h) {
          xr[h] = b[h][q].x * m[h];
          xi[h] = b[h][q].y * (sB * m[h]);
        }
        bf_split<NS>(xr, br[q]);
        bf_split<NS>(xi, bi[q]);
      }
#pragma unroll
      for (int q = 0; q < (M2 ? 2 : 1); ++q) {
        float xr[GS], xi[GS];
#pragma unroll
        for (int h = 0; h < GS; ++h) {
          xr[h] = a[h][q].x;
          xi[h] = a[h][q].y * sA;
        }
        BV ar[NS], ai[NS], an[NS];
        bf_split<NS>(xr, ar);
        bf_split<NS>(xi, ai);
#pragma unroll
        for (int s = 0; s < NS; ++s) an[s] = bf_neg(ai[s]);
        if (q == 0) {
          bf_cmac<NS>(ar, ai, an, br[0], bi[0], c00r, c00i);
          if (N2) bf_cmac<NS>(ar, ai, an, br[1], bi[1], c01r, c01i);
        } else {
          bf_cmac<NS>(ar, ai, an, br[0], bi[0], c10r, c10i);
          if (N2) bf_cmac<NS>(ar, ai, an, br[1], bi[1], c11r, c11i);
        }
      }
    }
    if (F32 && ++since == FLUSH) {
      flush();
      since = 0;
    }
    if (++cp == ngrp) {
      // end of a chunk: store it and start the next from zero
      const int cn0 = n0 + 32 * cc;
      if constexpr (F32) {
        flush();
        since = 0;
        store(cn0, 0, 0, s00r, s00i);
        if (N2) store(cn0, 0, 1, s01r, s01i);
        if (M2) store(cn0, 1, 0, s10r, s10i);
        if (M2 && N2) store(cn0, 1, 1, s11r, s11i);
        s00r = d4{0, 0, 0, 0};
        s00i = s00r;
        s01r = s00r;
        s01i = s00r;
        s10r = s00r;
        s10i = s00r;
        s11r = s00r;
        s11i = s00r;
      } else {
        store(cn0, 0, 0, re_of(c00r, c00i), im_of(c00r, c00i, c00x));
        if (N2) store(cn0, 0, 1, re_of(c01r, c01i), im_of(c01r, c01i, c01x));
        if (M2) store(cn0, 1, 0, re_of(c10r, c10i), im_of(c10r, c10i, c10x));
        if (M2 && N2) store(cn0, 1, 1, re_of(c11r, c11i), im_of(c11r, c11i, c11x));
        c00r = A4{0, 0, 0, 0};
        c00i = c00r;
        c00x = c00r;
        c01r = c00r;
        c01i = c00r;
        c01x = c00r;
        c10r = c00r;
        c10i = c00r;
        c10x = c00r;
        c11r = c00r;
        c11i = c00r;
        c11x = c00r;
      }
      cp = 0;
      ++cc;
    }
  }
  if (total == 0) {   // an empty K-segment range: the tile (or its partial slot) is zero
    const d4 z = {0, 0, 0, 0};
    for (int ch = 0; ch < nchunk; ++ch) {
      const int cn0 = n0 + 32 * ch;
      store(cn0, 0, 0, z, z);
      if (N2) store(cn0, 0, 1, z, z);
      if (M2) store(cn0, 1, 0, z, z);
      if (M2 && N2) store(cn0, 1, 1, z, z);
    }
  }
}

template <int AR, int TAG, bool KL>
void launch_wgemm_tag(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, unsigned mask) {
  const GemmProblem* pr = (const GemmProblem*)p.probs;
  const GemmTile* tl = (const GemmTile*)p.tiles;
  double2* pa = (double2*)partials;
  // the tile list is sorted by shape: 16x16, 16x32, 32x16, 32x32, counts in p.shape
  int at = 0;
  for (int sh = 0; sh < 4; ++sh) {
    const int n = p.shape[sh];
    if (n == 0) continue;
    const dim3 g(n), t(64);
    const GemmTile* ts = tl + at;
    switch (sh) {
      case 0: hipLaunchKernelGGL((k_wgemm<AR, TAG, false, false, KL>), g, t, 0, s, pr, ts, b, pa, mask); break;
      case 1: hipLaunchKernelGGL((k_wgemm<AR, TAG, false, true, KL>), g, t, 0, s, pr, ts, b, pa, mask); break;
      case 2: hipLaunchKernelGGL((k_wgemm<AR, TAG, true, false, KL>), g, t, 0, s, pr, ts, b, pa, mask); break;
      default: hipLaunchKernelGGL((k_wgemm<AR, TAG, true, true, KL>), g, t, 0, s, pr, ts, b, pa, mask); break;
    }
    at += n;
  }
}

// the polarization (1) and self-energy orbital (3) contractions take the K-segment form for
// the launches whose plan walks lists
template <int AR>
void launch_wgemm_t(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag, unsigned mask) {
  switch (tag) {
    case 1:
      p.lists ? launch_wgemm_tag<AR, 1, true>(p, b, partials, s, mask) : launch_wgemm_tag<AR, 1, false>(p, b, partials, s, mask);
      break;
    case 2: launch_wgemm_tag<AR, 2, false>(p, b, partials, s, mask); break;
    case 3:
      p.lists ? launch_wgemm_tag<AR, 3, true>(p, b, partials, s, mask) : launch_wgemm_tag<AR, 3, false>(p, b, partials, s, mask);
      break;
    default: launch_wgemm_tag<AR, 0, false>(p, b, partials, s, mask); break;
  }
}

void launch_wgemm(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag, int arith,
                  unsigned f32mask) {
  if (p.ntiles > 0) {
    const bool k16 = p.kdepth == 16, deep = p.prefetch == 4;
    switch (arith) {
      case 1: deep ? launch_wgemm_t<7>(p, b, partials, s, tag, f32mask) : launch_wgemm_t<1>(p, b, partials, s, tag, f32mask); break;
      case 2: k16 ? launch_wgemm_t<4>(p, b, partials, s, tag, f32mask) : launch_wgemm_t<2>(p, b, partials, s, tag, f32mask); break;
      case 3: k16 ? launch_wgemm_t<5>(p, b, partials, s, tag, f32mask) : launch_wgemm_t<3>(p, b, partials, s, tag, f32mask); break;
      default: deep ? launch_wgemm_t<6>(p, b, partials, s, tag, f32mask) : launch_wgemm_t<0>(p, b, partials, s, tag, f32mask); break;
    }
  }
  launch_reduce_tag(p, b, partials, s, tag, f32mask);
}

template <typename R>
void launch_brgemm_t(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag, unsigned mask) {
  const dim3 g(p.ntiles), t(256);
  const GemmProblem* pr = (const GemmProblem*)p.probs;
  const GemmTile* tl = (const GemmTile*)p.tiles;
  double2* pa = (double2*)partials;
  switch (tag) {
    case 1: hipLaunchKernelGGL((k_brgemm<R, 1>), g, t, 0, s, pr, tl, b, pa, mask); break;
    case 2: hipLaunchKernelGGL((k_brgemm<R, 2>), g, t, 0, s, pr, tl, b, pa, mask); break;
    case 3: hipLaunchKernelGGL((k_brgemm<R, 3>), g, t, 0, s, pr, tl, b, pa, mask); break;
    default: hipLaunchKernelGGL((k_brgemm<R, 0>), g, t, 0, s, pr, tl, b, pa, mask); break;
  }
}

void launch_brgemm(const GemmPlanDev& p, const Bases& b, void* partials, hipStream_t s, int tag, bool fp32,
                   unsigned f32mask) {
  if (p.ntiles > 0) {
    if (fp32) launch_brgemm_t<float>(p, b, partials, s, tag, f32mask);
    else launch_brgemm_t<double>(p, b, partials, s, tag, f32mask);
  }
  launch_reduce_tag(p, b, partials, s, tag, f32mask);
}

// FP64 -> FP32 copy of n complex numbers
__global__ void k_to_f32(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    out[e] = make_float2(float(in[e].x), float(in[e].y));
}

void launch_to_f32(const void* in, void* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_to_f32, dim3(unsigned(blocks)), dim3(256), 0, s, (const double2*)in, (float2*)out, n);
}

// ----------------------------------------------------------------------------
// Packed-block helpers.

// out[blk] = Y[blk] + Y[blk]^H for every segment (one n x n block each).
__global__ __launch_bounds__(256) void k_herm(const CopySeg* __restrict__ segs, Bases bases) {
  const CopySeg sg = segs[blockIdx.x];
  const double2* Y = reinterpret_cast<const double2*>(bases.p[sg.inbuf]) + sg.in_off;
  double2* X = reinterpret_cast<double2*>(bases.p[sg.outbuf]) + sg.out_off;
  const int n = sg.n;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int a = e / n, b = e % n;
    X[e] = cadd(Y[a * n + b], cconj(Y[b * n + a]));
  }
}

// plain copies of contiguous runs (tau mirror of P0)
__global__ __launch_bounds__(256) void k_copy(const CopySeg* __restrict__ segs, Bases bases) {
  const CopySeg sg = segs[blockIdx.x];
  const double2* a = reinterpret_cast<const double2*>(bases.p[sg.inbuf]) + sg.in_off;
  double2* o = reinterpret_cast<double2*>(bases.p[sg.outbuf]) + sg.out_off;
  for (int64_t e = threadIdx.x; e < sg.len; e += 256) o[e] = a[e];
}

// Hermitian fill of n x n blocks whose lower triangle holds the result: X[a][b] = conj(X[b][a])
// for a < b, in place; with out_off >= 0 the whole block is also copied there (the tau mirror,
// or an aligned partner block).  flags & 1: the source is only read (its own segment fills it).
__global__ __launch_bounds__(256) void k_herm_fill(const CopySeg* __restrict__ segs, Bases bases) {
  const CopySeg sg = segs[blockIdx.x];
  double2* X = reinterpret_cast<double2*>(bases.p[sg.inbuf]) + sg.in_off;
  double2* M = sg.out_off >= 0 ? reinterpret_cast<double2*>(bases.p[sg.outbuf]) + sg.out_off : nullptr;
  const int n = sg.n;
  const bool fill = !(sg.flags & 1);
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    const double2 v = a >= b ? X[e] : cconj(X[b * n + a]);
    if (a < b && fill) X[e] = v;
    if (M) M[e] = v;
  }
}

void launch_herm_fill(const void* segs, int nseg, const Bases& b, hipStream_t s) {
  if (nseg) hipLaunchKernelGGL(k_herm_fill, dim3(nseg), dim3(256), 0, s, (const CopySeg*)segs, b);
}

// gather an n x n block with leading dimension len into a contiguous n x n block
__global__ __launch_bounds__(256) void k_pack(const CopySeg* __restrict__ segs, Bases bases) {
  const CopySeg sg = segs[blockIdx.x];
  const double2* a = reinterpret_cast<const double2*>(bases.p[sg.inbuf]) + sg.in_off;
  double2* o = reinterpret_cast<double2*>(bases.p[sg.outbuf]) + sg.out_off;
  const int n = sg.n;
  for (int e = threadIdx.x; e < n * n; e += 256) o[e] = a[int64_t(e / n) * sg.len + e % n];
}

void launch_pack(const void* segs, int nseg, const Bases& b, hipStream_t s) {
  if (nseg) hipLaunchKernelGGL(k_pack, dim3(nseg), dim3(256), 0, s, (const CopySeg*)segs, b);
}

// ----------------------------------------------------------------------------
// Tile norms of V in the block bases (Sec. 4.3): for one pair and one auxiliary block, the
// squared Frobenius norm of every (orbital block r, orbital block r') tile, summed over the
// block's auxiliary functions.  Element (Q, a, b) of the pair sits at v_off + Q sQ + a sa + b sb;
// r and r' come from the block tables at bta (a) and btb (b), whose blocks tile [0, no) in
// order.  Each thread sums its (a, b) elements over Q, then adds them into its tile in LDS.
__global__ __launch_bounds__(256) void k_tile_norm(const TileNormItem* __restrict__ items, const double2* __restrict__ V,
                                                   const int* __restrict__ btab, double* __restrict__ out, int no) {
  const TileNormItem it = items[blockIdx.x];
  __shared__ double acc[TN_MAXB * TN_MAXB];
  __shared__ int ra[TN_MAXN], rb[TN_MAXN];
  const int* ta = btab + it.bta;
  const int* tb = btab + it.btb;
  const int nra = ta[0], nrb = tb[0];
  for (int x = threadIdx.x; x < no; x += 256) {
    int r = 0;
    while (r + 1 < nra && ta[1 + 3 * (r + 1)] <= x) ++r;
    ra[x] = r;
    int q = 0;
    while (q + 1 < nrb && tb[1 + 3 * (q + 1)] <= x) ++q;
    rb[x] = q;
  }
  for (int e = threadIdx.x; e < nra * nrb; e += 256) acc[e] = 0.0;
  __syncthreads();
  const double2* v = V + it.v_off;
  for (int e = threadIdx.x; e < no * no; e += 256) {
    const int a = e / no, b = e - a * no;
    const double2* x = v + int64_t(it.q0) * it.sQ + a * it.sa + b * it.sb;
    double s = 0.0;
    for (int q = 0; q < it.nq; ++q) {
      const double2 y = x[int64_t(q) * it.sQ];
      s = fma(y.x, y.x, fma(y.y, y.y, s));
    }
    atomicAdd(&acc[ra[a] * nrb + rb[b]], s);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nra * nrb; e += 256) out[it.out_off + e] = acc[e];
}

void launch_tile_norm(const void* items, int nitems, const void* V, const int* btab, double* out, int no,
                      hipStream_t s) {
  if (nitems) hipLaunchKernelGGL(k_tile_norm, dim3(nitems), dim3(256), 0, s, (const TileNormItem*)items,
                                 (const double2*)V, btab, out, no);
}

void launch_herm(const void* segs, int nseg, const Bases& b, hipStream_t s) {
  if (nseg) hipLaunchKernelGGL(k_herm, dim3(nseg), dim3(256), 0, s, (const CopySeg*)segs, b);
}
void launch_copy(const void* segs, int nseg, const Bases& b, hipStream_t s) {
  if (nseg) hipLaunchKernelGGL(k_copy, dim3(nseg), dim3(256), 0, s, (const CopySeg*)segs, b);
}

// ----------------------------------------------------------------------------
// Batched Gauss-Jordan inverse with partial pivoting, one workgroup per matrix.
//   mode INV_P:     A = I - X,                 out = A^{-1} - I    (eq. P02P)
//   mode INV_G:     A = (i w + mu) I - F - X,  out = A^{-1}        (eq. dyson)
//   mode INV_TRACE: as INV_G, writes Tr A^{-1} to trace[item] only
// Matrices with n <= INV_LDS_N are factorised in LDS, larger ones in place in `out`.

constexpr int INV_LDS_N = 48;
constexpr int INV_WAVE_N = 16;   // matrices up to this size take the one-wave kernel

__device__ void gauss_jordan(double2* A, int n, int* piv, double2* fcol, double* red, int* redi, int* sing) {
  const int tid = threadIdx.x;
  for (int c = 0; c < n; ++c) {
    // pivot search over rows c..n-1
    double best = -1.0;
    int bi = c;
    for (int r = c + tid; r < n; r += 256) {
      const double2 v = A[r * n + c];
      const double m = fabs(v.x) + fabs(v.y);
      if (m > best) { best = m; bi = r; }
    }
    red[tid] = best;
    redi[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        const double o = red[tid + w];
        const int oi = redi[tid + w];
        if (o > red[tid] || (o == red[tid] && oi < redi[tid])) { red[tid] = o; redi[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = redi[0];
    if (red[0] <= 0.0 && tid == 0) *sing = 1;
    if (tid == 0) piv[c] = p;
    if (p != c)
      for (int j = tid; j < n; j += 256) {
        const double2 t = A[c * n + j];
        A[c * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    __syncthreads();
    const double2 d = cdiv(make_double2(1.0, 0.0), A[c * n + c]);
    __syncthreads();
    for (int j = tid; j < n; j += 256) A[c * n + j] = (j == c) ? d : cmul(A[c * n + j], d);
    for (int r = tid; r < n; r += 256) fcol[r] = A[r * n + c];
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int r = e / n, j = e % n;
      if (r == c) continue;
      const double2 f = fcol[r];
      if (j == c) A[e] = cmul(make_double2(-f.x, -f.y), d);
      else A[e] = csub(A[e], cmul(f, A[c * n + j]));
    }
    __syncthreads();
  }
  for (int c = n - 1; c >= 0; --c) {
    const int p = piv[c];
    if (p != c)
      for (int r = tid; r < n; r += 256) {
        const double2 t = A[r * n + c];
        A[r * n + c] = A[r * n + p];
        A[r * n + p] = t;
      }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_inverse(const InvItem* __restrict__ items, Bases bases, int mode,
                                                 const double* __restrict__ mu, double* __restrict__ trace,
                                                 int* __restrict__ status) {
  __shared__ double2 Alds[INV_LDS_N * INV_LDS_N];
  __shared__ double2 fcol[512];
  __shared__ int piv[512];
  __shared__ double red[256];
  __shared__ int redi[256];
  __shared__ int sing;
  const InvItem it = items[blockIdx.x];
  const int n = it.n, tid = threadIdx.x;
  if (n <= INV_WAVE_N) return;   // done by k_inverse_w
  if (tid == 0) sing = 0;
  const double2* X = reinterpret_cast<const double2*>(bases.p[it.xbuf]) + it.x_off;
  const double2* F = it.f_off >= 0 ? reinterpret_cast<const double2*>(bases.p[it.fbuf]) + it.f_off : nullptr;
  double2* out = reinterpret_cast<double2*>(bases.p[it.outbuf]) + it.out_off;
  double2* A = (n <= INV_LDS_N) ? Alds : out;
  const double shift = (mode == INV_P) ? 0.0 : *mu;
  for (int e = tid; e < n * n; e += 256) {
    const int r = e / n, j = e % n;
    const double2 x = X[e];
    double2 a;
    if (mode == INV_P) {
      a = make_double2(-x.x, -x.y);
      if (r == j) a.x += 1.0;
    } else {
      const double2 f = F[e];
      a = make_double2(-f.x - x.x, -f.y - x.y);
      if (r == j) { a.x += shift; a.y += it.w; }
    }
    A[e] = a;
  }
  __syncthreads();
  gauss_jordan(A, n, piv, fcol, red, redi, &sing);
  __syncthreads();
  if (sing && tid == 0) atomicOr(status, 1);
  if (mode == INV_TRACE) {
    double2 s = make_double2(0.0, 0.0);
    for (int r = tid; r < n; r += 256) s = cadd(s, A[r * n + r]);
    red[tid] = s.x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    double re = red[0];
    __syncthreads();
    red[tid] = s.y;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      trace[2 * blockIdx.x] = re;
      trace[2 * blockIdx.x + 1] = red[0];
    }
    return;
  }
  for (int e = tid; e < n * n; e += 256) {
    double2 v = A[e];
    if (mode == INV_P && (e / n) == (e % n)) v.x -= 1.0;
    out[e] = v;
  }
}

// The same inverses for matrices of at most INV_WAVE_N rows: one wave per matrix, four per
// workgroup, each in its own LDS region; no workgroup barriers (a wave's LDS accesses are
// performed in order), the pivot search is a cross-lane reduction.
__global__ __launch_bounds__(256) void k_inverse_w(const InvItem* __restrict__ items, int nitems, Bases bases,
                                                   int mode, const double* __restrict__ mu,
                                                   double* __restrict__ trace, int* __restrict__ status) {
  __shared__ double2 lds[4][INV_WAVE_N * INV_WAVE_N];
  __shared__ int pivs[4][INV_WAVE_N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int idx = blockIdx.x * 4 + wave;
  if (idx >= nitems) return;
  const InvItem it = items[idx];
  const int n = it.n;
  if (n > INV_WAVE_N) return;
  double2* A = lds[wave];
  int* piv = pivs[wave];
  const double2* X = reinterpret_cast<const double2*>(bases.p[it.xbuf]) + it.x_off;
  const double2* F = it.f_off >= 0 ? reinterpret_cast<const double2*>(bases.p[it.fbuf]) + it.f_off : nullptr;
  double2* out = reinterpret_cast<double2*>(bases.p[it.outbuf]) + it.out_off;
  const double shift = (mode == INV_P) ? 0.0 : *mu;
  constexpr int EPL = INV_WAVE_N * INV_WAVE_N / 64;   // elements per lane
  int er[EPL], ej[EPL];
#pragma unroll
  for (int q = 0; q < EPL; ++q) {
    const int e = lane + 64 * q;
    er[q] = e / n;
    ej[q] = e - er[q] * n;
  }
#pragma unroll
  for (int q = 0; q < EPL; ++q) {
    const int e = lane + 64 * q;
    if (e >= n * n) continue;
    const double2 x = X[e];
    double2 a;
    if (mode == INV_P) {
      a = make_double2(-x.x, -x.y);
      if (er[q] == ej[q]) a.x += 1.0;
    } else {
      const double2 f = F[e];
      a = make_double2(-f.x - x.x, -f.y - x.y);
      if (er[q] == ej[q]) { a.x += shift; a.y += it.w; }
    }
    A[e] = a;
  }
  __builtin_amdgcn_wave_barrier();
  bool sing = false;
  for (int c = 0; c < n; ++c) {
    // pivot: largest |Re| + |Im| in column c at rows >= c, lowest row on ties
    double best = -1.0;
    int bi = c;
    if (lane >= c && lane < n) {
      const double2 v = A[lane * n + c];
      best = fabs(v.x) + fabs(v.y);
      bi = lane;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int p = bi;
    sing = sing || best <= 0.0;
    if (lane == 0) piv[c] = p;
    if (p != c && lane < n) {
      const double2 t = A[c * n + lane];
      A[c * n + lane] = A[p * n + lane];
      A[p * n + lane] = t;
    }
    __builtin_amdgcn_wave_barrier();
    const double2 d = cdiv(make_double2(1.0, 0.0), A[c * n + c]);
    __builtin_amdgcn_wave_barrier();
    if (lane < n) A[c * n + lane] = (lane == c) ? d : cmul(A[c * n + lane], d);
    __builtin_amdgcn_wave_barrier();
    double2 fv[EPL], rv[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const int e = lane + 64 * q;
      if (e < n * n) {
        fv[q] = A[er[q] * n + c];
        rv[q] = A[c * n + ej[q]];
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const int e = lane + 64 * q;
      if (e >= n * n || er[q] == c) continue;
      if (ej[q] == c) A[e] = cmul(make_double2(-fv[q].x, -fv[q].y), d);
      else A[e] = csub(A[e], cmul(fv[q], rv[q]));
    }
    __builtin_amdgcn_wave_barrier();
  }
  for (int c = n - 1; c >= 0; --c) {
    const int p = piv[c];
    if (p != c && lane < n) {
      const double2 t = A[lane * n + c];
      A[lane * n + c] = A[lane * n + p];
      A[lane * n + p] = t;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (sing && lane == 0) atomicOr(status, 1);
  if (mode == INV_TRACE) {
    double2 t = make_double2(0.0, 0.0);
    if (lane < n) t = A[lane * n + lane];
    for (int off = 32; off > 0; off >>= 1) {
      t.x += __shfl_xor(t.x, off);
      t.y += __shfl_xor(t.y, off);
    }
    if (lane == 0) {
      trace[2 * idx] = t.x;
      trace[2 * idx + 1] = t.y;
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < EPL; ++q) {
    const int e = lane + 64 * q;
    if (e >= n * n) continue;
    double2 v = A[e];
    if (mode == INV_P && er[q] == ej[q]) v.x -= 1.0;
    out[e] = v;
  }
}

void launch_inverse(const void* items, int nitems, int nmax, const Bases& b, int mode, const double* mu,
                    double* trace, int* status, hipStream_t s) {
  if (nitems == 0) return;
  hipLaunchKernelGGL(k_inverse_w, dim3((nitems + 3) / 4), dim3(256), 0, s, (const InvItem*)items, nitems, b, mode, mu,
                     trace, status);
  if (nmax > INV_WAVE_N)
    hipLaunchKernelGGL(k_inverse, dim3(nitems), dim3(256), 0, s, (const InvItem*)items, b, mode, mu, trace, status);
}

// ----------------------------------------------------------------------------
// Hartree term of the static self-energy (eq. sigma_hf, J).  Three small launches over the
// diagonal pairs V_S^{k0,k0}(s) (block basis, q = 0):
//   R[i][s]  = sum over the diagonal blocks of G^{k0}(beta)_ab conj(V_S^{k0,k0}(s)_ab)
//   rho[s]   = sum_s' Pi[s][s'] sum_i w_i R[i][s']   (Pi: projector onto the invariant
//              auxiliary functions; w_i folds -1 from gamma = -G(beta), s/Nk and |star|)
//   J^{k0}   = sum_s V_S^{k0,k0}(s) rho[s] on the diagonal blocks, into the F layout.
// All reductions run in a fixed order (no atomics).

__device__ inline double2 block_sum256(double2 v, double2* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  return red[0];
}

// grid (naux, nib): one workgroup per (s, irreducible point)
__global__ __launch_bounds__(256) void k_hartree_rho(const HartreeItem* __restrict__ items,
                                                     const int* __restrict__ first, Bases bases, int naux, int nao,
                                                     double2* __restrict__ R) {
  __shared__ double2 red[256];
  const int sx = blockIdx.x, i = blockIdx.y;
  const double2* VS = reinterpret_cast<const double2*>(bases.p[B_VS]);
  const double2* G = reinterpret_cast<const double2*>(bases.p[B_G]);
  double2 acc = make_double2(0.0, 0.0);
  for (int t = first[i]; t < first[i + 1]; ++t) {
    const HartreeItem it = items[t];
    const double2* v = VS + it.v_off + int64_t(sx) * nao * nao;
    const double2* g = G + it.g_off;
    for (int e = threadIdx.x; e < it.n * it.n; e += 256) {
      const int a = it.off + e / it.n, b = it.off + e % it.n;
      acc = cadd(acc, cmul(g[e], cconj(v[a * nao + b])));
    }
  }
  const double2 r = block_sum256(acc, red);
  if (threadIdx.x == 0) R[int64_t(i) * naux + sx] = r;
}

// grid ceil(naux / 4): one wave per auxiliary function s
__global__ __launch_bounds__(256) void k_hartree_mix(const double2* __restrict__ R, const double* __restrict__ w,
                                                     int nib, const double2* __restrict__ proj, int naux,
                                                     double2* __restrict__ rho) {
  const int lane = threadIdx.x & 63;
  const int sx = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (sx >= naux) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int t = lane; t < naux; t += 64) {
    double2 m = make_double2(0.0, 0.0);
    for (int i = 0; i < nib; ++i) {
      const double2 r = R[int64_t(i) * naux + t];
      m.x += w[i] * r.x;
      m.y += w[i] * r.y;
    }
    acc = cadd(acc, cmul(proj[int64_t(sx) * naux + t], m));
  }
  for (int o = 32; o > 0; o >>= 1) {
    acc.x += __shfl_xor(acc.x, o, 64);
    acc.y += __shfl_xor(acc.y, o, 64);
  }
  if (lane == 0) rho[sx] = acc;
}

// grid (nitems): one workgroup per diagonal block.  With add != null the output is
// J + add (+ the output's previous value when accumulate != 0), for F = H0 + J + K.
__global__ __launch_bounds__(256) void k_hartree_j(const HartreeItem* __restrict__ items, Bases bases, int naux,
                                                   int nao, const double2* __restrict__ rho,
                                                   const double2* __restrict__ add, int accumulate) {
  const HartreeItem it = items[blockIdx.x];
  const double2* VS = reinterpret_cast<const double2*>(bases.p[B_VS]) + it.v_off;
  double2* J = reinterpret_cast<double2*>(bases.p[B_OUT]) + it.f_off;
  const int64_t slab = int64_t(nao) * nao;
  for (int e = threadIdx.x; e < it.n * it.n; e += 256) {
    const int a = it.off + e / it.n, b = it.off + e % it.n;
    const double2* v = VS + a * nao + b;
    double2 acc = make_double2(0.0, 0.0);
    for (int sx = 0; sx < naux; ++sx) acc = cadd(acc, cmul(v[sx * slab], rho[sx]));
    if (add) acc = cadd(acc, add[it.f_off + e]);
    if (accumulate) acc = cadd(acc, J[e]);
    J[e] = acc;
  }
}

void launch_hartree(const void* items, const int* first, int nib, int nitems, const double* w, const void* proj,
                    int naux, int nao, void* rpart, void* rho, const void* add, int accumulate, const Bases& b,
                    hipStream_t s) {
  if (nib == 0 || nitems == 0 || naux == 0) return;
  const HartreeItem* it = static_cast<const HartreeItem*>(items);
  hipLaunchKernelGGL(k_hartree_rho, dim3(naux, nib), dim3(256), 0, s, it, first, b, naux, nao,
                     static_cast<double2*>(rpart));
  hipLaunchKernelGGL(k_hartree_mix, dim3((naux + 3) / 4), dim3(256), 0, s, static_cast<const double2*>(rpart), w,
                     nib, static_cast<const double2*>(proj), naux, static_cast<double2*>(rho));
  hipLaunchKernelGGL(k_hartree_j, dim3(nitems), dim3(256), 0, s, it, b, naux, nao, static_cast<const double2*>(rho),
                     static_cast<const double2*>(add), accumulate);
}

// ----------------------------------------------------------------------------
// Chemical potential bisection (one workgroup): N(mu) from the traces of G(i w_n) at the
// current mu, then the bracket update.  state = [lo, hi, mu].  probe 0 is one bisection step;
// probe 1 checks the result after the last step: |N(mu) - N_target| above 1e-8 max(1, N_target)
// means the bracket did not hold the root (status bit 2).

__global__ __launch_bounds__(256) void k_mu_update(const MuItem* __restrict__ items, int nitems,
                                                   const double2* __restrict__ trace, const double2* __restrict__ Blast,
                                                   double scale, double ntarget, double* __restrict__ state,
                                                   double* __restrict__ mu_out, int probe, int* __restrict__ status) {
  __shared__ double red[256];
  double s = 0.0;
  for (int e = threadIdx.x; e < nitems; e += 256) {
    const MuItem it = items[e];
    // Tr G(beta) = 2 Re sum_n B[ntau-1][n] Tr G(i w_n)
    const double2 v = cmul(Blast[it.n], trace[e]);
    s += 2.0 * v.x * it.weight;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double N = -scale * red[0];
    if (probe) {
      if (!(fabs(N - ntarget) <= 1e-8 * fmax(1.0, fabs(ntarget)))) atomicOr(status, 2);
      return;
    }
    double lo = state[0], hi = state[1];
    const double mid = state[2];
    if (N < ntarget) lo = mid; else hi = mid;
    state[0] = lo;
    state[1] = hi;
    state[2] = 0.5 * (lo + hi);
    *mu_out = state[2];
  }
}

// state = [eps_min - 20, eps_max + 20, midpoint]
__global__ void k_mu_init(const double* __restrict__ eps_range, double* __restrict__ state, double* __restrict__ mu) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    state[0] = eps_range[0] - 20.0;
    state[1] = eps_range[1] + 20.0;
    state[2] = 0.5 * (state[0] + state[1]);
    *mu = state[2];
  }
}

void launch_mu_init(const double* eps_range, double* state, double* mu, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_init, dim3(1), dim3(64), 0, s, eps_range, state, mu);
}
void launch_mu_update(const void* items, int nitems, const double* trace, const void* Blast, double scale,
                      double ntarget, double* state, double* mu, int probe, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_update, dim3(1), dim3(256), 0, s, (const MuItem*)items, nitems, (const double2*)trace,
                     (const double2*)Blast, scale, ntarget, state, mu, probe, status);
}

// ----------------------------------------------------------------------------
// Free G0 per block: Jacobi eigen-decomposition of F_r - mu I (parallel cyclic ordering),
// then G0(tau_j) = -V diag(g(e, tau_j)) V^H with g = exp(-e tau)/(1 + exp(-beta e)) in a
// form that never overflows.  Also writes per-block occupations and eigenvalue range.

// A (at most JAC_N x JAC_N) lives in LDS; the eigenvector matrix V lives in a global
// workspace slice of JAC_N * JAC_N per item, so that the workgroup stays under 64 KB of LDS.
__global__ __launch_bounds__(256) void k_jacobi_g0(const EigItem* __restrict__ items, Bases bases,
                                                   const double* __restrict__ tau, int ntau, double beta, double mu,
                                                   double* __restrict__ occ, double* __restrict__ erange,
                                                   double2* __restrict__ vwork) {
  __shared__ double2 A[JAC_N * JAC_N];
  __shared__ double ev[JAC_N];
  const EigItem it = items[blockIdx.x];
  const int n = it.n, tid = threadIdx.x;
  const int m = (n + 1) & ~1;  // even size for the round-robin pairing (index n is a dummy)
  double2* V = vwork + int64_t(blockIdx.x) * JAC_N * JAC_N;
  const double2* F = reinterpret_cast<const double2*>(bases.p[it.fbuf]) + it.f_off;
  for (int e = tid; e < m * m; e += 256) {
    const int r = e / m, c = e % m;
    double2 v = make_double2(0.0, 0.0);
    if (r < n && c < n) {
      v = F[r * n + c];
      if (r == c) v.x -= mu;
    }
    A[e] = v;
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Cyclic Jacobi by one lane (blocks are small and G0 is computed once): each rotation
  // removes the phase of the pivot A_pq with diag(1, e^{-i phi}) and then applies the real
  // rotation that zeroes it, J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]], A <- J^H A J, V <- V J.
  if (tid == 0) {
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
          const double2 v = A[r * m + c];
          const double w = v.x * v.x + v.y * v.y;
          tot += w;
          if (r != c) off += w;
        }
      if (off <= 1e-34 * tot) break;
      for (int p = 0; p < m; ++p)
        for (int q = p + 1; q < m; ++q) {
          const double2 b = A[p * m + q];
          const double ab = sqrt(b.x * b.x + b.y * b.y);
          if (ab < 1e-300) continue;
          const double2 ep = make_double2(b.x / ab, b.y / ab), em = cconj(ep);
          const double a = A[p * m + p].x, dd = A[q * m + q].x;
          const double th = (dd - a) / (2.0 * ab);
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
          for (int k = 0; k < m; ++k) {
            const double2 akp = A[k * m + p], t1 = cmul(em, A[k * m + q]);
            A[k * m + p] = make_double2(c * akp.x - s * t1.x, c * akp.y - s * t1.y);
            A[k * m + q] = make_double2(s * akp.x + c * t1.x, s * akp.y + c * t1.y);
            const double2 vkp = V[k * m + p], t2 = cmul(em, V[k * m + q]);
            V[k * m + p] = make_double2(c * vkp.x - s * t2.x, c * vkp.y - s * t2.y);
            V[k * m + q] = make_double2(s * vkp.x + c * t2.x, s * vkp.y + c * t2.y);
          }
          for (int k = 0; k < m; ++k) {
            const double2 apk = A[p * m + k], t1 = cmul(ep, A[q * m + k]);
            A[p * m + k] = make_double2(c * apk.x - s * t1.x, c * apk.y - s * t1.y);
            A[q * m + k] = make_double2(s * apk.x + c * t1.x, s * apk.y + c * t1.y);
          }
          A[p * m + q] = make_double2(0.0, 0.0);
          A[q * m + p] = make_double2(0.0, 0.0);
          A[p * m + p].y = 0.0;
          A[q * m + q].y = 0.0;
        }
    }
  }
  __syncthreads();
  if (tid < n) ev[tid] = A[tid * m + tid].x;
  __syncthreads();
  // occupations f(e) = 1/(1 + exp(beta e)) and eigenvalue range (of F, i.e. e + mu)
  if (tid == 0) {
    double o = 0.0, lo = 1e300, hi = -1e300;
    for (int l = 0; l < n; ++l) {
      const double e = ev[l];
      o += e >= 0 ? exp(-beta * e) / (1.0 + exp(-beta * e)) : 1.0 / (1.0 + exp(beta * e));
      lo = fmin(lo, e + mu);
      hi = fmax(hi, e + mu);
    }
    occ[blockIdx.x] = o;
    erange[2 * blockIdx.x] = lo;
    erange[2 * blockIdx.x + 1] = hi;
  }
  double2* G = reinterpret_cast<double2*>(bases.p[it.gbuf]) + it.g_off;
  for (int j = 0; j < ntau; ++j) {
    const double t = tau[j];
    for (int e = tid; e < n * n; e += 256) {
      const int a = e / n, b = e % n;
      double2 s = make_double2(0.0, 0.0);
      for (int l = 0; l < n; ++l) {
        const double el = ev[l];
        const double g = el >= 0 ? exp(-el * t) / (1.0 + exp(-beta * el)) : exp(el * (beta - t)) / (1.0 + exp(beta * el));
        const double2 va = V[a * m + l], vb = V[b * m + l];
        const double2 pr = cmul(va, cconj(vb));
        s.x -= g * pr.x;
        s.y -= g * pr.y;
      }
      G[int64_t(j) * it.g_stride + e] = s;
    }
  }
}

void launch_jacobi_g0(const void* items, int nitems, const Bases& b, const double* tau, int ntau, double beta,
                      double mu, double* occ, double* erange, void* vwork, hipStream_t s) {
  if (nitems)
    hipLaunchKernelGGL(k_jacobi_g0, dim3(nitems), dim3(256), 0, s, (const EigItem*)items, b, tau, ntau, beta, mu, occ,
                       erange, (double2*)vwork);
}

// sum of per-block occupations with star weights, and the global eigenvalue range
__global__ __launch_bounds__(256) void k_g0_reduce(const double* __restrict__ occ, const double* __restrict__ w,
                                                   const double* __restrict__ erange, int nitems, double scale,
                                                   double* __restrict__ nfree, double* __restrict__ eps) {
  __shared__ double s1[256], s2[256], s3[256];
  double a = 0.0, lo = 1e300, hi = -1e300;
  for (int e = threadIdx.x; e < nitems; e += 256) {
    a += w[e] * occ[e];
    lo = fmin(lo, erange[2 * e]);
    hi = fmax(hi, erange[2 * e + 1]);
  }
  s1[threadIdx.x] = a; s2[threadIdx.x] = lo; s3[threadIdx.x] = hi;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      s1[threadIdx.x] += s1[threadIdx.x + k];
      s2[threadIdx.x] = fmin(s2[threadIdx.x], s2[threadIdx.x + k]);
      s3[threadIdx.x] = fmax(s3[threadIdx.x], s3[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (nfree) *nfree = scale * s1[0];
    eps[0] = s2[0];
    eps[1] = s3[0];
  }
}

void launch_g0_reduce(const double* occ, const double* w, const double* erange, int nitems, double scale,
                      double* nfree, double* eps, hipStream_t s) {
  hipLaunchKernelGGL(k_g0_reduce, dim3(1), dim3(256), 0, s, occ, w, erange, nitems, scale, nfree, eps);
}

}  // namespace gw
