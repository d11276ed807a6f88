// Block-diagonal multiplies of the contractions on the matrix cores (gfx950).
//
// The Green's function factors of eq. P0 and eq. sigma are block-diagonal in the symmetry
// adapted basis (eq. mat_blk): each orbital block r of size n_r multiplies only the n_r
// matching rows or columns of the three-index slabs.  Both kernels here form these products
// as 16 x 16 output tiles on the MFMA (16 x 16 x 4 per instruction, four real instructions
// per complex K step), with the K range of a tile cut to the blocks that touch it: an output
// column c only sums over the k of its own block, and the entries of the block-diagonal
// factor outside the blocks are zeros fed to the MFMA.
//
//  k_bd_right  out[r][:] = in[r][:] G (and out2 = in G2 with the same blocks) for the rows of a
//              slab of row length n: the self-energy's Z = Y G^{k'}(tau) for a tau and its
//              mirror, and the exchange term.  Operands stream from global memory.
//  k_bd_both   X_s -> Gl^H X_s Gr^H for the S square n x n matrices side by side in a row-major
//              n x (S n) slice of a slab: the polarization's W = G^k(beta-tau)^H V G^{k+q}(tau)^H.
//              The slice sits in LDS; the right product is written back in place, the left one
//              goes to global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "kernel_api.hpp"

namespace gw {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename V2> struct Mf;
template <> struct Mf<double2> {
  using R = double;
  using A4 = d4;
  static __device__ __forceinline__ d4 mma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held by register j of lane l (column l % 16)
  static __device__ __forceinline__ int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};
template <> struct Mf<float2> {
  using R = float;
  using A4 = f4;
  static __device__ __forceinline__ f4 mma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};

// Complex accumulate c += a b on one 16 x 16 tile with three real MFMAs (3M): cr, ci and cx
// collect sum a_r b_r, sum a_i b_i and sum (a_r + a_i)(b_r + b_i); the tile's value is
// (cr - ci) + i (cx - cr - ci).  a is the row (A) fragment and b the column (B) fragment; as
// and bs are a_r + a_i and b_r + b_i, formed once where a held operand is loaded.
template <typename V2>
__device__ __forceinline__ void cmma(const V2 a, typename Mf<V2>::R as, const V2 b, typename Mf<V2>::R bs,
                                     typename Mf<V2>::A4& cr, typename Mf<V2>::A4& ci, typename Mf<V2>::A4& cx) {
  cr = Mf<V2>::mma(a.x, b.x, cr);
  ci = Mf<V2>::mma(a.y, b.y, ci);
  cx = Mf<V2>::mma(as, bs, cx);
}

// the same with four real MFMAs (4M), for kernels whose registers cannot hold a third accumulator
template <typename V2>
__device__ __forceinline__ void cmma4(const V2 a, const V2 b, typename Mf<V2>::A4& cr, typename Mf<V2>::A4& ci) {
  cr = Mf<V2>::mma(a.x, b.x, cr);
  ci = Mf<V2>::mma(a.x, b.y, ci);
  cr = Mf<V2>::mma(-a.y, b.y, cr);
  ci = Mf<V2>::mma(a.y, b.x, ci);
}

template <typename V2>
__device__ __forceinline__ V2 cval(const typename Mf<V2>::A4& cr, const typename Mf<V2>::A4& ci,
                                   const typename Mf<V2>::A4& cx, int j) {
  using R = typename Mf<V2>::R;
  return V2{R(cr[j] - ci[j]), R(cx[j] - cr[j] - ci[j])};
}

// Per index x < n of a basis: first index, size and packed offset of its block.
struct BlkOf {
  int off, sz, po;
};

__device__ __forceinline__ BlkOf blk_lookup(const int* __restrict__ bt, int x) {
  const int nb = bt[0];
  int b = 0;
  while (b + 1 < nb && x >= bt[1 + 3 * (b + 1)]) ++b;
  return BlkOf{bt[1 + 3 * b], bt[2 + 3 * b], bt[3 + 3 * b]};
}

// K range [lo, hi) of the blocks that meet the index tile [t0, t0 + 16) (indices < n)
__device__ __forceinline__ void tile_span(const int* __restrict__ bt, int t0, int n, int& lo, int& hi) {
  const BlkOf f = blk_lookup(bt, t0);
  const BlkOf l = blk_lookup(bt, min(t0 + 15, n - 1));
  lo = f.off;
  hi = l.off + l.sz;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// One 16 x 16 output tile over the K range of its blocks: the block-diagonal factor's
// fragments (one per lane and K step of four) are loaded into registers first, all at once, so
// their latencies overlap; the other operand's fragments come from LDS inside the MFMA loop.
// KS_MAX: K steps of the widest tile (n <= 4 KS_MAX).
constexpr int KS_MAX = 16;

// k_bd_right: a workgroup of four waves stages 64 rows of one slab in LDS (row stride n + 1).
// Wave w owns one column tile (w mod nct) and a share of the four row tiles; it loads the
// fragments of G (and, for a segment with out_off2 >= 0, of G2) for that column tile once and
// reuses them for all of its row tiles.  out[r][c] = sum_k in[r][k] G[k][c], k in the block of c.
template <typename V2>
__global__ __launch_bounds__(256) void k_bd_right(const RowSeg* __restrict__ segs, Bases bases,
                                                  const int* __restrict__ btab, int n) {
  using M = Mf<V2>;
  using R = typename M::R;
  using A4 = typename M::A4;
  extern __shared__ double2 lds_right[];
  V2* rows = reinterpret_cast<V2*>(lds_right);
  const RowSeg sg = segs[blockIdx.y];
  const int r0 = blockIdx.x * 64;
  if (r0 >= sg.nrows) return;
  const int nr = min(64, sg.nrows - r0), ld = n + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, kq = lane >> 4;
  const V2* in = reinterpret_cast<const V2*>(bases.p[sg.inbuf]) + sg.in_off + int64_t(r0) * n;
  for (int e = threadIdx.x; e < nr * n; e += 256) {
    const int r = e / n;
    rows[r * ld + (e - r * n)] = in[e];
  }
  __syncthreads();
  const bool dual = sg.out_off2 >= 0;   // uniform over the workgroup
  const int nct = (n + 15) / 16, nrt = (nr + 15) / 16;
  if (wave >= 4 / nct * nct) return;    // three column tiles: the fourth wave has none
  const int ct = wave % nct, rstep = 4 / nct;
  const int* bt = btab + sg.blk;
  const V2* G = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + sg.g_off;
  const V2* G2 = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + (dual ? sg.g_off2 : sg.g_off);
  int lo, hi;
  tile_span(bt, 16 * ct, n, lo, hi);
  const int k0 = lo & ~3, nks = (hi - k0 + 3) / 4;
  const int c = 16 * ct + li;
  const BlkOf cb = blk_lookup(bt, min(c, n - 1));
  const int cc = min(c, n - 1) - cb.off;
  // every lane loads an in-block address (its own column's first element when k is outside
  // the block) and zeroes what lies outside: no branches, so the loads stay in flight together
  V2 gf[KS_MAX], gf2[KS_MAX];
#pragma unroll
  for (int ks = 0; ks < KS_MAX; ++ks) {
    const int kk = k0 + 4 * ks + kq - cb.off;
    const bool in_b = ks < nks && c < n && kk >= 0 && kk < cb.sz;
    const int ge = cb.po + (in_b ? kk : 0) * cb.sz + cc;
    const V2 g = G[ge], g2 = G2[ge];
    gf[ks] = in_b ? g : V2{0, 0};
    gf2[ks] = in_b ? g2 : V2{0, 0};
  }
  V2* out = reinterpret_cast<V2*>(bases.p[sg.outbuf]) + sg.out_off + int64_t(r0) * n;
  V2* out2 = reinterpret_cast<V2*>(bases.p[sg.outbuf]) + (dual ? sg.out_off2 : sg.out_off) + int64_t(r0) * n;
  for (int rt = wave / nct; rt < nrt; rt += rstep) {   // uniform
    const V2* arow = rows + min(16 * rt + li, nr - 1) * ld;
    A4 cr = A4{0, 0, 0, 0}, ci = cr, dr = cr, di = cr;
#pragma unroll
    for (int ks = 0; ks < KS_MAX; ++ks) {
      if (ks < nks) {   // uniform
        const int k = k0 + 4 * ks + kq;
        V2 a = arow[min(k, n - 1)];
        if (k >= n) a = V2{0, 0};
        cmma4<V2>(a, gf[ks], cr, ci);
        if (dual) cmma4<V2>(a, gf2[ks], dr, di);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * rt + M::row(lane, j);
      if (c < n && r < nr) {
        out[int64_t(r) * n + c] = V2{R(cr[j]), R(ci[j])};
        if (dual) out2[int64_t(r) * n + c] = V2{R(dr[j]), R(di[j])};
      }
    }
  }
}

void launch_rowblock_right(const RowSegList& l, const Bases& b, const int* btab, int ncol, hipStream_t s, bool fp32) {
  if (l.nseg == 0) return;
  const dim3 g((l.maxrows + 63) / 64, l.nseg);
  const RowSeg* sg = (const RowSeg*)l.segs;
  const size_t lds = size_t(64) * (ncol + 1) * (fp32 ? sizeof(float2) : sizeof(double2));
  if (fp32) hipLaunchKernelGGL(k_bd_right<float2>, g, dim3(256), lds, s, sg, b, btab, ncol);
  else hipLaunchKernelGGL(k_bd_right<double2>, g, dim3(256), lds, s, sg, b, btab, ncol);
}

// ---------------------------------------------------------------------------------------
// k_bd_both: eight waves; the slice of S matrices (n x S n, row stride ld = S n + 1 in LDS).
// Right product Y = X Gr^H over the rows (s, a) (items: row tile x column tile, at most four
// per wave, held in registers until every wave has read the slice, then written back in
// place); left product W = Gl^H Y over the columns (s, b) (written to global memory).
template <typename V2>
__global__ __launch_bounds__(512) void k_bd_both(const RowSeg* __restrict__ segs, Bases bases,
                                                 const int* __restrict__ btab, int n, int S) {
  using M = Mf<V2>;
  using R = typename M::R;
  using A4 = typename M::A4;
  extern __shared__ double2 lds_both[];
  V2* tile = reinterpret_cast<V2*>(lds_both);
  const RowSeg sg = segs[blockIdx.y];
  const int ncols = sg.nrows;   // slab width: na matrices of n columns side by side
  const int s0 = blockIdx.x * S;
  if (s0 * n >= ncols) return;
  const int sv = min(S, ncols / n - s0), w = sv * n, ld = S * n + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, kq = lane >> 4;
  const V2* in = reinterpret_cast<const V2*>(bases.p[sg.inbuf]) + sg.in_off + s0 * n;
  V2* out = reinterpret_cast<V2*>(bases.p[sg.outbuf]) + sg.out_off + s0 * n;
  const V2* Gl = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + sg.g_off;
  const V2* Gr = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + sg.g_off2;
  const int* btl = btab + sg.blk;
  const int* btr = btab + sg.blk2;
  for (int e = threadIdx.x; e < n * w; e += 512) {
    const int a = e / w, j = e - a * w;
    tile[a * ld + j] = in[int64_t(a) * ncols + j];
  }
  __syncthreads();
  // ---- right: rows r = (s, a) = s n + a of [0, w), columns c of [0, n), K = b in the block of c.
  // Wave w owns column tile w mod nct (Gr fragments loaded once) and every (8 / nct)-th row tile.
  const int nrt = (w + 15) / 16, nct = (n + 15) / 16, rstep = 8 / nct;
  A4 yr[4], yi[4], yx[4];
  int gct = -1, k0 = 0, nks = 0;
  V2 gf[KS_MAX];
  R gs[KS_MAX];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    yr[q] = A4{0, 0, 0, 0};
    yi[q] = yr[q];
    yx[q] = yr[q];
    const int ct = wave % nct, rt = wave / nct + rstep * q;
    if (wave >= rstep * nct || rt >= nrt) continue;
    const int c = 16 * ct + li;
    if (ct != gct) {
      gct = ct;
      int lo, hi;
      tile_span(btr, 16 * ct, n, lo, hi);
      k0 = lo & ~3;
      nks = (hi - k0 + 3) / 4;
      const BlkOf cb = blk_lookup(btr, min(c, n - 1));
      const int cc = min(c, n - 1) - cb.off;
#pragma unroll
      for (int ks = 0; ks < KS_MAX; ++ks) {
        const int kk = k0 + 4 * ks + kq - cb.off;
        const bool in = ks < nks && c < n && kk >= 0 && kk < cb.sz;
        V2 g = Gr[cb.po + cc * cb.sz + (in ? kk : 0)];   // (Gr^H)[k][c] = conj Gr[c][k]
        g.y = -g.y;
        gf[ks] = in ? g : V2{0, 0};
        gs[ks] = gf[ks].x + gf[ks].y;
      }
    }
    const int r = min(16 * rt + li, w - 1), s = r / n, a = r - s * n;
    const V2* arow = tile + a * ld + s * n;
#pragma unroll
    for (int ks = 0; ks < KS_MAX; ++ks) {
      if (ks < nks) {
        const int k = k0 + 4 * ks + kq;
        V2 x = arow[min(k, n - 1)];
        if (k >= n) x = V2{0, 0};
        cmma<V2>(x, x.x + x.y, gf[ks], gs[ks], yr[q], yi[q], yx[q]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ct = wave % nct, rt = wave / nct + rstep * q, c = 16 * ct + li;
    if (wave >= rstep * nct || rt >= nrt) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * rt + M::row(lane, j);
      if (c < n && r < w) {
        const int s = r / n, a = r - s * n;
        tile[a * ld + s * n + c] = cval<V2>(yr[q], yi[q], yx[q], j);
      }
    }
  }
  __syncthreads();
  // ---- left: rows a' of [0, n), columns j of [0, w), K = a in the block of a'.  Wave w owns
  // row tile w mod nrt2 (Gl fragments loaded once) and every (8 / nrt2)-th column tile.
  const int nrt2 = (n + 15) / 16, nct2 = (w + 15) / 16, cstep = 8 / nrt2;
  int grt = -1;
  for (int ct = wave / nrt2; ct < nct2 && wave < cstep * nrt2; ct += cstep) {
    const int rt = wave % nrt2;
    const int ap = 16 * rt + li;
    if (rt != grt) {
      grt = rt;
      int lo, hi;
      tile_span(btl, 16 * rt, n, lo, hi);
      k0 = lo & ~3;
      nks = (hi - k0 + 3) / 4;
      const BlkOf rb = blk_lookup(btl, min(ap, n - 1));
      const int aa = min(ap, n - 1) - rb.off;
#pragma unroll
      for (int ks = 0; ks < KS_MAX; ++ks) {
        const int kk = k0 + 4 * ks + kq - rb.off;
        const bool in = ks < nks && ap < n && kk >= 0 && kk < rb.sz;
        V2 g = Gl[rb.po + (in ? kk : 0) * rb.sz + aa];   // (Gl^H)[a'][k] = conj Gl[k][a']
        g.y = -g.y;
        gf[ks] = in ? g : V2{0, 0};
        gs[ks] = gf[ks].x + gf[ks].y;
      }
    }
    const int jc = min(16 * ct + li, w - 1);
    A4 cr = A4{0, 0, 0, 0}, ci = cr, cx = cr;
#pragma unroll
    for (int ks = 0; ks < KS_MAX; ++ks) {
      if (ks < nks) {
        const int k = k0 + 4 * ks + kq;
        V2 y = tile[min(k, n - 1) * ld + jc];
        if (k >= n) y = V2{0, 0};
        cmma<V2>(gf[ks], gs[ks], y, y.x + y.y, cr, ci, cx);
      }
    }
    const int j = 16 * ct + li;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int a = 16 * rt + M::row(lane, jj);
      if (a < n && j < w) out[int64_t(a) * ncols + j] = cval<V2>(cr, ci, cx, jj);
    }
  }
}

// matrices per workgroup: the right product's rows (s, a) fill at most eight 16-row tiles, so
// that its items fit four per wave
inline int both_S(int n) { return std::max(1, 128 / n); }

void launch_rowblock_both(const RowSegList& l, const Bases& b, const int* btab, int n, hipStream_t s, bool fp32) {
  if (l.nseg == 0) return;
  const int S = both_S(n);
  const dim3 g((l.maxrows / n + S - 1) / S, l.nseg);
  const RowSeg* sg = (const RowSeg*)l.segs;
  const size_t lds = size_t(n) * (S * n + 1) * (fp32 ? sizeof(float2) : sizeof(double2));
  if (fp32) hipLaunchKernelGGL(k_bd_both<float2>, g, dim3(512), lds, s, sg, b, btab, n, S);
  else hipLaunchKernelGGL(k_bd_both<double2>, g, dim3(512), lds, s, sg, b, btab, n, S);
}

}  // namespace gw
