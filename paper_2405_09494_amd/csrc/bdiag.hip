// Block-diagonal multiplies of the contractions on the matrix cores (gfx950).
//
// The Green's function factors of eq. P0 and eq. sigma are block-diagonal in the symmetry
// adapted basis (eq. mat_blk): each orbital block r of size n_r multiplies only the n_r
// matching rows or columns of the three-index slabs.  Both kernels here form these products
// as 16 x 16 output tiles on the MFMA (16 x 16 x 4 per instruction, three real instructions
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
// Each 16 x 16 output tile runs over the K range of its blocks only.  The block-diagonal
// factor's fragments (one per lane and K step of four) are loaded into registers once per
// workgroup, branch-free, so their latencies overlap; the other operand's fragments come from
// LDS inside the MFMA loop.

// k_bd_right: out[r][c] = sum_k in[r][k] G[k][c] (k in the block of c) over the rows of one
// segment, and, for a segment with out_off2 >= 0, out2 the same with G2.  A workgroup of eight
// waves walks `per` consecutive chunks of ROWS rows of one segment: each wave owns one column
// tile, with as many waves per column tile as its K range calls for, and a share of the row
// tiles; it loads its fragments of G (and G2) once and keeps them for every chunk; the next
// chunk is loaded into registers (all loads in flight at once) while the current one is
// multiplied out of LDS.  KS: K steps of the widest column tile (n <= 4 KS); PF: chunk
// elements per thread (ROWS n / 512).

template <typename V2, int KS, int PF, int ROWS>
__global__ __launch_bounds__(512) void k_bd_right(const RowSeg* __restrict__ segs, Bases bases,
                                                  const int* __restrict__ btab, int n, int per) {
  using M = Mf<V2>;
  using R = typename M::R;
  using A4 = typename M::A4;
  constexpr int RT = ROWS / 16;   // row tiles per chunk, shared between the waves
  extern __shared__ double2 lds_right[];
  V2* rows = reinterpret_cast<V2*>(lds_right);
  const RowSeg sg = segs[blockIdx.y];
  const int nch = (sg.nrows + ROWS - 1) / ROWS;
  const int c0 = blockIdx.x * per;
  if (c0 >= nch) return;
  const int c1 = min(nch, c0 + per), ld = n + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, kq = lane >> 4;
  const bool dual = sg.out_off2 >= 0;   // uniform over the workgroup
  const int nct = (n + 15) / 16;
  const int* bt = btab + sg.blk;
  // waves per column tile in proportion to its K steps (the blocks make them differ): start
  // with one each and give every further wave to the tile whose share of the chunk's row
  // tiles takes longest; wave -> (column tile ct, rank j of w_ct)
  int ct = 0, rj = 0, rstep = 1;
  {
    int cost[4] = {0, 0, 0, 0}, wn[4] = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < nct) {
        int lo, hi;
        tile_span(bt, 16 * t, n, lo, hi);
        cost[t] = (hi - (lo & ~3) + 3) / 4 + 1;
        wn[t] = 1;
      }
    for (int extra = 8 - nct; extra > 0; --extra) {
      int best = 0, bv = -1;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int v = t < nct ? (RT + wn[t] - 1) / wn[t] * cost[t] : -1;
        if (v > bv) {
          bv = v;
          best = t;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t == best) ++wn[t];
    }
    int first = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (wave >= first && wave < first + wn[t]) {
        ct = t;
        rj = wave - first;
        rstep = wn[t];
      }
      first += wn[t];
    }
  }
  const bool act = true;
  const V2* G = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + sg.g_off;
  const V2* G2 = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + (dual ? sg.g_off2 : sg.g_off);
  int lo, hi;
  tile_span(bt, 16 * ct, n, lo, hi);
  const int k0 = lo & ~3, nks = (hi - k0 + 3) / 4;
  const int c = 16 * ct + li;
  V2 gf[KS], gf2[KS];
  {
    const BlkOf cb = blk_lookup(bt, min(c, n - 1));
    const int cc = min(c, n - 1) - cb.off;
    // every lane loads an in-block address and zeroes what lies outside: no branches
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kk = k0 + 4 * ks + kq - cb.off;
      const bool in_b = act && ks < nks && c < n && kk >= 0 && kk < cb.sz;
      const int ge = cb.po + (in_b ? kk : 0) * cb.sz + cc;
      const V2 g = G[ge], g2 = G2[ge];
      gf[ks] = in_b ? g : V2{0, 0};
      gf2[ks] = in_b ? g2 : V2{0, 0};
    }
  }
  const V2* in = reinterpret_cast<const V2*>(bases.p[sg.inbuf]) + sg.in_off;
  V2* out = reinterpret_cast<V2*>(bases.p[sg.outbuf]) + sg.out_off;
  V2* out2 = reinterpret_cast<V2*>(bases.p[sg.outbuf]) + (dual ? sg.out_off2 : sg.out_off);
  R pfx[PF], pfy[PF];   // real and imaginary parts apart: arrays of scalars stay in registers
  auto height = [&](int ch) { return min(ROWS, sg.nrows - ROWS * ch); };
  // physical element offset of logical row r (rows in groups of rw, ld apart, when rw > 0)
  const int rw = sg.rw;
  const int64_t gstride = int64_t(sg.ld) * n;
  auto prow = [&](int r) -> int64_t {
    if (rw <= 0) return int64_t(r) * n;
    const int g = r / rw;
    return g * gstride + int64_t(r - g * rw) * n;
  };
  auto fetch = [&](int ch) {   // past the chunk's end every lane reloads element 0: no branches
    const int ne = height(ch) * n;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = tid + 512 * t, ec = e < ne ? e : 0, r = ec / n;
      const V2 v = in[prow(ROWS * ch + r) + (ec - r * n)];
      pfx[t] = v.x;
      pfy[t] = v.y;
    }
  };
  auto stash = [&](int ch) {
    const int ne = height(ch) * n;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = tid + 512 * t;
      if (e < ne) {
        const int r = e / n;
        rows[r * ld + (e - r * n)] = V2{pfx[t], pfy[t]};
      }
    }
  };
  fetch(c0);
  stash(c0);
  if (c0 + 1 < c1) fetch(c0 + 1);
  __syncthreads();
  for (int ch = c0; ch < c1; ++ch) {
    const int nr = height(ch), nrt = (nr + 15) / 16;
    if (act) {
      for (int rt = rj; rt < nrt; rt += rstep) {   // uniform
        const V2* arow = rows + min(16 * rt + li, nr - 1) * ld;
        // one output at a time with three real products each (3M): the two outputs of a dual
        // segment read the chunk's rows from LDS twice, which costs less than a fourth
        // product and a second set of accumulators
        auto product = [&](const V2 (&g)[KS], V2* o) __attribute__((always_inline)) {
          A4 cr = A4{0, 0, 0, 0}, ci = cr, cx = cr;
          // each step's LDS read is issued one step ahead (addresses clamped into the row)
          V2 an = arow[min(k0 + kq, n - 1)];
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            if (ks < nks) {   // uniform
              const int k = k0 + 4 * ks + kq;
              V2 a = an;
              if (ks + 1 < KS) an = arow[min(k + 4, n - 1)];
              if (k >= n) a = V2{0, 0};
              cmma<V2>(a, a.x + a.y, g[ks], g[ks].x + g[ks].y, cr, ci, cx);
            }
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int r = 16 * rt + M::row(lane, j);
            if (c < n && r < nr) o[prow(ROWS * ch + r) + c] = cval<V2>(cr, ci, cx, j);
          }
        };
        product(gf, out);
        if (dual) product(gf2, out2);
      }
    }
    if (ch + 1 < c1) {
      __syncthreads();   // every wave is done with this chunk's rows
      stash(ch + 1);
      if (ch + 2 < c1) fetch(ch + 2);
      __syncthreads();
    }
  }
}

void launch_rowblock_right(const RowSegList& l, const Bases& b, const int* btab, int ncol, hipStream_t s, bool fp32) {
  if (l.nseg == 0) return;
  const int rows = ncol <= 52 ? 128 : 64;   // rows per chunk (the n > 52 form keeps its registers)
  const int nch = (l.maxrows + rows - 1) / rows;   // chunks of the tallest segment
  // about sixteen workgroups per CU over the launch, each walking `per` chunks of one segment
  const int ptarget = int(std::max<long>(1, std::min<long>(nch, long(nch) * l.nseg / 4096)));
  const int parts = (nch + ptarget - 1) / ptarget;
  const int per = (nch + parts - 1) / parts;
  const dim3 g(parts, l.nseg);
  const RowSeg* sg = (const RowSeg*)l.segs;
  const size_t lds = size_t(rows) * (ncol + 1) * (fp32 ? sizeof(float2) : sizeof(double2));
  if (ncol <= 52) {   // 128 rows x 52 over 512 threads: 13 elements each
    if (fp32) hipLaunchKernelGGL((k_bd_right<float2, 13, 13, 128>), g, dim3(512), lds, s, sg, b, btab, ncol, per);
    else hipLaunchKernelGGL((k_bd_right<double2, 13, 13, 128>), g, dim3(512), lds, s, sg, b, btab, ncol, per);
  } else {            // 64 rows x 64 over 512 threads: 8 elements each
    if (fp32) hipLaunchKernelGGL((k_bd_right<float2, 16, 8, 64>), g, dim3(512), lds, s, sg, b, btab, ncol, per);
    else hipLaunchKernelGGL((k_bd_right<double2, 16, 8, 64>), g, dim3(512), lds, s, sg, b, btab, ncol, per);
  }
}

// ---------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------
// k_bd_both: W_s = Gl^H X_s Gr^H for the matrices s of one segment (a slab of n rows and
// na n columns, matrix s in columns [s n, (s + 1) n)).  A workgroup of eight waves walks `per`
// consecutive groups of S matrices (S n <= 64) of one segment.  Each wave loads its fragments
// of Gr^H (one column tile) and Gl^H (one row tile) once and keeps them for every group; a
// group's slice of X is loaded into registers while the previous group is being multiplied,
// then stored to LDS (X), the right product goes to a second LDS buffer (Y) and the left
// product straight to global memory.
// KS: K steps of the widest tile (n <= 4 KS); PF: slice elements per thread, n (S n) / 512.
constexpr int BOTH_WAVES = 8;

template <typename V2, int KS, int PF>
__global__ __launch_bounds__(512) void k_bd_both(const RowSeg* __restrict__ segs, Bases bases,
                                                 const int* __restrict__ btab, int n, int S, int per) {
  using M = Mf<V2>;
  using R = typename M::R;
  using A4 = typename M::A4;
  extern __shared__ double2 lds_both[];
  const RowSeg sg = segs[blockIdx.y];
  const int wseg = sg.nrows;   // matrices of n columns side by side; row stride ncols
  const int64_t ncols = sg.ld > 0 ? sg.ld : wseg;
  const int nmat = wseg / n, ngrp = (nmat + S - 1) / S;
  const int g0 = blockIdx.x * per;
  if (g0 >= ngrp) return;
  const int g1 = min(ngrp, g0 + per);
  const int ld = S * n + 1;
  V2* X = reinterpret_cast<V2*>(lds_both);
  V2* Y = X + n * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, kq = lane >> 4;
  const V2* in = reinterpret_cast<const V2*>(bases.p[sg.inbuf]) + sg.in_off;
  V2* out = reinterpret_cast<V2*>(bases.p[sg.outbuf]) + sg.out_off;
  const V2* Gl = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + sg.g_off;
  const V2* Gr = reinterpret_cast<const V2*>(bases.p[sg.gbuf]) + sg.g_off2;
  const int* btl = btab + sg.blk;
  const int* btr = btab + sg.blk2;

  // ---- held fragments.  Right product: wave -> column tile ctr = wave mod nct, row tiles
  // wave / nct + rstep j.  Left product: wave -> row tile rtl = wave mod nrt2, column tiles
  // wave / nrt2 + cstep j.  nct, nrt2 <= 4, so each wave has at most two items per pass.
  const int nct = (n + 15) / 16, rstep = BOTH_WAVES / nct;
  const int nrt2 = nct, cstep = rstep;
  const bool act = wave < rstep * nct;   // waves beyond the last full round have no items
  const int ctr = wave % nct, rtl = wave % nrt2;
  int k0r, nksr, k0l, nksl;
  V2 gr[KS], gl[KS];
  {
    int lo, hi;
    tile_span(btr, 16 * ctr, n, lo, hi);
    k0r = lo & ~3;
    nksr = (hi - k0r + 3) / 4;
    const int c = 16 * ctr + li;
    const BlkOf cb = blk_lookup(btr, min(c, n - 1));
    const int cc = min(c, n - 1) - cb.off;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kk = k0r + 4 * ks + kq - cb.off;
      const bool ok = act && ks < nksr && c < n && kk >= 0 && kk < cb.sz;
      V2 g = Gr[cb.po + cc * cb.sz + (ok ? kk : 0)];   // (Gr^H)[k][c] = conj Gr[c][k]
      g.y = -g.y;
      gr[ks] = ok ? g : V2{0, 0};
    }
    tile_span(btl, 16 * rtl, n, lo, hi);
    k0l = lo & ~3;
    nksl = (hi - k0l + 3) / 4;
    const int ap = 16 * rtl + li;
    const BlkOf rb = blk_lookup(btl, min(ap, n - 1));
    const int aa = min(ap, n - 1) - rb.off;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kk = k0l + 4 * ks + kq - rb.off;
      const bool ok = act && ks < nksl && ap < n && kk >= 0 && kk < rb.sz;
      V2 g = Gl[rb.po + (ok ? kk : 0) * rb.sz + aa];   // (Gl^H)[a'][k] = conj Gl[k][a']
      g.y = -g.y;
      gl[ks] = ok ? g : V2{0, 0};
    }
  }

  // ---- slices: element e = a w + j of group g (w = matrices of the group times n)
  R pfx[PF], pfy[PF];   // real and imaginary parts apart: arrays of scalars stay in registers
  auto width = [&](int g) { return min(S, nmat - g * S) * n; };
  auto fetch = [&](int g) {   // past the slice's end every lane reloads element 0: no branches
    const int w = width(g);
    const V2* src = in + int64_t(g) * S * n;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = tid + 512 * t, ec = e < n * w ? e : 0;
      const int a = ec / w, j = ec - a * w;
      const V2 v = src[int64_t(a) * ncols + j];
      pfx[t] = v.x;
      pfy[t] = v.y;
    }
  };
  auto stash = [&](int g) {
    const int w = width(g);
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = tid + 512 * t;
      if (e < n * w) {
        const int a = e / w, j = e - a * w;
        X[a * ld + j] = V2{pfx[t], pfy[t]};
      }
    }
  };
  fetch(g0);
  stash(g0);
  if (g0 + 1 < g1) fetch(g0 + 1);
  __syncthreads();
  for (int g = g0; g < g1; ++g) {
    const int w = width(g), nrt = (w + 15) / 16;
    // right: Y[a][s n + c] = sum_b X[a][s n + b] Gr^H[b][c], rows r = s n + a of [0, w)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int rt = wave / nct + rstep * jt;
      if (!act || rt >= nrt) break;   // uniform per wave
      const int r = min(16 * rt + li, w - 1), s = r / n, a = r - s * n;
      const V2* arow = X + a * ld + s * n;
      A4 cr = A4{0, 0, 0, 0}, ci = cr, cx = cr;
      // each step's LDS read is issued one step ahead (addresses clamped into the row)
      V2 xn = arow[min(k0r + kq, n - 1)];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks < nksr) {
          const int k = k0r + 4 * ks + kq;
          V2 x = xn;
          if (ks + 1 < KS) xn = arow[min(k + 4, n - 1)];
          if (k >= n) x = V2{0, 0};
          cmma<V2>(x, x.x + x.y, gr[ks], gr[ks].x + gr[ks].y, cr, ci, cx);
        }
      }
      const int c = 16 * ctr + li;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = 16 * rt + M::row(lane, j);
        if (c < n && rr < w) {
          const int s2 = rr / n, a2 = rr - s2 * n;
          Y[a2 * ld + s2 * n + c] = cval<V2>(cr, ci, cx, j);
        }
      }
    }
    __syncthreads();   // Y complete, X free
    if (g + 1 < g1) {
      stash(g + 1);
      if (g + 2 < g1) fetch(g + 2);
    }
    // left: W[a'][s n + b] = sum_a Gl^H[a'][a] Y[a][s n + b], to global memory
    V2* dst = out + int64_t(g) * S * n;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int ct = wave / nrt2 + cstep * jt;
      if (!act || ct >= nrt) break;   // column tiles of the group: same count as row tiles above
      const int jc = min(16 * ct + li, w - 1);
      A4 cr = A4{0, 0, 0, 0}, ci = cr, cx = cr;
      V2 yn = Y[min(k0l + kq, n - 1) * ld + jc];   // one step ahead, as above
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks < nksl) {
          const int k = k0l + 4 * ks + kq;
          V2 y = yn;
          if (ks + 1 < KS) yn = Y[min(k + 4, n - 1) * ld + jc];
          if (k >= n) y = V2{0, 0};
          cmma<V2>(gl[ks], gl[ks].x + gl[ks].y, y, y.x + y.y, cr, ci, cx);
        }
      }
      const int jj = 16 * ct + li;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = 16 * rtl + M::row(lane, j);
        if (a < n && jj < w) dst[int64_t(a) * ncols + jj] = cval<V2>(cr, ci, cx, j);
      }
    }
    __syncthreads();   // Y free, the next slice in X
  }
}

// groups of S matrices: the right product's rows (s, a) fill at most four 16-row tiles
inline int both_S(int n) { return std::max(1, 64 / n); }

void launch_rowblock_both(const RowSegList& l, const Bases& b, const int* btab, int n, hipStream_t s, bool fp32) {
  if (l.nseg == 0) return;
  const int S = both_S(n);
  const int ngrp = (l.maxrows / n + S - 1) / S;   // groups of the widest segment
  // about sixteen workgroups per CU over the launch, each walking `per` groups of one segment
  const int ptarget = int(std::max<long>(1, std::min<long>(ngrp, long(ngrp) * l.nseg / 4096)));
  const int parts = (ngrp + ptarget - 1) / ptarget;
  const int per = (ngrp + parts - 1) / parts;
  const dim3 g(parts, l.nseg);
  const RowSeg* sg = (const RowSeg*)l.segs;
  const size_t lds = 2 * size_t(n) * (S * n + 1) * (fp32 ? sizeof(float2) : sizeof(double2));
  // n <= 52: n (S n) <= 52 * 52 (S = 1) or 64 * 32 (S >= 2), six elements per thread
  if (n <= 52) {
    if (fp32) hipLaunchKernelGGL((k_bd_both<float2, 13, 6>), g, dim3(512), lds, s, sg, b, btab, n, S, per);
    else hipLaunchKernelGGL((k_bd_both<double2, 13, 6>), g, dim3(512), lds, s, sg, b, btab, n, S, per);
  } else {
    if (fp32) hipLaunchKernelGGL((k_bd_both<float2, 16, 8>), g, dim3(512), lds, s, sg, b, btab, n, S, per);
    else hipLaunchKernelGGL((k_bd_both<double2, 16, 8>), g, dim3(512), lds, s, sg, b, btab, n, S, per);
  }
}

}  // namespace gw
