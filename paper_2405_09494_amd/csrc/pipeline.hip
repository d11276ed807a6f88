// Device-side orchestration of libgwsym: memory, the precomputed work lists of every stage
// and the order of launches.  All work lists are built once (device_init / load_V) with
// buffer ids and element offsets; each call only passes the current base pointers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <unordered_map>
#include <mutex>
#include <cmath>
#include <atomic>
#include <thread>
#include <cstdlib>
#include <cstdio>
#include <chrono>
#include <cstring>
#include <numeric>
#include <tuple>

#include "kernel_api.hpp"

namespace gw {

namespace {
// GWSYM_VERBOSE set in the environment: host set-up phases print their wall time to stderr
struct PhaseClock {
  bool on = std::getenv("GWSYM_VERBOSE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[gwsym] %s: %.2f s\n", what, std::chrono::duration<double>(now - t).count());
    t = now;
  }
};
}  // namespace

namespace {

struct Range {
  int t0 = 0, nt = 0, r0 = 0, nr = 0;
  double macs = 0;   // complex multiply-accumulates requested by the launch
  double bytes = 0;  // algorithmic bytes moved (memory-bound launches)
  int shape[4] = {0, 0, 0, 0};   // wave-tile launches: tiles per shape class, in list order
  int kdepth = 32;               // k values per bfloat16 MFMA in the split-bfloat16 forms
  int prefetch = 2;              // FP64 / FP32: K sub-steps per group of the wave-tile GEMM
  int lists = 0;                 // wave-tile launches: tiles walk K-segment lists
};

// Workgroup p of a launch runs on XCD p % 8, and each XCD has its own L2.  Tiles that read
// the same operand rows (the same A rows over the same outer range, or the same B columns)
// are gathered into one group, each group is given to the least loaded XCD, and the list is
// interleaved so that a group's tiles run on that XCD one after another.  Short queues are
// padded with empty tiles (prob = -1).
// mode 2: every problem (with its batch and outer range) is one group, its tiles ordered by
// column chunk and then row tile, so the row tiles that read the same B columns run together.
inline void xcd_order_tiles(std::vector<GemmTile>& tiles, int t0, const std::vector<GemmProblem>& probs,
                            int mode = 1) {
  constexpr int NX = 8;
  const int n = int(tiles.size()) - t0;
  if (n <= NX) return;
  // mode 3: a band of BAND row tiles of one problem (and outer range) is one group, swept column
  // chunk by column chunk: the band's row panels of A stay in L2 while each column panel of B
  // is read once for the whole band
  constexpr int BAND = 8;
  if (mode == 2)
    std::stable_sort(tiles.begin() + t0, tiles.end(), [](const GemmTile& a, const GemmTile& b) {
      return std::make_tuple(a.prob, a.batch, a.t0, a.tn, a.tm) < std::make_tuple(b.prob, b.batch, b.t0, b.tn, b.tm);
    });
  if (mode == 3)
    std::stable_sort(tiles.begin() + t0, tiles.end(), [](const GemmTile& a, const GemmTile& b) {
      return std::make_tuple(a.prob, a.batch, a.t0, a.tm / (2 * BAND), a.tn, a.tm) <
             std::make_tuple(b.prob, b.batch, b.t0, b.tm / (2 * BAND), b.tn, b.tm);
    });
  using Key = std::array<i64, 5>;
  struct KeyHash {
    size_t operator()(const Key& k) const {
      uint64_t h = 0x9e3779b97f4a7c15ull;
      for (i64 v : k) h = (h ^ uint64_t(v)) * 0x100000001b3ull + (h >> 29);
      return size_t(h);
    }
  };
  using Count = std::unordered_map<Key, int, KeyHash>;
  auto keyA = [&](const GemmTile& t) {
    const GemmProblem& p = probs[t.prob];
    return Key{p.abuf, p.aoff + i64(t.batch) * p.sAb, t.tm, t.t0, 0};
  };
  auto keyB = [&](const GemmTile& t) {
    const GemmProblem& p = probs[t.prob];
    return Key{p.bbuf, p.boff + i64(t.batch) * p.sBb, t.tn, t.t0, 1};
  };
  // hashed counts: the lists reach millions of tiles at the 6x6x6 workloads
  Count ca, cb;
  ca.reserve(size_t(n));
  cb.reserve(size_t(n));
  for (int i = t0; i < int(tiles.size()); ++i) {
    ca[keyA(tiles[i])]++;
    cb[keyB(tiles[i])]++;
  }
  Count gid;
  std::vector<std::vector<int>> groups;
  // a problem whose operands fit in an L2 comfortably keeps all its tiles on one XCD
  auto small = [&](const GemmTile& t) {
    const GemmProblem& p = probs[t.prob];
    return 16.0 * double(p.K) * p.T * (double(p.M) + p.N) <= 1.0e6;
  };
  for (int i = t0; i < int(tiles.size()); ++i) {
    const Key ka = keyA(tiles[i]), kb = keyB(tiles[i]);
    const Key k = mode == 3 ? Key{tiles[i].prob, tiles[i].batch, tiles[i].t0, tiles[i].tm / (2 * BAND), 3}
                  : mode == 2 || small(tiles[i]) ? Key{tiles[i].prob, tiles[i].batch, mode == 2 ? tiles[i].t0 : 0, 0, 2}
                                                 : (ca[ka] >= cb[kb] ? ka : kb);
    auto it = gid.find(k);
    if (it == gid.end()) {
      it = gid.emplace(k, int(groups.size())).first;
      groups.emplace_back();
    }
    groups[it->second].push_back(i);
  }
  std::vector<std::vector<int>> q(NX);
  for (const auto& g : groups) {
    int x = 0;
    for (int y = 1; y < NX; ++y)
      if (q[y].size() < q[x].size()) x = y;
    q[x].insert(q[x].end(), g.begin(), g.end());
  }
  size_t len = 0;
  for (const auto& v : q) len = std::max(len, v.size());
  std::vector<GemmTile> out;
  out.reserve(len * NX);
  for (size_t i = 0; i < len; ++i)
    for (int x = 0; x < NX; ++x) {
      if (i < q[x].size()) out.push_back(tiles[q[x][i]]);
      else out.push_back(GemmTile{-1, 0, 0, 0, 0, 0, -1, 1, 1, 0});
    }
  tiles.resize(t0);
  tiles.insert(tiles.end(), out.begin(), out.end());
}

struct GemmStage {
  std::vector<GemmProblem> probs;
  std::vector<GemmTile> tiles;
  std::vector<GemmReduce> reds;
  std::vector<Range> launches;
  std::vector<int> pending;   // problems of the launch being built
  std::vector<KSeg> klist;    // K-segment lists of the problems that have one
  void* d_probs = nullptr;
  void* d_tiles = nullptr;
  void* d_reds = nullptr;
  void* d_klist = nullptr;
  int max_slots = 0;
  double macs = 0;

  // algo_macs: the multiply-accumulates the algorithm needs when the problem computes more
  // (e.g. zero off-diagonal blocks); by default the problem's own M N K T batch.  The
  // algorithmic bytes of a problem are one read of each operand and one write of C, in
  // complex128 (the fused block-diagonal factor is small and cached).
  // herm: the problem's output is Hermitian within each column batch (C[r][c] with c taken
  // modulo cdiv); only the tiles that touch its lower triangle are generated, and the caller
  // fills the upper triangle afterwards
  std::vector<char> herm;
  void add(const GemmProblem& p, double algo_macs = -1.0, bool lower_only = false) {
    pending.push_back(int(probs.size()));
    probs.push_back(p);
    herm.push_back(lower_only ? 1 : 0);
    const double m = algo_macs >= 0 ? algo_macs : double(p.M) * p.N * p.K * double(p.T) * p.batch;
    macs += m;
    pending_macs += m;
    pending_bytes += 16.0 * p.batch * (double(p.K) * p.T * (double(p.M) + p.N) + double(p.M) * p.N);
  }
  double pending_macs = 0, pending_bytes = 0;
  // Closes a launch: records its problems and the plan settings; the tiles are made later by
  // finalize(), for every closed launch at once (in parallel), in launch order.
  bool wave = false;   // tiles for the wave-tile kernel: 32-column chunks, more of them
  // wave-tile plan: workgroups a launch aims for, 32-column chunks per tile, XCD order,
  // bfloat16 k depth (0: per launch)
  int target = 8192, per = 1, kdepth = 0, prefetch = 2;
  int xcd = 1;   // 0 plain order, 1 grouped by shared operand rows, 2 grouped by problem
  struct Deferred {
    std::vector<int> ids;
    int target, per, kdepth, prefetch, xcd;
    bool wave;
  };
  std::vector<Deferred> deferred;   // launches [built, launches.size()) not yet made into tiles
  size_t built = 0;
  void close() {
    Range r;
    r.macs = pending_macs;
    r.bytes = pending_bytes;
    pending_macs = 0;
    pending_bytes = 0;
    launches.push_back(r);
    deferred.push_back({std::move(pending), target, per, kdepth, prefetch, xcd, wave});
    pending.clear();
  }
  // One launch's tiles (problems with a long outer loop split so that the launch has about
  // `target` workgroups) and split-K reductions, with slot numbers local to the launch.
  struct Built {
    std::vector<GemmTile> tiles;
    std::vector<GemmReduce> reds;
    int shape[4] = {0, 0, 0, 0};
    int kdepth = 32, slots = 0, lists = 0;
  };
  // A launch walks its problems' K-segment lists only where they leave out at least a fifth of
  // the k steps (of 4) of the full outer range, counted over its output tiles: a list entry
  // costs branches and scalar loads in the k loop, which a bandwidth-bound launch pays for.
  bool walk_lists(const Deferred& L) const {
    double full = 0, kept = 0;
    for (int id : L.ids) {
      const GemmProblem& p = probs[id];
      if (p.kseg < 0) return false;
      const double w = double(p.batch) * ((p.M + 15) / 16) * ((p.N + 15) / 16);
      full += w * p.T * ((p.K + 3) / 4);
      for (int e = 0; e < p.nkseg; ++e) {
        const KSeg& q = klist[size_t(p.kseg) + e];
        kept += w * q.np * ((q.ke - q.kb + 3) / 4);
      }
    }
    return full > 0 && kept <= 0.8 * full;
  }
  Built build(const Deferred& L) const {
    const int target = L.wave ? L.target : 2048;
    Built out;
    std::vector<GemmTile>& tiles = out.tiles;
    std::vector<GemmReduce>& reds = out.reds;
    // tiles of 32 rows (columns), the last one 16 when the remainder allows
    auto units = [](int n) { return (n + 15) / 16; };
    long base = 0;
    for (int id : L.ids) {
      const GemmProblem& p = probs[id];
      base += long(p.batch) * ((units(p.M) + 1) / 2) * ((units(p.N) + 1) / 2);
    }
    int slots = 0;
    // a tile of rows [16 i, 16 (i + mh)) and columns [16 j, 16 (j + nn)) of a lower-only problem
    // is needed when some row r and column c in it have r >= c mod cdiv
    auto keep = [&](int id, int i, int mh, int j, int nn) {
      const GemmProblem& p = probs[id];
      if (!herm[id]) return true;
      const int rmax = std::min(16 * (i + mh), p.M) - 1;
      const int c0 = 16 * j, c1 = std::min(16 * (j + nn), p.N);
      const int cmin = (c0 / p.cdiv != (c1 - 1) / p.cdiv) ? 0 : c0 % p.cdiv;
      return rmax >= cmin;
    };
    std::vector<long> pre;
    out.lists = L.wave && walk_lists(L);
    for (int id : L.ids) {
      const GemmProblem& p = probs[id];
      const int mu = units(p.M), nu = units(p.N);
      // with lists a problem splits its entries (cut where the k sub-steps before them reach
      // s / split of the total), without them its outer range
      const bool lst = out.lists;
      const int tn = lst ? p.nkseg : p.T;
      if (lst) {
        pre.assign(size_t(tn) + 1, 0);
        for (int e = 0; e < tn; ++e) {
          const KSeg& q = klist[size_t(p.kseg) + e];
          pre[e + 1] = pre[e] + long(q.np) * ((q.ke - q.kb + 3) / 4);
        }
      }
      auto cut = [&](int s, int split) {
        if (!lst) return int(long(s) * tn / split);
        const long goal = (pre[tn] * s + split - 1) / split;
        return int(std::lower_bound(pre.begin(), pre.end(), goal) - pre.begin());
      };
      auto nsub = [&](int t0, int t1) { return lst ? int(pre[t1] - pre[t0]) : 0; };
      int split = 1;
      if (base < target && tn >= 8)
        split = int(std::min<long>(std::min<long>(tn / 4, 256), (target + base - 1) / std::max(1L, base)));
      split = std::max(1, split);
      // the parts' first entries, without empty parts (a list cut at sub-step quantiles can
      // give two equal cut points)
      std::vector<int> cuts{0};
      for (int s = 1; s <= split; ++s) {
        const int x = cut(s, split);
        if (x > cuts.back() || s == split) cuts.push_back(x);
      }
      if (cuts.size() > 2 && cuts[cuts.size() - 1] == cuts[cuts.size() - 2]) cuts.pop_back();
      split = int(cuts.size()) - 1;
      const int whole = nsub(0, tn);
      for (int b = 0; b < p.batch; ++b)
        for (int i = 0; i < mu; i += 2) {
          const int mh = std::min(2, mu - i);
          if (split == 1) {
            if (L.wave) {
              // one full 32-column chunk per wave (a wave can walk several: nn = 2 x chunks),
              // a last 16-column unit on its own
              const int full = nu / 2;
              for (int j = 0; j < full; j += L.per) {
                const int nn = 2 * std::min(L.per, full - j);
                if (keep(id, i, mh, 2 * j, nn)) tiles.push_back({id, b, i, 2 * j, 0, tn, -1, mh, nn, whole});
              }
              if (nu % 2 && keep(id, i, mh, 2 * full, 1)) tiles.push_back({id, b, i, 2 * full, 0, tn, -1, mh, 1, whole});
              continue;
            }
            for (int j = 0; j < nu; j += 16)   // up to eight 32-column chunks per workgroup
              if (keep(id, i, mh, j, std::min(16, nu - j)))
                tiles.push_back({id, b, i, j, 0, tn, -1, mh, std::min(16, nu - j), whole});
            continue;
          }
          for (int j = 0; j < nu; j += 2) {
            const int nh = std::min(2, nu - j);
            if (!keep(id, i, mh, j, nh)) continue;
            const int s0 = slots;
            for (int s = 0; s < split; ++s) {
              const int t0 = cuts[s], t1 = cuts[s + 1];
              tiles.push_back({id, b, i, j, t0, t1, s0 + s, mh, nh, nsub(t0, t1)});
            }
            reds.push_back({id, b, i, j, s0, split, mh, nh});
            slots += split;
          }
        }
    }
    if (L.wave) {
      // sort by shape class (rows 32? columns 32?), each class in XCD order of its own
      std::vector<GemmTile> all(std::move(tiles));
      tiles.clear();
      for (int sh = 0; sh < 4; ++sh) {
        const int c0 = int(tiles.size());
        for (const GemmTile& t : all)
          if ((t.mh == 2) * 2 + (t.nn >= 2) == sh) tiles.push_back(t);
        if (L.xcd) xcd_order_tiles(tiles, c0, probs, L.xcd);
        out.shape[sh] = int(tiles.size()) - c0;
      }
    } else {
      xcd_order_tiles(tiles, 0, probs);
    }
    // k depth of the bfloat16 MFMA: a tile walks ceil(K/4) sub-steps per outer index in groups
    // of 8 (32-deep) or 4 (16-deep), the last group padded; 16-deep where 32 would pad more
    // than a quarter of the work
    double sub = 0, pad8 = 0;
    for (size_t t = 0; t < tiles.size(); ++t) {
      const GemmTile& tl = tiles[t];
      if (tl.prob < 0) continue;
      const double n = out.lists ? double(tl.nsub) : double(tl.t1 - tl.t0) * ((probs[tl.prob].K + 3) / 4);
      sub += n;
      pad8 += 8.0 * std::ceil(n / 8.0);
    }
    out.kdepth = L.kdepth ? L.kdepth : pad8 > 1.25 * sub ? 16 : 32;
    out.slots = slots;
    return out;
  }
  void finalize() {
    const size_t n0 = built, n = launches.size();
    if (n == n0) return;
    std::vector<Built> out(n - n0);
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<size_t> next{0};
    auto work = [&]() {
      for (size_t i; (i = next.fetch_add(1)) < out.size();) out[i] = build(deferred[i]);
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < std::min<size_t>(nth, out.size()); ++t) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    for (size_t i = 0; i < out.size(); ++i) {
      Range& r = launches[n0 + i];
      const Deferred& L = deferred[i];
      r.t0 = int(tiles.size());
      r.r0 = int(reds.size());
      tiles.insert(tiles.end(), out[i].tiles.begin(), out[i].tiles.end());
      reds.insert(reds.end(), out[i].reds.begin(), out[i].reds.end());
      r.nt = int(tiles.size()) - r.t0;
      r.nr = int(reds.size()) - r.r0;
      for (int sh = 0; sh < 4; ++sh) r.shape[sh] = out[i].shape[sh];
      r.kdepth = out[i].kdepth;
      r.prefetch = L.prefetch;
      r.lists = out[i].lists;
      max_slots = std::max(max_slots, out[i].slots);
    }
    deferred.clear();
    built = n;
  }
};

struct RowStage {
  std::vector<RowSeg> segs;
  std::vector<Range> launches;  // t0 = first segment, nt = count, r0 = max rows
  void* d = nullptr;
  int start = 0, maxr = 0;
  double macs = 0, bytes = 0;
  // m: complex MACs; the slab is read and written once: 32 bytes per complex element
  void add(const RowSeg& s, double m, double elems) {
    segs.push_back(s);
    maxr = std::max(maxr, s.nrows);
    macs += m;
    bytes += 32.0 * elems;
  }
  void close() {
    Range r;
    r.t0 = start;
    r.nt = int(segs.size()) - start;
    r.r0 = maxr;
    r.macs = macs;
    r.bytes = bytes;
    launches.push_back(r);
    start = int(segs.size());
    maxr = 0;
    macs = 0;
    bytes = 0;
  }
};

// Live per-class timing with HIP events on the launch stream (enabled on request).
enum ProfClass { PC_P0 = 0, PC_SA, PC_SC, PC_RIGHT, PC_LEFT, PC_XFORM, PC_INV, PC_OTHER, PC_N };

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> recs;
  double macs[PC_N] = {};
  double bytes[PC_N] = {};
};

template <class T>
struct ListStage {
  std::vector<T> items;
  std::vector<Range> launches;
  void* d = nullptr;
  int start = 0;
  int nmax = 0;   // inverse lists: largest matrix
  void close() {
    Range r;
    r.t0 = start;
    r.nt = int(items.size()) - start;
    launches.push_back(r);
    start = int(items.size());
  }
};

}  // namespace

struct DevState {
  // tables
  void* U = nullptr;        // U_ao [nk][nao][nao] then U_aux [nk][naux][naux]
  void* TR = nullptr;       // Tf, Tb [nw][ntau]; Bf, Bb [ntau][nw]
  double* tau = nullptr;
  int* btab = nullptr;
  std::vector<int> bt_ao, bt_aux;   // offsets into btab per irreducible point
  double* wts = nullptr;            // star weight per g0 item
  // V
  void* VP = nullptr;
  void* VS = nullptr;
  void* VP32 = nullptr;     // FP32 copies for the FP32 contraction mode
  void* VS32 = nullptr;
  void* G32 = nullptr;
  void* P32 = nullptr;
  void* WT = nullptr;       // per-pair rotation matrices for the polarization copy of V
  // workspaces
  void* W1 = nullptr;
  void* W2 = nullptr;
  size_t ws_elems = 0;
  size_t ws_min = 0;        // workspace elements the non-contraction stages need
  size_t scr_tau = 0;       // tau slabs SCR holds
  bool ws_exact = false;    // the next plan sizes the workspaces exactly (also shrinks them)
  void* partials = nullptr;
  size_t nslots = 0, partial_cap = 0;
  double* mu_state = nullptr;  // mu state (3), eps range (2), internal n_free (1)
  double* trace = nullptr;
  double* occ = nullptr;
  double* erange = nullptr;
  void* vwork = nullptr;     // Jacobi eigenvectors, JAC_N^2 complex per g0 item
  int* status = nullptr;
  int tau_chunk = 1;
  // stages
  GemmStage p0_gemm, s_gemmA, s_gemmC, scr_fwd, scr_bwd, dys_fwd, dys_bwd, tb_1[3], tb_2[3], fb_1[3], fb_2[3];
  GemmStage lv1, lv2, lv3;
  RowStage p0_both, s_right;
  // exchange part of the static self-energy (eq. sigma_hf, K term), one launch set per k0
  GemmStage hx_gemm;
  RowStage hx_right;
  ListStage<CopySeg> hx_pack;
  // Hartree part (eq. sigma_hf, J term): diagonal blocks, per-point item ranges, weights,
  // the invariant-subspace projector of the auxiliary basis at q = 0 and two small buffers
  void* hj_items = nullptr;
  int* hj_first = nullptr;
  double* hj_w = nullptr;
  void* hj_proj = nullptr;
  void* hj_r = nullptr;
  void* hj_rho = nullptr;
  int hj_nitems = 0;
  ListStage<CopySeg> p0_mirror, scr_herm, dys_herm, s_pack;
  // launch order of the contractions: per step one block-multiply launch and ranges of GEMM
  // launches (one step per tau chunk; in the unbatched schedule one per pair)
  struct P0Step {
    int both, g0, g1;
  };
  struct SStep {
    int a0, a1, right, c0, c1;
  };
  std::vector<P0Step> p0_steps;
  std::vector<SStep> s_steps;
  std::vector<std::array<int, 3>> s_chunks;   // (first step, end step, gather launch) per chunk
  void* SCR = nullptr;      // full nao x nao self-energy products of one tau chunk
  ListStage<InvItem> scr_inv, dys_inv, mu_inv;
  ListStage<MuItem> mu_items;
  ListStage<EigItem> g0_items;
  std::vector<void*> allocs;
  Prof prof;
  hipGraphExec_t graph_exec = nullptr;   // captured iteration and the arguments it was captured with
  std::vector<const void*> graph_key;
  double graph_ntarget = 0;
};

namespace {

#define HIPCHECK(x)                                              \
  do {                                                           \
    hipError_t e_ = (x);                                         \
    if (e_ != hipSuccess) {                                      \
      c.err = std::string(#x " failed: ") + hipGetErrorString(e_); \
      return GWSYM_EHIP;                                         \
    }                                                            \
  } while (0)

int dalloc(Ctx& c, DevState& d, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    c.err = "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
    *p = nullptr;
    return GWSYM_ENOMEM;
  }
  d.allocs.push_back(*p);
  return GWSYM_OK;
}

template <class T>
int upload(Ctx& c, DevState& d, const std::vector<T>& v, void** p, hipStream_t s) {
  int st = dalloc(c, d, p, v.size() * sizeof(T));
  if (st) return st;
  if (!v.empty()) HIPCHECK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return GWSYM_OK;
}

int upload_stage(Ctx& c, DevState& d, GemmStage& g, hipStream_t s) {
  int st;
  g.finalize();
  if ((st = upload(c, d, g.klist, &g.d_klist, s))) return st;
  if ((st = upload(c, d, g.probs, &g.d_probs, s))) return st;
  if ((st = upload(c, d, g.tiles, &g.d_tiles, s))) return st;
  if ((st = upload(c, d, g.reds, &g.d_reds, s))) return st;
  d.nslots = std::max(d.nslots, size_t(g.max_slots));
  return GWSYM_OK;
}

GemmPlanDev plan_of(const GemmStage& g, const Range& r) {
  GemmPlanDev p;
  p.probs = g.d_probs;
  p.tiles = static_cast<GemmTile*>(g.d_tiles) + r.t0;
  p.reds = static_cast<GemmReduce*>(g.d_reds) + r.r0;
  p.ntiles = r.nt;
  p.nreds = r.nr;
  for (int i = 0; i < 4; ++i) p.shape[i] = r.shape[i];
  p.kdepth = r.kdepth;
  p.prefetch = r.prefetch;
  p.lists = r.lists;
  return p;
}

GemmProblem gp(int M, int N, int K, int T, int batch, int abuf, i64 aoff, i64 lda, i64 sAt, i64 sAb, int opA, int bbuf,
               i64 boff, i64 ldb, i64 sBt, i64 sBb, int opB, int cbuf, i64 coff, i64 ldc, i64 sCb, double are = 1.0,
               double aim = 0.0, int beta = 0) {
  GemmProblem p{};
  p.M = M; p.N = N; p.K = K; p.T = T; p.batch = batch;
  p.abuf = abuf; p.aoff = aoff; p.lda = lda; p.sAt = sAt; p.sAb = sAb; p.opA = opA;
  p.bbuf = bbuf; p.boff = boff; p.ldb = ldb; p.sBt = sBt; p.sBb = sBb; p.opB = opB;
  p.cbuf = cbuf; p.coff = coff; p.ldc = ldc; p.sCb = sCb;
  p.alpha_re = are; p.alpha_im = aim; p.beta = beta;
  p.rdiv = M; p.cdiv = N;
  p.kseg = -1;
  return p;
}

// mesh arithmetic
struct Mesh {
  int n;
  int idx(int a, int b, int c) const { return ((((a % n) + n) % n) * n + (((b % n) + n) % n)) * n + (((c % n) + n) % n); }
  void pt(int k, int m[3]) const { m[0] = k / (n * n); m[1] = (k / n) % n; m[2] = k % n; }
  int add(int k1, int k2) const { int a[3], b[3]; pt(k1, a); pt(k2, b); return idx(a[0] + b[0], a[1] + b[1], a[2] + b[2]); }
  int sub(int k1, int k2) const { int a[3], b[3]; pt(k1, a); pt(k2, b); return idx(a[0] - b[0], a[1] - b[1], a[2] - b[2]); }
};

i64 U_off(const Ctx& c, bool aux, int k) {
  return aux ? i64(c.nk) * c.nao * c.nao + i64(k) * c.naux * c.naux : i64(k) * c.nao * c.nao;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// The contraction work lists (eq. P0 / Alg. 3 and eq. sigma / Alg. 4) for the plan in
// c.tune: tau chunk, and per GEMM stage the workgroup target, tile width, XCD order and
// bfloat16 k depth.  Replaces the previous lists (their device copies are freed), grows the
// workspaces to the chunk and drops a captured iteration graph.

namespace {

void dfree(DevState& d, void*& p) {
  if (!p) return;
  hipFree(p);
  auto it = std::find(d.allocs.begin(), d.allocs.end(), p);
  if (it != d.allocs.end()) d.allocs.erase(it);
  p = nullptr;
}

void reset_gemm(DevState& d, GemmStage& g) {
  dfree(d, g.d_probs);
  dfree(d, g.d_tiles);
  dfree(d, g.d_reds);
  dfree(d, g.d_klist);
  g = GemmStage{};
  g.wave = true;
}

}  // namespace

int plan_contractions(Ctx& c, DevState& d, hipStream_t s) {
  const int nk = c.nk, no = c.nao, na = c.naux, nt = c.ntau, nib = c.nibz;
  int st;
  // the lists and workspaces being replaced may still be read by queued work on any stream
  if (d.p0_gemm.d_tiles) HIPCHECK(hipDeviceSynchronize());
  reset_gemm(d, d.p0_gemm);
  reset_gemm(d, d.s_gemmA);
  reset_gemm(d, d.s_gemmC);
  GemmStage* gs[3] = {&d.p0_gemm, &d.s_gemmA, &d.s_gemmC};
  for (int g = 0; g < 3; ++g) {
    gs[g]->target = c.tune.wg_target[g];
    gs[g]->per = c.tune.cols[g] / 32;
    gs[g]->xcd = c.tune.xcd_order[g];
    gs[g]->kdepth = c.tune.kdepth[g];
    gs[g]->prefetch = c.tune.prefetch[g];
  }
  for (RowStage* r : {&d.p0_both, &d.s_right}) {
    dfree(d, r->d);
    *r = RowStage{};
  }
  for (auto* l : {&d.p0_mirror, &d.s_pack}) {
    dfree(d, l->d);
    *l = ListStage<CopySeg>{};
  }
  d.p0_steps.clear();
  d.s_steps.clear();
  d.s_chunks.clear();
  for (int x = 4; x < 8; ++x) c.vt_stats[x] = 0;
  // unbatched: every pair's block multiply and every (pair, block) GEMM its own launch, in order
  const bool ub = c.prm.sched == GWSYM_SCHED_UNBATCHED;
  if (d.graph_exec) {
    hipGraphExecDestroy(d.graph_exec);
    d.graph_exec = nullptr;
    d.graph_key.clear();
  }

  // tau chunk: contraction workspaces hold J * nk * naux * nao^2 complex numbers each
  const i64 slab = i64(nk) * na * no * no;
  int J = c.tune.tau_chunk;
  if (J <= 0) {
    // 2 GB per workspace, or as many tau slabs as the workspaces hold anyway for the other
    // stages (the readout of P over every k)
    const double budget = std::max(2.0e9 / 16.0, double(d.ws_min));  // elements per workspace
    J = int(std::max(1.0, std::min(double(nt), budget / double(slab))));
  }
  J = std::min(J, nt);
  if (c.prm.half_tau && nt >= 2) J = std::max(J, 2);   // a tau and its mirror share a chunk
  d.tau_chunk = J;
  c.tune.tau_chunk = J;
  const int nthalf = c.prm.half_tau ? (nt + 1) / 2 : nt;
  const size_t ws = std::max(d.ws_min, size_t(J) * size_t(slab));
  if (ws > d.ws_elems || (d.ws_exact && ws < d.ws_elems)) {
    dfree(d, d.W1);
    dfree(d, d.W2);
    d.ws_elems = ws;
    if ((st = dalloc(c, d, &d.W1, d.ws_elems * 16))) return st;
    if ((st = dalloc(c, d, &d.W2, d.ws_elems * 16))) return st;
  }
  if (size_t(J) > d.scr_tau || (d.ws_exact && size_t(J) < d.scr_tau)) {
    dfree(d, d.SCR);
    d.scr_tau = size_t(J);
    if ((st = dalloc(c, d, &d.SCR, size_t(J) * no * no * 16))) return st;
  }

  PhaseClock clk;
  // maximal runs (first index, length) of consecutive leading blocks: the functions whose
  // values are computed (the others repeat an aligned partner block and are copied)
  auto lead_runs = [](const Blocks& B) {
    std::vector<std::pair<int, int>> runs;
    for (size_t r = 0; r < B.size.size(); ++r) {
      if (B.lead[r] != int(r)) continue;
      if (!runs.empty() && runs.back().first + runs.back().second == B.off[r]) runs.back().second += B.size[r];
      else runs.push_back({B.off[r], B.size[r]});
    }
    return runs;
  };
  Mesh mesh{c.n};
  // K-segment lists of the contractions that sum over orbital functions b of V (Sec. 4.3: only
  // the tiles of V that are not zero by symmetry take part).  For an outer index run (a run of
  // the orbital functions a, or of the auxiliary functions Q, of one block), the windows are the
  // runs of consecutive b blocks whose tiles are kept; without tile flags (V not loaded yet)
  // every tile is kept.  Windows that save less than a quarter of the run's k steps (of 4) are
  // replaced by the whole range: short entries cost more in list steps and partly filled k
  // steps than they save.  Entries of one list are merged while they continue each other with
  // the same window, up to 64 outer indices, so that a split of the sum has entries to cut at.
  const bool have_tiles = !c.vt_nz[0].empty();
  std::vector<std::pair<int, int>> win;
  auto windows = [&](const Blocks& Bb, auto&& kept) {
    win.clear();
    for (size_t r2 = 0; r2 < Bb.size.size(); ++r2) {
      if (!kept(int(r2))) continue;
      const int b0 = Bb.off[r2], b1 = b0 + Bb.size[r2];
      if (!win.empty() && win.back().second == b0) win.back().second = b1;
      else win.push_back({b0, b1});
    }
    int steps = 0;
    for (const auto& w : win) steps += (w.second - w.first + 3) / 4;
    if (!win.empty() && 4 * steps > 3 * ((no + 3) / 4)) win.assign(1, {0, no});
  };
  auto push_seg = [](GemmStage& g, size_t start, int t0, int np, int kb, int ke) {
    if (g.klist.size() > start) {
      KSeg& l = g.klist.back();
      if (l.kb == kb && l.ke == ke && l.t0 + l.np == t0 && l.np + np <= 64) {
        l.np += np;
        return;
      }
    }
    g.klist.push_back({t0, np, kb, ke});
  };
  // windows per piece; returns the list's entry count and adds the kept MACs per output
  // element pair of the problem (sum over entries of np (ke - kb)) to `kept`
  std::map<std::array<int, 4>, std::array<i64, 3>> p0_lists, s_lists;
  // polarization problem (i, aux block sg): pieces (k, a) for k in [k0, k0 + nkc), a at k, K = b
  // at k + q0; copy 1 of the tile flags
  auto p0_list = [&](GemmProblem& p, int i, int sg, int k0, int nkc, double& kept) {
    const std::array<int, 4> key{i, sg, k0, nkc};
    auto it = p0_lists.find(key);
    if (it == p0_lists.end()) {
      GemmStage& g = d.p0_gemm;
      const size_t start = g.klist.size();
      double mk = 0;
      const int q0 = c.ibz[i];
      for (int k = k0; k < k0 + nkc; ++k) {
        const Blocks& Ba = c.bao[c.rep[k]];
        const Blocks& Bb = c.bao[c.rep[mesh.add(k, q0)]];
        const int nra = int(Ba.size.size()), nrb = int(Bb.size.size());
        const uint8_t* nz = have_tiles ? c.vt_nz[1].data() + c.vt_off[1][size_t(i) * nk + k] : nullptr;
        for (int r = 0; r < nra; ++r) {
          windows(Bb, [&](int r2) { return !nz || nz[(size_t(sg) * nra + r) * nrb + r2]; });
          for (const auto& w : win) {
            push_seg(g, start, (k - k0) * no + Ba.off[r], Ba.size[r], w.first, w.second);
            mk += double(Ba.size[r]) * (w.second - w.first);
          }
        }
      }
      it = p0_lists.emplace(key, std::array<i64, 3>{i64(start), i64(g.klist.size() - start), i64(mk)}).first;
    }
    p.kseg = it->second[0];
    p.nkseg = int(it->second[1]);
    kept = double(it->second[2]);
  };
  // self-energy orbital problem (i, bin of k0's orbital functions [r0, r0 + nb)): pieces
  // (k', Q) for k' in [kp0, kp0 + nkc), Q at q = k0 - k', K = b at k'; copy 0 of the flags.  A
  // window serves the whole bin (the union over its blocks); `kept` counts per block of the
  // bin, weighted by n_r^2, what the block itself needs
  auto s_list = [&](GemmStage& g, GemmProblem& p, int i, int r0, int nb, int kp0, int nkc, bool tiles,
                    double& kept) {
    const std::array<int, 4> key{i, r0 * 4096 + nb, kp0, nkc};
    auto it = tiles ? s_lists.find(key) : s_lists.end();
    if (it == s_lists.end()) {
      const size_t start = g.klist.size();
      const int k0 = c.ibz[i];
      const Blocks& Ba = c.bao[i];
      std::vector<int> rs;
      for (size_t r = 0; r < Ba.size.size(); ++r)
        if (Ba.off[r] >= r0 && Ba.off[r] < r0 + nb) rs.push_back(int(r));
      double mk = 0;
      const int nra = int(Ba.size.size());
      for (int kp = kp0; kp < kp0 + nkc; ++kp) {
        const Blocks& BQ = c.baux[c.rep[mesh.sub(k0, kp)]];
        const Blocks& Bb = c.bao[c.rep[kp]];
        const int nrb = int(Bb.size.size());
        const uint8_t* nz =
            tiles && have_tiles ? c.vt_nz[0].data() + c.vt_off[0][size_t(i) * nk + kp] : nullptr;
        for (size_t sg = 0; sg < BQ.size.size(); ++sg) {
          auto flag = [&](int r, int r2) { return !nz || nz[(sg * nra + r) * nrb + r2]; };
          for (int r : rs) {
            windows(Bb, [&](int r2) { return flag(r, r2); });
            for (const auto& w : win) mk += double(Ba.size[r]) * Ba.size[r] * BQ.size[sg] * (w.second - w.first);
          }
          windows(Bb, [&](int r2) {
            for (int r : rs)
              if (flag(r, r2)) return true;
            return false;
          });
          for (const auto& w : win) push_seg(g, start, (kp - kp0) * na + BQ.off[sg], BQ.size[sg], w.first, w.second);
        }
      }
      const std::array<i64, 3> v{i64(start), i64(g.klist.size() - start), i64(mk)};
      if (!tiles) {
        p.kseg = v[0];
        p.nkseg = int(v[1]);
        kept = mk;
        return;
      }
      it = s_lists.emplace(key, v).first;
    }
    p.kseg = it->second[0];
    p.nkseg = int(it->second[1]);
    kept = double(it->second[2]);
  };
  // ---------------- polarization (eq. P0, Alg. 3) ----------------
  std::vector<double> sumsq_ao(nib, 0.0);  // sum of squared orbital block sizes
  for (int i = 0; i < nib; ++i)
    for (int sz : c.bao[i].size) sumsq_ao[i] += double(sz) * sz;
  const double pscale = -c.prm.spin / nk;
  // P0^q(tau_j)[Q, Q'] = -(s/Nk) sum_k sum_(a,b) Vp(Q)_ab conj(W(Q')_ab) with
  // W(Q') = G^k(beta - tau_j)^H Vp(Q') G^(k+q)(tau_j)^H, which equals the trace of eq. P0;
  // W comes from one pass of the both-sided block multiply, then a plain grouped GEMM.
  for (int i = 0; i < nib; ++i) {
    const int q0 = c.ibz[i];
    const Blocks& BA = c.baux[i];
    std::vector<int> kq(nk);
    for (int k = 0; k < nk; ++k) kq[k] = mesh.add(k, q0);
    for (int j0 = 0; j0 < nthalf; j0 += J) {
      const int j1 = std::min(nthalf, j0 + J), jc = j1 - j0;
      // W is needed only for the auxiliary functions of leading blocks (the GEMM reads no other)
      const auto qruns = lead_runs(BA);
      auto segs = [&](int k) {
        const int ik = c.rep[k], ikq = c.rep[kq[k]];
        for (int j = j0; j < j1; ++j) {
          const i64 vp = (i64(i) * nk + k) * na * no * no;
          const i64 wo = (i64(j - j0) * nk + k) * na * no * no;
          for (const auto& run : qruns) {
            RowSeg r{};
            r.inbuf = B_VP; r.outbuf = B_W2; r.gbuf = B_G;
            r.blk = d.bt_ao[ik]; r.g_off = c.g_off[ik] + i64(nt - 1 - j) * c.bao[ik].packed;
            r.blk2 = d.bt_ao[ikq]; r.g_off2 = c.g_off[ikq] + i64(j) * c.bao[ikq].packed;
            r.in_off = vp + i64(run.first) * no; r.out_off = wo + i64(run.first) * no;
            r.nrows = run.second * no;
            r.ld = na * no;
            d.p0_both.add(r, double(run.second) * no * (sumsq_ao[ik] + sumsq_ao[ikq]), double(run.second) * no * no);
          }
        }
      };
      // one problem per auxiliary block for all tau of the chunk: the columns are (tau, Q'), so
      // the Vp rows of the block are read once for every tau and small blocks fill the tiles;
      // the outer sum runs over the nkc points from k0 (all of them, or one pair unbatched)
      auto gemm = [&](size_t sg, int k0, int nkc, int beta) {
        const int m = BA.size[sg], off = BA.off[sg];
        // A_(k,a) = Vp[i][k][a][rows of block sg][:], B_(k,a) = W[tau][k][a][rows of block sg][:]
        const i64 ko = i64(k0) * na * no * no;
        GemmProblem p = gp(m, jc * m, no, nkc * no, 1, B_VP, i64(i) * nk * na * no * no + ko + i64(off) * no, no,
                           i64(na) * no, 0, OP_N, B_W2, ko + i64(off) * no, no, i64(na) * no, 0, OP_H, B_OUT,
                           c.p_off[i] + i64(j0) * BA.packed + BA.poff[sg], m, 0, pscale, 0.0, beta);
        p.cdiv = m;
        p.sBcb = slab;
        p.sCcb = BA.packed;
        double kept = 0;
        p0_list(p, i, int(sg), k0, nkc, kept);
        // P0^q(tau) is Hermitian (so is every term of the k sum, G being Hermitian): only the
        // tiles on or below the diagonal are computed
        const double tri = double(jc) * m * (m + 1) / 2;
        c.vt_stats[4] += tri * no * nkc * no;
        c.vt_stats[5] += tri * kept;
        d.p0_gemm.add(p, tri * kept, true);
      };
      // aligned partner blocks repeat their leading block: only leading blocks are computed
      if (!ub) {
        for (int k = 0; k < nk; ++k) segs(k);
        for (size_t sg = 0; sg < BA.size.size(); ++sg)
          if (BA.lead[sg] == int(sg)) gemm(sg, 0, nk, 0);
        d.p0_both.close();
        d.p0_gemm.close();
        const int l = int(d.p0_gemm.launches.size());
        d.p0_steps.push_back({int(d.p0_both.launches.size()) - 1, l - 1, l});
      } else {
        for (int k = 0; k < nk; ++k) {
          segs(k);
          d.p0_both.close();
          const int g0 = int(d.p0_gemm.launches.size());
          for (size_t sg = 0; sg < BA.size.size(); ++sg) {
            if (BA.lead[sg] != int(sg)) continue;
            gemm(sg, k, 1, k > 0);
            d.p0_gemm.close();
          }
          d.p0_steps.push_back({int(d.p0_both.launches.size()) - 1, g0, int(d.p0_gemm.launches.size())});
        }
      }
    }
    // upper triangles from the lower ones; with half tau also the mirrored tau; a partner
    // block that repeats a leading one is written from the leader's lower triangle
    for (int j = 0; j < nthalf; ++j)
      for (size_t sg = 0; sg < BA.size.size(); ++sg) {
        const int l = BA.lead[sg];
        const i64 o = c.p_off[i] + i64(j) * BA.packed + BA.poff[sg];
        const i64 ol = c.p_off[i] + i64(j) * BA.packed + BA.poff[l];
        const bool mir = c.prm.half_tau && nt - 1 - j != j;
        const i64 om = c.p_off[i] + i64(nt - 1 - j) * BA.packed + BA.poff[sg];
        if (l == int(sg)) {
          d.p0_mirror.items.push_back({B_OUT, B_OUT, BA.size[sg], 0, o, mir ? om : -1, 0});
        } else {
          d.p0_mirror.items.push_back({B_OUT, B_OUT, BA.size[sg], 1, ol, o, 0});
          if (mir) d.p0_mirror.items.push_back({B_OUT, B_OUT, BA.size[sg], 1, ol, om, 0});
        }
      }
  }
  d.p0_mirror.close();

  clk.mark("polarization work lists");
  // ---------------- self-energy (eq. sigma, Alg. 4) ----------------
  // bins of consecutive orbital blocks, at most 16 rows each (a larger block is a bin alone)
  // of the leading blocks only (a block repeating an aligned partner is gathered from it)
  std::vector<std::vector<std::pair<int, int>>> bins_ao(nib);
  for (int i = 0; i < nib; ++i) {
    const Blocks& B = c.bao[i];
    int r0 = 0, nb = 0;
    for (size_t r = 0; r < B.size.size(); ++r) {
      if (B.lead[r] != int(r)) {
        if (nb > 0) bins_ao[i].push_back({r0, nb});
        r0 = B.off[r] + B.size[r];
        nb = 0;
        continue;
      }
      if (nb > 0 && nb + B.size[r] > 16) {
        bins_ao[i].push_back({r0, nb});
        r0 += nb;
        nb = 0;
      }
      nb += B.size[r];
    }
    if (nb > 0) bins_ao[i].push_back({r0, nb});
  }
  // Y(k', s') = P_blk^T Vs (per auxiliary block), Z = Y G^{k'}(tau_j) (block multiply),
  // Sigma = -(1/Nk) sum_(k', s') Z Vs^H on the diagonal squares of the bins, then the diagonal
  // blocks are gathered into Sigma_blk; only the block work is counted.
  // tau units: with time reversal P(beta - tau) = P(tau) (the reading that mirrors P0), so
  // Y(tau) = Y(beta - tau): a unit is a tau of the first half with its mirror, Y is formed
  // once per unit, and the block multiply, the orbital contraction and the gather run for both.
  std::vector<std::pair<int, int>> units;   // (j, mirror or -1); the j are consecutive
  if (c.prm.half_tau) {
    for (int j = 0; j < (nt + 1) / 2; ++j) units.push_back({j, nt - 1 - j != j ? nt - 1 - j : -1});
  } else {
    for (int j = 0; j < nt; ++j) units.push_back({j, -1});
  }
  for (int i = 0; i < nib; ++i) {
    const int k0 = c.ibz[i];
    const Blocks& BO = c.bao[i];
    const auto aruns = lead_runs(BO);
    for (size_t u0 = 0; u0 < units.size();) {
      // units of this chunk: at most J tau (workspace slabs) in all
      size_t u1 = u0;
      int nslot = 0;
      while (u1 < units.size() && nslot + (units[u1].second >= 0 ? 2 : 1) <= J) nslot += units[u1++].second >= 0 ? 2 : 1;
      const int nu = int(u1 - u0), j0 = units[u0].first;
      std::vector<int> slot_tau;   // tau of each workspace slot
      std::vector<int> slot_unit;  // unit (Y slab) of each slot
      for (int uu = 0; uu < nu; ++uu) {
        slot_tau.push_back(units[u0 + uu].first);
        slot_unit.push_back(uu);
        if (units[u0 + uu].second >= 0) {
          slot_tau.push_back(units[u0 + uu].second);
          slot_unit.push_back(uu);
        }
      }
      // Y = P_blk^T Vs with the rows (unit, s') in one problem per (k', auxiliary block): the Vs
      // rows are read once for every tau of the chunk
      // Y's columns (a, b) only for the orbital functions a of k0's leading blocks: the orbital
      // GEMM reads no other rows of Z = Y G
      auto gemmA = [&](int kp, bool each) {
        const int q = mesh.sub(k0, kp), iq = c.rep[q];
        const Blocks& BQ = c.baux[iq];
        const i64 vs = (i64(i) * nk + kp) * na * no * no;
        for (size_t sg = 0; sg < BQ.size.size(); ++sg) {
          const int m = BQ.size[sg], off = BQ.off[sg];
          for (const auto& run : aruns) {
            const i64 ca = i64(run.first) * no;
            GemmProblem p = gp(nu * m, run.second * no, m, 1, 1, B_P, c.p_off[iq] + i64(j0) * BQ.packed + BQ.poff[sg],
                               m, 0, 0, OP_T, B_VS, vs + i64(off) * no * no + ca, i64(no) * no, 0, 0, OP_N, B_W1,
                               i64(kp) * na * no * no + i64(off) * no * no + ca, i64(no) * no, 0);
            p.rdiv = m;
            p.sArb = BQ.packed;
            p.sCrb = slab;
            d.s_gemmA.add(p);
          }
          if (each) d.s_gemmA.close();
        }
      };
      // Z(tau) = Y(unit) G^{k'}(tau) for every tau of the chunk; a unit's Y is read once for
      // both of its tau
      auto right = [&](int kp) {
        const int ik = c.rep[kp];
        for (int sl = 0; sl < nslot; ++sl) {
          if (sl > 0 && slot_unit[sl] == slot_unit[sl - 1]) continue;   // the mirror slot, done below
          const bool pair = sl + 1 < nslot && slot_unit[sl + 1] == slot_unit[sl];
          RowSeg r{};
          r.inbuf = B_W1; r.outbuf = B_W2; r.gbuf = B_G; r.blk = d.bt_ao[ik];
          r.in_off = (i64(slot_unit[sl]) * nk + kp) * na * no * no;
          r.out_off = (i64(sl) * nk + kp) * na * no * no;
          r.g_off = c.g_off[ik] + i64(slot_tau[sl]) * c.bao[ik].packed;
          r.out_off2 = -1;
          if (pair) {
            r.out_off2 = (i64(sl + 1) * nk + kp) * na * no * no;
            r.g_off2 = c.g_off[ik] + i64(slot_tau[sl + 1]) * c.bao[ik].packed;
          }
          // rows (s', a) for the leading runs of a only: groups of the run's width, nao apart
          for (const auto& run : aruns) {
            RowSeg rr = r;
            rr.in_off += i64(run.first) * no;
            rr.out_off += i64(run.first) * no;
            if (pair) rr.out_off2 += i64(run.first) * no;
            rr.rw = run.second;
            rr.ld = no;
            rr.nrows = na * run.second;
            d.s_right.add(rr, double(na) * run.second * sumsq_ao[ik] * (pair ? 2 : 1),
                          double(na) * run.second * no * (pair ? 1.5 : 1));
          }
        }
      };
      // only the diagonal blocks of Sigma are kept: consecutive orbital blocks are grouped into
      // bins of at most 16 rows and each bin's diagonal square is one problem, with the rows
      // (slot, a) of all tau of the chunk stacked; the outer sum runs over the nkc points from kp0
      auto gemmC = [&](int kp0, int nkc, bool each) {
        for (const auto& bn : bins_ao[i]) {
          const int r0 = bn.first, nb = bn.second;
          const i64 ko = i64(kp0) * na * no * no;
          GemmProblem p = gp(nslot * nb, nb, no, nkc * na, 1, B_W2, ko + i64(r0) * no, no, i64(no) * no, 0, OP_N, B_VS,
                             i64(i) * nk * na * no * no + ko + i64(r0) * no, no, i64(no) * no, 0, OP_H, B_SCR,
                             i64(r0) * no + r0, no, 0, -1.0 / nk, 0.0, kp0 > 0 ? 1 : 0);
          p.rdiv = nb;
          p.sArb = slab;
          p.sCrb = i64(no) * no;
          double algo = 0;
          for (size_t rb = 0; rb < BO.size.size(); ++rb)
            if (BO.off[rb] >= r0 && BO.off[rb] < r0 + nb) algo += double(BO.size[rb]) * BO.size[rb];
          double kept = 0;
          s_list(d.s_gemmC, p, i, r0, nb, kp0, nkc, true, kept);
          c.vt_stats[6] += double(nslot) * algo * no * double(nkc) * na;
          c.vt_stats[7] += double(nslot) * kept;
          d.s_gemmC.add(p, double(nslot) * kept);
          if (each) d.s_gemmC.close();
        }
      };
      const int step0 = int(d.s_steps.size());
      if (!ub) {
        for (int kp = 0; kp < nk; ++kp) gemmA(kp, false);
        for (int kp = 0; kp < nk; ++kp) right(kp);
        gemmC(0, nk, false);
        d.s_gemmA.close();
        d.s_right.close();
        d.s_gemmC.close();
        const int la = int(d.s_gemmA.launches.size()), lc = int(d.s_gemmC.launches.size());
        d.s_steps.push_back({la - 1, la, int(d.s_right.launches.size()) - 1, lc - 1, lc});
      } else {
        for (int kp = 0; kp < nk; ++kp) {
          const int a0 = int(d.s_gemmA.launches.size());
          gemmA(kp, true);
          right(kp);
          d.s_right.close();
          const int c0 = int(d.s_gemmC.launches.size());
          gemmC(kp, 1, true);
          d.s_steps.push_back({a0, int(d.s_gemmA.launches.size()), int(d.s_right.launches.size()) - 1, c0,
                               int(d.s_gemmC.launches.size())});
        }
      }
      for (int sl = 0; sl < nslot; ++sl)
        for (size_t rb = 0; rb < BO.size.size(); ++rb) {
          const int n = BO.size[rb], off = BO.off[size_t(BO.lead[rb])];
          d.s_pack.items.push_back({B_SCR, B_OUT, n, 0, i64(sl) * no * no + i64(off) * no + off,
                                    c.g_off[i] + i64(slot_tau[sl]) * BO.packed + BO.poff[rb], no});
        }
      d.s_pack.close();
      d.s_chunks.push_back({step0, int(d.s_steps.size()), int(d.s_pack.launches.size()) - 1});
      u0 = u1;
    }
  }

  clk.mark("self-energy work lists");
  for (GemmStage* g : gs)
    if ((st = upload_stage(c, d, *g, s))) return st;
  // launches that walk K-segment lists, per stage
  c.vt_stats[8] = c.vt_stats[9] = 0;
  for (const Range& r : d.p0_gemm.launches) c.vt_stats[8] += r.lists;
  for (const Range& r : d.s_gemmC.launches) c.vt_stats[9] += r.lists;
  c.vt_stats[10] = double(d.p0_gemm.launches.size());
  c.vt_stats[11] = double(d.s_gemmC.launches.size());
  for (RowStage* r : {&d.p0_both, &d.s_right})
    if ((st = upload(c, d, r->segs, &r->d, s))) return st;
  for (auto* l : {&d.p0_mirror, &d.s_pack})
    if ((st = upload(c, d, l->items, &l->d, s))) return st;
  HIPCHECK(hipStreamSynchronize(s));
  clk.mark("contraction work lists uploaded");
  return GWSYM_OK;
}

int init_noalloc_scratch(Ctx& c);

// ---------------------------------------------------------------------------------------
// device_init: tables, workspaces and the work lists that do not depend on V.

int device_init(Ctx& c, void* stream) {
  PhaseClock clk;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState* dp = new DevState();
  c.dev_state = dp;
  DevState& d = *dp;
  const int nk = c.nk, no = c.nao, na = c.naux, nt = c.ntau, nw = c.nw, nib = c.nibz;
  d.p0_gemm.wave = d.s_gemmA.wave = d.s_gemmC.wave = true;
  int st;
  // U tables
  {
    std::vector<cplx> u;
    u.reserve(size_t(nk) * (no * no + na * na));
    for (int k = 0; k < nk; ++k) u.insert(u.end(), c.U_ao[k].a.begin(), c.U_ao[k].a.end());
    for (int k = 0; k < nk; ++k) u.insert(u.end(), c.U_aux[k].a.begin(), c.U_aux[k].a.end());
    if ((st = upload(c, d, u, &d.U, s))) return st;
  }
  {
    std::vector<cplx> tr;
    tr.insert(tr.end(), c.Tf.begin(), c.Tf.end());
    tr.insert(tr.end(), c.Tb.begin(), c.Tb.end());
    tr.insert(tr.end(), c.Bf.begin(), c.Bf.end());
    tr.insert(tr.end(), c.Bb.begin(), c.Bb.end());
    if ((st = upload(c, d, tr, &d.TR, s))) return st;
    void* t;
    if ((st = upload(c, d, c.tau, &t, s))) return st;
    d.tau = static_cast<double*>(t);
  }
  const i64 TF = 0, TB = i64(nw) * nt, BF = 2 * i64(nw) * nt, BB = 3 * i64(nw) * nt;
  // block tables: count, then (off, size, poff) per block
  {
    std::vector<int> bt;
    for (int i = 0; i < nib; ++i) {
      d.bt_ao.push_back(int(bt.size()));
      const Blocks& B = c.bao[i];
      bt.push_back(int(B.size.size()));
      for (size_t r = 0; r < B.size.size(); ++r) {
        bt.push_back(B.off[r]);
        bt.push_back(B.size[r]);
        bt.push_back(int(B.poff[r]));
      }
    }
    for (int i = 0; i < nib; ++i) {
      d.bt_aux.push_back(int(bt.size()));
      const Blocks& B = c.baux[i];
      bt.push_back(int(B.size.size()));
      for (size_t r = 0; r < B.size.size(); ++r) {
        bt.push_back(B.off[r]);
        bt.push_back(B.size[r]);
        bt.push_back(int(B.poff[r]));
      }
    }
    void* t;
    if ((st = upload(c, d, bt, &t, s))) return st;
    d.btab = static_cast<int*>(t);
  }
  // star weights
  std::vector<int> star(nib, 0);
  for (int k = 0; k < nk; ++k) star[c.rep[k]]++;

  // frequency and readout sizes; the contraction plan adds its tau slabs to the workspaces
  std::vector<i64> pw_off(nib + 1, 0), gw_off(nib + 1, 0);
  for (int i = 0; i < nib; ++i) {
    pw_off[i + 1] = pw_off[i] + i64(nw) * c.baux[i].packed;
    gw_off[i + 1] = gw_off[i] + i64(nw) * c.bao[i].packed;
  }
  i64 ws = std::max(pw_off[nib], gw_off[nib]);
  ws = std::max<i64>(ws, i64(nk) * nt * std::max(no * no, na * na));   // from_block of P over every k
  ws = std::max<i64>(ws, c.p_off[nib] + c.g_off[nib]);
  d.ws_min = size_t(ws);
  if (no > 64) {   // the block multiplies give each orbital column one lane
    c.err = "orbital basis larger than 64 functions";
    return GWSYM_ESHAPE;
  }
  clk.mark("tables, workspaces");
  if ((st = plan_contractions(c, d, s))) return st;
  clk.t = std::chrono::steady_clock::now();

  // ---------------- exchange (eq. sigma_hf, K term) ----------------
  // K^{k0} = -(1/Nk) sum_{k', Q} V^{k0,k'}(Q) gamma^{k'} V^{k0,k'}(Q)^H with gamma = -G(beta):
  // Z(k') = V_S[k0][k'] G^{k'}(beta) (block multiply), then +(1/Nk) sum_{(k',s)} Z V_S^H on the
  // diagonal squares of the same orbital bins as the self-energy, gathered into the F layout.
  d.hx_gemm.wave = true;
  {
    const i64 slab1 = i64(nk) * na * no * no;
    // the orbital GEMM walks every (k', Q) over all b: one list for all its problems
    for (int t = 0; t < nk * na; t += 64) d.hx_gemm.klist.push_back({t, std::min(64, nk * na - t), 0, no});
    for (int i = 0; i < nib; ++i) {
      const Blocks& BO = c.bao[i];
      for (int kp = 0; kp < nk; ++kp) {
        const int ik = c.rep[kp];
        RowSeg r{};
        r.inbuf = B_VS; r.outbuf = B_W2; r.gbuf = B_G; r.blk = d.bt_ao[ik];
        r.in_off = (i64(i) * nk + kp) * na * no * no;
        r.out_off = i64(kp) * na * no * no;
        r.g_off = c.g_off[ik] + i64(nt - 1) * c.bao[ik].packed;
        r.out_off2 = -1;
        r.nrows = na * no;
        double sq = 0;
        for (int sz : c.bao[ik].size) sq += double(sz) * sz;
        d.hx_right.add(r, double(na) * no * sq, double(na) * no * no);
      }
      int r0 = 0, nb = 0;
      std::vector<std::pair<int, int>> bins;
      for (size_t rb = 0; rb < BO.size.size(); ++rb) {
        if (nb > 0 && nb + BO.size[rb] > 16) {
          bins.push_back({r0, nb});
          r0 += nb;
          nb = 0;
        }
        nb += BO.size[rb];
      }
      if (nb > 0) bins.push_back({r0, nb});
      for (const auto& bn : bins) {
        GemmProblem p = gp(bn.second, bn.second, no, nk * na, 1, B_W2, i64(bn.first) * no, no, i64(no) * no, 0, OP_N,
                           B_VS, i64(i) * slab1 + i64(bn.first) * no, no, i64(no) * no, 0, OP_H, B_SCR,
                           i64(bn.first) * no + bn.first, no, 0, 1.0 / nk);
        p.kseg = 0;
        p.nkseg = int(d.hx_gemm.klist.size());
        d.hx_gemm.add(p);
      }
      for (size_t rb = 0; rb < BO.size.size(); ++rb)
        d.hx_pack.items.push_back({B_SCR, B_OUT, BO.size[rb], 0, i64(BO.off[rb]) * no + BO.off[rb],
                                   c.f_off[i] + BO.poff[rb], no});
      d.hx_right.close();
      d.hx_gemm.close();
      d.hx_pack.close();
    }
    if ((st = upload_stage(c, d, d.hx_gemm, s))) return st;
    if ((st = upload(c, d, d.hx_right.segs, &d.hx_right.d, s))) return st;
    if ((st = upload(c, d, d.hx_pack.items, &d.hx_pack.d, s))) return st;
  }

  // ---------------- Hartree (eq. sigma_hf, J term) ----------------
  // rho = sum over the whole zone of Tr[gamma^{k'} V^{k'k'}(Q)].  Only the irreducible points
  // hold V^{k'k'}: a star's points add the rotated copies of the representative's density,
  // whose sum is |star| times its projection onto the invariant auxiliary functions.
  {
    Mesh mesh{c.n};
    std::vector<HartreeItem> items;
    std::vector<int> first(size_t(nib) + 1, 0);
    std::vector<double> w(size_t(nib), 0.0);
    for (int k = 0; k < nk; ++k) w[size_t(c.rep[k])] += 1.0;
    for (int i = 0; i < nib; ++i) {
      w[size_t(i)] *= -c.prm.spin / nk;   // gamma = -G(beta); s/Nk; star size
      const Blocks& BO = c.bao[i];
      first[size_t(i)] = int(items.size());
      for (size_t rb = 0; rb < BO.size.size(); ++rb)
        items.push_back({BO.off[rb], BO.size[rb], c.g_off[i] + i64(nt - 1) * BO.packed + BO.poff[rb],
                         (i64(i) * nk + c.ibz[i]) * na * no * no, c.f_off[i] + BO.poff[rb]});
    }
    first[size_t(nib)] = int(items.size());
    d.hj_nitems = int(items.size());
    // V_S(s) = sum_Q U_{Qs} V(Q), so a density vector maps as rho_s = (U^H rho)_s and the
    // projector (1/|G|) sum_g Obar(g) becomes U^H Pi U
    const int kg = mesh.sub(c.ibz[0], c.ibz[0]);
    // (without symmetry every point is summed explicitly: no projection)
    CMat Pi = CMat::eye(na);
    if (c.prm.mode != GWSYM_MODE_FULL) {
      Pi = CMat(na, na);
      for (int a = 0; a < c.nop; ++a) {
        const CMat O = orbital_rep(c, true, a, kg);
        for (size_t e = 0; e < Pi.a.size(); ++e) Pi.a[e] += O.a[e] / double(c.nop);
      }
    }
    const CMat P2 = matmul(Pi, Pi);
    double dev2 = 0;
    for (size_t e = 0; e < Pi.a.size(); ++e) dev2 = std::max(dev2, std::abs(P2.a[e] - Pi.a[e]));
    if (dev2 > 1e-10) {
      c.err = "the auxiliary representation at q = 0 does not average to a projector";
      return GWSYM_EINVAL;
    }
    const CMat Ps = matmul(adjoint(c.U_aux[kg]), matmul(Pi, c.U_aux[kg]));
    if ((st = upload(c, d, items, &d.hj_items, s))) return st;
    void* fp = nullptr;
    if ((st = upload(c, d, first, &fp, s))) return st;
    d.hj_first = static_cast<int*>(fp);
    void* wp = nullptr;
    if ((st = upload(c, d, w, &wp, s))) return st;
    d.hj_w = static_cast<double*>(wp);
    if ((st = upload(c, d, Ps.a, &d.hj_proj, s))) return st;
    if ((st = dalloc(c, d, &d.hj_r, size_t(nib) * na * 16))) return st;
    if ((st = dalloc(c, d, &d.hj_rho, size_t(na) * 16))) return st;
  }

  // ---------------- screened interaction (eq. P02P) ----------------
  for (int i = 0; i < nib; ++i) {
    const Blocks& B = c.baux[i];
    d.scr_fwd.add(gp(nw, int(B.packed), nt, 1, 1, B_TR, TB, nt, 0, 0, OP_N, B_IN, c.p_off[i], B.packed, 0, 0, OP_N, B_W1,
                     pw_off[i], B.packed, 0));
    d.scr_bwd.add(gp(nt, int(B.packed), nw, 1, 1, B_TR, BB, nw, 0, 0, OP_N, B_W2, pw_off[i], B.packed, 0, 0, OP_N, B_W1,
                     c.p_off[i], B.packed, 0));
    for (int n = 0; n < nw; ++n)
      for (size_t sg = 0; sg < B.size.size(); ++sg) {
        InvItem it{};
        it.n = B.size[sg]; it.xbuf = B_W1; it.fbuf = B_W1; it.outbuf = B_W2;
        it.x_off = pw_off[i] + i64(n) * B.packed + B.poff[sg]; it.f_off = -1; it.out_off = it.x_off; it.w = 0;
        d.scr_inv.items.push_back(it);
      }
    for (int j = 0; j < nt; ++j)
      for (size_t sg = 0; sg < B.size.size(); ++sg) {
        const i64 o = c.p_off[i] + i64(j) * B.packed + B.poff[sg];
        d.scr_herm.items.push_back({B_W1, B_OUT, B.size[sg], 0, o, o, 0});
      }
  }
  d.scr_fwd.close();
  d.scr_bwd.close();
  d.scr_inv.close();
  for (const InvItem& it : d.scr_inv.items) d.scr_inv.nmax = std::max(d.scr_inv.nmax, it.n);
  d.scr_herm.close();

  // ---------------- Dyson equation and mu (eq. dyson, N_e) ----------------
  std::vector<double> g0w;
  for (int i = 0; i < nib; ++i) {
    const Blocks& B = c.bao[i];
    d.dys_fwd.add(gp(nw, int(B.packed), nt, 1, 1, B_TR, TF, nt, 0, 0, OP_N, B_IN, c.g_off[i], B.packed, 0, 0, OP_N, B_W1,
                     gw_off[i], B.packed, 0));
    d.dys_bwd.add(gp(nt, int(B.packed), nw, 1, 1, B_TR, BF, nw, 0, 0, OP_N, B_W2, gw_off[i], B.packed, 0, 0, OP_N, B_W1,
                     c.g_off[i], B.packed, 0));
    for (int n = 0; n < nw; ++n)
      for (size_t r = 0; r < B.size.size(); ++r) {
        InvItem it{};
        it.n = B.size[r]; it.xbuf = B_W1; it.fbuf = B_F; it.outbuf = B_W2;
        it.x_off = gw_off[i] + i64(n) * B.packed + B.poff[r]; it.f_off = c.f_off[i] + B.poff[r];
        it.out_off = it.x_off; it.w = (2.0 * c.nfreq_f[n] + 1.0) * M_PI / c.prm.beta;
        d.dys_inv.items.push_back(it);
        d.mu_inv.items.push_back(it);
        d.mu_items.items.push_back({n, 0, double(star[i])});
      }
    for (int j = 0; j < nt; ++j)
      for (size_t r = 0; r < B.size.size(); ++r) {
        const i64 o = c.g_off[i] + i64(j) * B.packed + B.poff[r];
        d.dys_herm.items.push_back({B_W1, B_OUT, B.size[r], 0, o, o, 0});
      }
    for (size_t r = 0; r < B.size.size(); ++r) {
      EigItem e{};
      e.n = B.size[r]; e.fbuf = B_F; e.gbuf = B_OUT;
      e.f_off = c.f_off[i] + B.poff[r]; e.g_off = c.g_off[i] + B.poff[r]; e.g_stride = B.packed;
      d.g0_items.items.push_back(e);
      g0w.push_back(double(star[i]));
    }
  }
  d.dys_fwd.close();
  d.dys_bwd.close();
  d.dys_inv.close();
  d.mu_inv.close();
  for (const InvItem& it : d.dys_inv.items) d.dys_inv.nmax = std::max(d.dys_inv.nmax, it.n);
  d.mu_inv.nmax = d.dys_inv.nmax;
  d.mu_items.close();
  d.dys_herm.close();
  d.g0_items.close();

  // ---------------- to_block / from_block (eq. mat_blk, eq. mat_rot) ----------------
  for (int kind = 0; kind < 3; ++kind) {
    const bool aux = kind == GWSYM_KIND_P;
    const int nb = aux ? na : no;
    const int ntk = kind == GWSYM_KIND_F ? 1 : nt;
    const std::vector<i64>& boff = kind == GWSYM_KIND_F ? c.f_off : kind == GWSYM_KIND_G ? c.g_off : c.p_off;
    for (int i = 0; i < nib; ++i) {
      const Blocks& B = aux ? c.baux[i] : c.bao[i];
      const i64 uo = U_off(c, aux, c.ibz[i]);
      const i64 fo = i64(i) * ntk * nb * nb;
      d.tb_1[kind].add(gp(nb, nb, nb, 1, ntk, B_IN, fo, nb, 0, i64(nb) * nb, OP_N, B_U, uo, nb, 0, 0, OP_N, B_W1, fo, nb,
                          i64(nb) * nb));
      for (size_t r = 0; r < B.size.size(); ++r)
        d.tb_2[kind].add(gp(B.size[r], B.size[r], nb, 1, ntk, B_U, uo + B.off[r], nb, 0, 0, OP_H, B_W1, fo + B.off[r], nb, 0,
                            i64(nb) * nb, OP_N, B_OUT, boff[i] + B.poff[r], B.size[r], B.packed));
    }
    d.tb_1[kind].close();
    d.tb_2[kind].close();
    for (int k = 0; k < nk; ++k) {
      const int i = c.rep[k];
      const Blocks& B = aux ? c.baux[i] : c.bao[i];
      const i64 uo = U_off(c, aux, k);
      const i64 fo = i64(k) * ntk * nb * nb;
      for (size_t r = 0; r < B.size.size(); ++r)
        d.fb_1[kind].add(gp(nb, B.size[r], B.size[r], 1, ntk, B_U, uo + B.off[r], nb, 0, 0, OP_N, B_IN, boff[i] + B.poff[r],
                            B.size[r], 0, B.packed, OP_N, B_W1, fo + B.off[r], nb, i64(nb) * nb));
      d.fb_2[kind].add(gp(nb, nb, nb, 1, ntk, B_W1, fo, nb, 0, i64(nb) * nb, OP_N, B_U, uo, nb, 0, 0, OP_H, B_OUT, fo, nb,
                          i64(nb) * nb));
    }
    d.fb_1[kind].close();
    d.fb_2[kind].close();
  }

  for (GemmStage* g : {&d.scr_fwd, &d.scr_bwd, &d.dys_fwd, &d.dys_bwd})
    if ((st = upload_stage(c, d, *g, s))) return st;
  for (int kind = 0; kind < 3; ++kind)
    for (GemmStage* g : {&d.tb_1[kind], &d.tb_2[kind], &d.fb_1[kind], &d.fb_2[kind]})
      if ((st = upload_stage(c, d, *g, s))) return st;
  for (auto* l : {&d.scr_herm, &d.dys_herm})
    if ((st = upload(c, d, l->items, &l->d, s))) return st;
  for (auto* l : {&d.scr_inv, &d.dys_inv, &d.mu_inv})
    if ((st = upload(c, d, l->items, &l->d, s))) return st;
  if ((st = upload(c, d, d.mu_items.items, &d.mu_items.d, s))) return st;
  if ((st = upload(c, d, d.g0_items.items, &d.g0_items.d, s))) return st;
  {
    void* t;
    if ((st = upload(c, d, g0w, &t, s))) return st;
    d.wts = static_cast<double*>(t);
  }
  void* t;
  if ((st = dalloc(c, d, &t, 16 * sizeof(double)))) return st;
  d.mu_state = static_cast<double*>(t);
  if ((st = dalloc(c, d, &t, std::max<size_t>(1, d.mu_inv.items.size()) * 2 * sizeof(double)))) return st;
  d.trace = static_cast<double*>(t);
  if ((st = dalloc(c, d, &t, std::max<size_t>(1, d.g0_items.items.size()) * sizeof(double)))) return st;
  d.occ = static_cast<double*>(t);
  if ((st = dalloc(c, d, &t, std::max<size_t>(1, d.g0_items.items.size()) * 2 * sizeof(double)))) return st;
  d.erange = static_cast<double*>(t);
  if ((st = dalloc(c, d, &d.vwork, std::max<size_t>(1, d.g0_items.items.size()) * JAC_N * JAC_N * 16))) return st;
  if ((st = dalloc(c, d, &t, sizeof(int)))) return st;
  d.status = static_cast<int*>(t);
  HIPCHECK(hipMemsetAsync(d.status, 0, sizeof(int), s));
  HIPCHECK(hipMemsetAsync(d.mu_state, 0, 16 * sizeof(double), s));
  HIPCHECK(hipStreamSynchronize(s));
  if ((st = init_noalloc_scratch(c))) return st;
  clk.mark("exchange, Hartree, Dyson and mu lists");
  c.dev = true;
  return GWSYM_OK;
}

void device_free(Ctx& c) {
  DevState* d = static_cast<DevState*>(c.dev_state);
  if (!d) return;
  for (hipEvent_t e : d->prof.pool) hipEventDestroy(e);
  if (d->graph_exec) hipGraphExecDestroy(d->graph_exec);
  for (void* p : d->allocs) hipFree(p);
  delete d;
  c.dev_state = nullptr;
  c.dev = false;
  c.vloaded = false;
}

namespace {

template <class F>
void timed(DevState& d, hipStream_t s, int cls, double macs, F f, double bytes = 0) {
  Prof& p = d.prof;
  if (!p.on) {
    f();
    return;
  }
  while (p.pool.size() < p.used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      f();
      return;
    }
    p.pool.push_back(e);
  }
  const size_t i = p.used;
  p.used += 2;
  hipEventRecord(p.pool[i], s);
  f();
  hipEventRecord(p.pool[i + 1], s);
  p.recs.push_back({cls, i});
  p.macs[cls] += macs;
  p.bytes[cls] += bytes;
}

int nmax_of(const ListStage<InvItem>& l) { return l.nmax; }

Bases bases_of(DevState& d) {
  Bases b{};
  b.p[B_VP] = d.VP;
  b.p[B_VS] = d.VS;
  b.p[B_W1] = d.W1;
  b.p[B_W2] = d.W2;
  b.p[B_TR] = d.TR;
  b.p[B_U] = d.U;
  b.p[B_WT] = d.WT;
  b.p[B_SCR] = d.SCR;
  b.p[B_BT] = d.btab;
  return b;
}

}  // namespace

// Split-K partial tiles: one 32 x 32 complex slot each, sized for the largest launch.
int need_partials(Ctx& c, DevState& d) {
  if (d.nslots <= d.partial_cap) return GWSYM_OK;
  if (d.partials) {
    hipFree(d.partials);
    d.allocs.erase(std::find(d.allocs.begin(), d.allocs.end(), d.partials));
    d.partials = nullptr;
  }
  const int st = dalloc(c, d, &d.partials, d.nslots * 32 * 32 * 16);
  if (st == GWSYM_OK) d.partial_cap = d.nslots;
  return st;
}

// ---------------------------------------------------------------------------------------
// load_V: block-transformed copies of V for the two contractions (eq. C_blk, Sec. 4.2).

namespace {

// Flags of the (auxiliary block, orbital block, orbital block) tiles of both block-form copies
// of V (Sec. 4.3: only the non-zero blocks of V are used): squared Frobenius norms on the
// device, then on the host a tile is kept when its norm exceeds 1e-13 times that of its pair.
// Bases with more functions or blocks than the tile-norm pass takes keep every tile.
int vtile_flags(Ctx& c, DevState& d, hipStream_t s) {
  const int nk = c.nk, no = c.nao, na = c.naux, nib = c.nibz;
  const i64 pe = i64(na) * no * no;
  Mesh mesh{c.n};
  for (int cp = 0; cp < 2; ++cp) {
    c.vt_nz[cp].clear();
    c.vt_off[cp].clear();
  }
  for (int x = 0; x < 4; ++x) c.vt_stats[x] = 0;
  bool fits = no <= TN_MAXN;
  for (const Blocks& B : c.bao) fits &= B.size.size() <= size_t(TN_MAXB);
  if (!fits) return GWSYM_OK;
  std::vector<TileNormItem> items;
  std::vector<i64> off[2];
  size_t nitems0 = 0;
  i64 total = 0;
  for (int cp = 0; cp < 2; ++cp) {
    off[cp].assign(size_t(nib) * nk + 1, 0);
    for (int i = 0; i < nib; ++i)
      for (int k = 0; k < nk; ++k) {
        const size_t p = size_t(i) * nk + k;
        off[cp][p] = total;
        // self-energy copy [i][k'][Q][a][b]: a at k0, b at k', Q at k0 - k'; polarization copy
        // [i][k][a][Q][b]: a at k, b at k + q0, Q at q0
        const int ia = cp == 0 ? i : c.rep[k];
        const int ib = cp == 0 ? c.rep[k] : c.rep[mesh.add(k, c.ibz[i])];
        const Blocks& BQ = cp == 0 ? c.baux[c.rep[mesh.sub(c.ibz[i], k)]] : c.baux[i];
        const i64 nt = i64(c.bao[ia].size.size()) * i64(c.bao[ib].size.size());
        for (size_t sg = 0; sg < BQ.size.size(); ++sg) {
          TileNormItem it{};
          it.v_off = i64(p) * pe;
          it.out_off = total;
          it.sQ = cp == 0 ? i64(no) * no : no;
          it.sa = cp == 0 ? no : na * no;
          it.sb = 1;
          it.q0 = BQ.off[sg];
          it.nq = BQ.size[sg];
          it.bta = d.bt_ao[ia];
          it.btb = d.bt_ao[ib];
          items.push_back(it);
          total += nt;
        }
      }
    off[cp][size_t(nib) * nk] = total;
    if (cp == 0) nitems0 = items.size();
  }
  void *ditems = nullptr, *dout = nullptr;
  int st;
  if ((st = upload(c, d, items, &ditems, s))) return st;
  if ((st = dalloc(c, d, &dout, size_t(total) * 8))) return st;
  launch_tile_norm(ditems, int(nitems0), d.VS, d.btab, static_cast<double*>(dout), no, s);
  launch_tile_norm(static_cast<TileNormItem*>(ditems) + nitems0, int(items.size() - nitems0), d.VP, d.btab,
                   static_cast<double*>(dout), no, s);
  HIPCHECK(hipGetLastError());
  std::vector<double> nrm(static_cast<size_t>(total), 0.0);
  HIPCHECK(hipMemcpyAsync(nrm.data(), dout, size_t(total) * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  dfree(d, ditems);
  dfree(d, dout);
  for (int cp = 0; cp < 2; ++cp) {
    std::vector<uint8_t>& nz = c.vt_nz[cp];
    nz.assign(size_t(off[cp][size_t(nib) * nk] - off[cp][0]), 0);
    for (size_t p = 0; p < size_t(nib) * nk; ++p) {
      double pair = 0;
      for (i64 t = off[cp][p]; t < off[cp][p + 1]; ++t) pair += nrm[size_t(t)];
      for (i64 t = off[cp][p]; t < off[cp][p + 1]; ++t) {
        const bool kept = nrm[size_t(t)] > 1e-26 * pair;
        nz[size_t(t - off[cp][0])] = kept;
        c.vt_stats[2 * cp + 1] += kept;
      }
      c.vt_stats[2 * cp] += double(off[cp][p + 1] - off[cp][p]);
    }
    c.vt_off[cp].assign(off[cp].begin(), off[cp].end());
    const i64 base = c.vt_off[cp][0];
    for (i64& o : c.vt_off[cp]) o -= base;
  }
  return GWSYM_OK;
}

}  // namespace

int device_load_V(Ctx& c, const void* Vin, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  const int nk = c.nk, no = c.nao, na = c.naux, nib = c.nibz;
  const i64 pe = i64(na) * no * no;  // elements per pair
  int st;
  if (!d.VP) {
    if ((st = dalloc(c, d, &d.VP, size_t(nib) * nk * pe * 16))) return st;
    if ((st = dalloc(c, d, &d.VS, size_t(nib) * nk * pe * 16))) return st;
  }
  Mesh mesh{c.n};
  // inverse operations
  std::vector<int> opinv(c.nop, -1);
  for (int a = 0; a < c.nop; ++a)
    for (int b = 0; b < c.nop; ++b) {
      int prod[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          int sum = 0;
          for (int k = 0; k < 3; ++k) sum += c.W[9 * a + 3 * i + k] * c.W[9 * b + 3 * k + j];
          prod[3 * i + j] = sum;
        }
      bool id = true;
      for (int j = 0; j < 9; ++j) id &= prod[j] == (j % 4 == 0 ? 1 : 0);
      if (id) opinv[a] = b;
    }
  // Per-pair source and rotation matrices for the polarization copy: V^{k,k+q0} with
  // k = alpha k1 (k1 representative) equals the rotation of V^{k1,k''}, k'' = k1 + alpha^{-1} q0.
  struct Pair {
    int src;          // pair index in the input [i][k'] layout
    bool ident;       // alpha = identity: rotations are U^H / U only
    i64 wl, wr, wa;   // offsets in WT (or U)
  };
  std::vector<Pair> pp(size_t(nib) * nk);
  std::vector<cplx> wt;
  for (int i = 0; i < nib; ++i) {
    const int q0 = c.ibz[i];
    for (int k = 0; k < nk; ++k) {
      const int i1 = c.rep[k], k1 = c.ibz[i1], a = c.alpha[k];
      const int kpp = mesh.add(k1, c.kmap[size_t(opinv[a]) * nk + q0]);
      const int kq = mesh.add(k, q0);
      if (c.kmap[size_t(a) * nk + kpp] != kq) return c.err = "inconsistent k rotation in load_V", GWSYM_EINVAL;
      Pair p{};
      p.src = i1 * nk + kpp;
      p.ident = a == 0;
      if (!p.ident) {
        const CMat Ok1 = orbital_rep(c, false, a, k1);
        const CMat Okpp = orbital_rep(c, false, a, kpp);
        const CMat Oq = orbital_rep(c, true, a, mesh.sub(kpp, k1));
        const CMat WL = adjoint(matmul(adjoint(Ok1), c.U_ao[k]));     // U^{k H} O^{k1}(a)
        const CMat WR = matmul(adjoint(Okpp), c.U_ao[kq]);            // O^{k''}(a)^H U^{k+q0}
        const CMat WA = adjoint(matmul(adjoint(Oq), c.U_aux[q0]));    // U_aux^{q0 H} Obar^{k''-k1}(a)
        p.wl = i64(wt.size());
        wt.insert(wt.end(), WL.a.begin(), WL.a.end());
        p.wr = i64(wt.size());
        wt.insert(wt.end(), WR.a.begin(), WR.a.end());
        p.wa = i64(wt.size());
        wt.insert(wt.end(), WA.a.begin(), WA.a.end());
      }
      pp[size_t(i) * nk + k] = p;
    }
  }
  if (d.WT) { /* reloading: the previous table is kept in the allocation list */ }
  if ((st = upload(c, d, wt, &d.WT, s))) return st;
  // work lists, processed in chunks of pairs that fit the two workspaces
  const int chunk = int(std::max<i64>(1, i64(d.ws_elems) / pe));
  GemmStage g1, g2, g3;
  const int npairs = nib * nk;
  for (int which = 0; which < 2; ++which) {        // 0: self-energy copy, 1: polarization copy
    for (int p0 = 0; p0 < npairs; p0 += chunk) {
      const int p1 = std::min(npairs, p0 + chunk);
      for (int p = p0; p < p1; ++p) {
        const int i = p / nk, k = p % nk;
        const i64 w = i64(p - p0) * pe;
        if (which == 0) {
          // Vs(s) = sum_Q U^q_{Qs} [U^{k0 H} V(Q) U^{k'}],  q = k0 - k'
          const int k0 = c.ibz[i], q = mesh.sub(k0, k);
          g1.add(gp(na * no, no, no, 1, 1, B_IN, i64(p) * pe, no, 0, 0, OP_N, B_U, U_off(c, false, k), no, 0, 0, OP_N,
                    B_W1, w, no, 0));
          g2.add(gp(no, no, no, 1, na, B_U, U_off(c, false, k0), no, 0, 0, OP_H, B_W1, w, no, 0, i64(no) * no, OP_N, B_W2,
                    w, no, i64(no) * no));
          g3.add(gp(na, no * no, na, 1, 1, B_U, U_off(c, true, q), na, 0, 0, OP_T, B_W2, w, i64(no) * no, 0, 0, OP_N, B_VS,
                    i64(p) * pe, i64(no) * no, 0));
        } else {
          const Pair& pr = pp[p];
          const int q0 = c.ibz[i], kq = mesh.add(k, q0);
          const i64 src = i64(pr.src) * pe;
          if (pr.ident) {
            g1.add(gp(na * no, no, no, 1, 1, B_IN, src, no, 0, 0, OP_N, B_U, U_off(c, false, kq), no, 0, 0, OP_N, B_W1, w,
                      no, 0));
            g2.add(gp(no, no, no, 1, na, B_U, U_off(c, false, k), no, 0, 0, OP_H, B_W1, w, no, 0, i64(no) * no, OP_N, B_W2,
                      w, no, i64(no) * no));
            // a-major output [a][s][b]: batch over a
            g3.add(gp(na, no, na, 1, no, B_U, U_off(c, true, q0), na, 0, 0, OP_H, B_W2, w, i64(no) * no, 0, no, OP_N, B_VP,
                      i64(p) * pe, no, i64(na) * no));
          } else {
            g1.add(gp(na * no, no, no, 1, 1, B_IN, src, no, 0, 0, OP_N, B_WT, pr.wr, no, 0, 0, OP_N, B_W1, w, no, 0));
            g2.add(gp(no, no, no, 1, na, B_WT, pr.wl, no, 0, 0, OP_N, B_W1, w, no, 0, i64(no) * no, OP_N, B_W2, w, no,
                      i64(no) * no));
            g3.add(gp(na, no, na, 1, no, B_WT, pr.wa, na, 0, 0, OP_N, B_W2, w, i64(no) * no, 0, no, OP_N, B_VP, i64(p) * pe,
                      no, i64(na) * no));
          }
        }
      }
      g1.close();
      g2.close();
      g3.close();
    }
  }
  for (GemmStage* g : {&g1, &g2, &g3})
    if ((st = upload_stage(c, d, *g, s))) return st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_IN] = const_cast<void*>(Vin);
  for (size_t l = 0; l < g1.launches.size(); ++l) {
    launch_brgemm(plan_of(g1, g1.launches[l]), b, d.partials, s);
    launch_brgemm(plan_of(g2, g2.launches[l]), b, d.partials, s);
    launch_brgemm(plan_of(g3, g3.launches[l]), b, d.partials, s);
  }
  // the vanishing tiles, then the contraction lists that skip them
  if ((st = vtile_flags(c, d, s)) || (st = plan_contractions(c, d, s))) return st;
  if (c.prm.precision != GWSYM_FP64) {
    const size_t n = size_t(nib) * nk * pe;
    if (!d.VP32) {
      if ((st = dalloc(c, d, &d.VP32, n * 8))) return st;
      if ((st = dalloc(c, d, &d.VS32, n * 8))) return st;
      if ((st = dalloc(c, d, &d.G32, size_t(c.g_off[nib]) * 8 + 16))) return st;
      if ((st = dalloc(c, d, &d.P32, size_t(c.p_off[nib]) * 8 + 16))) return st;
    }
    launch_to_f32(d.VP, d.VP32, i64(n), s);
    launch_to_f32(d.VS, d.VS32, i64(n), s);
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  if (c.prm.precision != GWSYM_FP64) {   // the contractions read only the FP32 copies
    dfree(d, d.VP);
    dfree(d, d.VS);
  }
  c.vloaded = true;
  return GWSYM_OK;
}

// ---------------------------------------------------------------------------------------

int device_to_block(Ctx& c, int kind, const void* full, void* blk, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_IN] = const_cast<void*>(full);
  b.p[B_OUT] = blk;
  launch_brgemm(plan_of(d.tb_1[kind], d.tb_1[kind].launches[0]), b, d.partials, s);
  launch_brgemm(plan_of(d.tb_2[kind], d.tb_2[kind].launches[0]), b, d.partials, s);
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

int device_from_block(Ctx& c, int kind, const void* blk, void* full, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_IN] = const_cast<void*>(blk);
  b.p[B_OUT] = full;
  launch_brgemm(plan_of(d.fb_1[kind], d.fb_1[kind].launches[0]), b, d.partials, s);
  launch_brgemm(plan_of(d.fb_2[kind], d.fb_2[kind].launches[0]), b, d.partials, s);
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

int device_g0(Ctx& c, const void* F, double mu, void* G, double* nfree, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  for (const EigItem& e : d.g0_items.items)
    if (e.n > JAC_N) return c.err = "orbital block larger than 60 in g0", GWSYM_ESHAPE;
  Bases b = bases_of(d);
  b.p[B_F] = const_cast<void*>(F);
  b.p[B_OUT] = G;
  const int n = int(d.g0_items.items.size());
  launch_jacobi_g0(d.g0_items.d, n, b, d.tau, c.ntau, c.prm.beta, mu, d.occ, d.erange, d.vwork, s);
  launch_g0_reduce(d.occ, d.wts, d.erange, n, c.prm.spin / c.nk, nfree ? nfree : d.mu_state + 5, d.mu_state + 3, s);
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

int device_polarization(Ctx& c, const void* G, void* P0, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_G] = const_cast<void*>(G);
  b.p[B_OUT] = P0;
  b.p[B_KL] = d.p0_gemm.d_klist;
  // FP32 and split-bfloat16 contractions: FP32 copies of V (made once) and of G (here); W2
  // holds float2
  const bool f32 = c.prm.precision != GWSYM_FP64;
  const int arith = c.prm.precision;
  unsigned mask = 0;
  if (f32) {
    launch_to_f32(G, d.G32, c.g_off[c.nibz], s);
    b.p[B_G] = d.G32;
    b.p[B_VP] = d.VP32;
    mask = 1u << B_W2;
  }
  for (const auto& st : d.p0_steps) {
    const Range& rb = d.p0_both.launches[st.both];
    RowSegList L{static_cast<RowSeg*>(d.p0_both.d) + rb.t0, rb.nt, rb.r0};
    timed(d, s, PC_LEFT, rb.macs, [&] { launch_rowblock_both(L, b, d.btab, c.nao, s, f32); }, rb.bytes);
    for (int l = st.g0; l < st.g1; ++l) {
      const Range& rg = d.p0_gemm.launches[l];
      timed(d, s, PC_P0, rg.macs, [&] { launch_wgemm(plan_of(d.p0_gemm, rg), b, d.partials, s, 1, arith, mask); },
            rg.bytes);
    }
  }
  const Range& m = d.p0_mirror.launches[0];
  timed(d, s, PC_OTHER, 0, [&] { launch_herm_fill(static_cast<CopySeg*>(d.p0_mirror.d) + m.t0, m.nt, b, s); });
  HIPCHECK(hipGetLastError());
  c.last_macs[0] = d.p0_gemm.macs;
  return GWSYM_OK;
}

int device_self_energy(Ctx& c, const void* G, const void* P, void* S, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_G] = const_cast<void*>(G);
  b.p[B_P] = const_cast<void*>(P);
  b.p[B_OUT] = S;
  b.p[B_KL] = d.s_gemmC.d_klist;
  const bool f32 = c.prm.precision != GWSYM_FP64;
  const int arith = c.prm.precision;
  unsigned mask = 0;
  if (f32) {
    launch_to_f32(G, d.G32, c.g_off[c.nibz], s);
    launch_to_f32(P, d.P32, c.p_off[c.nibz], s);
    b.p[B_G] = d.G32;
    b.p[B_P] = d.P32;
    b.p[B_VS] = d.VS32;
    mask = (1u << B_W1) | (1u << B_W2);
  }
  for (const auto& ch : d.s_chunks) {
    for (int si = ch[0]; si < ch[1]; ++si) {
      const auto& st = d.s_steps[si];
      for (int l = st.a0; l < st.a1; ++l) {
        const Range& ra = d.s_gemmA.launches[l];
        timed(d, s, PC_SA, ra.macs, [&] { launch_wgemm(plan_of(d.s_gemmA, ra), b, d.partials, s, 2, arith, mask); },
              ra.bytes);
      }
      const Range& rr = d.s_right.launches[st.right];
      RowSegList R{static_cast<RowSeg*>(d.s_right.d) + rr.t0, rr.nt, rr.r0};
      timed(d, s, PC_RIGHT, rr.macs, [&] { launch_rowblock_right(R, b, d.btab, c.nao, s, f32); }, rr.bytes);
      for (int l = st.c0; l < st.c1; ++l) {
        const Range& rc = d.s_gemmC.launches[l];
        timed(d, s, PC_SC, rc.macs, [&] { launch_wgemm(plan_of(d.s_gemmC, rc), b, d.partials, s, 3, arith, mask); },
              rc.bytes);
      }
    }
    const Range& rp = d.s_pack.launches[ch[2]];
    timed(d, s, PC_OTHER, 0, [&] { launch_pack(static_cast<CopySeg*>(d.s_pack.d) + rp.t0, rp.nt, b, s); });
  }
  HIPCHECK(hipGetLastError());
  c.last_macs[1] = d.s_gemmA.macs + d.s_gemmC.macs;
  return GWSYM_OK;
}

int device_exchange(Ctx& c, const void* G, void* K, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  if (c.prm.precision != GWSYM_FP64) {
    c.err = "the exchange term is computed in FP64 only (the reduced modes keep FP32 copies of V)";
    return GWSYM_EINVAL;
  }
  int st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_G] = const_cast<void*>(G);
  b.p[B_OUT] = K;
  b.p[B_KL] = d.hx_gemm.d_klist;
  for (size_t l = 0; l < d.hx_gemm.launches.size(); ++l) {
    const Range& rr = d.hx_right.launches[l];
    RowSegList R{static_cast<RowSeg*>(d.hx_right.d) + rr.t0, rr.nt, rr.r0};
    timed(d, s, PC_RIGHT, rr.macs, [&] { launch_rowblock_right(R, b, d.btab, c.nao, s, false); }, rr.bytes);
    const Range& rc = d.hx_gemm.launches[l];
    timed(d, s, PC_SC, rc.macs, [&] { launch_wgemm(plan_of(d.hx_gemm, rc), b, d.partials, s, 3, 0, 0u); }, rc.bytes);
    const Range& rp = d.hx_pack.launches[l];
    timed(d, s, PC_OTHER, 0, [&] { launch_pack(static_cast<CopySeg*>(d.hx_pack.d) + rp.t0, rp.nt, b, s); });
  }
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

int device_hartree(Ctx& c, const void* G, void* J, const void* add, int accumulate, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  if (c.prm.precision != GWSYM_FP64) {
    c.err = "the Hartree term is computed in FP64 only (the reduced modes keep FP32 copies of V)";
    return GWSYM_EINVAL;
  }
  Bases b = bases_of(d);
  b.p[B_G] = const_cast<void*>(G);
  b.p[B_OUT] = J;
  timed(d, s, PC_OTHER, 0, [&] {
    launch_hartree(d.hj_items, d.hj_first, c.nibz, d.hj_nitems, d.hj_w, d.hj_proj, c.naux, c.nao, d.hj_r, d.hj_rho,
                   add, accumulate, b, s);
  });
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

// F = H0 + J + K (eq. sigma_hf): the exchange term written into F, then J and H0 added
int device_fock(Ctx& c, const void* H0, const void* G, void* F, void* stream) {
  int st;
  if ((st = device_exchange(c, G, F, stream))) return st;
  return device_hartree(c, G, F, H0, 1, stream);
}

int device_screened(Ctx& c, const void* P0, void* P, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  for (const InvItem& it : d.scr_inv.items)
    if (it.n > 512) return c.err = "auxiliary block larger than 512", GWSYM_ESHAPE;
  Bases b = bases_of(d);
  b.p[B_IN] = const_cast<void*>(P0);
  b.p[B_OUT] = P;
  timed(d, s, PC_XFORM, d.scr_fwd.launches[0].macs,
        [&] { launch_brgemm(plan_of(d.scr_fwd, d.scr_fwd.launches[0]), b, d.partials, s); });
  timed(d, s, PC_INV, 0,
        [&] { launch_inverse(d.scr_inv.d, int(d.scr_inv.items.size()), nmax_of(d.scr_inv), b, INV_P, nullptr, nullptr,
                       d.status, s); });
  timed(d, s, PC_XFORM, d.scr_bwd.launches[0].macs,
        [&] { launch_brgemm(plan_of(d.scr_bwd, d.scr_bwd.launches[0]), b, d.partials, s); });
  timed(d, s, PC_OTHER, 0, [&] { launch_herm(d.scr_herm.d, int(d.scr_herm.items.size()), b, s); });
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

namespace {

// eq. dyson on the bases given: Sigma(tau) -> Sigma(i w) into B_W1, the inverses into B_W2,
// i w -> tau into B_W1 and the Hermitian sum into G.  The two frequency workspaces and the
// split-K partial tiles are whatever the caller passes.
void dyson_launches(Ctx& c, DevState& d, Bases& b, void* partials, const double* mu, hipStream_t s, bool prof) {
  auto run = [&](int cls, double macs, auto f) {
    if (prof) timed(d, s, cls, macs, f);
    else f();
  };
  run(PC_XFORM, d.dys_fwd.launches[0].macs,
      [&] { launch_brgemm(plan_of(d.dys_fwd, d.dys_fwd.launches[0]), b, partials, s); });
  run(PC_INV, 0.0, [&] {
    launch_inverse(d.dys_inv.d, int(d.dys_inv.items.size()), nmax_of(d.dys_inv), b, INV_G, mu, nullptr, d.status, s);
  });
  run(PC_XFORM, d.dys_bwd.launches[0].macs,
      [&] { launch_brgemm(plan_of(d.dys_bwd, d.dys_bwd.launches[0]), b, partials, s); });
  run(PC_OTHER, 0.0, [&] { launch_herm(d.dys_herm.d, int(d.dys_herm.items.size()), b, s); });
}

}  // namespace

int device_dyson(Ctx& c, const void* F, const void* S, const double* mu, void* G, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  Bases b = bases_of(d);
  b.p[B_IN] = const_cast<void*>(S);
  b.p[B_F] = const_cast<void*>(F);
  b.p[B_OUT] = G;
  dyson_launches(c, d, b, d.partials, mu, s, true);
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

// ---------------------------------------------------------------------------------------
// Allocation-free form of the Dyson step for callers that cannot allocate (code under graph
// capture, tight serving loops): its frequency workspaces and split-K partial tiles live in one
// file-scope device array instead of the context's buffers, so a call allocates nothing.  Each
// GPU holds its own copy of the array until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device (set up in device_init).  Calls
// that overlap on one GPU share the array and race.

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};   // device address of `scratch` per device id
}  // namespace

// once per device, with that device current
int init_noalloc_scratch(Ctx& c) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return c.err = "device id beyond the scratch table", GWSYM_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return GWSYM_OK;
  void* p = nullptr;
  HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return c.err = "no device address for the scratch array", GWSYM_EHIP;
  g_scratch_dev[dev] = p;
  return GWSYM_OK;
}

int device_dyson_noalloc(Ctx& c, const void* F, const void* S, const double* mu, void* G, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  void* base = (dev >= 0 && dev < MAX_DEVICES) ? g_scratch_dev[dev] : nullptr;
  if (!base) return c.err = "the scratch array was not set up on this device (gwsym_device_init runs there first)",
                    GWSYM_ESTATE;
  // layout: W1 (frequency Sigma, then G(tau) before the Hermitian sum), W2 (G(i w)), partials
  const size_t wf = size_t(c.nw) * size_t(c.g_off[c.nibz]);
  const size_t wt = size_t(c.g_off[c.nibz]);
  const size_t w1 = (std::max(wf, wt) * 16 + 255) & ~size_t(255), w2 = (wf * 16 + 255) & ~size_t(255);
  const size_t slots = size_t(std::max(d.dys_fwd.max_slots, d.dys_bwd.max_slots));
  const size_t need = w1 + w2 + slots * 32 * 32 * 16;
  if (need > NOALLOC_BYTES) {
    c.err = "the allocation-free Dyson step needs " + std::to_string(need) + " bytes of scratch, more than its " +
            std::to_string(NOALLOC_BYTES) + "-byte array";
    return GWSYM_ESHAPE;
  }
  Bases b = bases_of(d);
  unsigned char* p = static_cast<unsigned char*>(base);
  b.p[B_W1] = p;
  b.p[B_W2] = p + w1;
  b.p[B_IN] = const_cast<void*>(S);
  b.p[B_F] = const_cast<void*>(F);
  b.p[B_OUT] = G;
  dyson_launches(c, d, b, p + w1 + w2, mu, s, false);
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

int device_find_mu(Ctx& c, const void* F, const void* S, double ntarget, double* mu, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int st;
  if ((st = need_partials(c, d))) return st;
  for (const EigItem& e : d.g0_items.items)
    if (e.n > JAC_N) return c.err = "orbital block larger than 60 in find_mu", GWSYM_ESHAPE;
  Bases b = bases_of(d);
  b.p[B_IN] = const_cast<void*>(S);
  b.p[B_F] = const_cast<void*>(F);
  // bracket from the spectrum of the F passed in: the block eigen-solver of g0 with no tau
  // points (eigenvalue range only, no Green's function written)
  const int ng = int(d.g0_items.items.size());
  timed(d, s, PC_OTHER, 0, [&] {
    launch_jacobi_g0(d.g0_items.d, ng, b, d.tau, 0, c.prm.beta, 0.0, d.occ, d.erange, d.vwork, s);
    launch_g0_reduce(d.occ, d.wts, d.erange, ng, c.prm.spin / c.nk, d.mu_state + 5, d.mu_state + 3, s);
  });
  timed(d, s, PC_XFORM, d.dys_fwd.launches[0].macs,
        [&] { launch_brgemm(plan_of(d.dys_fwd, d.dys_fwd.launches[0]), b, d.partials, s); });
  const void* Blast = static_cast<const cplx*>(d.TR) + 2 * i64(c.nw) * c.ntau + i64(c.ntau - 1) * c.nw;
  launch_mu_init(d.mu_state + 3, d.mu_state, mu, s);
  const int n = int(d.mu_inv.items.size());
  // a fixed 64 bisection steps, all on the device, then N at the result: a residual above
  // 1e-8 N_target is flagged (the root was outside the bracket)
  for (int it = 0; it < 65; ++it) {
    const int probe = it == 64;
    timed(d, s, PC_INV, 0, [&] { launch_inverse(d.mu_inv.d, n, nmax_of(d.mu_inv), b, INV_TRACE, mu, d.trace, d.status, s); });
    timed(d, s, PC_OTHER, 0, [&] {
      launch_mu_update(d.mu_items.d, n, d.trace, Blast, c.prm.spin / c.nk, ntarget, d.mu_state, mu, probe, d.status, s);
    });
  }
  HIPCHECK(hipGetLastError());
  return GWSYM_OK;
}

// Reads and clears the device status word of the context after the work queued on `stream`:
// bit 0 a singular matrix in a Dyson inverse, bit 1 a chemical potential search whose result
// missed N_target.
int device_check(Ctx& c, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  int h = 0;
  HIPCHECK(hipMemcpyAsync(&h, d.status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (h == 0) return GWSYM_OK;
  HIPCHECK(hipMemsetAsync(d.status, 0, sizeof(int), s));
  HIPCHECK(hipStreamSynchronize(s));
  if (h & 1) {
    c.err = "a matrix of a Dyson equation (I - P0 or (i w + mu) - F - Sigma) was singular";
    return GWSYM_ESINGULAR;
  }
  c.err = "the chemical potential search missed N_target (its root was outside the bracket)";
  return GWSYM_ENOCONV;
}

int device_iteration(Ctx& c, const void* H0, const void* F, void* G, void* P0, void* P, void* S, double* mu,
                     double ntarget, int use_graph, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  auto body = [&]() -> int {
    int st;
    // self-consistent form: F = H0 + J + K from the same G as the polarization and Sigma (the
    // mu search brackets its root from the spectrum of this new F)
    if (H0 && (st = device_fock(c, H0, G, const_cast<void*>(F), stream))) return st;
    if ((st = device_polarization(c, G, P0, stream))) return st;
    if ((st = device_screened(c, P0, P, stream))) return st;
    if ((st = device_self_energy(c, G, P, S, stream))) return st;
    if (ntarget > 0 && (st = device_find_mu(c, F, S, ntarget, mu, stream))) return st;
    return device_dyson(c, F, S, mu, G, stream);
  };
  if (!use_graph) return body();
  int st;
  if ((st = need_partials(c, d))) return st;   // no allocation may happen inside the capture
  const std::vector<const void*> key{H0, F, G, P0, P, S, mu, stream};
  if (!d.graph_exec || key != d.graph_key || ntarget != d.graph_ntarget) {
    if (d.graph_exec) {
      hipGraphExecDestroy(d.graph_exec);
      d.graph_exec = nullptr;
    }
    const bool prof = d.prof.on;
    d.prof.on = false;  // no event records inside the graph
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    st = body();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    d.prof.on = prof;
    if (st) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    HIPCHECK(e);
    const hipError_t ei = hipGraphInstantiate(&d.graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIPCHECK(ei);
    d.graph_key = key;
    d.graph_ntarget = ntarget;
  }
  HIPCHECK(hipGraphLaunch(d.graph_exec, s));
  return GWSYM_OK;
}

int device_profile(Ctx& c, int enable) {
  DevState& d = *static_cast<DevState*>(c.dev_state);
  d.prof.on = enable != 0;
  return GWSYM_OK;
}

int device_profile_read(Ctx& c, double* ms, int64_t* launches, double* macs, double* bytes) {
  DevState& d = *static_cast<DevState*>(c.dev_state);
  Prof& p = d.prof;
  for (int k = 0; k < PC_N; ++k) {
    ms[k] = 0;
    launches[k] = 0;
    macs[k] = p.macs[k];
    bytes[k] = p.bytes[k];
    p.bytes[k] = 0;
    p.macs[k] = 0;
  }
  for (const auto& r : p.recs) {
    HIPCHECK(hipEventSynchronize(p.pool[r.second + 1]));
    float t = 0;
    HIPCHECK(hipEventElapsedTime(&t, p.pool[r.second], p.pool[r.second + 1]));
    ms[r.first] += t;
    launches[r.first] += 1;
  }
  p.recs.clear();
  p.used = 0;
  return GWSYM_OK;
}

// ---------------------------------------------------------------------------------------
// Contraction plans: rebuild from c.tune, or choose c.tune by timing candidates.

int device_replan(Ctx& c, void* stream) {
  DevState& d = *static_cast<DevState*>(c.dev_state);
  d.ws_exact = true;
  const int st = plan_contractions(c, d, static_cast<hipStream_t>(stream));
  d.ws_exact = false;
  return st;
}

namespace {

// device buffers and events that live for one autotune call
struct TuneScratch {
  std::vector<void*> bufs;
  hipEvent_t e[2] = {nullptr, nullptr};
  ~TuneScratch() {
    for (void* p : bufs) hipFree(p);
    for (hipEvent_t x : e)
      if (x) hipEventDestroy(x);
  }
};

}  // namespace

int device_autotune(Ctx& c, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevState& d = *static_cast<DevState*>(c.dev_state);
  const int nk = c.nk, no = c.nao, na = c.naux, nt = c.ntau, nib = c.nibz;
  int st;
  TuneScratch ts;
  // zero G and P inputs: the launch sequence and the operand traffic do not depend on values
  void* buf[4];
  const size_t gbytes = size_t(c.g_off[nib]) * 16 + 16, pbytes = size_t(c.p_off[nib]) * 16 + 16;
  const size_t sizes[4] = {gbytes, pbytes, pbytes, gbytes};   // G, P, P0, Sigma
  for (int b = 0; b < 4; ++b) {
    HIPCHECK(hipMalloc(&buf[b], sizes[b]));
    ts.bufs.push_back(buf[b]);
    HIPCHECK(hipMemsetAsync(buf[b], 0, sizes[b], s));
  }
  HIPCHECK(hipEventCreate(&ts.e[0]));
  HIPCHECK(hipEventCreate(&ts.e[1]));
  const bool prof_on = d.prof.on;
  d.prof.on = false;
  // which: 1 polarization, 2 self-energy, 3 both; best of two runs after one warm-up run
  auto time_calls = [&](int which, float& best) -> int {
    best = 3.4e38f;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHECK(hipEventRecord(ts.e[0], s));
      if ((which & 1) && (st = device_polarization(c, buf[0], buf[2], s))) return st;
      if ((which & 2) && (st = device_self_energy(c, buf[0], buf[1], buf[3], s))) return st;
      HIPCHECK(hipEventRecord(ts.e[1], s));
      HIPCHECK(hipEventSynchronize(ts.e[1]));
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, ts.e[0], ts.e[1]));
      if (rep > 0) best = std::min(best, ms);
    }
    return GWSYM_OK;
  };
  gwsym_tuning best = c.tune;
  float best_ms = 3.4e38f;
  auto trial = [&](const gwsym_tuning& t, int which) -> int {
    c.tune = t;
    float ms;
    if ((st = plan_contractions(c, d, s)) || (st = time_calls(which, ms))) {
      d.prof.on = prof_on;
      return st;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c.tune;   // with the tau chunk the plan actually used
    }
    return GWSYM_OK;
  };
  // 1. tau chunk: powers of two up to the tau count of one contraction pass, within the
  //    workspace budget (the current workspaces count as free)
  size_t freeb = 0, totalb = 0;
  HIPCHECK(hipMemGetInfo(&freeb, &totalb));
  const double slab_bytes = 16.0 * nk * na * double(no) * no;
  const double cap = std::min(16.0e9, 0.25 * (double(freeb) + 32.0 * double(d.ws_elems)));
  const int nthalf = c.prm.half_tau ? (nt + 1) / 2 : nt;
  const int J0 = d.tau_chunk, Jmin = c.prm.half_tau ? 2 : 1;
  std::vector<int> js;
  for (int J = Jmin; J < nthalf; J *= 2) js.push_back(J);
  js.push_back(nthalf);
  js.push_back(J0);
  std::sort(js.begin(), js.end());
  js.erase(std::unique(js.begin(), js.end()), js.end());
  for (int J : js) {
    if (J != J0 && J > Jmin && J * slab_bytes > cap) continue;
    gwsym_tuning t = best;
    t.tau_chunk = J;
    if ((st = trial(t, 3))) return st;
  }
  // 2. per GEMM stage, one knob at a time, timed on the call that contains the stage
  const bool bf = c.prm.precision == GWSYM_BF16X6 || c.prm.precision == GWSYM_BF16X3;
  for (int g = 0; g < 3; ++g) {
    const int which = g == 0 ? 1 : 2;
    best_ms = 3.4e38f;
    if ((st = trial(best, which))) return st;
    for (int v : {2048, 4096, 16384, 32768}) {
      gwsym_tuning t = best;
      t.wg_target[g] = v;
      if ((st = trial(t, which))) return st;
    }
    {
      gwsym_tuning t = best;
      t.cols[g] = t.cols[g] == 32 ? 64 : 32;
      if ((st = trial(t, which))) return st;
    }
    for (int v : {0, 1, 2, 3}) {
      gwsym_tuning t = best;
      if (v == t.xcd_order[g]) continue;
      t.xcd_order[g] = v;
      if ((st = trial(t, which))) return st;
    }
    if (bf)
      for (int v : {16, 32}) {
        gwsym_tuning t = best;
        t.kdepth[g] = v;
        if ((st = trial(t, which))) return st;
      }
    else {
      gwsym_tuning t = best;
      t.prefetch[g] = t.prefetch[g] == 2 ? 4 : 2;
      if ((st = trial(t, which))) return st;
    }
  }
  d.prof.on = prof_on;
  c.tune = best;
  return device_replan(c, stream);
}

}  // namespace gw
