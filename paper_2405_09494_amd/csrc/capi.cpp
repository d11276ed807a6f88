// The extern "C" boundary of libgwsym (declared in include/gwsym.h).
#include <cstring>
#include <new>

#include "internal.hpp"

using namespace gw;

struct gwsym_ctx {
  Ctx c;
};

namespace {

const char* g_static_err = "no context";

int check_params(const gwsym_params* p, std::string& err) {
  if (!p) return err = "params is NULL", GWSYM_EINVAL;
  if (!(p->beta > 0)) return err = "beta must be positive", GWSYM_EINVAL;
  if (p->grid != GWSYM_GRID_CHEBYSHEV && p->grid != GWSYM_GRID_IR) return err = "unknown grid", GWSYM_EINVAL;
  if (p->grid == GWSYM_GRID_IR) {
    if (!(p->ir_wmax > 0)) return err = "ir_wmax must be positive", GWSYM_EINVAL;
    if (!(p->ir_eps >= 1e-14 && p->ir_eps <= 1e-2)) return err = "ir_eps must lie in [1e-14, 1e-2]", GWSYM_EINVAL;
    if (!(p->beta * p->ir_wmax >= 1.0 && p->beta * p->ir_wmax <= 1e5))
      return err = "beta ir_wmax must lie in [1, 1e5]", GWSYM_EINVAL;
  } else {
    if (p->ntau < 3) return err = "ntau must be >= 3", GWSYM_EINVAL;
    if (p->nw < 1) return err = "nw must be >= 1", GWSYM_EINVAL;
    if (2 * p->nw - 1 < p->ntau) return err = "need 2 nw - 1 >= ntau for the inverse transform", GWSYM_EINVAL;
  }
  if (p->mode < 0 || p->mode > 2) return err = "unknown mode", GWSYM_EINVAL;
  if (p->precision < GWSYM_FP64 || p->precision > GWSYM_BF16X3) return err = "unknown precision", GWSYM_EINVAL;
  if (p->tau_chunk < 0) return err = "tau_chunk must be >= 0", GWSYM_EINVAL;
  if (!(p->spin > 0)) return err = "spin factor must be positive", GWSYM_EINVAL;
  if (p->sched != GWSYM_SCHED_GROUPED && p->sched != GWSYM_SCHED_UNBATCHED) return err = "unknown schedule", GWSYM_EINVAL;
  if (p->blocks != GWSYM_BLOCKS_ISOTYPIC && p->blocks != GWSYM_BLOCKS_PARTNER) return err = "unknown block kind", GWSYM_EINVAL;
  return GWSYM_OK;
}

template <class T>
int copy_out(const std::vector<T>& v, void* out, int64_t nbytes) {
  const int64_t need = int64_t(v.size() * sizeof(T));
  if (nbytes < need) return GWSYM_ESHAPE;
  if (need) std::memcpy(out, v.data(), size_t(need));
  return GWSYM_OK;
}

// Builds the named host table; returns false if the name is unknown.
bool table(const Ctx& c, const std::string& name, std::vector<int64_t>& iv, std::vector<double>& dv,
           std::vector<cplx>& cv, int& kind) {
  kind = 0;
  auto ints = [&](const std::vector<int>& v) { iv.assign(v.begin(), v.end()); };
  if (name == "dims") {
    iv = {c.nk, c.nibz, c.nao, c.naux, c.ntau, c.nw, c.nop, c.prm.mode};
  } else if (name == "ibz") {
    ints(c.ibz);
  } else if (name == "rep") {
    ints(c.rep);
  } else if (name == "alpha") {
    ints(c.alpha);
  } else if (name == "kmap") {
    ints(c.kmap);
  } else if (name == "ao_blocks" || name == "aux_blocks") {
    const bool aux = name == "aux_blocks";
    const int nb = aux ? c.naux : c.nao;
    iv.assign(size_t(c.nibz) * (1 + nb), 0);
    for (int i = 0; i < c.nibz; ++i) {
      const Blocks& B = aux ? c.baux[i] : c.bao[i];
      iv[size_t(i) * (1 + nb)] = int64_t(B.size.size());
      for (size_t r = 0; r < B.size.size(); ++r) iv[size_t(i) * (1 + nb) + 1 + r] = B.size[r];
    }
  } else if (name == "ao_lead" || name == "aux_lead") {
    const bool aux = name == "aux_lead";
    const int nb = aux ? c.naux : c.nao;
    iv.assign(size_t(c.nibz) * nb, -1);
    for (int i = 0; i < c.nibz; ++i) {
      const Blocks& B = aux ? c.baux[i] : c.bao[i];
      for (size_t r = 0; r < B.lead.size(); ++r) iv[size_t(i) * nb + r] = B.lead[r];
    }
  } else if (name == "g_off") {
    iv = c.g_off;
  } else if (name == "p_off") {
    iv = c.p_off;
  } else if (name == "f_off") {
    iv = c.f_off;
  } else if (name == "U_ao" || name == "U_aux") {
    kind = 2;
    const auto& U = name == "U_ao" ? c.U_ao : c.U_aux;
    for (const auto& m : U) cv.insert(cv.end(), m.a.begin(), m.a.end());
  } else if (name == "O_ao" || name == "O_aux") {
    kind = 2;
    for (int a = 0; a < c.nop; ++a)
      for (int k = 0; k < c.nk; ++k) {
        const CMat O = orbital_rep(c, name == "O_aux", a, k);
        cv.insert(cv.end(), O.a.begin(), O.a.end());
      }
  } else if (name == "vtile_flags_s" || name == "vtile_flags_p") {
    const auto& v = c.vt_nz[name == "vtile_flags_p"];
    iv.assign(v.begin(), v.end());
  } else if (name == "vtile_off_s" || name == "vtile_off_p") {
    iv = c.vt_off[name == "vtile_off_p"];
  } else if (name == "vtile_stats") {
    kind = 1;
    dv.assign(c.vt_stats, c.vt_stats + 12);
  } else if (name == "freq_f") {
    ints(c.nfreq_f);
  } else if (name == "freq_b") {
    ints(c.nfreq_b);
  } else if (name == "tau") {
    kind = 1;
    dv = c.tau;
  } else if (name == "Tf") {
    kind = 2, cv = c.Tf;
  } else if (name == "Tb") {
    kind = 2, cv = c.Tb;
  } else if (name == "Bf") {
    kind = 2, cv = c.Bf;
  } else if (name == "Bb") {
    kind = 2, cv = c.Bb;
  } else {
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

int gwsym_create(const gwsym_params* params, gwsym_ctx** out) {
  if (!out) return GWSYM_EINVAL;
  std::string err;
  const int st = check_params(params, err);
  if (st != GWSYM_OK) return st;
  gwsym_ctx* ctx = new (std::nothrow) gwsym_ctx();
  if (!ctx) return GWSYM_ENOMEM;
  ctx->c.prm = *params;
  gwsym_tuning& t = ctx->c.tune;
  t.tau_chunk = params->tau_chunk;
  for (int g = 0; g < 3; ++g) {
    t.wg_target[g] = 8192;
    t.cols[g] = 32;
    t.xcd_order[g] = 1;
    t.kdepth[g] = 0;
    t.prefetch[g] = 2;
  }
  // the P0 GEMM's tiles read V_P rows and W columns of one problem: bands of its row tiles on
  // one XCD swept column by column keep both in L2 better (6 % faster at 6x6x6), and its long
  // sums over (k, a) split into more parts fill the chip better (16384 workgroups instead of
  // 8192: 13 % faster on that stage at 6x6x6)
  t.xcd_order[0] = 3;
  t.wg_target[0] = 16384;
  *out = ctx;
  return GWSYM_OK;
}

void gwsym_destroy(gwsym_ctx* ctx) {
  if (!ctx) return;
  device_free(ctx->c);
  delete ctx;
}

const char* gwsym_last_error(const gwsym_ctx* ctx) { return ctx ? ctx->c.err.c_str() : g_static_err; }

int gwsym_build_symmetry_basis(gwsym_ctx* ctx, const gwsym_crystal* crystal) {
  if (!ctx) return GWSYM_EINVAL;
  Ctx& c = ctx->c;
  if (c.built) return c.err = "symmetry basis already built", GWSYM_ESTATE;
  try {
    build_grids(c);   // first: the packed layouts count tau points
    const int st = build_symmetry(c, crystal);
    if (st != GWSYM_OK) return st;
  } catch (const std::bad_alloc&) {
    return c.err = "host allocation failed", GWSYM_ENOMEM;
  } catch (const std::exception& e) {
    return c.err = e.what(), GWSYM_EINVAL;
  }
  c.built = true;
  return GWSYM_OK;
}

int64_t gwsym_table_size(const gwsym_ctx* ctx, const char* name) {
  if (!ctx || !name) return GWSYM_EINVAL;
  if (!ctx->c.built) return GWSYM_ESTATE;
  std::vector<int64_t> iv;
  std::vector<double> dv;
  std::vector<cplx> cv;
  int kind;
  if (!table(ctx->c, name, iv, dv, cv, kind)) return GWSYM_EINVAL;
  return kind == 0 ? int64_t(iv.size() * 8) : kind == 1 ? int64_t(dv.size() * 8) : int64_t(cv.size() * 16);
}

int gwsym_get(const gwsym_ctx* ctx, const char* name, void* out, int64_t nbytes) {
  if (!ctx || !name || !out) return GWSYM_EINVAL;
  if (!ctx->c.built) return GWSYM_ESTATE;
  std::vector<int64_t> iv;
  std::vector<double> dv;
  std::vector<cplx> cv;
  int kind;
  if (!table(ctx->c, name, iv, dv, cv, kind)) return GWSYM_EINVAL;
  return kind == 0 ? copy_out(iv, out, nbytes) : kind == 1 ? copy_out(dv, out, nbytes) : copy_out(cv, out, nbytes);
}

#define NEED(cond, code, msg) \
  do {                        \
    if (!(cond)) {            \
      ctx->c.err = msg;       \
      return code;            \
    }                         \
  } while (0)

int gwsym_device_init(gwsym_ctx* ctx, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.built, GWSYM_ESTATE, "gwsym_build_symmetry_basis must come first");
  NEED(!ctx->c.dev, GWSYM_ESTATE, "device already initialised");
  return device_init(ctx->c, stream);
}

int gwsym_load_V(gwsym_ctx* ctx, const void* V_ibz, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(V_ibz, GWSYM_EINVAL, "V_ibz is NULL");
  return device_load_V(ctx->c, V_ibz, stream);
}

int gwsym_to_block(gwsym_ctx* ctx, int kind, const void* full, void* blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(full && blk, GWSYM_EINVAL, "NULL buffer");
  NEED(kind >= 0 && kind <= 2, GWSYM_EINVAL, "unknown kind");
  return device_to_block(ctx->c, kind, full, blk, stream);
}

int gwsym_from_block(gwsym_ctx* ctx, int kind, const void* blk, void* full, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(full && blk, GWSYM_EINVAL, "NULL buffer");
  NEED(kind >= 0 && kind <= 2, GWSYM_EINVAL, "unknown kind");
  return device_from_block(ctx->c, kind, blk, full, stream);
}

int gwsym_g0(gwsym_ctx* ctx, const void* F_blk, double mu, void* G_blk, double* n_free, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(F_blk && G_blk, GWSYM_EINVAL, "NULL buffer");
  return device_g0(ctx->c, F_blk, mu, G_blk, n_free, stream);
}

int gwsym_polarization(gwsym_ctx* ctx, const void* G_blk, void* P0_blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(G_blk && P0_blk, GWSYM_EINVAL, "NULL buffer");
  return device_polarization(ctx->c, G_blk, P0_blk, stream);
}

int gwsym_screened_interaction(gwsym_ctx* ctx, const void* P0_blk, void* P_blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(P0_blk && P_blk, GWSYM_EINVAL, "NULL buffer");
  return device_screened(ctx->c, P0_blk, P_blk, stream);
}

int gwsym_self_energy(gwsym_ctx* ctx, const void* G_blk, const void* P_blk, void* Sigma_blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(G_blk && P_blk && Sigma_blk, GWSYM_EINVAL, "NULL buffer");
  return device_self_energy(ctx->c, G_blk, P_blk, Sigma_blk, stream);
}

int gwsym_find_mu(gwsym_ctx* ctx, const void* F_blk, const void* Sigma_blk, double n_target, double* mu,
                  void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(F_blk && Sigma_blk && mu, GWSYM_EINVAL, "NULL buffer");
  NEED(n_target > 0, GWSYM_EINVAL, "n_target must be positive");
  return device_find_mu(ctx->c, F_blk, Sigma_blk, n_target, mu, stream);
}

int gwsym_dyson_G(gwsym_ctx* ctx, const void* F_blk, const void* Sigma_blk, const double* mu, void* G_blk,
                  void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(F_blk && Sigma_blk && mu && G_blk, GWSYM_EINVAL, "NULL buffer");
  return device_dyson(ctx->c, F_blk, Sigma_blk, mu, G_blk, stream);
}

int gwsym_dyson_G_noalloc(gwsym_ctx* ctx, const void* F_blk, const void* Sigma_blk, const double* mu, void* G_blk,
                          void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(F_blk && Sigma_blk && mu && G_blk, GWSYM_EINVAL, "NULL buffer");
  return device_dyson_noalloc(ctx->c, F_blk, Sigma_blk, mu, G_blk, stream);
}

int gwsym_iteration(gwsym_ctx* ctx, const void* F_blk, void* G_blk, void* P0_blk, void* P_blk, void* Sigma_blk,
                    double* mu, double n_target, int use_graph, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(F_blk && G_blk && P0_blk && P_blk && Sigma_blk && mu, GWSYM_EINVAL, "NULL buffer");
  NEED(!(use_graph && stream == nullptr), GWSYM_EINVAL, "graph capture needs a created stream");
  return device_iteration(ctx->c, nullptr, F_blk, G_blk, P0_blk, P_blk, Sigma_blk, mu, n_target, use_graph, stream);
}

int gwsym_scf_iteration(gwsym_ctx* ctx, const void* H0_blk, void* F_blk, void* G_blk, void* P0_blk, void* P_blk,
                        void* Sigma_blk, double* mu, double n_target, int use_graph, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(H0_blk && F_blk && G_blk && P0_blk && P_blk && Sigma_blk && mu, GWSYM_EINVAL, "NULL buffer");
  NEED(F_blk != H0_blk && F_blk != G_blk, GWSYM_EINVAL, "F_blk must not alias H0_blk or G_blk");
  NEED(ctx->c.prm.precision == GWSYM_FP64, GWSYM_EINVAL, "the F update is computed in FP64 only");
  NEED(!(use_graph && stream == nullptr), GWSYM_EINVAL, "graph capture needs a created stream");
  return device_iteration(ctx->c, H0_blk, F_blk, G_blk, P0_blk, P_blk, Sigma_blk, mu, n_target, use_graph, stream);
}

int gwsym_check(gwsym_ctx* ctx, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  return device_check(ctx->c, stream);
}

int gwsym_profile(gwsym_ctx* ctx, int enable) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  return device_profile(ctx->c, enable);
}

int gwsym_profile_read(gwsym_ctx* ctx, double* ms, int64_t* launches, double* macs, double* bytes) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(ms && launches && macs && bytes, GWSYM_EINVAL, "NULL buffer");
  return device_profile_read(ctx->c, ms, launches, macs, bytes);
}

int gwsym_exchange(gwsym_ctx* ctx, const void* G_blk, void* K_blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(G_blk && K_blk, GWSYM_EINVAL, "NULL buffer");
  return device_exchange(ctx->c, G_blk, K_blk, stream);
}

int gwsym_hartree(gwsym_ctx* ctx, const void* G_blk, void* J_blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(G_blk && J_blk, GWSYM_EINVAL, "NULL buffer");
  return device_hartree(ctx->c, G_blk, J_blk, nullptr, 0, stream);
}

int gwsym_fock(gwsym_ctx* ctx, const void* H0_blk, const void* G_blk, void* F_blk, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  NEED(H0_blk && G_blk && F_blk, GWSYM_EINVAL, "NULL buffer");
  NEED(F_blk != H0_blk && F_blk != G_blk, GWSYM_EINVAL, "F_blk must not alias H0_blk or G_blk");
  return device_fock(ctx->c, H0_blk, G_blk, F_blk, stream);
}

int gwsym_autotune(gwsym_ctx* ctx, void* stream, gwsym_tuning* out) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(ctx->c.vloaded, GWSYM_ESTATE, "gwsym_load_V must come first");
  const int st = device_autotune(ctx->c, stream);
  if (st == GWSYM_OK && out) *out = ctx->c.tune;
  return st;
}

int gwsym_get_tuning(const gwsym_ctx* ctx, gwsym_tuning* out) {
  if (!ctx || !out) return GWSYM_EINVAL;
  *out = ctx->c.tune;
  return GWSYM_OK;
}

int gwsym_set_tuning(gwsym_ctx* ctx, const gwsym_tuning* t, void* stream) {
  if (!ctx) return GWSYM_EINVAL;
  NEED(t, GWSYM_EINVAL, "NULL tuning");
  NEED(ctx->c.dev, GWSYM_ESTATE, "gwsym_device_init must come first");
  NEED(t->tau_chunk >= 0, GWSYM_EINVAL, "tau_chunk must be >= 0");
  for (int g = 0; g < 3; ++g) {
    NEED(t->wg_target[g] >= 256 && t->wg_target[g] <= (1 << 20), GWSYM_EINVAL, "wg_target out of [256, 2^20]");
    NEED(t->cols[g] == 32 || t->cols[g] == 64, GWSYM_EINVAL, "cols must be 32 or 64");
    NEED(t->xcd_order[g] >= 0 && t->xcd_order[g] <= 3, GWSYM_EINVAL, "xcd_order must be 0, 1, 2 or 3");
    NEED(t->kdepth[g] == 0 || t->kdepth[g] == 16 || t->kdepth[g] == 32, GWSYM_EINVAL, "kdepth must be 0, 16 or 32");
    NEED(t->prefetch[g] == 2 || t->prefetch[g] == 4, GWSYM_EINVAL, "prefetch must be 2 or 4");
  }
  ctx->c.tune = *t;
  return device_replan(ctx->c, stream);
}

int gwsym_flop_counts(const gwsym_ctx* ctx, double* out2) {
  if (!ctx || !out2) return GWSYM_EINVAL;
  out2[0] = ctx->c.last_macs[0];
  out2[1] = ctx->c.last_macs[1];
  return GWSYM_OK;
}

}  // extern "C"
