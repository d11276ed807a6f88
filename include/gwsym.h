/*
 * gwsym: symmetry-adapted finite-temperature GW hot path for AMD MI355X (gfx950).
 *
 * One GW iteration (Alg. 2 of the paper) on density-fitted three-index Coulomb
 * tensors V^{k1,k2}(Q), restricted to the irreducible wedge of the Brillouin zone
 * and block-diagonalised into the isotypic blocks found by simultaneous
 * diagonalisation of Dirac characters (Sec. 3.4, Alg. 1):
 *
 *   polarization          P0^q(tau)  (eq. P0, Alg. 3)
 *   screened_interaction  P^q = [I - P0^q]^{-1} P0^q at bosonic frequencies (eq. P02P)
 *   self_energy           Sigma~^k(tau)  (eq. sigma, Alg. 4)
 *   find_mu, dyson_G      G^k(i w_n) = [(i w_n + mu) S - F - Sigma(i w_n)]^{-1} (eq. dyson), N_e fixed
 *   exchange, hartree     K^k and J^k of the static self-energy (eq. sigma_hf)
 *   fock, scf_iteration   F = H0 + J + K, alone or as the first step of each iteration
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im) IEEE doubles (C99 double _Complex layout).
 *   - Matrices are row-major.
 *   - "Device" pointers are MI355X global-memory addresses (hipMalloc / torch CUDA tensors);
 *     "host" pointers are ordinary CPU memory.  Every device pointer argument must stay
 *     valid until the work queued on `stream` has finished.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  Every device-side
 *     call only enqueues work on `stream` and returns; no call synchronises the host unless
 *     it says so.  A context is used from one host thread at a time.
 *   - Errors: every call returns GWSYM_OK (0) or a negative gwsym_status; arguments are
 *     checked before anything is enqueued.  gwsym_last_error() gives the message.  A fault
 *     inside a kernel surfaces at the next synchronising HIP call of the caller.
 *   - Ownership: the context owns its symmetry tables, the transformed V tensors and every
 *     workspace (allocated in gwsym_device_init / gwsym_load_V, freed by gwsym_destroy).
 *     The caller owns every buffer it passes in.
 *
 * Block-packed layouts ("blk"), read with gwsym_get ("ao_blocks", "g_off", ...):
 *   For each irreducible point i (in increasing mesh-index order of the representatives)
 *   the orbital blocks r of sizes n_r (sum n_r = nao) are stored one after another, each
 *   n_r x n_r row-major: "packed_ao(i)" = sum_r n_r^2 complex numbers.  Likewise the
 *   auxiliary blocks s of sizes m_s: "packed_aux(i)" = sum_s m_s^2.
 *     F_blk     : [i][packed_ao(i)]
 *     G_blk, Sigma_blk : [i][tau][packed_ao(i)]        (offset of i: query "g_off")
 *     P0_blk, P_blk    : [i][tau][packed_aux(i)]       (offset of i: query "p_off")
 *   In GWSYM_MODE_FULL every mesh point is its own representative and each matrix is a
 *   single block, so "blk" is simply the full matrix.
 *
 * k mesh: Gamma-centred n x n x n; point m = (m0, m1, m2) has fractional reciprocal
 * coordinates m / n and linear index (m0 n + m1) n + m2.
 */
#ifndef GWSYM_H
#define GWSYM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gwsym_ctx gwsym_ctx;

typedef enum {
  GWSYM_OK = 0,
  GWSYM_EINVAL = -1,     /* bad argument value or NULL pointer */
  GWSYM_ESHAPE = -2,     /* sizes inconsistent with the context */
  GWSYM_ENOMEM = -3,     /* host or device allocation failed */
  GWSYM_EHIP = -4,       /* a HIP runtime call failed */
  GWSYM_ESINGULAR = -5,  /* a matrix of a Dyson equation was singular (reported by gwsym_check) */
  GWSYM_ENOCONV = -6,    /* an iterative routine did not converge, or the chemical-potential
                            search missed N_e (reported by gwsym_check) */
  GWSYM_ESTATE = -7      /* call made out of order (e.g. before build_symmetry_basis) */
} gwsym_status;

typedef enum {
  GWSYM_MODE_FULL = 0,   /* no symmetry: every k point, full matrices */
  GWSYM_MODE_ROTATE = 1, /* irreducible wedge, full matrices rotated by O^k(alpha) (eq. mat_rot) */
  GWSYM_MODE_BLOCK = 2   /* irreducible wedge and isotypic blocks (eq. mat_blk, eq. C_blk) */
} gwsym_mode;

/* Arithmetic of the P0 and Sigma contractions (eq. P0, eq. sigma).  In every mode the
   Fourier transforms, the Dyson inverses, the chemical-potential search and the G transform
   stay FP64, and every tensor passed through this interface is complex128. */
typedef enum {
  GWSYM_FP64 = 0,        /* FP64 operands on the FP64 MFMA */
  GWSYM_FP32 = 1,        /* FP32 operands, FP32 MFMA accumulation per tile, split sums in FP64 */
  GWSYM_BF16X6 = 2,      /* FP32 operands, each split into three bfloat16 pieces x = hi + mid + lo
                            (round to nearest even from the remainder); the six piece products
                            with piece indices adding to at most 2 on the bfloat16 MFMA, FP32
                            accumulation: FP32-level error */
  GWSYM_BF16X3 = 3       /* two pieces hi + lo and three products: faster, about 1e-5 relative */
} gwsym_precision;

/* Launch schedule of the contractions (eq. P0, eq. sigma). */
typedef enum {
  GWSYM_SCHED_GROUPED = 0,   /* every stage of a tau chunk is one launch over all pairs and blocks */
  GWSYM_SCHED_UNBATCHED = 1  /* one launch per pair for the block multiplies and per (pair, block)
                                for the GEMMs, issued one after another: the per-block baseline */
} gwsym_sched;

/* Imaginary-time and Matsubara grids (Sec. 5.1). */
typedef enum {
  GWSYM_GRID_CHEBYSHEV = 0,  /* ntau Chebyshev-Gauss-Lobatto points, frequencies n = 0 .. nw-1 */
  GWSYM_GRID_IR = 1          /* sparse sampling on the intermediate-representation basis of the
                                logistic kernel with Lambda = beta ir_wmax and cutoff ir_eps: tau = 0,
                                the zeros of the first dropped basis function and beta; the
                                Matsubara indices where its transform changes sign.  ntau and nw
                                are chosen by the library (pass 0; read them from "dims"), the
                                frequency indices from "freq_f" / "freq_b". */
} gwsym_grid;

/* Blocks of the symmetry-adapted bases (Sec. 3.4). */
typedef enum {
  GWSYM_BLOCKS_ISOTYPIC = 0,  /* one block per irrep of the little group (simultaneous eigenspaces
                                 of the Dirac characters, Alg. 1): size multiplicity x dimension */
  GWSYM_BLOCKS_PARTNER = 1    /* each isotypic block of an irrep of dimension d further split into
                                 d partner-function blocks of the multiplicity's size: operators
                                 that commute with the group act as X (x) I_d there */
} gwsym_blocks;

typedef struct {
  double beta;        /* inverse temperature (1/Ha) */
  int ntau;           /* GWSYM_GRID_CHEBYSHEV: tau points on [0, beta], >= 3 */
  int nw;             /* GWSYM_GRID_CHEBYSHEV: Matsubara frequencies stored for n >= 0 (fermionic
                         and bosonic) */
  double spin;        /* spin factor s multiplying P0 and N_e (2 for closed shells) */
  int mode;           /* gwsym_mode */
  int precision;      /* gwsym_precision */
  int half_tau;       /* 1: inputs are time-reversal symmetric, P0 is evaluated for
                         tau_j with j < ceil(ntau/2) and mirrored (Alg. 3 tau loop) */
  int tau_chunk;      /* tau points per contraction launch (0 = library default) */
  int sched;          /* gwsym_sched */
  int grid;           /* gwsym_grid */
  double ir_wmax;     /* GWSYM_GRID_IR: real-frequency cutoff omega_max (Ha) of the basis */
  double ir_eps;      /* GWSYM_GRID_IR: singular values kept above ir_eps times the largest */
  int blocks;         /* gwsym_blocks */
} gwsym_params;

typedef struct {
  double lattice[9];        /* row-major 3x3 whose columns are the primitive vectors a_i */
  int natom;
  const double* positions;  /* host, natom x 3 fractional coordinates */
  int nop;                  /* space-group operations {alpha | v(alpha)} (Sec. 3.1); op 0 = identity */
  const int* rot;           /* host, nop x 9, integer rotation W on fractional coordinates, row-major */
  const double* trans;      /* host, nop x 3, fractional translation v(alpha) */
  int kmesh;                /* n of the Gamma-centred n^3 mesh */
  int nshell_ao;            /* orbital shells, in basis order; functions m = -l..l per shell */
  const int* ao_atom;       /* host, atom of each shell */
  const int* ao_l;          /* host, angular momentum of each shell, 0..4 */
  int nshell_aux;           /* auxiliary (density-fitting) shells */
  const int* aux_atom;
  const int* aux_l;
} gwsym_crystal;

/* Kinds for gwsym_to_block / gwsym_from_block. */
typedef enum {
  GWSYM_KIND_F = 0,       /* orbital matrix, one per k:          full [nk_in][nao][nao]        */
  GWSYM_KIND_G = 1,       /* orbital matrix per k and tau:       full [nk_in][ntau][nao][nao]  */
  GWSYM_KIND_P = 2        /* auxiliary matrix per q and tau:     full [nk_in][ntau][naux][naux] */
} gwsym_kind;

/* Creates a context.  params is copied.  *out receives the new context (host). */
int gwsym_create(const gwsym_params* params, gwsym_ctx** out);

/* Frees the context, its device tables, the transformed V tensors and every workspace. */
void gwsym_destroy(gwsym_ctx* ctx);

/* Message describing the last error of ctx (a static string when ctx is NULL). */
const char* gwsym_last_error(const gwsym_ctx* ctx);

/* Alg. 1 (Sec. 3.2-3.4), on the host: builds the operation tables, the stars and
 * irreducible representatives of the k mesh (Sec. 4.2), the orbital and auxiliary
 * representations O^k(alpha) (eq. basis_rot, with the phases exp(-i k~ . v_x^alpha)),
 * the projective representations D^k and factors lambda^k (eq. projrep, eq. factor),
 * the Dirac characters of every little co-group (eq. dirac) and, in GWSYM_MODE_BLOCK, the
 * unitary U^k that block-diagonalises every invariant matrix (eq. mat_blk).  Also builds
 * the tau grid and the Matsubara transform matrices.  Host only; makes no HIP call.
 * Fails with GWSYM_EINVAL if an operation does not map the crystal onto itself. */
int gwsym_build_symmetry_basis(gwsym_ctx* ctx, const gwsym_crystal* crystal);

/* Size in bytes of the table `name` (see gwsym_get). Negative status if unknown. */
int64_t gwsym_table_size(const gwsym_ctx* ctx, const char* name);

/* Copies the host table `name` into out (host, nbytes >= gwsym_table_size).
 * Integer tables are int64; real tables double; complex tables interleaved doubles.
 *   "dims"        int64[8]: nk, nibz, nao, naux, ntau, nw, nop, mode
 *   "ibz"         int64[nibz]: mesh index of each irreducible representative
 *   "rep"         int64[nk]: irreducible index i of rep(k)
 *   "alpha"       int64[nk]: operation alpha_k with alpha_k rep(k) = k
 *   "kmap"        int64[nop*nk]: index of alpha k
 *   "ao_blocks"   int64[nibz*(1+nao)]: per i: count, then sizes
 *   "aux_blocks"  int64[nibz*(1+naux)]
 *   "ao_lead", "aux_lead" int64[nibz*n]: per i and block r, the block whose values block r
 *                 repeats (aligned partner blocks), r itself if none; -1 past the last block
 *   "g_off","p_off","f_off"  int64[nibz+1]: packed offsets (complex elements)
 *   "U_ao"        complex[nk][nao][nao]: U^k for every mesh point (columns = block basis)
 *   "U_aux"       complex[nk][naux][naux]
 *   "O_ao"        complex[nop][nk][nao][nao]: O^k(alpha) mapping k to alpha k
 *   "O_aux"       complex[nop][nk][naux][naux]
 *   "tau"         double[ntau];  "Tf","Tb" complex[nw][ntau];  "Bf","Bb" complex[ntau][nw]
 *   "vtile_flags_s", "vtile_flags_p"  int64: after gwsym_load_V, per pair of the self-energy copy
 *                 (k0 in IBZ, k') or of the polarization copy (q0 in IBZ, k), pair p = i nk + k,
 *                 1 for each (auxiliary block s, orbital block r, orbital block r') tile of V in
 *                 the block bases that the contractions use, 0 for one they skip (Sec. 4.3: its
 *                 Frobenius norm is at most 1e-13 times that of its pair), at
 *                 off[p] + (s nr + r) nr' + r'.  Self-energy copy: Q at k0 - k', r at k0, r' at
 *                 k'; polarization copy: Q at q0, r at k, r' at k + q0.  Empty before load_V.
 *   "vtile_off_s", "vtile_off_p"      int64[nibz*nk+1]: the offsets off[p] of those flags
 *   "vtile_stats" double[12]: tiles and used tiles of the self-energy copy, the same for the
 *                 polarization copy, then per iteration the complex MACs of the P0 GEMM over all
 *                 tiles and over the used ones, the same for the Sigma orbital GEMM, then the
 *                 P0 and Sigma orbital GEMM launches that skip the unused tiles and the launches
 *                 of those two stages (a launch whose used tiles keep more than four fifths of
 *                 its k steps runs over all tiles: skipping costs it more than it saves)
 *   "freq_f","freq_b" int64[nw]: Matsubara index n of each stored fermionic / bosonic frequency
 *                 (X(tau) = Y + Y^H with Y = B X(i nu); for bosons the n = 0 column
 *                  carries half weight)
 */
int gwsym_get(const gwsym_ctx* ctx, const char* name, void* out, int64_t nbytes);

/* Allocates the device tables and workspaces on the current HIP device and uploads the
 * symmetry tables.  Must follow gwsym_build_symmetry_basis.  Synchronises `stream`.
 * Size limits (GWSYM_ESHAPE otherwise): nao <= 64; orbital blocks <= 60 functions (free
 * G0); auxiliary blocks <= 512 functions (screened-interaction inverse). */
int gwsym_device_init(gwsym_ctx* ctx, void* stream);

/* Sec. 4.2-4.3 / eq. C_blk: takes V^{k0,k'}(Q) for every representative k0 (in "ibz"
 * order; every mesh point in GWSYM_MODE_FULL) and every k' (device, complex
 * [nibz][nk][naux][nao][nao]) and builds the two block-transformed copies the
 * contractions read: one indexed by (k0, k') for the self-energy and one indexed by
 * (q0, k) with q0 irreducible, rotated with O^k(alpha) and O_aux^q(alpha), for the
 * polarization.  The input is only read; it may be freed once `stream` is done.  Device
 * memory: two copies of the input's size in GWSYM_FP64; in the reduced-precision modes the
 * FP64 copies are replaced by FP32 ones (half the size each) before this call returns.
 * Sec. 4.3: the (auxiliary block, orbital block, orbital block) tiles of both copies whose
 * Frobenius norm is at most 1e-13 times that of their pair are flagged (tables "vtile_*"),
 * and the contraction work lists are rebuilt so that the P0 GEMM and the Sigma orbital GEMM
 * skip them; a captured iteration graph is dropped. */
int gwsym_load_V(gwsym_ctx* ctx, const void* V_ibz, void* stream);

/* eq. mat_blk: full matrices at the irreducible points (device, layout by kind with
 * nk_in = nibz) -> block-packed (device).  Off-block elements are dropped. */
int gwsym_to_block(gwsym_ctx* ctx, int kind, const void* full, void* blk, void* stream);

/* Inverse of eq. mat_blk followed by eq. mat_rot / eq. prot: block-packed (device) ->
 * full matrices at every mesh point (device, layout by kind with nk_in = nk). */
int gwsym_from_block(gwsym_ctx* ctx, int kind, const void* blk, void* full, void* stream);

/* Free Green's function G0^k(tau) = -U diag(exp(-e tau)/(1 + exp(-beta e))) U^H of
 * F^k - mu = U diag(e) U^H, per block, from F_blk (device).  Writes G_blk (device) and
 * the free electron count (s/Nk) sum_k sum_i 1/(1 + exp(beta e_i)) to *n_free (device
 * double; may be NULL). */
int gwsym_g0(gwsym_ctx* ctx, const void* F_blk, double mu, void* G_blk, double* n_free,
             void* stream);

/* eq. P0 / Alg. 3: P0_blk (device) from G_blk (device) and the loaded V. */
int gwsym_polarization(gwsym_ctx* ctx, const void* G_blk, void* P0_blk, void* stream);

/* eq. P02P: tau -> i Omega_n, P = [I - P0]^{-1} P0 per auxiliary block, i Omega_n -> tau.
 * P0_blk, P_blk device. */
int gwsym_screened_interaction(gwsym_ctx* ctx, const void* P0_blk, void* P_blk, void* stream);

/* eq. sigma / Alg. 4: Sigma_blk (device) from G_blk, P_blk (device) and the loaded V. */
int gwsym_self_energy(gwsym_ctx* ctx, const void* G_blk, const void* P_blk, void* Sigma_blk,
                      void* stream);

/* Chemical potential for a fixed electron count (Sec. 4.1, N_e): bisection over 64
 * steps on N(mu) = (s/Nk) sum_k Tr[-G^k(beta; mu)], G from eq. dyson with F_blk and
 * Sigma_blk (device).  Bracket: [lowest, highest] eigenvalue of the F_blk passed in -/+ 20 Ha
 * (a block eigen-solve of F on the device, no earlier call needed).  N is evaluated once more
 * at the result: |N(mu) - n_target| above 1e-8 max(1, n_target) (the root was outside the
 * bracket) sets a device flag that the next gwsym_check reports as GWSYM_ENOCONV.  Writes *mu
 * (device double).  Asynchronous and graph-capturable like the other device calls.  Orbital
 * blocks <= 60 (GWSYM_ESHAPE). */
int gwsym_find_mu(gwsym_ctx* ctx, const void* F_blk, const void* Sigma_blk, double n_target,
                  double* mu, void* stream);

/* Waits for the work queued on `stream`, then reads and clears the context's device status
 * word, which the device calls set without synchronising: GWSYM_ESINGULAR when a batched
 * inverse of eq. P02P (I - P0) or eq. dyson ((i w_n + mu) - F - Sigma) met an exactly zero
 * pivot column since the last check (the results of that call are then not finite);
 * GWSYM_ENOCONV when a gwsym_find_mu result missed n_target; else GWSYM_OK.
 * Synchronises `stream`. */
int gwsym_check(gwsym_ctx* ctx, void* stream);

/* eq. dyson: Sigma(tau) -> Sigma(i w_n), G(i w_n) = [(i w_n + mu) I - F - Sigma(i w_n)]^{-1}
 * per block, i w_n -> tau.  mu is a device double.  Writes G_blk (device). */
int gwsym_dyson_G(gwsym_ctx* ctx, const void* F_blk, const void* Sigma_blk, const double* mu,
                  void* G_blk, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gwsym_dyson_G with the same arguments and result,
 * whose frequency workspaces and split-K partial tiles live in a file-scope device array of the
 * library (64 MiB per GPU, held until the process ends) instead of the context's buffers; the
 * call allocates nothing.  GWSYM_ESHAPE when the workload needs more than the array
 * (2 nw sum_i packed_ao(i) complex numbers plus the partial tiles: the small and 4x4x4
 * workloads fit, the 6x6x6 ones do not).  Every call on one GPU shares the array: calls that
 * overlap on a GPU (other streams, other contexts) race. */
int gwsym_dyson_G_noalloc(gwsym_ctx* ctx, const void* F_blk, const void* Sigma_blk, const double* mu,
                          void* G_blk, void* stream);

/* eq. sigma_hf, exchange term: K^k = -(1/Nk) sum_{k'} sum_Q V^{k,k'}(Q) gamma^{k'} V^{k',k}(Q)
 * with the density matrix gamma^k = G^k(0^-) = -G^k(beta), taken from the last tau point of
 * G_blk (device, G layout).  Writes K_blk (device) in the F layout: block-packed, one matrix
 * per irreducible point ("f_off").  Spin-diagonal, so no spin factor.  F is not updated by
 * this call: the caller forms F = H0 + J + K.  GWSYM_FP64 only (GWSYM_EINVAL in the
 * reduced-precision modes, which keep only FP32 copies of V).  Uses the contraction
 * workspaces: not concurrent with the other calls of this context. */
int gwsym_exchange(gwsym_ctx* ctx, const void* G_blk, void* K_blk, void* stream);

/* eq. sigma_hf, Hartree term: J^k = (s/Nk) sum_Q V^{k,k}(Q) rho(Q) with the density on the
 * auxiliary functions rho(Q) = sum_{k'} Tr[gamma^{k'} V^{k',k'}(Q)] over the whole zone,
 * gamma^k = -G^k(beta) from the last tau point of G_blk (device, G layout), s the spin factor
 * of the parameters (the equation's spin sum).  Needs V^{k,k}(Q) Hermitian in the orbital
 * indices (as the pairing V^{k',k} = V^{k,k'}^H of gwsym_load_V implies).  Writes J_blk
 * (device, F layout).  GWSYM_FP64 only (GWSYM_EINVAL otherwise).  Uses two small buffers of
 * the context: not concurrent with other calls of this context. */
int gwsym_hartree(gwsym_ctx* ctx, const void* G_blk, void* J_blk, void* stream);

/* The one-body matrix of the self-consistent loop (eq. sigma_hf with eq. dyson):
 * F = H0 + J + K, J and K as gwsym_hartree and gwsym_exchange compute them from the density
 * matrix of G_blk.  H0_blk (the non-interacting one-body matrix), G_blk and F_blk are device
 * buffers (F layout, G layout, F layout); F_blk must not alias H0_blk or G_blk (GWSYM_EINVAL).
 * Pass F_blk to the next gwsym_iteration / gwsym_dyson_G.  GWSYM_FP64 only. */
int gwsym_fock(gwsym_ctx* ctx, const void* H0_blk, const void* G_blk, void* F_blk, void* stream);

/* One GW iteration in the order of Alg. 2: polarization(G) -> screened interaction ->
 * self-energy(G, P) -> (find_mu when n_target > 0, else mu is read as given) -> dyson_G,
 * which overwrites G_blk.  All buffers are device memory of the layouts above; mu is one
 * device double.  use_graph != 0: the work is captured once into a HIP graph on `stream`
 * (a created stream, not the null stream) and that graph is replayed by later calls with the
 * same arguments; changing any pointer or n_target captures a new graph.  The capture
 * contains kernels only (no memset, no allocation). */
int gwsym_iteration(gwsym_ctx* ctx, const void* F_blk, void* G_blk, void* P0_blk, void* P_blk, void* Sigma_blk,
                    double* mu, double n_target, int use_graph, void* stream);

/* One iteration of the self-consistent loop (eq. dyson with eq. sigma_hf): first
 * F_blk = H0_blk + J + K from the density matrix of G_blk (as gwsym_fock), then the steps of
 * gwsym_iteration with that F, all from the same G.  H0_blk is the non-interacting one-body
 * matrix (device, F layout); F_blk is written (device, F layout, must not alias H0_blk or
 * G_blk).  The chemical-potential search brackets the root by the lowest and highest
 * eigenvalue of the new F -/+ 20 Ha, as gwsym_find_mu does.  use_graph as for gwsym_iteration (the F update is captured with the
 * rest).  GWSYM_FP64 only (GWSYM_EINVAL otherwise). */
int gwsym_scf_iteration(gwsym_ctx* ctx, const void* H0_blk, void* F_blk, void* G_blk, void* P0_blk, void* P_blk,
                        void* Sigma_blk, double* mu, double n_target, int use_graph, void* stream);

/* Launch plan of the contractions (eq. P0 and eq. sigma work lists).  Index 0 is the
 * polarization GEMM, 1 the self-energy auxiliary GEMM (P^T V), 2 the self-energy orbital
 * GEMM (on the diagonal blocks).  Every choice leaves the results unchanged up to rounding
 * order. */
typedef struct {
  int tau_chunk;      /* tau points per contraction launch (the workspaces hold this many
                         tau slabs of nk * naux * nao^2 complex numbers each) */
  int wg_target[3];   /* workgroups a launch aims for: outer sums are split (and the parts
                         summed in a fixed order) until the tile list reaches this size */
  int cols[3];        /* output columns per wave tile: 32 or 64 */
  int xcd_order[3];   /* 1: tiles sharing operand rows queued on one XCD in sequence; 2: all
                         tiles of a problem on one XCD, the row tiles of a column chunk
                         together; 3: bands of 256 rows of a problem, each on one XCD and
                         swept column chunk by column chunk; 0: plain order */
  int kdepth[3];      /* split-bfloat16 modes: k values per bfloat16 MFMA, 16 or 32; 0 picks
                         per launch (16 where 32 would pad more than a quarter of the sums) */
  int prefetch[3];    /* FP64 / FP32 modes: K steps of 4 fetched ahead per wave, 2 or 4 */
} gwsym_tuning;

/* Autotuner: times candidate launch plans of the polarization and self-energy on this GPU
 * with the loaded V and keeps the fastest: first the tau chunk (powers of two up to the
 * half-tau count, within a workspace budget of a quarter of free device memory and 16 GB
 * per workspace), then per GEMM stage the workgroup target, tile width, XCD order and (in
 * the split-bfloat16 modes) the k depth, else the prefetch depth, one at a time.  Must follow
 * gwsym_load_V.
 * Allocates and frees temporary device buffers (zero G and P inputs) and may grow the
 * workspaces; synchronises `stream`.  *out (host, may be NULL) receives the chosen plan. */
int gwsym_autotune(gwsym_ctx* ctx, void* stream, gwsym_tuning* out);

/* The plan in use (host struct). */
int gwsym_get_tuning(const gwsym_ctx* ctx, gwsym_tuning* out);

/* Rebuilds the contraction plans from *t (host) without timing, e.g. a plan cached from an
 * earlier gwsym_autotune for the same workload and device.  Must follow gwsym_device_init.
 * GWSYM_EINVAL for out-of-range fields; synchronises `stream`. */
int gwsym_set_tuning(gwsym_ctx* ctx, const gwsym_tuning* t, void* stream);

/* Algorithm and executed complex multiply-accumulate counts of the last
 * polarization / self_energy call, for throughput accounting (host).
 * out[0] = P0 MACs, out[1] = Sigma MACs (as executed, padding excluded). */
int gwsym_flop_counts(const gwsym_ctx* ctx, double* out2);

/* Live timing of the launches the context enqueues, with HIP events recorded on the
 * launch stream around every launch (enable != 0) or not at all (enable = 0, default).
 * Classes: 0 polarization contraction (grouped GEMM), 1 self-energy auxiliary contraction,
 * 2 self-energy orbital contraction, 3 block-diagonal multiply from the right, 4 two-sided
 * block-diagonal multiply, 5 Matsubara transforms, 6 batched inverses, 7 other. */
int gwsym_profile(gwsym_ctx* ctx, int enable);

/* Waits for the recorded events and returns, per class (arrays of 8, host): total
 * milliseconds, number of launches, complex multiply-accumulates requested by those
 * launches and, for the block-diagonal multiplies, the algorithmic bytes they read and
 * write, since the previous read; then clears the record. */
int gwsym_profile_read(gwsym_ctx* ctx, double* ms, int64_t* launches, double* macs, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* GWSYM_H */
