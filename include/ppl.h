/*
 * ppl.h -- C ABI of the MI355X (gfx950) particle-particle ladder library.
 *
 * The library evaluates the ladder term of the spin-free closed-shell CCD/CCSD
 * vector function (Sec. 2, eq. (ppl-term)) with Cholesky-decomposed integrals
 * (eq. (cholesky)), i.e. eq. (vfunction-chol):
 *
 *     R_ij^ab = sum_{c,d} (ac|bd) t_ij^cd,     (ac|bd) = sum_P L^P_ac L^P_bd,
 *
 * on one GPU, and iterates the linearized doubles equations
 * t <- (V + PPL(t)) / D built on it, with V_ij^ab = (ia|jb) and
 * D_ij^ab = e_i + e_j - e_a - e_b.
 *
 * Conventions shared by every entry point:
 *   - Orbitals are ordered occupied first: p = 0..o-1 occupied, o..o+v-1 virtual.
 *   - L is a device pointer to FP64 [naux][o+v][o+v], C-contiguous; each
 *     L[P] must be symmetric (real orbitals, Sec. 2 after eq. (cholesky)).
 *   - Amplitudes and results are device FP64 [o][o][v][v] (i, j, a, b),
 *     C-contiguous. Amplitudes must be pair-symmetric, t_ij^ab = t_ji^ba
 *     (eq. (2)): only the i <= j half is read.
 *   - Every pointer argument that names device memory is owned by the caller.
 *     The library never allocates or frees device memory: all its device
 *     storage lives in one caller-provided workspace (ppl_bind_workspace).
 *   - Work is enqueued asynchronously on the plan's stream unless stated.
 *   - Functions return PPL_OK (0) or a negative PPL_E_* code; nothing throws
 *     or aborts across the ABI, and there is no CPU fallback. ppl_last_error()
 *     returns a thread-local description of the last failure.
 *   - A plan is bound to one stream and one device and is not thread-safe.
 */
#ifndef PPL_H
#define PPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define PPL_OK             0
#define PPL_E_ARG         -1  /* invalid argument (sizes, null pointers, alignment) */
#define PPL_E_NOMEM       -2  /* budget or workspace too small for even one row batch */
#define PPL_E_HIP         -3  /* a HIP runtime call or kernel launch failed (or no device) */
#define PPL_E_NONFINITE   -4  /* NaN/Inf met in inputs or in a residual */
#define PPL_E_NOCONV      -5  /* iteration hit max_sweeps before reaching tol */
#define PPL_E_DIVERGED    -6  /* residual grew by more than the guard factor */
#define PPL_E_STATE       -7  /* call out of order (no workspace bound, V+- not built, ...) */
#define PPL_E_UNSUPPORTED -8  /* combination not implemented */

/* precision of the two PPL GEMMs (integral build and contraction) */
typedef enum {
  PPL_FP64   = 0,  /* FP64 operands, FP64 MFMA, FP64 accumulation */
  PPL_FP32   = 1,  /* FP32 operands, FP32 MFMA, FP32 accumulation */
  PPL_BF16X3 = 2,  /* x = hi + lo (two bf16 terms), hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation */
  PPL_BF16X6 = 3   /* x = hi + mid + lo (three bf16 terms, the 24 bits of FP32), the six products
                      whose plane indices sum to at most two on BF16 MFMA, FP32 accumulation:
                      about FP32 accuracy (Henry, Tang and Heinecke, ARITH 2019) */
} ppl_prec_t;

typedef struct ppl_plan_s* ppl_plan_t;

/* ppl_desc_t.flags: the plan serves ppl_contract, ppl_contract_tau and ppl_hhl only. It
 * keeps none of the iteration's buffers ((ia|jb), their scratch, the checked-start copy),
 * which leaves more of the budget to V+- rows (larger streaming steps); ppl_iterate and
 * ppl_mp2 return PPL_E_STATE on it. */
#define PPL_PLAN_CONTRACT_ONLY 1
/* ppl_desc_t.flags: the plan also reserves the buffers of the ring terms
 * (ppl_ring_scratch_bytes plus two [o][o][v][v] FP64 tensors, and for a low-precision plan
 * the ring integrals J and K in that precision), so that ppl_iterate can add them to every
 * sweep (ppl_iter_opts_t.ring). PPL_E_ARG together with PPL_PLAN_CONTRACT_ONLY. */
#define PPL_PLAN_RING 2

/* Problem description (input of ppl_plan). */
typedef struct {
  int32_t  o;           /* occupied orbitals, >= 1 */
  int32_t  v;           /* virtual orbitals, >= 2 */
  int32_t  naux;        /* Cholesky vectors, >= 1 */
  int32_t  prec;        /* ppl_prec_t of the PPL GEMMs */
  int32_t  keep_fp64;   /* prec != FP64: also keep an FP64 copy of V+- for refinement sweeps */
  int32_t  tile_contract; /* contraction tile id, -1 = planner's choice (see ppl_tile_count) */
  uint64_t hbm_budget;  /* bytes the workspace may use; 0 = 90% of the device's free memory */
  void*    stream;      /* hipStream_t every call of this plan enqueues on (NULL = null stream) */
  uint64_t build_scratch; /* bytes of integral-build scratch (0 = up to 4 GiB); larger = fewer build steps */
  int32_t  diis_max;    /* DIIS subspace capacity kept in the workspace, 0 .. PPL_DIIS_MAX (0 = none);
                           costs 2 * diis_max packed FP64 amplitude vectors */
  int32_t  flags;       /* PPL_PLAN_* bits */
  const char* tune_cache; /* optional path of a text file of tuned contraction configurations (NULL =
                             none): ppl_plan takes the last entry for (prec, o, v) if there is one
                             (an explicit tile_contract wins); ppl_autotune appends its choice.
                             One entry per line: "ppl-tune 1 <prec> <o> <v> <tile+> <splits+>
                             <tile-> <splits->". A missing or unreadable file is no entry. */
} ppl_desc_t;

/* What the planner decided (output of ppl_plan_query). */
typedef struct {
  uint64_t workspace_bytes;   /* bytes ppl_bind_workspace needs (256-byte aligned base) */
  uint64_t vpm_bytes;         /* bytes of V+ and V- in the compute precision (all rows) */
  int32_t  n_batches;         /* V+- row batches; 1 means all rows resident */
  int32_t  resident;          /* 1: V+- stay resident between calls; 0: rebuilt per contraction */
  int32_t  a_per_batch;       /* virtual rows a (pairs a<=b) per batch */
  int32_t  tile_build;        /* tile id of the integral-build GEMM */
  int32_t  tile_contract;     /* tile id of the contraction GEMM */
  int32_t  n_plus;            /* N+ = o(o+1)/2 occupied pairs i<=j */
  int32_t  n_minus;           /* N- = o(o-1)/2 occupied pairs i<j */
  int32_t  p_plus;            /* P+ = v(v+1)/2 virtual pairs a<=b */
  int32_t  p_minus;           /* P- = v(v-1)/2 virtual pairs a<b */
  int32_t  splits_contract;   /* split-K slices of the R+ contraction GEMM (1 = none, 0 = stream-K) */
  int32_t  tile_contract_minus;   /* tile id of the R- contraction GEMM */
  int32_t  splits_contract_minus; /* split-K slices of the R- contraction GEMM (0 = stream-K) */
  uint64_t build_scratch_bytes;   /* bytes of the integral-build scratch */
  int64_t  max_step_pairs;        /* largest number of (a<=b) pairs one build step holds */
  double   flops_build;       /* useful flops of one integral build: naux (P+^2 + v(v+1)(2v+1)/6)
                                 (upper triangle over packed column pairs: resident and FP64
                                 streaming plans) or 2 naux v^2 P+ (other streaming plans, full rows) */
  double   flops_contract;    /* useful flops of one contraction: 2 (P+^2 N+ + P-^2 N-) */
} ppl_plan_info_t;

/*
 * ppl_plan: validate sizes and choose the V+- row batches, tiles and the
 * workspace layout for the symmetric/antisymmetric pair method:
 *   V+_ab,cd = ((ac|bd) + (ad|bc))/2 (a<=b, c<=d),  V-_ab,cd = ((ac|bd) - (ad|bc))/2 (a<b, c<d).
 * Pure host logic: allocates no device memory and launches nothing. With
 * hbm_budget == 0 it queries the free device memory (PPL_E_HIP without a GPU).
 * Returns PPL_E_ARG for o<1, v<2, naux<1, an unknown precision or sizes whose
 * byte counts overflow 64 bits, and PPL_E_NOMEM when the budget cannot hold the
 * fixed buffers plus one batch of V+- rows. A resident plan, and an FP64 streaming
 * plan, builds the upper triangle of V+- only (see ppl_build_batch); the environment
 * variable PPL_SYM_BUILD=0, read here, makes the plan build full rows instead (for
 * comparisons).
 */
int ppl_plan(const ppl_desc_t* desc, ppl_plan_t* out);

/* ppl_plan_query: copy the planner's decisions into *info. */
int ppl_plan_query(ppl_plan_t plan, ppl_plan_info_t* info);

/*
 * ppl_bind_workspace: hand the plan `bytes` of device memory at `dptr`
 * (256-byte aligned, at least info.workspace_bytes). The caller keeps
 * ownership and must keep it alive until ppl_destroy; the library only
 * partitions it. Enqueues a one-time setup (pair tables, zeroed padding).
 */
int ppl_bind_workspace(ppl_plan_t plan, void* dptr, uint64_t bytes);

/*
 * ppl_build_batch: form V+- rows from the Cholesky vectors (eq. (cholesky)).
 * Every L^P must be symmetric (real orbitals, as the paper assumes), which makes
 * V+ and V- symmetric matrices: a resident plan builds their upper triangle
 * (rows (a, c >= a) of the integrals against the packed column pairs (b <= d), since
 * (ac|bd) = (ac|db)) and writes each entry and its mirror entry as it packs a batch;
 * an FP64 streaming plan builds upper-triangle steps as well (contracted as U and
 * U^T), other streaming plans build full rows. Plans that build upper triangles
 * first check (batch 0 or -1) that the virtual block of L is symmetric to a relative
 * Frobenius asymmetry of 1e-10 and return PPL_E_ARG otherwise. batch in [0, n_batches) builds one row
 * batch, -1 builds every batch of a resident plan. The plan remembers L; a non-resident plan rebuilds its
 * batches from it inside ppl_contract, so L must stay valid until the next
 * ppl_build_batch or ppl_destroy.
 */
int ppl_build_batch(ppl_plan_t plan, const double* L, int32_t batch);

/*
 * ppl_contract: R = beta * R + alpha * PPL(t2) for one amplitude tensor
 * (eq. (vfunction-chol)). t2 and R are device FP64 [o][o][v][v]; t2 must be
 * pair-symmetric; R may not alias t2. The V+- rows must have been built
 * (PPL_E_STATE otherwise).
 */
int ppl_contract(ppl_plan_t plan, const double* t2, double* R, double alpha, double beta);

/*
 * ppl_contract_tau: the ladder term of CCSD, R = beta * R + alpha * PPL(tau) with
 * tau_ij^cd = t_ij^cd + t_i^c t_j^d (the standard closed-shell CCSD ladder; the paper
 * treats the doubles part, eq. (vfunction-chol)). t1 is device FP64 [o][v]; tau is
 * formed while packing, never stored. Same layouts, state and errors as ppl_contract;
 * PPL_E_ARG for a null t1.
 */
int ppl_contract_tau(ppl_plan_t plan, const double* t2, const double* t1, double* R, double alpha,
                     double beta);

/*
 * ppl_hhl: the hole-hole ladder of the doubles residual, R = beta * R + alpha * HHL(t2)
 * with HHL_ij^ab = sum_kl (ki|lj) t_kl^ab and (ki|lj) = sum_P L^P_ki L^P_lj from the
 * occupied block of L (eq. (cholesky) applied to occupied indices). In the pair space:
 * W+-_{ij,kl} = ((ki|lj) +- (li|kj)) / 2, a K = N+ (N-) FP64 MFMA contraction against the
 * packed amplitudes, unpacked with the same signs as ppl_contract. L is device FP64
 * [naux][o+v][o+v], t2 and R device FP64 [o][o][v][v], t2 pair-symmetric, R not
 * aliasing t2. Uses the plan's build scratch, so it must not run concurrently with
 * another call of the same plan; V+- are not needed (any bound plan).
 */
int ppl_hhl(ppl_plan_t plan, const double* L, const double* t2, double* R, double alpha, double beta);

/*
 * ppl_ring: the ring (particle-hole) terms of the closed-shell linearized doubles
 * residual, R = beta * R + alpha * RING(t2) with RING_ij^ab = Y_ij^ab + Y_ji^ba and
 *   Y_ij^ab = sum_kc [ (2 t_ik^ac - t_ik^ca) (kc|jb) - t_ik^ac (kj|bc) - t_ik^cb (kj|ac) ],
 * the standard closed-shell CCD terms next to the ladder (the paper batches them with
 * its generic engine; integrals from the same Cholesky vectors, eq. (cholesky)). Three
 * FP64 MFMA GEMMs of (o v) x (o v) x (o v) over pair matrices: (2A - B) J + (-A) K and
 * B K with A[(i,a)][(k,c)] = t_ik^ac, B[(i,a)][(k,c)] = t_ik^ca, J[(k,c)][(j,b)] = (kc|jb),
 * K[(k,c)][(j,b)] = (kj|bc) (both symmetric), 2 (o v)^3 flops each. Needs no plan: L
 * device FP64 [naux][o+v][o+v], t2 and R device FP64 [o][o][v][v] (t2 pair-symmetric, R
 * not aliasing t2), `scratch` device memory of at least ppl_ring_scratch_bytes(o, v,
 * naux) bytes (256-byte aligned, caller-owned, its contents overwritten), `stream` a
 * hipStream_t (NULL = default). Asynchronous. PPL_E_ARG for bad sizes, null or aliased
 * pointers, misalignment or too small a scratch.
 */
uint64_t ppl_ring_scratch_bytes(int32_t o, int32_t v, int32_t naux);
int ppl_ring(int32_t o, int32_t v, int32_t naux, const double* L, const double* t2, double* R, double alpha,
             double beta, void* scratch, uint64_t scratch_bytes, void* stream);

/*
 * ppl_ring_static: ppl_ring for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc). It takes no
 * scratch argument: its scratch is a static device array of PPL_RING_STATIC_BYTES that
 * every GPU the library runs on holds until the process ends, so sizes whose
 * ppl_ring_scratch_bytes(o, v, naux) exceeds that (about (o, v, naux) = (10, 100, 300)
 * and beyond) return PPL_E_ARG. It allocates nothing and runs the same kernels as
 * ppl_ring, with the same arguments, layouts and results; `stream` (NULL = default)
 * must belong to the current device (PPL_E_ARG otherwise). Every call on one GPU shares
 * that GPU's array, which keeps the last call's contents (each call rewrites what it
 * reads first): calls that overlap on one GPU, on different streams or host threads,
 * race and must not be issued.
 */
#define PPL_RING_STATIC_BYTES (128ull << 20)
int ppl_ring_static(int32_t o, int32_t v, int32_t naux, const double* L, const double* t2, double* R,
                    double alpha, double beta, void* stream);

/* ------------------------------------------------ linearized doubles iteration */
#define PPL_START_MP2   0  /* start from t = V / D */
#define PPL_START_GIVEN 1  /* start from the t2 passed in */
#define PPL_START_GIVEN_CHECKED 2  /* start from t2, but restart from MP2 if its first residual is larger,
                                      or at once if t2 holds a NaN or Inf (no sweep from it then) */
#define PPL_DIIS_MAX 16            /* largest DIIS subspace */

typedef struct {
  int32_t max_sweeps;       /* hard cap on sweeps (all precisions), >= 1 */
  int32_t start;            /* PPL_START_* */
  double  tol;              /* stop when the FP64 residual ||t_new - t||_F < tol (0 = never) */
  double  switch_tol;       /* mixed: go to FP64 sweeps when the residual < switch_tol (0 = 1e-6 for BF16X3, 1e-7 for FP32 and BF16X6) */
  double  stagnation;       /* mixed: go to FP64 sweeps when r_n / r_{n-1} > stagnation */
  int32_t min_fp64_sweeps;  /* mixed: at least this many FP64 sweeps after the switch */
  int32_t fail_on_noconv;   /* 1: return PPL_E_NOCONV when max_sweeps is reached (else OK) */
  double  diverge_factor;   /* PPL_E_DIVERGED when r > diverge_factor * r_first (0 = off) */
  double* history;          /* optional host array of max_sweeps residuals (NULL = none) */
  int32_t diis;             /* DIIS subspace size (<= the plan's diis_max); 0 or 1 = plain Jacobi */
  int32_t hhl;              /* 1: sweeps solve t = (V + PPL(t) + HHL(t)) / D (hole-hole ladder, ppl_hhl;
                               resident plans only, PPL_E_UNSUPPORTED otherwise) */
  int32_t ring;             /* 1: sweeps also add the ring terms RING(t) (ppl_ring) of the FP64
                               amplitudes, their three GEMMs in the sweep's precision (low-precision
                               sweeps: the plan's precision with FP32 accumulation; FP64 sweeps:
                               FP64); needs a resident PPL_PLAN_RING plan (PPL_E_STATE otherwise) */
} ppl_iter_opts_t;

typedef struct {
  int32_t sweeps_lp;        /* sweeps done with the low-precision GEMMs */
  int32_t sweeps_fp64;      /* sweeps done with the FP64 GEMMs */
  int32_t status;           /* PPL_OK / PPL_E_NOCONV / PPL_E_DIVERGED / PPL_E_NONFINITE */
  int32_t restarted_mp2;    /* 1 if a PPL_START_GIVEN_CHECKED start was rejected */
  double  residual;         /* last FP64-update residual ||t_new - t||_F */
  double  energy;           /* E = sum V (2 t_ij^ab - t_ij^ba) of the final t */
  double  energy_start;     /* the same energy of the starting amplitudes */
  double  first_residual;   /* residual of the first sweep */
  int32_t diis_dropped;     /* sweeps dropped from the DIIS subspace because its system was singular */
} ppl_iter_report_t;

/* Fill *opts with the defaults: 100 sweeps, MP2 start, tol 1e-7, switch_tol 0 (automatic),
 * stagnation 0.95, min_fp64_sweeps 2, fail_on_noconv 1, diverge_factor 1e3, diis 0. */
void ppl_iter_opts_default(ppl_iter_opts_t* opts);

/*
 * ppl_iterate: Jacobi sweeps t <- (V + PPL(t)) / D from an MP2 or given start,
 * all in the packed pair space; the update, residual and energy are FP64.
 * With a low-precision plan and keep_fp64 the sweeps first use the
 * low-precision GEMMs, then switch to FP64 (switch_tol / stagnation) and run
 * FP64 sweeps to tol. L, e_occ [o], e_vir [v] and t2 are device FP64; t2
 * holds the start (PPL_START_GIVEN*) on entry and the last iterate on return.
 * Synchronous: it reads two scalars back per sweep. Builds V+- itself.
 *
 * With opts->diis = m >= 2 the sweeps are accelerated by direct inversion in the
 * iterative subspace (DIIS; P. Pulay, Chem. Phys. Lett. 73, 393 (1980)): sweep k
 * maps t_k to t'_k = (V + PPL(t_k)) / D with error e_k = t'_k - t_k (its norm is the
 * residual above); unless converged, the next input is sum_i c_i t'_i over the last m
 * sweeps, c minimizing ||sum_i c_i e_i||_F subject to sum_i c_i = 1 (inner products
 * over the full tensors, in FP64). A singular subspace system drops its oldest sweep.
 * The subspace restarts when a mixed run switches to FP64 sweeps; the sweeps of a
 * checked start are plain. The returned t2 is t'_k of the last sweep, as without DIIS.
 * PPL_E_ARG when m exceeds the plan's diis_max.
 */
int ppl_iterate(ppl_plan_t plan, const double* L, const double* e_occ, const double* e_vir,
                double* t2, const ppl_iter_opts_t* opts, ppl_iter_report_t* report);

/*
 * ppl_mp2: first-order amplitudes t = V / D into t2_out [o][o][v][v] (device
 * FP64), V_ij^ab = (ia|jb) from the occupied-virtual block of L; e_mp2 (host,
 * optional) receives sum V (2 t_ij^ab - t_ij^ba). Synchronous when e_mp2 != NULL.
 */
int ppl_mp2(ppl_plan_t plan, const double* L, const double* e_occ, const double* e_vir, double* t2_out,
            double* e_mp2);

/* ------------------------------------------------ learned start (MLP) */
/*
 * A 4 -> 128 -> 128 -> 1 network with SiLU after both hidden layers maps the
 * per-element features x = (t_MP2/sigma, D_ij^ab, e_i + e_j, e_a + e_b) of an
 * instance to f(x); the guess is t = t_MP2 + sigma * f(x). Parameters, Adam
 * state and training scratch live in one caller-provided device workspace.
 * Flat parameter order (FP32): W1 [128][4], b1 [128], W2 [128][128], b2 [128],
 * W3 [128], b3 [1]. All MLP calls enqueue on the stream given at creation;
 * calls that take a plan must use the same stream as the plan.
 */
typedef struct ppl_mlp_s* ppl_mlp_t;

/* width must be 128; max_batch bounds the rows of one training step. */
int ppl_mlp_create(int32_t width, int64_t max_batch, void* stream, ppl_mlp_t* out);
int ppl_mlp_workspace_bytes(ppl_mlp_t mlp, uint64_t* bytes);
int ppl_mlp_bind_workspace(ppl_mlp_t mlp, void* dptr, uint64_t bytes);
/* number of FP32 parameters (17281 for width 128) */
int ppl_mlp_param_count(ppl_mlp_t mlp);
/* uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases from a seeded host generator; resets Adam */
int ppl_mlp_init(ppl_mlp_t mlp, uint64_t seed);
/* host <-> device copies of the flat parameter vector (n must equal the count); set resets Adam */
int ppl_mlp_set_params(ppl_mlp_t mlp, const float* host_params, int64_t n);
int ppl_mlp_get_params(ppl_mlp_t mlp, float* host_params, int64_t n);
/*
 * ppl_mlp_grad: mean-squared-error loss and its gradient for X [n][4], Y [n]
 * (device FP32) without updating; host_grad receives param_count floats.
 * Synchronous. Gradient partials are summed in a fixed order.
 */
int ppl_mlp_grad(ppl_mlp_t mlp, const float* X, const float* Y, int64_t n, float* host_grad, float* host_loss);
/* ppl_mlp_train_step: one Adam step (beta 0.9/0.999, eps 1e-8) on the batch; host_loss (optional) syncs. */
int ppl_mlp_train_step(ppl_mlp_t mlp, const float* X, const float* Y, int64_t n, float lr, float* host_loss);
/* sigma = RMS of t_mp2 [o][o][v][v] over the whole tensor (host double). Synchronous. */
int ppl_mlp_sigma(ppl_plan_t plan, const double* t_mp2, double* sigma);
/*
 * ppl_mlp_samples: features X [n][4] (and targets Y [n] = (t_star - t_mp2)/sigma
 * when t_star and Y are not NULL) at the flat element indices idx [n] of the
 * [o][o][v][v] tensors (device int64).
 */
int ppl_mlp_samples(ppl_plan_t plan, const double* t_mp2, const double* t_star, const double* e_occ,
                    const double* e_vir, double sigma, const int64_t* idx, int64_t n, float* X, float* Y);
/* ppl_mlp_guess: t2_out = t_mp2 + sigma * f(x) for every element (BF16 MFMA hidden layer). */
int ppl_mlp_guess(ppl_mlp_t mlp, ppl_plan_t plan, const double* t_mp2, const double* e_occ,
                  const double* e_vir, double sigma, double* t2_out);
int ppl_mlp_destroy(ppl_mlp_t mlp);

/* ------------------------------------------------ contraction tile configuration */
/*
 * ppl_set_contract_config: choose the tile id (0 .. ppl_tile_count()-1) and the
 * K decomposition of the R+ and R- contraction GEMMs: 1 .. 8 = that many split-K
 * slices, 0 = stream-K (the (tile, K chunk) iterations cut into equal ranges, one
 * per workgroup the device holds at once; tiles shared by several workgroups are
 * summed afterwards in workgroup order). Split-K slices are summed in slice order,
 * so a fixed configuration on a given device gives bitwise reproducible results.
 * The planner (and ppl_autotune) give PPL_BF16X6 plans K slices of at most 12288
 * elements, because its error grows with the length of each FP32 accumulation; a
 * configuration set here with fewer slices, or stream-K, runs but is less accurate.
 * PPL_E_ARG for out-of-range values.
 */
int ppl_set_contract_config(ppl_plan_t plan, int32_t tile_plus, int32_t splits_plus,
                            int32_t tile_minus, int32_t splits_minus);

/*
 * ppl_autotune: time every (tile, K decomposition) candidate of both contraction
 * GEMMs `reps` times on the bound workspace with HIP events (V+- must be built;
 * operand values do not matter), after a few untimed launches that bring the
 * device to its steady clock; the four fastest are timed again over three
 * interleaved rounds and the fastest on average is kept. The operands are the
 * ones in the workspace (the last packed amplitudes): the matrix-core rate depends
 * on operand values through the power draw, so tune after a contraction of
 * representative amplitudes. Synchronous. best_ms (optional, 2 doubles)
 * receives the winning average times. With a tune cache (ppl_desc_t.tune_cache) the
 * choice is appended to it; PPL_E_ARG if the file cannot be written.
 */
int ppl_autotune(ppl_plan_t plan, int32_t reps, double* best_ms);

/* ------------------------------------------------ batched instances (one persistent launch) */
/*
 * Many independent, uneven (o, v, naux) instances of the ladder term share one
 * workspace; their contractions run as one persistent grouped launch whose
 * workgroups pull (instance, R+/R-, tile) items from a queue sorted
 * longest-first, each instance with its own tile shape. ppl_batch_build runs the
 * integral builds of the instances as concurrent branches on side streams of the
 * batch (joined back into its stream). The contraction sequence (packing, grouped
 * launch, unpacking), or the builds and the contraction together, can be captured
 * once in a hipGraph and replayed. All instances use one precision (FP64 or FP32) and
 * the stream of descs[0]; graph capture needs a non-default stream.
 */
typedef struct ppl_batch_s* ppl_batch_t;

int ppl_batch_plan(int32_t n, const ppl_desc_t* descs, ppl_batch_t* out);
/* workspace bytes and the current number of queue items (after build / autotune) */
int ppl_batch_query(ppl_batch_t batch, uint64_t* workspace_bytes, int32_t* n_items);
int ppl_batch_bind_workspace(ppl_batch_t batch, void* dptr, uint64_t bytes);
/* L: host array of n device pointers, one Cholesky tensor per instance */
int ppl_batch_build(ppl_batch_t batch, const double* const* L);
/*
 * Tile choice of the grouped launch, timed on the launch itself with HIP events
 * (synchronous; operand values do not matter). Candidates: the model's tile for
 * every instance GEMM (the default before autotuning: least row padding times the
 * tile's measured throughput), and for each grouped tile t, t for every GEMM whose
 * occupied-pair rows it pads by at most a quarter. The fastest assignment is kept.
 */
int ppl_batch_autotune(ppl_batch_t batch, int32_t reps);
/* t2, R: host arrays of n device pointers; R_k = PPL_k(t2_k) */
int ppl_batch_contract(ppl_batch_t batch, const double* const* t2, double* const* R);
/* record ppl_batch_contract on these pointers into a graph (replaces a previous one) */
int ppl_batch_graph_capture(ppl_batch_t batch, const double* const* t2, double* const* R);
/*
 * ppl_batch_graph_capture_build: record the whole evaluation of every instance into one graph
 * (replaces a previous one): the integral builds from L[k] (staging and build steps, one
 * instance after another on the batch stream) followed by the packing, the grouped
 * contraction and the unpacking of ppl_batch_contract. One replay
 * (ppl_batch_graph_launch) computes R_k = PPL_k(t2_k) from L and t2. L, t2, R: host arrays of
 * n device pointers, kept by the graph. ppl_batch_build must have run once (it checks that
 * every L is symmetric, which a replay does not re-check). PPL_E_STATE before that,
 * PPL_E_ARG for null pointers or the default stream.
 */
int ppl_batch_graph_capture_build(ppl_batch_t batch, const double* const* L, const double* const* t2,
                                  double* const* R);
int ppl_batch_graph_launch(ppl_batch_t batch);
int ppl_batch_destroy(ppl_batch_t batch);

/* ------------------------------------------------ kernel timing (HIP events) */
#define PPL_PROF_BUILD_GEMM     0  /* integral-build GEMM launches */
#define PPL_PROF_BUILD_PACK     1  /* G -> V+- packing launches */
#define PPL_PROF_CONTRACT_PLUS  2  /* R+ = S' V+ GEMM launches */
#define PPL_PROF_CONTRACT_MINUS 3  /* R- = A' V- GEMM launches */
#define PPL_PROF_UPDATE         4  /* packed Jacobi update + reductions */
#define PPL_PROF_OTHER          5  /* staging, packing of t2, unpacking, (ia|jb) */
#define PPL_PROF_KINDS          6

typedef struct {
  int64_t launches[PPL_PROF_KINDS];  /* timed launches per kind */
  double  ms[PPL_PROF_KINDS];        /* summed event time per kind (milliseconds) */
  double  flops[PPL_PROF_KINDS];     /* summed useful flops of those launches (GEMM kinds) */
} ppl_profile_t;

/*
 * ppl_profile_enable: on != 0 starts (and clears) per-launch timing: every
 * library launch on the plan's stream is bracketed by a pair of HIP events.
 * on == 0 stops recording. Events are created lazily and kept by the plan.
 */
int ppl_profile_enable(ppl_plan_t plan, int on);

/* ppl_profile_read: synchronize the plan's stream and sum the recorded event pairs by kind. */
int ppl_profile_read(ppl_plan_t plan, ppl_profile_t* out);

/* ppl_destroy: free the plan's host metadata (never the workspace). NULL is a no-op. */
int ppl_destroy(ppl_plan_t plan);

/* Thread-local text of the last error ("" if none). Valid until the next call on this thread. */
const char* ppl_last_error(void);

/* Number of contraction tile configurations compiled into the library. */
int ppl_tile_count(void);

/*
 * ppl_tile_dims: rows (bm, of the occupied-pair operand) and columns (bn, of the
 * virtual-pair operand) of the C tile of contraction tile `tile`, and the threads
 * per workgroup of its kernels. Host only. PPL_E_ARG for an unknown tile id or a
 * NULL output.
 */
int ppl_tile_dims(int32_t tile, int32_t* bm, int32_t* bn, int32_t* threads);

/* Library version string. */
const char* ppl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PPL_H */
