// Internal definitions shared by the host side and the kernels of libppl.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ppl.h"

namespace ppl {

// ------------------------------------------------------------------ pair indices
// Row-major packed upper triangles of an n x n index space:
//   plus : pairs (a, b) with a <= b, index a*n - a(a+1)/2 + b
//   minus: pairs (a, b) with a <  b, index a*(n-1) - a(a+1)/2 + b - 1
__host__ __device__ inline int64_t pair_plus(int64_t a, int64_t b, int64_t n) {
  return a * n - a * (a + 1) / 2 + b;
}
__host__ __device__ inline int64_t pair_minus(int64_t a, int64_t b, int64_t n) {
  return a * (n - 1) - a * (a + 1) / 2 + b - 1;
}
__host__ __device__ inline int64_t npairs_plus(int64_t n) { return n * (n + 1) / 2; }
__host__ __device__ inline int64_t npairs_minus(int64_t n) { return n * (n - 1) / 2; }

// pair tables store (a << 16) | b
__host__ __device__ inline int pair_first(int packed) { return packed >> 16; }
__host__ __device__ inline int pair_second(int packed) { return packed & 0xffff; }

// leading dimension of every packed operand row: a multiple of 64 elements,
// so the GEMM K loop never needs a bounds check (the padding is kept zero)
// K elements staged per LDS chunk by the GEMM tiles (FP64 / FP32 and BF16 operands);
// leading dimensions (pad_ld) are multiples of both.
#ifndef PPL_KC64
#define PPL_KC64 16
#endif
constexpr int kKcF64 = PPL_KC64;
constexpr int kKcF32 = 32;
__host__ __device__ constexpr int kc_of_prec(int prec) { return prec == PPL_FP64 ? kKcF64 : kKcF32; }
// BF16x3 tiles stage 64 K elements per chunk (two MFMA k-steps between barriers) when
// two workgroups still fit in the 160 KB of LDS (two buffers of both bf16 planes: 512
// bytes per staged row), 32 otherwise: measured on gfx950, one workgroup per CU with
// the longer chunk is slower than two with the shorter one
__host__ __device__ constexpr int bf3_kc(int bm, int bn) { return 2 * (bm + bn) * 512 <= 160 * 1024 ? 64 : 32; }
static_assert(64 % kKcF64 == 0 && 64 % kKcF32 == 0 && 64 % bf3_kc(0, 0) == 0,
              "K chunk must divide the leading-dimension padding");

__host__ __device__ inline int64_t pad_ld(int64_t k) { return (k + 63) / 64 * 64; }

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
#define PPL_HIP_TRY(expr)                                                                 \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return ::ppl::fail(PPL_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                         __FILE__, __LINE__);                                             \
  } while (0)
#define PPL_TRY(expr)            \
  do {                           \
    int _rc = (expr);            \
    if (_rc != PPL_OK) return _rc; \
  } while (0)

// ------------------------------------------------------------------ workspace
struct Region {
  uint64_t off = 0, bytes = 0;
};

// One set of packed operands in one compute precision.
struct OperandSet {
  int prec = PPL_FP64;     // element precision of Xt / V+- / S' / A'
  bool present = false;
  Region xt, xt_lo;        // staged virtual block of L, transposed to [(a,c)][P]; lo plane for BF16X3
  Region vp, vp_lo;        // V+ rows [rows][ldp]
  Region vm, vm_lo;        // V- rows [rows][ldm]
  Region sp, sp_lo;        // S' [N+][ldp]
  Region am, am_lo;        // A' [N-][ldm]
  bool built = false;      // resident V+- complete
  // contraction tiles and K decompositions of the FP64 copy of a mixed plan (the
  // primary set uses the plan's, which the autotuner and ppl_set_contract_config set)
  int tile_p = 0, split_p = 1, tile_m = 0, split_m = 1;
};

struct Batch {
  int a0, a1;              // virtual rows a in [a0, a1)
  int64_t p0, p1;          // V+ rows [p0, p1)
  int64_t q0, q1;          // V- rows [q0, q1)
};

}  // namespace ppl

struct ppl_plan_s {
  // problem
  int o = 0, v = 0, naux = 0, prec = PPL_FP64, keep_fp64 = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  uint64_t budget = 0;
  // pair counts and padded leading dimensions
  int64_t Pp = 0, Pm = 0, Np = 0, Nm = 0;
  int64_t ldp = 0, ldm = 0, ldx = 0;   // row lengths of +, - operands and of Xt (K = naux)
  // batching
  bool resident = true;
  std::vector<ppl::Batch> batches;
  int a_per_batch = 0;
  int64_t g_pairs_cap = 0;             // pairs (a<=b) one build step may hold in G
  int64_t ld_part = 0;                 // row length of split-K partial slices (streaming: one batch wide)
  // tiles
  int tile_build = 0, tile_contract = 0;
  int tile_build64 = 0;                // build tile of the FP64 copy of a mixed plan (ops[1])
  int split_p = 1, tile_m = 0, split_m = 1;   // split-K of the R+ GEMM; tile and split-K of the R- GEMM
  // workspace
  uint64_t ws_bytes_needed = 0;
  char* ws = nullptr;
  uint64_t ws_bytes = 0;
  ppl::OperandSet ops[2];              // [0] = compute precision, [1] = FP64 refinement copy (if any)
  ppl::Region g;                       // build scratch G [pairs][v][v] (also the V-setup scratch)
  bool g_external = false;             // G lies outside the plan's layout (batched instances share one per
                                       // build branch); g_bytes_wanted is its size
  uint64_t g_bytes_wanted = 0;
  ppl::Region rp, rm;                  // R+ [N+][ldp], R- [N-][ldm] (accumulator type of the GEMM)
  ppl::Region part;                    // split-K slices of one contraction GEMM
  ppl::Region s64, a64;                // FP64 master amplitudes in S'/A' form when ops[*] are not FP64
  ppl::Region vs, va;                  // packed (ia|jb): VS [N+][ldp], VA [N-][ldm] (FP64)
  ppl::Region bs, ba;                  // FP64 copy of S'/A' kept across the two first sweeps of a checked start
  ppl::Region xov;                     // staged occupied-virtual block [(i,a)][ldx] (FP64)
  ppl::Region tab_vp, tab_vm, tab_op, tab_om;  // pair tables (int32)
  ppl::Region red;                     // reduction partials
  int diis_max = 0;                    // DIIS subspace capacity
  bool contract_only = false;          // no iteration buffers (PPL_PLAN_CONTRACT_ONLY)
  bool ring = false;                   // ring-term buffers reserved (PPL_PLAN_RING)
  ppl::Region ring_ws, tfull, rfull;   // ring scratch, full amplitudes and ring result
  std::string tune_cache;              // path of the tuned-configuration file ("" = none)
  int64_t diis_slot_n = 0;             // doubles per DIIS slot: S' rows [N+][ldp], then A' rows [N-][ldm]
  ppl::Region diis_t, diis_e;          // diis_max slots of amplitudes t' and of errors t' - t (S'/A' scaling)
  ppl::Region diis_red;                // DIIS inner-product partials and results
  ppl::Region tiles;                   // per-batch (row tile, column tile) lists of the build GEMM (int32 pairs)
  bool sym_build = false;              // build the upper triangle of V+- (resident: then mirror it;
                                       // streaming: contract U and U^T of each step, V = U + U^T)
  int64_t ldq = 0, ldqm = 0;           // row lengths of the transposed streaming results (pad N+, N-)
  int64_t ldk = 0;                     // row length of a transposed row block (its K range)
  ppl::Region r2p, r2m;                // streaming U^T term, transposed: [P+][ldq], [P-][ldqm] (FP64)
  ppl::Region ut;                      // one transposed row block of U+ or U-: [P+][ldk] (FP64)
  ppl::Region cols;                    // operand rows of the upper-triangle build's columns (int32, v(v+1)/2)
  ppl::Region cube_off;                // resident upper-triangle builds: cubes below each virtual (int64, v + 1)
  std::vector<int> cols_host;
  std::vector<int> tiles_host;         // host copy of the tile tables (kept alive for the async copy)
  std::vector<int64_t> tiles_off;      // element offset of each batch's list in `tiles`, [set][batch]
  std::vector<int64_t> tiles_n;        // tiles in each batch's list, [set][batch]
  int tile_sets = 1;                   // 2 when the FP64 copy builds on a tile of its own
  const double* L_last = nullptr;
  bool setup_done = false;
  // kernel timing
  struct ProfRec {
    int kind;
    int ev;          // index of the first of two events in prof_pool
    double flops;
  };
  bool prof_on = false;
  std::vector<hipEvent_t> prof_pool;
  std::vector<ProfRec> prof_recs;
  int prof_next = 0;
};

namespace ppl {

template <class T>
inline T* at(ppl_plan_t p, const Region& r) {
  return reinterpret_cast<T*>(p->ws + r.off);
}

// ------------------------------------------------------------------ kernels (launchers)
// All launchers enqueue on the given stream and return PPL_OK or PPL_E_HIP.

// Dense NT GEMM, C[M][N] = alpha * sum_k A[m][k] B[n][k] + beta * C (FP64 only; used
// for the occupied-virtual integrals). K must be padded to ld with zeros.
int gemm_store_f64(hipStream_t s, int64_t M, int64_t N, int64_t Kpad, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc);

// Contraction C[N][P] = sum_k S[n][k] V[p][k] for one operand set (R+ or R-).
// Output in the accumulator precision (double for FP64, float otherwise).
// S_lo / V_lo (and Xt_lo of the builds) point at the second bf16 plane: lo for BF16x3,
// mid for BF16x6, whose lo plane lies one plane further on (mid + (mid - hi)).
// splits > 1 splits K into that many slices written to `partial` ([splits][Nrows][partial_ld],
// accumulator type) and summed in slice order into C. accumulate: C += the product (one
// K slice only; PPL_E_ARG with split-K or stream-K).
int gemm_contract(hipStream_t s, int prec, int tile, int64_t Nrows, int64_t Prows, int64_t Kpad,
                  const void* S, const void* S_lo, int64_t lds_, const void* V, const void* V_lo,
                  int64_t ldv, void* C, int64_t ldc, int64_t c_col0, int splits, void* partial,
                  int64_t partial_ld, uint64_t partial_bytes, bool accumulate = false);
// bytes of partial slots a stream-K contraction (splits == 0) with this tile needs at most
uint64_t streamk_part_bytes(int tile, int prec, int64_t Nrows, int64_t Prows, int64_t Kpad);
int64_t contract_jobs(int tile, int prec, int64_t Nrows, int64_t Prows, int64_t Kpad, int splits);
// fewest K slices the planner and the autotuner use for a precision (more than one only
// for BF16x6, whose accuracy is limited by the length of its FP32 accumulations)
int contract_min_splits(int prec, int64_t Kpad);
// *tile_out >= 0 on entry fixes the tile and only chooses the split count
void contract_choose(int prec, int64_t Nrows, int64_t Prows, int64_t Kpad, int max_splits, int* tile_out,
                     int* splits_out);
// contraction tile the integral build GEMM of a plan runs on (measured at (20, 200, 600),
// (30, 300, 900) and (40, 400, 1200): 64 x 128 with direct loads for FP64 operands,
// 128 x 128 for FP32, 96 x 128 for BF16x3 and BF16x6)
#ifndef PPL_BUILD_TILE
#define PPL_BUILD_TILE 1     // FP32 integral-build tile (contraction tile id)
#endif
#ifndef PPL_BUILD_TILE_F64
#define PPL_BUILD_TILE_F64 8 // FP64 integral-build tile
#endif
inline int build_tile_for_prec(int prec) {
  return prec == PPL_BF16X3 || prec == PPL_BF16X6 ? 5 : (prec == PPL_FP64 ? PPL_BUILD_TILE_F64 : PPL_BUILD_TILE);
}
constexpr int kMaxSplits = 8;          // split-K slices 1 .. kMaxSplits; 0 selects stream-K
constexpr int64_t kStreamKMaxGrid = 1024;   // stream-K workgroups at most (partial slots: 2 each)
constexpr int64_t kStreamKMinChunks = 8;    // and at least this many K chunks per workgroup

// grouped persistent contraction (batched instances)
struct GroupDesc {       // byte offsets from the launch's base pointer (the batch workspace)
  int64_t a_off;         // S' or A' rows [M][lda]
  int64_t b_off;         // V+ or V- rows [N][ldb]
  int64_t c_off;         // R+ or R- [M][ldc]
  int64_t M, N, nk, lda, ldb, ldc;
  int cfg, pad;
};
bool grouped_tile_ok(int tile);
int grouped_choose_tile(int prec, int64_t rows);
void grouped_tile_dims(int tile, int* bm, int* bn);
// one work queue per XCD (workgroups are dealt to the XCDs round robin)
constexpr int kGroupedQueues = 8;
int gemm_grouped(hipStream_t s, int prec, char* base, const GroupDesc* groups, const int4* items, int n_items,
                 const int* q_begin, int* counters, int grid);

// Integral build G[pair(a,b) - pair(a0,a0)][c][d] = sum_P Xt[(a,c)][P] Xt[(b,d)][P]
// for a in [a0, a1), b in [a, v).
int gemm_build(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad,
               const void* Xt, const void* Xt_lo, int64_t ldx, void* G, const int* tile_list,
               int64_t n_valid_tiles);
// host helper: the valid (row tile, column tile) pairs of a build step in launch order
// (two ints per tile)
void build_tile_table(int tile, int v, int a0, int a1, std::vector<int>& tiles, int& n_mtiles,
                      int& n_ntiles);
int build_tile_dims(int tile, int* bm, int* bn);
// Upper-triangle build of a resident plan: G[pair(a,b) - pair(a0,a0)][c - a0][d - a0] =
// (ac|bd) for a in [a0, a1), b >= a, c >= a, d >= a (W = v - a0); rows are the packed
// pairs (a, c >= a) decoded through tab_vp, columns the operand rows in `cols`
// (build_column_order).
int gemm_build_sym(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                   const void* Xt_lo, int64_t ldx, void* G, const int* tile_list, int64_t n_valid_tiles,
                   const int* tab_vp, const int* cols);
// The same build in the GEMM's natural layout (resident plans): T[pair(a,c) - pr0][pair(b,d) - pr0]
// = (ac|bd), row length (v - a0)(v - a0 + 1) / 2, pr0 = pair(a0, a0), for b <= d and b >= a.
int gemm_build_natural(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                       const void* Xt_lo, int64_t ldx, void* T, const int* tile_list, int64_t n_valid_tiles,
                       const int* tab_vp, const int* cols);
void build_tile_table_sym(int tile, int v, int a0, int a1, std::vector<int>& tiles, int& n_mtiles,
                          int& n_ntiles);
void build_column_order(int v, std::vector<int>& cols);
void contract_tile_dims(int tile, int* bm, int* bn, int* threads);
int contract_tile_count();
int contract_tile_default(int prec, int64_t Nrows);

// staging: Xt[(a,c)][P] = L[P][o+a][o+c] in the operand precision (zero padding up to ldx)
int stage_vv(hipStream_t s, int prec, const double* L, int o, int v, int naux, int64_t ldx, void* xt,
             void* xt_lo);
// staging: Xov[(i,a)][P] = L[P][i][o+a] (FP64)
int stage_ov(hipStream_t s, const double* L, int o, int v, int naux, int64_t ldx, double* xov);
// pack G (accumulator precision) into V+ / V- rows of one batch (operand precision)
int pack_vpm(hipStream_t s, int prec, int v, int a0, int a1, const void* G, void* vp, void* vp_lo,
             int64_t ldp, int64_t vp_row0, void* vm, void* vm_lo, int64_t ldm, int64_t vm_row0,
             const int* tab_vp, const int* tab_vm);
// upper triangle of V+- rows from an upper-triangle build step (gemm_build_sym); resident rows
// (resident: vp_row0 = vm_row0 = 0, half_diag = 0; streaming: rows relative to the
// step's first pair, diagonal halved so that V = U + U^T, columns from zp / zm up to
// the row's own pair zeroed)
int pack_vpm_sym(hipStream_t s, int prec, int v, int a0, int a1, const void* G, void* vp, void* vp_lo,
                 int64_t ldp, void* vm, void* vm_lo, int64_t ldm, const int* tab_vp, int64_t vp_row0 = 0,
                 int64_t vm_row0 = 0, int half_diag = 0, int64_t zp = 0, int64_t zm = 0);
// whole V+- rows (and their mirror entries) of a resident build step from gemm_build_natural's
// T (row length ldt); off[a] = cubes of the virtuals below a (pack_cubes.h), v + 1 entries
int pack_vpm_cubes(hipStream_t s, int prec, int v, int a0, int a1, const void* T, int64_t ldt, const int64_t* off,
                   void* vp, void* vp_lo, int64_t ldp, void* vm, void* vm_lo, int64_t ldm);
// C[q][p] += T[p][q] for q < nq, p < np (T FP64; C FP64 or FP32 by c_prec)
int add_transposed(hipStream_t s, int c_prec, void* C, int64_t ldc, const double* T, int64_t ldt, int64_t nq,
                   int64_t np);
// Y[p][q] = w X[q][p] (q < nq, p < np), and with pad zero for nq <= q < ldy; scaled:
// w = (2 - d_kl) / (2 - d_ab) with (k, l) = tab_q[q], (a, b) = tab_p[p]
int transpose_pm(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t nq, int64_t np,
                 const int* tab_q, const int* tab_p, int scaled, int pad = 1);
// Ut[r][k] = U[k0 + k - u0][c0 + r] for u0 <= k0 + k < u1, else 0 (r < nr, k < nk)
int transpose_block(hipStream_t s, int elem_bytes, const void* U, int64_t ldu, int64_t u0, int64_t u1, int64_t c0,
                    int64_t k0, void* Ut, int64_t ldt, int64_t nr, int64_t nk);
// V[r][q] = V[q][r] for q < r (bit copy of elem_bytes-wide elements)
int mirror_lower(hipStream_t s, int elem_bytes, void* V, int64_t n, int64_t ld);
// pair tables
int fill_tables(hipStream_t s, int o, int v, int* tab_vp, int* tab_vm, int* tab_op, int* tab_om);
// generic pack of an (i,j,a,b)-indexed FP64 tensor into + / - packed rows:
//   plus [q(i<=j)][p(a<=b)] = (a<b ? sp_off : sp_diag) * (X^ab + X^ba)
//   minus[q(i<j)][p(a<b)]   = am * (X^ab - X^ba)
// where, with t1 ([i][a], row length v), X_ij^ab stands for X_ij^ab + t1_i^a t1_j^b
int pack_pm(hipStream_t s, int o, int v, const double* X, int64_t si, int64_t sj, int64_t sa,
            int64_t sb, double sp_off, double sp_diag, double am, double* plus, int64_t ldp,
            double* minus, int64_t ldm, const int* tab_op, const int* tab_om, const int* tab_vp,
            const int* tab_vm, const double* t1 = nullptr);
// staging: Xoo[(k,i)][P] = L[P][k][i] (FP64)
int stage_oo(hipStream_t s, const double* L, int o, int v, int naux, int64_t ldx, double* xoo);

// convert FP64 packed rows to an operand precision (FP32 or BF16 hi/lo), zero padding kept
int convert_rows(hipStream_t s, int prec, const double* src, int64_t rows, int64_t cols, int64_t ld,
                 void* dst, void* dst_lo);
// unpack R = beta R + alpha (R+ +- R-) into [o][o][v][v]
int unpack_r(hipStream_t s, int acc_prec, int o, int v, const void* rp, int64_t ldp, const void* rm,
             int64_t ldm, double* R, double alpha, double beta);
// packed amplitudes S'/A' (FP64) back to the full pair-symmetric t2
int unpack_t(hipStream_t s, int o, int v, const double* sp, int64_t ldp, const double* am,
             int64_t ldm, double* t2);
// MP2 start S' = (2 - delta_ab) VS / D, A' = 2 VA / D (red_out[1] = its energy)
int mp2_start(hipStream_t s, int o, int v, const double* e_occ, const double* e_vir, const double* vs,
              const double* va, int64_t ldp, int64_t ldm, double* sp, double* am, const int* tab_op,
              const int* tab_om, const int* tab_vp, const int* tab_vm, double* partials,
              double* red_out);
// Jacobi update in packed space with FP64 residual^2 / energy partial sums
// (red_out[0] = r^2, red_out[1] = E, red_out[2] = non-finite count)
// tslot / eslot (both or neither): DIIS slots that also receive the new amplitudes and
// the error new - old in the packed scaling (padding columns untouched)
int update_sweep(hipStream_t s, int acc_prec, int o, int v, const double* e_occ, const double* e_vir,
                 const double* vs, const double* va, const void* rp, const void* rm, int64_t ldp,
                 int64_t ldm, double* sp, double* am, const int* tab_op, const int* tab_om,
                 const int* tab_vp, const int* tab_vm, double* partials, double* red_out,
                 double* tslot = nullptr, double* eslot = nullptr);
// DIIS: the vectors of a subspace (slot ids) and their extrapolation coefficients
constexpr int kDiisMax = 16;
static_assert(kDiisMax == PPL_DIIS_MAX, "one DIIS capacity limit");
struct DiisSet {
  int n;
  int id[kDiisMax];
  double c[kDiisMax];
};
// out[i] = <E_knew, E_id[i]> over the full tensors, i < set.n (partials: kReduceBlocks x kDiisMax)
int diis_dots(hipStream_t s, int o, int v, int64_t ldp, int64_t ldm, const int* tab_op, const int* tab_om,
              const int* tab_vp, const int* tab_vm, const double* E, int64_t slot_n, const DiisSet& set,
              int knew, double* partials, double* out);
// S'/A' = sum_i c_i T_id[i], zero padding
int diis_combine(hipStream_t s, int o, int v, int64_t ldp, int64_t ldm, const double* T, int64_t slot_n,
                 const DiisSet& set, double* sp, double* am);
// energy of the current packed amplitudes (red_out[1] = E)
int energy_only(hipStream_t s, int o, int v, const double* vs, const double* va, const double* sp,
                const double* am, int64_t ldp, int64_t ldm, const int* tab_op, const int* tab_om,
                const int* tab_vp, const int* tab_vm, double* partials, double* red_out);
// zero a device range (a fill kernel, never hipMemsetAsync)
int zero_bytes(hipStream_t s, void* p, uint64_t bytes);
// ring terms: (o v) x (o v) operands over the pairs (i,a), (k,c) (rows of ld elements)
int ring_pack(hipStream_t s, int o, int v, const double* t, int64_t ld, double* Xa, double* An, double* B);
// the same operands in precision prec (FP32, or bf16 planes: each *_lo is the lo / mid plane)
int ring_pack_lp(hipStream_t s, int prec, int o, int v, const double* t, int64_t ld, void* Xa, void* Xa_lo,
                 void* An, void* An_lo, void* B, void* B_lo);
int ring_exchange(hipStream_t s, int o, int v, const double* G, int64_t ldg, double* K, int64_t ld);
int ring_unpack(hipStream_t s, int o, int v, const double* C1, const double* C2, int64_t ld, double* R, double alpha,
                double beta);
int ring_unpack_f32(hipStream_t s, int o, int v, const float* C1, const float* C2, int64_t ld, double* R, double alpha,
                    double beta);
// rp[(ij)][(ab)] += (R_ij^ab + R_ij^ba) / 2 (i <= j, a <= b), rm[(ij)][(ab)] += (R_ij^ab - R_ij^ba) / 2
// (i < j, a < b): a pair-symmetric [o][o][v][v] tensor added to R+- (accumulator precision c_prec)
int add_pm(hipStream_t s, int c_prec, int o, int v, const double* R, void* rp, int64_t ldp, void* rm, int64_t ldm,
           const int* tab_op, const int* tab_om, const int* tab_vp, const int* tab_vm);
// red_out[0] = sum (L^P_ac - L^P_ca)^2, red_out[1] = sum (L^P_ac)^2 + (L^P_ca)^2 over a < c (virtual block)
int asymmetry_vv(hipStream_t s, const double* L, int o, int v, int naux, double* partials, double* red_out);
// count non-finite values of an FP64 array (red_out[2])
int count_nonfinite(hipStream_t s, const double* x, int64_t n, double* partials, double* red_out);

// learned start
int mlp_param_count();
int mlp_train_rows();
int mlp_train_launch(hipStream_t s, const float* prm, const float* X, const float* Y, int64_t n,
                     float* gpart, float* lpart, float* grad, float* loss);
int mlp_adam_launch(hipStream_t s, float* prm, const float* grad, float* m, float* v, float lr, int step,
                    float beta1, float beta2, float eps);
int mlp_samples_launch(hipStream_t s, int o, int v, const double* tm, const double* ts, const double* e_occ,
                       const double* e_vir, double sigma, const int64_t* idx, int64_t n, float* X, float* Y);
int mlp_infer_launch(hipStream_t s, const float* prm, int o, int v, const double* tm, const double* e_occ,
                     const double* e_vir, double sigma, const int* tab_om, const int* tab_vp, double* tout);
int sumsq_launch(hipStream_t s, const double* x, int64_t n, double* partials, double* red_out);

constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

}  // namespace ppl
