// MFMA GEMM tiles of the PPL hot path on gfx950.
//
// Every product of the method is an "NT" product of two K-contiguous operands,
//     C[m][n] = sum_k A[m][k] * B[n][k],
// which is the natural layout of the matrix-core fragments:
//   * integral build (eq. (cholesky)): A = B = Xt[(a,c)][P] (virtual block of L,
//     transposed), C = G_ab[c][d] = (ac|bd) for a <= b;
//   * contraction (eq. (vfunction-chol)): A = S'[(ij)][(cd)], B = V+[(ab)][(cd)]
//     (V+- are symmetric matrices, so their rows are also their columns),
//     C = R+[(ij)][(ab)]; the same for A'/V-/R-.
//
// Tiles: a workgroup of WAVES_M x WAVES_N wavefronts (64 lanes each) owns a
// BM x BN block of C; each wave owns WM x WN MFMA blocks of 16 x 16. K is
// consumed in chunks of KC staged through LDS with two buffers: the global
// loads of chunk k+1 are in flight while chunk k feeds the matrix cores.
// Operand rows are padded with zeros to a multiple of 64 elements, so the K
// loop never tests bounds; rows beyond M / N are clamped on load and masked
// on store.
//
// Fragment layouts (16x16 output blocks, 64 lanes, l = lane, r = 0..3), as
// measured on gfx950 with one-hot operands:
//   f64 16x16x4:   lane l holds A[l%16][l/16], B[l/16][l%16], D[4*r + l/16][l%16];
//   f32 16x16x4:   lane l holds A[l%16][l/16], B[l/16][l%16], D[4*(l/16) + r][l%16];
//   bf16 16x16x32: lane l holds A[l%16][8*(l/16)+0..7], B[8*(l/16)+0..7][l%16],
//                  D[4*(l/16) + r][l%16].
#include <cmath>

#include "ppl_internal.h"

namespace ppl {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// 16 bytes as a native vector (register staging of K chunks; HIP's uint4 is a struct
// with a union, which keeps loop-carried arrays of it in scratch memory)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// accumulator type and the row (within a 16x16 block) of accumulator register r of lane l
template <class T> struct AccOf;
template <> struct AccOf<double> {
  using type = double;
  using vec = d4;
  __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct AccOf<float> {
  using type = float;
  using vec = f4;
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct AccOf<__bf16> {
  using type = float;
  using vec = f4;
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Spread a launch over the 8 XCDs so that each XCD walks a contiguous run of
// logical tiles: consecutive workgroup ids land on different XCDs, so logical
// tile t of XCD x is x*q + min(x, r) + j for the j-th id it receives.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t total) {
  const int64_t x = bid % 8, j = bid / 8, q = total / 8, r = total % 8;
  return x * q + (x < r ? x : r) + j;
}

#ifndef PPL_SPLIT_OUTER
#define PPL_SPLIT_OUTER 1
#endif

// ------------------------------------------------------------------ tile maps
struct TileJob {
  int64_t m0, n0;        // first row / column of the C tile
  int64_t kc0, kc1;      // K chunks [kc0, kc1) of this job
  int split;             // split-K slice written by this job
};

// Dense grid with an optional split of K into `splits` slices. Logical order:
// row tile fastest, then column tile, then split, so jobs that read the same
// B rows run next to each other on one XCD and each XCD works on one K slice at
// a time: its resident workgroups then share that slice of the A rows in L2 (with
// the split innermost, every XCD streamed all slices of A at once and re-fetched
// them from HBM; R+ at (20, 200, 600) read 1.3x its algorithmic bytes, now 1.05x).
struct MapGrid {
  int64_t n_mt, n_nt;
  int bm, bn;
  int splits;
  int64_t nk, kps;       // K chunks in total and per split
  __device__ bool operator()(int64_t bid, TileJob& j) const {
    const int64_t t = xcd_remap(bid, n_mt * n_nt * splits);
#if PPL_SPLIT_OUTER
    const int64_t per = n_mt * n_nt, r = t % per;
    j.split = (int)(t / per);
    j.m0 = (r % n_mt) * bm;
    j.n0 = (r / n_mt) * bn;
#else
    const int64_t r = t / n_mt;
    j.m0 = (t % n_mt) * bm;
    j.split = (int)(r % splits);
    j.n0 = (r / splits) * bn;
#endif
    j.kc0 = j.split * kps;
    j.kc1 = j.kc0 + kps < nk ? j.kc0 + kps : nk;
    return true;
  }
};

struct MapBuild {        // block-upper-triangle of the (a,c) x (b,d) grid: only tiles with some b >= a
  const int* tiles;      // (row tile, column tile) of each job, in launch order
  int64_t total;
  int bm, bn;
  int64_t nk;
  __device__ bool operator()(int64_t bid, TileJob& j) const {
    const int64_t t = xcd_remap(bid, total);
    j.m0 = (int64_t)tiles[2 * t] * bm;
    j.n0 = (int64_t)tiles[2 * t + 1] * bn;
    j.kc0 = 0;
    j.kc1 = nk;
    j.split = 0;
    return true;
  }
};

// ------------------------------------------------------------------ epilogues
template <class Tc>
struct EpiStore {        // C[split][m][c_col0 + n] = alpha * acc + beta * C (beta == 0: no read)
  __device__ int64_t arow(int64_t r) const { return r; }   // operand rows of C row / column r
  __device__ int64_t brow(int64_t r) const { return r; }
  Tc* C;
  int64_t ldc, c_col0, M, N;
  double alpha, beta;
  int64_t split_stride;  // elements between split-K slices
  __device__ void row(int split, int64_t m, int64_t& base, bool& ok) const {
    ok = m < M;
    base = split * split_stride + m * ldc + c_col0;
  }
  __device__ void put(int64_t base, bool ok, int64_t n, typename AccOf<Tc>::type x) const {
    if (!ok || n >= N) return;
    Tc* p = C + base + n;
    if (beta == 0.0) *p = (Tc)(alpha * x);
    else *p = (Tc)(alpha * x + beta * (double)*p);
  }
};

template <class Tc>
struct EpiSK {           // stream-K: whole tiles go to C, shared tiles to a dense BM x BN partial slot
  __device__ int64_t arow(int64_t r) const { return r; }   // operand rows of C row / column r
  __device__ int64_t brow(int64_t r) const { return r; }
  Tc* C;
  int64_t ldc, c_col0, M, N;
  Tc* P;                 // partial slot of this tile (to_part) or unused
  int64_t m0, n0;
  int ldp;               // = BN
  bool to_part;
  __device__ void row(int, int64_t m, int64_t& base, bool& ok) const {
    if (to_part) {
      ok = true;
      base = (m - m0) * ldp - n0;
    } else {
      ok = m < M;
      base = m * ldc + c_col0;
    }
  }
  __device__ void put(int64_t base, bool ok, int64_t n, typename AccOf<Tc>::type x) const {
    if (to_part) P[base + n] = (Tc)x;
    else if (ok && n < N) C[base + n] = (Tc)x;
  }
};

template <class Tg>
struct EpiBuild {        // G[pair(a,b) - pair(a0,a0)][c][d] for b >= a
  __device__ int64_t arow(int64_t r) const { return r; }   // operand rows of C row / column r
  __device__ int64_t brow(int64_t r) const { return r; }
  Tg* G;
  int64_t M, N;
  int v, a0;
  // per-row: a, c; per-col: b, d
  __device__ void row(int, int64_t m, int64_t& base, bool& ok) const {
    ok = m < M;
    const int64_t arel = m / v, c = m - arel * v;
    // encode a (relative) and c in base: rows are combined with columns in put()
    base = (arel << 20) | c;
  }
  __device__ void put(int64_t base, bool ok, int64_t n, Tg x) const {
    if (!ok || n >= N) return;
    const int64_t arel = base >> 20, c = base & ((1 << 20) - 1);
    const int64_t brel = n / v, d = n - brel * v;
    if (brel < arel) return;
    const int64_t a = a0 + arel, b = a0 + brel;
    const int64_t pr = pair_plus(a, b, v) - pair_plus(a0, a0, v);
    G[(pr * v + c) * v + d] = x;
  }
};

// Upper-triangle build of a resident plan. Rows are the packed pairs (a, c), c >= a, of
// the step's virtuals a in [a0, a1) (packed pairs pr0 + m); columns are the packed pairs
// (b, d), b <= d, as operand rows b * v + d listed in `cols` (ordered by b, starting at
// b = a0). Only (ac|bd) with b, d >= a is kept: G[pair(a,b) - pr0][c - a0][d - a0] and its
// mirror G[pair(a,d) - pr0][c - a0][b - a0], W = v - a0.
template <class Tg>
struct EpiBuildSym {
  Tg* G;
  int64_t M, N;
  int v, a0, W;
  int64_t pr0;
  const int* tab;        // packed pair -> (first << 16) | second
  const int* cols;       // column n -> operand row b * v + d
  __device__ int64_t arow(int64_t m) const {
    const int ac = tab[pr0 + m];
    return (int64_t)pair_first(ac) * v + pair_second(ac);
  }
  __device__ int64_t brow(int64_t n) const { return cols[n]; }
  __device__ void row(int, int64_t m, int64_t& base, bool& ok) const {
    ok = m < M;
    const int ac = ok ? tab[pr0 + m] : 0;
    base = ((int64_t)pair_first(ac) << 20) | pair_second(ac);
  }
  // Column n is the packed pair (b <= d); (ac|bd) = (ac|db) for symmetric Cholesky vectors,
  // so the product fills G_ab[c][d] and G_ad[c][b].
  __device__ void put(int64_t base, bool ok, int64_t n, Tg x) const {
    if (!ok || n >= N) return;
    const int a = (int)(base >> 20), c = (int)(base & ((1 << 20) - 1));
    const int bd = cols[n];
    const int b = bd / v, d = bd - b * v;
    if (b < a) return;
    const int64_t cr = c - a0;
    G[((pair_plus(a, b, v) - pr0) * W + cr) * W + (d - a0)] = x;
    if (d != b) G[((pair_plus(a, d, v) - pr0) * W + cr) * W + (b - a0)] = x;
  }
};

// Upper-triangle build of a resident plan in the GEMM's natural layout: rows and columns
// as in EpiBuildSym, T[m * ldt + n] = (ac|bd) for row m = pair(a, c) - pr0 and column
// n = pair(b, d) - pr0 (b <= d; computed for b >= a of the row tile's first virtual). The
// packing (pack_vpm_cubes) reads both (ac|bd) and (ad|bc) from it.
template <class Tg>
struct EpiBuildT {
  Tg* T;
  int64_t M, N, ldt;
  int v;
  int64_t pr0;
  const int* tab;        // packed pair -> (first << 16) | second
  const int* cols;       // column n -> operand row b * v + d
  __device__ int64_t arow(int64_t m) const {
    const int ac = tab[pr0 + m];
    return (int64_t)pair_first(ac) * v + pair_second(ac);
  }
  __device__ int64_t brow(int64_t n) const { return cols[n]; }
  __device__ void row(int, int64_t m, int64_t& base, bool& ok) const {
    ok = m < M;
    base = m * ldt;
  }
  __device__ void put(int64_t base, bool ok, int64_t n, Tg x) const {
    if (ok && n < N) T[base + n] = x;
  }
};

// ------------------------------------------------------------------ the kernel (FP64 / FP32)
// LDS layout of a staged K chunk (BM or BN rows of KC elements, moved as 16-byte vectors):
//   0: each row padded by 16 bytes;
//   1: unpadded rows, vector kv of row r stored at vector slot kv ^ (r % (KC / VEC)).
// Fragment reads (PPL_FRAG_VEC):
//   0: one element per lane per MFMA (lane l holds k = l / 16 of the 4-wide step);
//   1: one 16-byte vector per lane covering VEC consecutive MFMA steps: in step e
//      lane l holds k = VEC * (l / 16) + e of the 4 * VEC-wide group. A and B use
//      the same assignment, so every k is paired exactly once.
#ifndef PPL_LDS_LAYOUT
#define PPL_LDS_LAYOUT 1
#endif
#ifndef PPL_FRAG_VEC
#define PPL_FRAG_VEC 1
#endif
#ifndef PPL_SCHED_FENCE
#define PPL_SCHED_FENCE 0
#endif
#ifndef PPL_DIRECT_LDS
#define PPL_DIRECT_LDS 0
#endif
#ifndef PPL_PREFETCH
#define PPL_PREFETCH 0
#endif
#ifndef PPL_BF3_DIRECT
#define PPL_BF3_DIRECT 1
#endif
#ifndef PPL_BF6_DIRECT
#define PPL_BF6_DIRECT 1
#endif
#ifndef PPL_FP_DIRECT3
#define PPL_FP_DIRECT3 1
#endif
#ifndef PPL_BUILD_DIRECT3
#define PPL_BUILD_DIRECT3 1
#endif
#ifndef PPL_GROUPED_DIRECT3
#define PPL_GROUPED_DIRECT3 1
#endif
constexpr int kLdsLayout = PPL_LDS_LAYOUT;
constexpr int kFragVec = PPL_FRAG_VEC;
constexpr int kSchedFence = PPL_SCHED_FENCE;
constexpr int kDirectLds = PPL_DIRECT_LDS;   // 1: chunks go global -> LDS without registers (layout 1 only)
constexpr int kPrefetch = PPL_PREFETCH;      // chunks in flight in registers: 1, 2, or 0 = per tile (below)
constexpr int kBf3Direct = PPL_BF3_DIRECT;   // 1: BF16x3 chunks go global -> LDS, three stages, two in flight
constexpr int kBf6Direct = PPL_BF6_DIRECT;   // 1: BF16x6 chunks go global -> LDS, two stages
constexpr int kFpDirect3 = PPL_FP_DIRECT3;   // 1: FP64 / FP32 contraction chunks go global -> LDS, three stages
static_assert(!kDirectLds || kLdsLayout == 1, "direct LDS loads need the unpadded swizzled layout");

template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC>
struct TileGeom {
  static constexpr int NT = 64 * WAVES_M * WAVES_N;
  static constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  static constexpr int LDSR = kLdsLayout == 0 ? KC + 16 / (int)sizeof(T) : KC;
  static constexpr int BUF_A = BM * LDSR, BUF_B = BN * LDSR;   // elements of one buffer
  static constexpr int LDS_BYTES = 2 * (BUF_A + BUF_B) * (int)sizeof(T);
};

// element offset of 16-byte vector kv of staged row r
template <int VEC, int VPR, int LDSR>
__device__ __forceinline__ int lds_vec_off(int r, int kv) {
  if constexpr (kLdsLayout == 0) return r * LDSR + kv * VEC;
  else return r * LDSR + ((kv ^ (r % VPR)) * VEC);
}

// Multiply one staged chunk (As: A rows, Bs: B rows, LDSR elements apart) into acc.
template <class T, int WM, int WN, int KC, int LDSR>
__device__ __forceinline__ void consume_chunk(typename AccOf<T>::vec (&acc)[WM][WN], const T* __restrict__ As,
                                              const T* __restrict__ Bs, int arow, int brow, int fq, int key) {
  constexpr int VEC = 16 / sizeof(T);
  if constexpr (kFragVec) {
#pragma unroll
    for (int kg = 0; kg < KC / (4 * VEC); ++kg) {
      const int col = ((kg * 4 + fq) ^ key) * VEC;
      union U { uint4 u; T e[VEC]; };
      U a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i].u = *reinterpret_cast<const uint4*>(&As[arow + i * 16 * LDSR + col]);
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j].u = *reinterpret_cast<const uint4*>(&Bs[brow + j * 16 * LDSR + col]);
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[i][j] = mfma16(a[i].e[e], b[j].e[e], acc[i][j]);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int c = kk + fq;
      const int col = ((c / VEC) ^ key) * VEC + c % VEC;
      T a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = As[arow + i * 16 * LDSR + col];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Bs[brow + j * 16 * LDSR + col];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
    }
  }
}

// Write the accumulators of one wave (16-row blocks i, 16-column blocks j) through the epilogue.
template <class T, int WM, int WN, class Epi>
__device__ __forceinline__ void store_acc(typename AccOf<T>::vec (&acc)[WM][WN], const TileJob& job, const Epi& epi,
                                          int wm, int wn, int lane) {
#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = job.m0 + wm * WM * 16 + i * 16 + AccOf<T>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(job.split, m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = job.n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r]);
      }
    }
  }
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void global_cvoid_t;

// The tile with chunks moved straight from global memory into LDS: one wave
// instruction fills 64 / VPR whole staged rows (1 KB, one 16-byte vector per lane),
// lane l taking the global vector that the swizzled layout keeps at its slot.
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi>
__device__ __forceinline__ void tile_body_direct(const TileJob& job, int64_t M, int64_t N, const T* __restrict__ A,
                                                 int64_t lda, const T* __restrict__ B, int64_t ldb, const Epi& epi,
                                                 T* __restrict__ a0, T* __restrict__ a1, T* __restrict__ b0,
                                                 T* __restrict__ b1) {
  using accv = typename AccOf<T>::vec;
  constexpr int NW = WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int LDSR = TileGeom<T, WM, WN, WAVES_M, WAVES_N, KC>::LDSR;
  constexpr int VPR = KC / VEC;
  constexpr int RPI = 64 / VPR;                   // staged rows per wave instruction
  constexpr int GA = BM / RPI, GB = BN / RPI;     // wave instructions per chunk
  constexpr int IA = (GA + NW - 1) / NW, IB = (GB + NW - 1) / NW;
  static_assert(LDSR == KC && 64 % VPR == 0 && BM % RPI == 0 && BN % RPI == 0, "direct LDS geometry");
  static_assert(KC % (4 * VEC) == 0 && 16 % VPR == 0, "bad KC");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int lr = lane / VPR, slot = lane % VPR;

  const T* pa[IA];
  const T* pb[IB];
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int g = wave + i * NW, r = g * RPI + lr;
    int64_t gr = job.m0 + r;
    if (gr > M - 1) gr = M - 1;
    pa[i] = A + epi.arow(gr) * lda + (slot ^ (r % VPR)) * VEC + job.kc0 * KC;
  }
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int g = wave + i * NW, r = g * RPI + lr;
    int64_t gr = job.n0 + r;
    if (gr > N - 1) gr = N - 1;
    pb[i] = B + epi.brow(gr) * ldb + (slot ^ (r % VPR)) * VEC + job.kc0 * KC;
  }
  // chunk c (relative to job.kc0) into LDS buffer `buf`
  auto issue = [&](int64_t c, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int g = wave + i * NW;
      if (g < GA)
        __builtin_amdgcn_global_load_lds((global_cvoid_t*)(pa[i] + c * KC),
                                         (lds_void_t*)((buf ? a1 : a0) + g * RPI * LDSR), 16, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int g = wave + i * NW;
      if (g < GB)
        __builtin_amdgcn_global_load_lds((global_cvoid_t*)(pb[i] + c * KC),
                                         (lds_void_t*)((buf ? b1 : b0) + g * RPI * LDSR), 16, 0, 0);
    }
  };

  accv acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = accv{0, 0, 0, 0};
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (wn * WN * 16 + (lane & 15)) * LDSR;
  const int fq = lane >> 4;
  const int key = (lane & 15) % VPR;
  const int64_t nk = job.kc1 - job.kc0;

  // two steps per loop trip so that every LDS access names its buffer (four distinct
  // objects: the compiler then needs no wait on the DMA into one buffer before
  // reading the other)
  issue(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  int64_t kt = 0;
  for (; kt + 2 < nk; kt += 2) {
    issue(kt + 1, 1);
    consume_chunk<T, WM, WN, KC, LDSR>(acc, a0, b0, arow, brow, fq, key);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's part of chunk kt+1 is in LDS
    __syncthreads();
    issue(kt + 2, 0);
    consume_chunk<T, WM, WN, KC, LDSR>(acc, a1, b1, arow, brow, fq, key);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  if (kt + 1 < nk) {   // chunks kt (buffer 0) and kt + 1 (buffer 1) remain
    issue(kt + 1, 1);
    consume_chunk<T, WM, WN, KC, LDSR>(acc, a0, b0, arow, brow, fq, key);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    consume_chunk<T, WM, WN, KC, LDSR>(acc, a1, b1, arow, brow, fq, key);
  } else {             // chunk kt (buffer 0) remains
    consume_chunk<T, WM, WN, KC, LDSR>(acc, a0, b0, arow, brow, fq, key);
  }
  store_acc<T, WM, WN>(acc, job, epi, wm, wn, lane);
}

// The FP64 / FP32 tile with chunks moved straight from global memory into LDS in three
// stages (the scheme of the BF16x3 tile below: step k reads its fragments of chunk k,
// issues chunk k+2 into the stage chunk k-1 left, multiplies, then waits for its part of
// chunk k+1 and meets the other waves). One stage holds BM rows of A, then BN rows of B.
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi>
__device__ __forceinline__ void tile_body_direct3(const TileJob& job, int64_t M, int64_t N, const T* __restrict__ A,
                                                  int64_t lda, const T* __restrict__ B, int64_t ldb, const Epi& epi,
                                                  T* __restrict__ st0, T* __restrict__ st1, T* __restrict__ st2) {
  using accv = typename AccOf<T>::vec;
  constexpr int NW = WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int LDSR = KC;
  constexpr int VPR = KC / VEC;                   // 16-byte vectors per staged row
  constexpr int RPI = 64 / VPR;                   // staged rows per wave instruction
  constexpr int GA = BM / RPI, GB = BN / RPI;
  constexpr int GT = GA + GB;                     // instructions per chunk
  constexpr int NI = (GT + NW - 1) / NW;          // per wave (the short waves repeat one)
  static_assert(kLdsLayout == 1 && 64 % VPR == 0 && BM % RPI == 0 && BN % RPI == 0 && GT >= NW && NI < 16,
                "direct LDS geometry");
  static_assert(KC % (4 * VEC) == 0 && 16 % VPR == 0, "bad KC");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int lr = lane / VPR, slot = lane % VPR;

  const T* src[NI];
  int dst[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    int q = wave + i * NW;
    if (q >= GT) q -= GT;
    if (q < GA) {
      const int r = q * RPI + lr;
      int64_t gr = job.m0 + r;
      if (gr > M - 1) gr = M - 1;
      src[i] = A + epi.arow(gr) * lda + (slot ^ (r % VPR)) * VEC + job.kc0 * KC;
      dst[i] = q * RPI * LDSR;
    } else {
      const int r = (q - GA) * RPI + lr;
      int64_t gr = job.n0 + r;
      if (gr > N - 1) gr = N - 1;
      src[i] = B + epi.brow(gr) * ldb + (slot ^ (r % VPR)) * VEC + job.kc0 * KC;
      dst[i] = (BM + (q - GA) * RPI) * LDSR;
    }
  }
  auto issue = [&](int64_t c, T* st) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
      __builtin_amdgcn_global_load_lds((global_cvoid_t*)(src[i] + c * KC), (lds_void_t*)(st + dst[i]), 16, 0, 0);
  };
  auto wait_one = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70 | NI);
    asm volatile("" ::: "memory");
  };
  auto wait_all = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    asm volatile("" ::: "memory");
  };
  auto meet = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  accv acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = accv{0, 0, 0, 0};
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (BM + wn * WN * 16 + (lane & 15)) * LDSR;
  const int fq = lane >> 4;
  const int key = (lane & 15) % VPR;
  const int64_t nk = job.kc1 - job.kc0;

  auto compute = [&](const T* __restrict__ st, bool go, int64_t c, T* nx) __attribute__((always_inline)) {
#pragma unroll
    for (int kg = 0; kg < KC / (4 * VEC); ++kg) {
      const int col = ((kg * 4 + fq) ^ key) * VEC;
      union U { uint4 u; T e[VEC]; };
      U a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i].u = *reinterpret_cast<const uint4*>(&st[arow + i * 16 * LDSR + col]);
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j].u = *reinterpret_cast<const uint4*>(&st[brow + j * 16 * LDSR + col]);
      if (kg == 0) {
        asm volatile("" ::: "memory");
        if (go) issue(c, nx);
      }
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[i][j] = mfma16(a[i].e[e], b[j].e[e], acc[i][j]);
    }
  };

  issue(0, st0);
  if (nk > 1) {
    issue(1, st1);
    wait_one();
  } else {
    wait_all();
  }
  meet();
  int64_t kt = 0;
  for (; kt + 7 < nk; kt += 6) {   // six steps whose k+2 exists
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      compute(st0, true, kt + 3 * u + 2, st2);
      wait_one();
      meet();
      compute(st1, true, kt + 3 * u + 3, st0);
      wait_one();
      meet();
      compute(st2, true, kt + 3 * u + 4, st1);
      wait_one();
      meet();
    }
  }
  for (int64_t j = kt; j < nk; ++j) {
    const int sj = (int)((j - kt) % 3);
    const T* cur = sj == 0 ? st0 : (sj == 1 ? st1 : st2);
    T* nx = sj == 0 ? st2 : (sj == 1 ? st0 : st1);
    compute(cur, j + 2 < nk, j + 2, nx);
    if (j + 1 < nk) {
      if (j + 2 < nk) wait_one();
      else wait_all();
      meet();
    }
  }
  store_acc<T, WM, WN>(acc, job, epi, wm, wn, lane);
}

// Fetch chunk c (relative to the job's first chunk) of the staged rows into registers,
// and store such registers into one LDS buffer.
template <class T, int NLA, int NLB, int KC>
__device__ __forceinline__ void chunk_load(u32x4 (&ra)[NLA], u32x4 (&rb)[NLB], const T* const (&pa)[NLA],
                                           const T* const (&pb)[NLB], int64_t c) {
#pragma unroll
  for (int i = 0; i < NLA; ++i) ra[i] = *reinterpret_cast<const u32x4*>(pa[i] + c * KC);
#pragma unroll
  for (int i = 0; i < NLB; ++i) rb[i] = *reinterpret_cast<const u32x4*>(pb[i] + c * KC);
}

template <class T, int NLA, int NLB>
__device__ __forceinline__ void chunk_store(const u32x4 (&ra)[NLA], const u32x4 (&rb)[NLB], T* sA, T* sB,
                                            const int (&oa)[NLA], const int (&ob)[NLB]) {
#pragma unroll
  for (int i = 0; i < NLA; ++i) *reinterpret_cast<u32x4*>(&sA[oa[i]]) = ra[i];
#pragma unroll
  for (int i = 0; i < NLB; ++i) *reinterpret_cast<u32x4*>(&sB[ob[i]]) = rb[i];
}

// One BM x BN tile of C over the K chunks [job.kc0, job.kc1); sA0 / sA1 (sB0 / sB1)
// are the two LDS buffers of BM (BN) staged rows.
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi>
__device__ __forceinline__ void tile_body(const TileJob& job, int64_t M, int64_t N, const T* __restrict__ A,
                                          int64_t lda, const T* __restrict__ B, int64_t ldb, const Epi& epi,
                                          T* __restrict__ sA0, T* __restrict__ sA1, T* __restrict__ sB0,
                                          T* __restrict__ sB1) {
  if constexpr (kDirectLds) {
    tile_body_direct<T, WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, A, lda, B, ldb, epi, sA0, sA1, sB0, sB1);
    return;
  }
  using accv = typename AccOf<T>::vec;
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int VEC = 16 / sizeof(T);             // elements per 16-byte vector
  constexpr int LDSR = TileGeom<T, WM, WN, WAVES_M, WAVES_N, KC>::LDSR;
  constexpr int VPR = KC / VEC;                   // 16-byte vectors per staged row
  constexpr int NLA = (BM * VPR + NT - 1) / NT;
  constexpr int NLB = (BN * VPR + NT - 1) / NT;
  static_assert(KC % (4 * VEC) == 0, "bad KC");
  static_assert(16 % VPR == 0, "swizzle period must divide the 16-row fragment blocks");
  const int64_t m0 = job.m0, n0 = job.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;

  const T* pa[NLA];
  int oa[NLA];
  const T* pb[NLB];
  int ob[NLB];
#pragma unroll
  for (int i = 0; i < NLA; ++i) {
    int idx = tid + i * NT;
    if (idx >= BM * VPR) idx = BM * VPR - 1;      // duplicates the last vector (harmless)
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = m0 + r;
    if (gr > M - 1) gr = M - 1;
    pa[i] = A + epi.arow(gr) * lda + kv * VEC + job.kc0 * KC;
    oa[i] = lds_vec_off<VEC, VPR, LDSR>(r, kv);
  }
#pragma unroll
  for (int i = 0; i < NLB; ++i) {
    int idx = tid + i * NT;
    if (idx >= BN * VPR) idx = BN * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = n0 + r;
    if (gr > N - 1) gr = N - 1;
    pb[i] = B + epi.brow(gr) * ldb + kv * VEC + job.kc0 * KC;
    ob[i] = lds_vec_off<VEC, VPR, LDSR>(r, kv);
  }

  accv acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = accv{0, 0, 0, 0};

  // fragment rows: row (lane & 15) of each 16-row block; a block start is a
  // multiple of 16, so the swizzle key of the row is (lane & 15) % VPR
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (wn * WN * 16 + (lane & 15)) * LDSR;
  const int fq = lane >> 4;
  const int key = kLdsLayout == 0 ? 0 : (lane & 15) % VPR;
  const int64_t nk = job.kc1 - job.kc0;

  // Two chunks in flight where the registers allow: every FP32 tile, and the FP64
  // tiles whose accumulators, two register sets and fragments come to at most 150
  // VGPRs by this count (the larger FP64 tiles spill with two sets; measured on gfx950).
  constexpr int kRegEst = WM * WN * 8 + 2 * (NLA + NLB) * 4 + (WM + WN) * 4;
  constexpr int kDepth = kPrefetch != 0 ? kPrefetch : ((sizeof(T) == 4 || kRegEst <= 150) ? 2 : 1);
  if constexpr (kDepth == 2) {
    // two register sets: at the top of step kt, LDS buffer kt & 1 holds chunk kt and
    // register set (kt + 1) & 1 holds chunk kt + 1, loaded one step earlier
    u32x4 ra0[NLA], rb0[NLB], ra1[NLA], rb1[NLB];
    chunk_load<T, NLA, NLB, KC>(ra0, rb0, pa, pb, 0);
    chunk_store<T, NLA, NLB>(ra0, rb0, sA0, sB0, oa, ob);
    // (loads past the last chunk re-read the last one: always in bounds, never stored)
    chunk_load<T, NLA, NLB, KC>(ra1, rb1, pa, pb, nk > 1 ? 1 : 0);
    __syncthreads();
    int64_t kt = 0;
    for (; kt + 2 < nk; kt += 2) {
      chunk_load<T, NLA, NLB, KC>(ra0, rb0, pa, pb, kt + 2);
      consume_chunk<T, WM, WN, KC, LDSR>(acc, sA0, sB0, arow, brow, fq, key);
      chunk_store<T, NLA, NLB>(ra1, rb1, sA1, sB1, oa, ob);
      __syncthreads();
      chunk_load<T, NLA, NLB, KC>(ra1, rb1, pa, pb, kt + 3 < nk ? kt + 3 : nk - 1);
      consume_chunk<T, WM, WN, KC, LDSR>(acc, sA1, sB1, arow, brow, fq, key);
      chunk_store<T, NLA, NLB>(ra0, rb0, sA0, sB0, oa, ob);
      __syncthreads();
    }
    if (kt + 1 < nk) {   // chunks kt (LDS buffer 0) and kt + 1 (register set 1) remain
      consume_chunk<T, WM, WN, KC, LDSR>(acc, sA0, sB0, arow, brow, fq, key);
      chunk_store<T, NLA, NLB>(ra1, rb1, sA1, sB1, oa, ob);
      __syncthreads();
      consume_chunk<T, WM, WN, KC, LDSR>(acc, sA1, sB1, arow, brow, fq, key);
    } else {
      consume_chunk<T, WM, WN, KC, LDSR>(acc, sA0, sB0, arow, brow, fq, key);
    }
    store_acc<T, WM, WN>(acc, job, epi, wm, wn, lane);
    return;
  }

  // chunk 0 straight into LDS buffer 0
  {
    u32x4 ra[NLA], rb[NLB];
#pragma unroll
    for (int i = 0; i < NLA; ++i) ra[i] = *reinterpret_cast<const u32x4*>(pa[i]);
#pragma unroll
    for (int i = 0; i < NLB; ++i) rb[i] = *reinterpret_cast<const u32x4*>(pb[i]);
#pragma unroll
    for (int i = 0; i < NLA; ++i) *reinterpret_cast<u32x4*>(&sA0[oa[i]]) = ra[i];
#pragma unroll
    for (int i = 0; i < NLB; ++i) *reinterpret_cast<u32x4*>(&sB0[ob[i]]) = rb[i];
  }
  __syncthreads();

  // steady state: chunk kt+1 is fetched into registers while chunk kt is consumed
  for (int64_t kt = 0; kt + 1 < nk; ++kt) {
    const int buf = (int)(kt & 1);
    const int64_t k1 = (kt + 1) * KC;
    u32x4 ra[NLA], rb[NLB];
#pragma unroll
    for (int i = 0; i < NLA; ++i) ra[i] = *reinterpret_cast<const u32x4*>(pa[i] + k1);
#pragma unroll
    for (int i = 0; i < NLB; ++i) rb[i] = *reinterpret_cast<const u32x4*>(pb[i] + k1);
    consume_chunk<T, WM, WN, KC, LDSR>(acc, buf ? sA1 : sA0, buf ? sB1 : sB0, arow, brow, fq, key);
#pragma unroll
    for (int i = 0; i < NLA; ++i) *reinterpret_cast<u32x4*>(&(buf ? sA0 : sA1)[oa[i]]) = ra[i];
#pragma unroll
    for (int i = 0; i < NLB; ++i) *reinterpret_cast<u32x4*>(&(buf ? sB0 : sB1)[ob[i]]) = rb[i];
    if constexpr (kSchedFence) {
      // order of this block: the global loads of the next chunk, then the LDS reads and
      // MFMAs of this chunk group by group, then the LDS stores (whose waits on the
      // global loads thereby come after every MFMA of the chunk)
      constexpr int NG = KC / (4 * VEC), MG = WM * WN * VEC;
      constexpr int EARLY = kSchedFence == 2 ? (MG < 4 ? MG : 4) : MG;
      __builtin_amdgcn_sched_group_barrier(0x020, NLA + NLB, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, WM + WN, 0);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        // with kSchedFence == 2 the fragments of group g+1 are read after the first
        // few MFMAs of group g
        __builtin_amdgcn_sched_group_barrier(0x008, EARLY, 0);
        if (g + 1 < NG) __builtin_amdgcn_sched_group_barrier(0x100, WM + WN, 0);
        if (MG > EARLY) __builtin_amdgcn_sched_group_barrier(0x008, MG - EARLY, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x200, NLA + NLB, 0);
    }
    __syncthreads();
  }
  {  // last chunk
    const int buf = (int)((nk - 1) & 1);
    consume_chunk<T, WM, WN, KC, LDSR>(acc, buf ? sA1 : sA0, buf ? sB1 : sB0, arow, brow, fq, key);
  }

  store_acc<T, WM, WN>(acc, job, epi, wm, wn, lane);
}

// Two workgroups' waves per SIMD where two workgroups fit in LDS; one where the three
// stages of the direct loads leave room for a single workgroup
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi>
struct GemmOccupancy {
  static constexpr bool build64 = PPL_BUILD_DIRECT3 && sizeof(T) == 8 && WM == 4 && WN == 2 && WAVES_M == 1 && WAVES_N == 4;
  static constexpr bool direct = kFpDirect3 && (std::is_same_v<Epi, EpiStore<T>> || build64);
  static constexpr int lds = 3 * 16 * (WM * WAVES_M + WN * WAVES_N) * KC * (int)sizeof(T);
  static constexpr int waves = (direct && 2 * lds > 160 * 1024) ? 1 : 2;
};

template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi, class Map>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
__attribute__((amdgpu_waves_per_eu(GemmOccupancy<T, WM, WN, WAVES_M, WAVES_N, KC, Epi>::waves)))
gemm_nt_kernel(int64_t M, int64_t N, int64_t Kpad, const T* __restrict__ A, int64_t lda,
               const T* __restrict__ B, int64_t ldb, Epi epi, Map map) {
  using G = TileGeom<T, WM, WN, WAVES_M, WAVES_N, KC>;
  (void)Kpad;
  TileJob job;
  // The contractions take the three-stage direct loads, and so do the FP64 integral
  // builds on their 64 x 128 tile (13.1 against 13.7 ms per build at (20, 200, 600), 307
  // against 321 ms at (40, 400, 1200), for the register-staged loop on the 128 x 128
  // tile); the other builds keep the register-staged loop (FP32 on 128 x 128: 171
  // against 195 ms with direct loads at (40, 400, 1200); the FP64 copy of a mixed plan,
  // built on the 96 x 128 tile of its low-precision operands).
  if constexpr (GemmOccupancy<T, WM, WN, WAVES_M, WAVES_N, KC, Epi>::direct) {
    __shared__ __attribute__((aligned(16))) T st0[G::BUF_A + G::BUF_B];
    __shared__ __attribute__((aligned(16))) T st1[G::BUF_A + G::BUF_B];
    __shared__ __attribute__((aligned(16))) T st2[G::BUF_A + G::BUF_B];
    if (!map(blockIdx.x, job)) return;
    tile_body_direct3<T, WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, A, lda, B, ldb, epi, st0, st1, st2);
  } else {
    __shared__ __attribute__((aligned(16))) T sA0[G::BUF_A];
    __shared__ __attribute__((aligned(16))) T sA1[G::BUF_A];
    __shared__ __attribute__((aligned(16))) T sB0[G::BUF_B];
    __shared__ __attribute__((aligned(16))) T sB1[G::BUF_B];
    if (!map(blockIdx.x, job)) return;
    tile_body<T, WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, A, lda, B, ldb, epi, sA0, sA1, sB0, sB1);
  }
}

// ------------------------------------------------------------------ the kernel (BF16 x 3)
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi); x*y ~ hi*hi + hi*lo + lo*hi,
// the two small cross products accumulated in their own FP32 register set and
// added to the hi*hi set once at the end.
template <int WM, int WN, int WAVES_M, int WAVES_N, int KC>
struct Bf3Geom {
  static constexpr int NT = 64 * WAVES_M * WAVES_N;
  static constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  // unpadded rows; 16-byte vector kv of row r at slot kv ^ key(r), with key(r) =
  // (r / 2) mod 4 for 64-byte rows and r mod 8 for rows of 128 bytes and more, so that
  // the eight lanes of a 16-byte access phase (rows r .. r+7, one vector each) hit
  // eight different 16-byte bank groups
  static constexpr int LDSR = KC;
  static constexpr int VPR = KC / 8;
  __host__ __device__ static constexpr int key(int r) { return VPR >= 8 ? (r & 7) : ((r >> 1) & 3); }
  static constexpr int LDS_A = 2 * BM * LDSR, LDS_B = 2 * BN * LDSR;   // per plane, two buffers
  // direct loads: one stage holds the hi and lo planes of A, then those of B
  static constexpr int STAGE = 2 * (BM + BN) * LDSR;
  static_assert(!kBf3Direct || 3 * STAGE * 2 <= 160 * 1024, "three BF16x3 stages exceed the LDS");
};

// The tile with chunks moved straight from global memory into LDS (global_load_lds, 16
// bytes a lane), in three stages: step k multiplies chunk k while chunk k+1 is still
// arriving and issues chunk k+2, so that the wait at the end of a step is never for
// loads issued in that step, and no registers or LDS store instructions stage them
// (measured at (40, 400, 1200), R+ on tile 9: 28.7 ms against 38.5 ms for the
// register-staged two-buffer loop, which stays as the PPL_BF3_DIRECT=0 build). One
// wave instruction fills 64 / VPR whole staged rows of one plane (1 KB); lane l loads the
// global vector that the swizzled layout keeps at slot l. The 2 (BM + BN) / (64 / VPR)
// instructions of a chunk are dealt round-robin over the waves; where they do not divide
// evenly, the waves short of one repeat one of the first instructions (the same bytes to
// the same place, before the same wait), so that every wave issues the same number.
template <int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi>
__device__ __forceinline__ void bf3_tile_body_direct(const TileJob& job, int64_t M, int64_t N,
                                                     const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al,
                                                     int64_t lda, const __bf16* __restrict__ Bh,
                                                     const __bf16* __restrict__ Bl, int64_t ldb, const Epi& epi,
                                                     __bf16* __restrict__ st0, __bf16* __restrict__ st1,
                                                     __bf16* __restrict__ st2) {
  using G = Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>;
  constexpr int NW = WAVES_M * WAVES_N;
  constexpr int BM = G::BM, BN = G::BN, LDSR = G::LDSR, VPR = G::VPR;
  constexpr int RPI = 64 / VPR;                    // staged rows per wave instruction
  constexpr int GA = BM / RPI, GB = BN / RPI;      // instructions per plane and chunk
  constexpr int GT = 2 * (GA + GB);                // instructions per chunk
  constexpr int NI = (GT + NW - 1) / NW;           // per wave
  static_assert(64 % VPR == 0 && BM % RPI == 0 && BN % RPI == 0 && GT >= NW, "direct LDS geometry");
  static_assert(KC == 32 || KC % 64 == 0, "the swizzle permutes aligned groups of 4 (or 8) 16-byte vectors");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int lr = lane / VPR, slot = lane % VPR;

  // instruction q = wave + i NW of a chunk (q - GT past the end): plane Ah (q < GA), Al,
  // Bh, then Bl; src is this lane's global vector, dst the instruction's 1 KB in a stage
  const __bf16* src[NI];
  int dst[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    int q = wave + i * NW;
    if (q >= GT) q -= GT;
    src[i] = Ah;
    dst[i] = 0;
    if (q < 2 * GA) {
      const int plane = q / GA, g = q % GA, r = g * RPI + lr;
      int64_t gr = job.m0 + r;
      if (gr > M - 1) gr = M - 1;
      src[i] = (plane ? Al : Ah) + epi.arow(gr) * lda + (slot ^ G::key(r)) * 8 + job.kc0 * KC;
      dst[i] = (plane * BM + g * RPI) * LDSR;
    } else if (q < GT) {
      const int plane = (q - 2 * GA) / GB, g = (q - 2 * GA) % GB, r = g * RPI + lr;
      int64_t gr = job.n0 + r;
      if (gr > N - 1) gr = N - 1;
      src[i] = (plane ? Bl : Bh) + epi.brow(gr) * ldb + (slot ^ G::key(r)) * 8 + job.kc0 * KC;
      dst[i] = (2 * BM + plane * BN + g * RPI) * LDSR;
    }
  }
  auto issue = [&](int64_t c, __bf16* st) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
      __builtin_amdgcn_global_load_lds((global_cvoid_t*)(src[i] + c * KC), (lds_void_t*)(st + dst[i]), 16, 0, 0);
  };
  // Wait until at most one chunk of this wave's loads is outstanding (vmcnt counts loads
  // in issue order), or none. The waits are s_waitcnt builtins (vmcnt only: expcnt and
  // lgkmcnt fields at their maxima), which the compiler folds into its own bookkeeping
  // of outstanding loads, so that it adds no wait of its own before reading a stage.
  static_assert(NI < 16, "vmcnt immediate");
  auto wait_one = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70 | NI);
    asm volatile("" ::: "memory");
  };
  auto wait_all = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    asm volatile("" ::: "memory");
  };
  // the workgroup barrier without the fence of __syncthreads, which would wait for every
  // load in flight (the chunk after next included); each meet() follows one of the waits
  // above, and the empty asm keeps the compiler from moving LDS reads above the barrier
  auto meet = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  f4 acc[WM][WN], accx[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc[i][j] = f4{0, 0, 0, 0};
      accx[i][j] = f4{0, 0, 0, 0};
    }
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (2 * BM + wn * WN * 16 + (lane & 15)) * LDSR;
  const int fsw = G::key(lane & 15);
  const int64_t nk = job.kc1 - job.kc0;

  // Multiply the chunk staged in st; when go, start chunk c into stage nx between the
  // LDS reads of the first 32-wide K group and its MFMAs (the empty asm keeps the reads
  // first, so that a wait the compiler may place before them never covers chunk c).
  auto compute = [&](const __bf16* __restrict__ st, bool go, int64_t c, __bf16* nx) __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 32) {
      const int col = ((((kk) >> 3) + (lane >> 4)) ^ fsw) * 8;
      bf8 ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ah[i] = *reinterpret_cast<const bf8*>(&st[arow + i * 16 * LDSR + col]);
        al[i] = *reinterpret_cast<const bf8*>(&st[BM * LDSR + arow + i * 16 * LDSR + col]);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        bh[j] = *reinterpret_cast<const bf8*>(&st[brow + j * 16 * LDSR + col]);
        bl[j] = *reinterpret_cast<const bf8*>(&st[BN * LDSR + brow + j * 16 * LDSR + col]);
      }
      if (kk == 0) {
        asm volatile("" ::: "memory");
        if (go) issue(c, nx);
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          accx[i][j] = mfma16(al[i], bh[j], accx[i][j]);
          accx[i][j] = mfma16(ah[i], bl[j], accx[i][j]);
          acc[i][j] = mfma16(ah[i], bh[j], acc[i][j]);
        }
    }
  };

  // Chunk j lives in stage j mod 3. Step k starts chunk k+2 into the stage that chunk
  // k-1 used (every wave is past it), multiplies chunk k, waits for this wave's part of
  // chunk k+1, and meets the other waves. The compiler adds a wait for every load in
  // flight at the loop head (it keeps no account of which stage a pending load fills
  // across the back edge); placed before that step's own loads it covers only chunk
  // kt+1, and a loop trip of 3 U steps pays it once.
  constexpr int U = 2;
  issue(0, st0);
  if (nk > 1) {
    issue(1, st1);
    wait_one();
  } else {
    wait_all();
  }
  meet();
  int64_t kt = 0;
  for (; kt + 3 * U + 1 < nk; kt += 3 * U) {   // 3 U steps whose k+2 exists
#pragma unroll
    for (int u = 0; u < U; ++u) {
      compute(st0, true, kt + 3 * u + 2, st2);
      wait_one();
      meet();
      compute(st1, true, kt + 3 * u + 3, st0);
      wait_one();
      meet();
      compute(st2, true, kt + 3 * u + 4, st1);
      wait_one();
      meet();
    }
  }
  // the last steps (at most 3 U + 1): chunk kt in st0, kt+1 (if any) in flight to st1
  for (int64_t j = kt; j < nk; ++j) {
    const int sj = (int)((j - kt) % 3);
    const __bf16* cur = sj == 0 ? st0 : (sj == 1 ? st1 : st2);
    __bf16* nx = sj == 0 ? st2 : (sj == 1 ? st0 : st1);   // the stage of chunk j+2
    compute(cur, j + 2 < nk, j + 2, nx);
    if (j + 1 < nk) {
      if (j + 2 < nk) wait_one();
      else wait_all();
      meet();
    }
  }

#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = job.m0 + wm * WM * 16 + i * 16 + AccOf<__bf16>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(job.split, m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = job.n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r] + accx[i][j][r]);
      }
    }
  }
}

// One BM x BN tile over the K chunks [job.kc0, job.kc1); the s* arrays hold two LDS
// buffers each of the hi and lo planes.
template <int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi>
__device__ __forceinline__ void bf3_tile_body(const TileJob& job, int64_t M, int64_t N, const __bf16* __restrict__ Ah,
                                              const __bf16* __restrict__ Al, int64_t lda,
                                              const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl,
                                              int64_t ldb, const Epi& epi, __bf16* __restrict__ sAh,
                                              __bf16* __restrict__ sAl, __bf16* __restrict__ sBh,
                                              __bf16* __restrict__ sBl) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int VEC = 8;                           // bf16 per 16-byte load
  constexpr int LDSR = Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>::LDSR;
  constexpr int VPR = KC / VEC;
  constexpr int NLA = (BM * VPR + NT - 1) / NT;
  constexpr int NLB = (BN * VPR + NT - 1) / NT;
  static_assert(KC % 32 == 0, "bad KC");
  const int64_t m0 = job.m0, n0 = job.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;

  int64_t ga[NLA], gb[NLB];
  int oa[NLA], ob[NLB];
#pragma unroll
  for (int i = 0; i < NLA; ++i) {
    int idx = tid + i * NT;
    if (idx >= BM * VPR) idx = BM * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = m0 + r;
    if (gr > M - 1) gr = M - 1;
    ga[i] = epi.arow(gr) * lda + kv * VEC + job.kc0 * KC;
    oa[i] = r * LDSR + (kv ^ Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>::key(r)) * VEC;
  }
#pragma unroll
  for (int i = 0; i < NLB; ++i) {
    int idx = tid + i * NT;
    if (idx >= BN * VPR) idx = BN * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = n0 + r;
    if (gr > N - 1) gr = N - 1;
    gb[i] = epi.brow(gr) * ldb + kv * VEC + job.kc0 * KC;
    ob[i] = r * LDSR + (kv ^ Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>::key(r)) * VEC;
  }
  f4 acc[WM][WN], accx[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc[i][j] = f4{0, 0, 0, 0};
      accx[i][j] = f4{0, 0, 0, 0};
    }

  // fragment rows start at multiples of 16, so a row's swizzle key is that of lane & 15
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (wn * WN * 16 + (lane & 15)) * LDSR;
  const int fsw = Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>::key(lane & 15);
  static_assert(KC == 32 || KC % 64 == 0, "the swizzle permutes aligned groups of 4 (or 8) 16-byte vectors");
  const int64_t nk = job.kc1 - job.kc0;

// element offset of this lane's 8-element fragment vector at K offset kk of a staged row
#define PPL_BF3_COL(kk) (((((kk) >> 3) + (lane >> 4)) ^ fsw) * 8)
#define PPL_BF3_LOAD(k0)                                                     \
  _Pragma("unroll") for (int i = 0; i < NLA; ++i) {                          \
    rah[i] = *reinterpret_cast<const uint4*>(Ah + ga[i] + (k0));             \
    ral[i] = *reinterpret_cast<const uint4*>(Al + ga[i] + (k0));             \
  }                                                                          \
  _Pragma("unroll") for (int i = 0; i < NLB; ++i) {                          \
    rbh[i] = *reinterpret_cast<const uint4*>(Bh + gb[i] + (k0));             \
    rbl[i] = *reinterpret_cast<const uint4*>(Bl + gb[i] + (k0));             \
  }
#define PPL_BF3_STORE(buf)                                                   \
  _Pragma("unroll") for (int i = 0; i < NLA; ++i) {                          \
    *reinterpret_cast<uint4*>(&sAh[(buf) * (BM * LDSR) + oa[i]]) = rah[i];                    \
    *reinterpret_cast<uint4*>(&sAl[(buf) * (BM * LDSR) + oa[i]]) = ral[i];                    \
  }                                                                          \
  _Pragma("unroll") for (int i = 0; i < NLB; ++i) {                          \
    *reinterpret_cast<uint4*>(&sBh[(buf) * (BN * LDSR) + ob[i]]) = rbh[i];                    \
    *reinterpret_cast<uint4*>(&sBl[(buf) * (BN * LDSR) + ob[i]]) = rbl[i];                    \
  }
#define PPL_BF3_COMPUTE(buf)                                                                   \
  _Pragma("unroll") for (int kk = 0; kk < KC; kk += 32) {                                      \
    bf8 ah[WM], al[WM], bh[WN], bl[WN];                                                        \
    _Pragma("unroll") for (int i = 0; i < WM; ++i) {                                           \
      ah[i] = *reinterpret_cast<const bf8*>(&sAh[(buf) * (BM * LDSR) + arow + i * 16 * LDSR + PPL_BF3_COL(kk)]); \
      al[i] = *reinterpret_cast<const bf8*>(&sAl[(buf) * (BM * LDSR) + arow + i * 16 * LDSR + PPL_BF3_COL(kk)]); \
    }                                                                                          \
    _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                           \
      bh[j] = *reinterpret_cast<const bf8*>(&sBh[(buf) * (BN * LDSR) + brow + j * 16 * LDSR + PPL_BF3_COL(kk)]); \
      bl[j] = *reinterpret_cast<const bf8*>(&sBl[(buf) * (BN * LDSR) + brow + j * 16 * LDSR + PPL_BF3_COL(kk)]); \
    }                                                                                          \
    _Pragma("unroll") for (int i = 0; i < WM; ++i)                                             \
    _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                           \
      accx[i][j] = mfma16(al[i], bh[j], accx[i][j]);                                           \
      accx[i][j] = mfma16(ah[i], bl[j], accx[i][j]);                                           \
      acc[i][j] = mfma16(ah[i], bh[j], acc[i][j]);                                             \
    }                                                                                          \
  }

  {
    uint4 rah[NLA], ral[NLA], rbh[NLB], rbl[NLB];
    PPL_BF3_LOAD(0)
    PPL_BF3_STORE(0)
  }
  __syncthreads();
  for (int64_t kt = 0; kt + 1 < nk; ++kt) {
    const int buf = (int)(kt & 1);
    uint4 rah[NLA], ral[NLA], rbh[NLB], rbl[NLB];
    PPL_BF3_LOAD((kt + 1) * KC)
    PPL_BF3_COMPUTE(buf)
    PPL_BF3_STORE(buf ^ 1)
    __syncthreads();
  }
  {
    const int buf = (int)((nk - 1) & 1);
    PPL_BF3_COMPUTE(buf)
  }
#undef PPL_BF3_LOAD
#undef PPL_BF3_STORE
#undef PPL_BF3_COMPUTE
#undef PPL_BF3_COL

#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM * 16 + i * 16 + AccOf<__bf16>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(job.split, m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r] + accx[i][j][r]);
      }
    }
  }
}

template <int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi, class Map>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
gemm_nt_bf16x3_kernel(int64_t M, int64_t N, int64_t Kpad, const __bf16* __restrict__ Ah,
                      const __bf16* __restrict__ Al, int64_t lda, const __bf16* __restrict__ Bh,
                      const __bf16* __restrict__ Bl, int64_t ldb, Epi epi, Map map) {
  using G = Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>;
  (void)Kpad;
  TileJob job;
  if constexpr (kBf3Direct) {
    // three distinct arrays, so that the compiler can tell the loads into one stage
    // from the reads of another
    __shared__ __attribute__((aligned(16))) __bf16 st0[G::STAGE];
    __shared__ __attribute__((aligned(16))) __bf16 st1[G::STAGE];
    __shared__ __attribute__((aligned(16))) __bf16 st2[G::STAGE];
    if (!map(blockIdx.x, job)) return;
    bf3_tile_body_direct<WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, Ah, Al, lda, Bh, Bl, ldb, epi, st0, st1, st2);
  } else {
    __shared__ __attribute__((aligned(16))) __bf16 sAh[G::LDS_A];
    __shared__ __attribute__((aligned(16))) __bf16 sAl[G::LDS_A];
    __shared__ __attribute__((aligned(16))) __bf16 sBh[G::LDS_B];
    __shared__ __attribute__((aligned(16))) __bf16 sBl[G::LDS_B];
    if (!map(blockIdx.x, job)) return;
    bf3_tile_body<WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, Ah, Al, lda, Bh, Bl, ldb, epi, sAh, sAl, sBh, sBl);
  }
}

// ------------------------------------------------------------------ the kernel (BF16 x 6)
// x (in FP32) = hi + mid + lo with hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid):
// 24 significant bits, those of FP32. x*y ~ the six products whose plane indices sum to at
// most two (hi*hi; hi*mid, mid*hi; mid*mid, hi*lo, lo*hi), the five small ones in a second
// FP32 register set added to the hi*hi set at the end (the bf16x6 scheme of Henry, Tang and
// Heinecke, ARITH 2019). The planes of an operand lie equally far apart in memory: hi at h,
// mid at m, lo at m + (m - h). K chunks of 32: two buffers of three planes of BM + BN rows
// take 384 (BM + BN) bytes of LDS, 132 KB for the largest tile (224 + 128 rows).
constexpr int kKcBf6 = 32;

template <int WM, int WN, int WAVES_M, int WAVES_N>
struct Bf6Geom {
  static constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  static constexpr int LDSR = kKcBf6;
  static constexpr int BUF_A = BM * LDSR, BUF_B = BN * LDSR;     // one buffer of one plane
  static constexpr int LDS_A = 6 * BUF_A, LDS_B = 6 * BUF_B;     // [plane][buffer]
  static_assert((LDS_A + LDS_B) * 2 <= 160 * 1024, "BF16x6 tile exceeds the LDS");
  static constexpr int STAGE = 3 * (BM + BN) * LDSR;              // direct loads: all planes
};

template <int WM, int WN, int WAVES_M, int WAVES_N, class Epi>
__device__ __forceinline__ void bf6_tile_body(const TileJob& job, int64_t M, int64_t N, const __bf16* Ah,
                                              const __bf16* Am, int64_t lda, const __bf16* Bh,
                                              const __bf16* Bm, int64_t ldb, const Epi& epi,
                                              __bf16* __restrict__ sA, __bf16* __restrict__ sB) {
  constexpr int KC = kKcBf6;
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  using G = Bf6Geom<WM, WN, WAVES_M, WAVES_N>;
  constexpr int BM = G::BM, BN = G::BN, LDSR = G::LDSR;
  constexpr int VEC = 8;                           // bf16 per 16-byte load
  constexpr int VPR = KC / VEC;                    // 4 vectors per staged row
  constexpr int NLA = (BM * VPR + NT - 1) / NT;
  constexpr int NLB = (BN * VPR + NT - 1) / NT;
  const int64_t m0 = job.m0, n0 = job.n0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const __bf16* Ap[3] = {Ah, Am, Am + (Am - Ah)};
  const __bf16* Bp[3] = {Bh, Bm, Bm + (Bm - Bh)};

  // swizzled slot of vector kv of staged row r (64-byte rows: key (r / 2) mod 4)
  auto key = [](int r) { return (r >> 1) & 3; };
  int64_t ga[NLA], gb[NLB];
  int oa[NLA], ob[NLB];
#pragma unroll
  for (int i = 0; i < NLA; ++i) {
    int idx = tid + i * NT;
    if (idx >= BM * VPR) idx = BM * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = m0 + r;
    if (gr > M - 1) gr = M - 1;
    ga[i] = epi.arow(gr) * lda + kv * VEC + job.kc0 * KC;
    oa[i] = r * LDSR + (kv ^ key(r)) * VEC;
  }
#pragma unroll
  for (int i = 0; i < NLB; ++i) {
    int idx = tid + i * NT;
    if (idx >= BN * VPR) idx = BN * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = n0 + r;
    if (gr > N - 1) gr = N - 1;
    gb[i] = epi.brow(gr) * ldb + kv * VEC + job.kc0 * KC;
    ob[i] = r * LDSR + (kv ^ key(r)) * VEC;
  }
  f4 acc[WM][WN], accx[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc[i][j] = f4{0, 0, 0, 0};
      accx[i][j] = f4{0, 0, 0, 0};
    }
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (wn * WN * 16 + (lane & 15)) * LDSR;
  const int col = (((lane >> 4)) ^ key(lane & 15)) * 8;   // this lane's 8-element fragment vector
  const int64_t nk = job.kc1 - job.kc0;

#define PPL_BF6_LOAD(k0)                                                                  \
  _Pragma("unroll") for (int q = 0; q < 3; ++q) {                                         \
    _Pragma("unroll") for (int i = 0; i < NLA; ++i)                                       \
      ra[q][i] = *reinterpret_cast<const uint4*>(Ap[q] + ga[i] + (k0));                   \
    _Pragma("unroll") for (int i = 0; i < NLB; ++i)                                       \
      rb[q][i] = *reinterpret_cast<const uint4*>(Bp[q] + gb[i] + (k0));                   \
  }
#define PPL_BF6_STORE(buf)                                                                \
  _Pragma("unroll") for (int q = 0; q < 3; ++q) {                                         \
    _Pragma("unroll") for (int i = 0; i < NLA; ++i)                                       \
      *reinterpret_cast<uint4*>(&sA[(2 * q + (buf)) * G::BUF_A + oa[i]]) = ra[q][i];      \
    _Pragma("unroll") for (int i = 0; i < NLB; ++i)                                       \
      *reinterpret_cast<uint4*>(&sB[(2 * q + (buf)) * G::BUF_B + ob[i]]) = rb[q][i];      \
  }
#define PPL_BF6_COMPUTE(buf)                                                                               \
  {                                                                                                        \
    bf8 a[3][WM], b[3][WN];                                                                                \
    _Pragma("unroll") for (int q = 0; q < 3; ++q) {                                                        \
      _Pragma("unroll") for (int i = 0; i < WM; ++i)                                                       \
        a[q][i] = *reinterpret_cast<const bf8*>(&sA[(2 * q + (buf)) * G::BUF_A + arow + i * 16 * LDSR + col]); \
      _Pragma("unroll") for (int j = 0; j < WN; ++j)                                                       \
        b[q][j] = *reinterpret_cast<const bf8*>(&sB[(2 * q + (buf)) * G::BUF_B + brow + j * 16 * LDSR + col]); \
    }                                                                                                      \
    _Pragma("unroll") for (int i = 0; i < WM; ++i)                                                         \
    _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                                       \
      accx[i][j] = mfma16(a[2][i], b[0][j], accx[i][j]);                                                   \
      accx[i][j] = mfma16(a[0][i], b[2][j], accx[i][j]);                                                   \
      accx[i][j] = mfma16(a[1][i], b[1][j], accx[i][j]);                                                   \
      accx[i][j] = mfma16(a[1][i], b[0][j], accx[i][j]);                                                   \
      accx[i][j] = mfma16(a[0][i], b[1][j], accx[i][j]);                                                   \
      acc[i][j] = mfma16(a[0][i], b[0][j], acc[i][j]);                                                     \
    }                                                                                                      \
  }

  {
    uint4 ra[3][NLA], rb[3][NLB];
    PPL_BF6_LOAD(0)
    PPL_BF6_STORE(0)
  }
  __syncthreads();
  for (int64_t kt = 0; kt + 1 < nk; ++kt) {
    const int buf = (int)(kt & 1);
    uint4 ra[3][NLA], rb[3][NLB];
    PPL_BF6_LOAD((kt + 1) * KC)
    PPL_BF6_COMPUTE(buf)
    PPL_BF6_STORE(buf ^ 1)
    __syncthreads();
  }
  {
    const int buf = (int)((nk - 1) & 1);
    PPL_BF6_COMPUTE(buf)
  }
#undef PPL_BF6_LOAD
#undef PPL_BF6_STORE
#undef PPL_BF6_COMPUTE

#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM * 16 + i * 16 + AccOf<__bf16>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(job.split, m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r] + accx[i][j][r]);
      }
    }
  }
}

// The BF16x6 tile with chunks moved straight from global memory into LDS, in two stages
// (three planes of 224 + 128 rows leave no room for a third): step k issues chunk k+1
// into the other stage, multiplies chunk k, then waits for its loads and meets the
// other waves. One stage holds the hi, mid and lo planes of A, then those
// of B; the instructions of a chunk are dealt over the waves as in the BF16x3 tile.
template <int WM, int WN, int WAVES_M, int WAVES_N, class Epi>
__device__ __forceinline__ void bf6_tile_body_direct(const TileJob& job, int64_t M, int64_t N, const __bf16* Ah,
                                                     const __bf16* Am, int64_t lda, const __bf16* Bh,
                                                     const __bf16* Bm, int64_t ldb, const Epi& epi,
                                                     __bf16* __restrict__ st0, __bf16* __restrict__ st1) {
  constexpr int KC = kKcBf6;
  using G = Bf6Geom<WM, WN, WAVES_M, WAVES_N>;
  constexpr int NW = WAVES_M * WAVES_N;
  constexpr int BM = G::BM, BN = G::BN, LDSR = G::LDSR;
  constexpr int VPR = KC / 8;                      // 4 vectors per staged row
  constexpr int RPI = 64 / VPR;                    // staged rows per wave instruction
  constexpr int GA = BM / RPI, GB = BN / RPI;      // instructions per plane and chunk
  constexpr int GT = 3 * (GA + GB);                // instructions per chunk
  constexpr int NI = (GT + NW - 1) / NW;           // per wave (the short waves repeat one)
  static_assert(BM % RPI == 0 && BN % RPI == 0 && GT >= NW && NI < 16, "direct LDS geometry");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int lr = lane / VPR, slot = lane % VPR;
  auto key = [](int r) { return (r >> 1) & 3; };
  auto plane_of = [](const __bf16* h, const __bf16* m, int q) { return q == 0 ? h : (q == 1 ? m : m + (m - h)); };

  const __bf16* src[NI];
  int dst[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    int q = wave + i * NW;
    if (q >= GT) q -= GT;
    if (q < 3 * GA) {
      const int plane = q / GA, g = q % GA, r = g * RPI + lr;
      int64_t gr = job.m0 + r;
      if (gr > M - 1) gr = M - 1;
      src[i] = plane_of(Ah, Am, plane) + epi.arow(gr) * lda + (slot ^ key(r)) * 8 + job.kc0 * KC;
      dst[i] = (plane * BM + g * RPI) * LDSR;
    } else {
      const int plane = (q - 3 * GA) / GB, g = (q - 3 * GA) % GB, r = g * RPI + lr;
      int64_t gr = job.n0 + r;
      if (gr > N - 1) gr = N - 1;
      src[i] = plane_of(Bh, Bm, plane) + epi.brow(gr) * ldb + (slot ^ key(r)) * 8 + job.kc0 * KC;
      dst[i] = (3 * BM + plane * BN + g * RPI) * LDSR;
    }
  }
  auto issue = [&](int64_t c, __bf16* st) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
      __builtin_amdgcn_global_load_lds((global_cvoid_t*)(src[i] + c * KC), (lds_void_t*)(st + dst[i]), 16, 0, 0);
  };
  // vmcnt(0) as a builtin (expcnt and lgkmcnt fields at their maxima), so that the
  // compiler knows no load is pending; then the barrier without the fence of
  // __syncthreads (the empty asm keeps LDS reads below it)
  auto wait_meet = []() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  f4 acc[WM][WN], accx[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc[i][j] = f4{0, 0, 0, 0};
      accx[i][j] = f4{0, 0, 0, 0};
    }
  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR;
  const int brow = (3 * BM + wn * WN * 16 + (lane & 15)) * LDSR;
  const int col = ((lane >> 4) ^ key(lane & 15)) * 8;   // this lane's 8-element fragment vector
  const int64_t nk = job.kc1 - job.kc0;

  // Multiply the chunk in st; when go, first issue chunk c into nx. The empty asm keeps
  // the LDS reads, and with them the MFMAs, below the loads: left to itself the compiler
  // sinks the loads below the MFMAs, and the wait that ends the step would then find
  // them just issued.
  auto compute = [&](const __bf16* __restrict__ st, bool go, int64_t c, __bf16* nx) __attribute__((always_inline)) {
    if (go) issue(c, nx);
    asm volatile("" ::: "memory");
    bf8 a[3][WM], b[3][WN];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
#pragma unroll
      for (int i = 0; i < WM; ++i) a[q][i] = *reinterpret_cast<const bf8*>(&st[q * BM * LDSR + arow + i * 16 * LDSR + col]);
#pragma unroll
      for (int j = 0; j < WN; ++j) b[q][j] = *reinterpret_cast<const bf8*>(&st[q * BN * LDSR + brow + j * 16 * LDSR + col]);
    }
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        accx[i][j] = mfma16(a[2][i], b[0][j], accx[i][j]);
        accx[i][j] = mfma16(a[0][i], b[2][j], accx[i][j]);
        accx[i][j] = mfma16(a[1][i], b[1][j], accx[i][j]);
        accx[i][j] = mfma16(a[1][i], b[0][j], accx[i][j]);
        accx[i][j] = mfma16(a[0][i], b[1][j], accx[i][j]);
        acc[i][j] = mfma16(a[0][i], b[0][j], acc[i][j]);
      }
  };

  // chunk j lives in stage j mod 2
  issue(0, st0);
  wait_meet();
  int64_t kt = 0;
  for (; kt + 2 < nk; kt += 2) {
    compute(st0, true, kt + 1, st1);
    wait_meet();
    compute(st1, true, kt + 2, st0);
    wait_meet();
  }
  // one or two chunks remain, chunk kt in st0
  compute(st0, kt + 1 < nk, kt + 1, st1);
  if (kt + 1 < nk) {
    wait_meet();
    compute(st1, false, 0, st0);
  }

#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = job.m0 + wm * WM * 16 + i * 16 + AccOf<__bf16>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(job.split, m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = job.n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r] + accx[i][j][r]);
      }
    }
  }
}

template <int WM, int WN, int WAVES_M, int WAVES_N, class Epi, class Map>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
gemm_nt_bf16x6_kernel(int64_t M, int64_t N, const __bf16* Ah, const __bf16* Am, int64_t lda, const __bf16* Bh,
                      const __bf16* Bm, int64_t ldb, Epi epi, Map map) {
  using G = Bf6Geom<WM, WN, WAVES_M, WAVES_N>;
  TileJob job;
  if constexpr (kBf6Direct) {
    __shared__ __attribute__((aligned(16))) __bf16 st0[G::STAGE];
    __shared__ __attribute__((aligned(16))) __bf16 st1[G::STAGE];
    if (!map(blockIdx.x, job)) return;
    bf6_tile_body_direct<WM, WN, WAVES_M, WAVES_N>(job, M, N, Ah, Am, lda, Bh, Bm, ldb, epi, st0, st1);
  } else {
    __shared__ __attribute__((aligned(16))) __bf16 sA[G::LDS_A];
    __shared__ __attribute__((aligned(16))) __bf16 sB[G::LDS_B];
    if (!map(blockIdx.x, job)) return;
    bf6_tile_body<WM, WN, WAVES_M, WAVES_N>(job, M, N, Ah, Am, lda, Bh, Bm, ldb, epi, sA, sB);
  }
}

// ------------------------------------------------------------------ tile configurations
struct TileCfg {
  int wm, wn, waves_m, waves_n;
  int bm() const { return 16 * wm * waves_m; }
  int bn() const { return 16 * wn * waves_n; }
};

// contraction tiles: BM spans occupied pairs (small), BN spans virtual pairs
static const TileCfg kContract[] = {
    {7, 2, 1, 4},   // 0: 112 x 128
    {4, 4, 2, 2},   // 1: 128 x 128
    {13, 1, 1, 4},  // 2: 208 x 64
    {2, 4, 1, 4},   // 3:  32 x 256
    {3, 4, 1, 4},   // 4:  48 x 256
    {6, 2, 1, 4},   // 5:  96 x 128
    {2, 2, 1, 4},   // 6:  32 x 128
    {3, 2, 1, 4},   // 7:  48 x 128
    {4, 2, 1, 4},   // 8:  64 x 128
    {7, 2, 2, 4},   // 9: 224 x 128, eight waves (one row tile covers up to 224 occupied pairs)
    {7, 1, 2, 4},   // 10: 224 x 64, eight waves
};
static const int kNumContract = sizeof(kContract) / sizeof(kContract[0]);

int contract_tile_count() { return kNumContract; }

void contract_tile_dims(int tile, int* bm, int* bn, int* threads) {
  const TileCfg& c = kContract[tile];
  *bm = c.bm();
  *bn = c.bn();
  *threads = 64 * c.waves_m * c.waves_n;
}

int contract_tile_default(int prec, int64_t Nrows) {
  (void)prec;
  // smallest padding waste of the occupied-pair dimension, ties to the larger tile
  int best = 0;
  double best_eff = -1.0;
  for (int t = 0; t < kNumContract; ++t) {
    const int bm = kContract[t].bm();
    const int64_t padded = (Nrows + bm - 1) / bm * bm;
    const double eff = (double)Nrows / (double)padded;
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = t;
    }
  }
  return best;
}

// The integral build runs on one of these contraction tiles (ids as in kContract).
// Row tiles per group in the launch order of the build tiles.
#ifndef PPL_BUILD_GROUP
#define PPL_BUILD_GROUP 8
#endif

bool build_tile_ok(int tile) { return tile == 0 || tile == 1 || tile == 5 || tile == 8 || tile == 9 || tile == 10; }

int build_tile_dims(int tile, int* bm, int* bn) {
  if (!build_tile_ok(tile)) return fail(PPL_E_ARG, "tile %d is not a build tile", tile);
  *bm = kContract[tile].bm();
  *bn = kContract[tile].bn();
  return PPL_OK;
}

// Valid (row tile, column tile) pairs of one build step in launch order: row tiles
// in groups of kBuildGroup, each group walked column tile by column tile with its row
// tiles innermost, so that workgroups running together on one XCD share operand rows
// in L2 (a column tile is re-read once per group instead of once per row tile).
// A row tile starting at a (relative to a0) needs the column tiles from the one
// holding b = a on; the earlier ones lie wholly below the diagonal b >= a.
void build_tile_table(int tile, int v, int a0, int a1, std::vector<int>& tiles, int& n_mt, int& n_nt) {
  constexpr int kBuildGroup = PPL_BUILD_GROUP;
  int bm, bn;
  build_tile_dims(tile, &bm, &bn);
  const int64_t M = (int64_t)(a1 - a0) * v, N = (int64_t)(v - a0) * v;
  n_mt = (int)((M + bm - 1) / bm);
  n_nt = (int)((N + bn - 1) / bn);
  tiles.clear();
  for (int g0 = 0; g0 < n_mt; g0 += kBuildGroup) {
    const int g1 = g0 + kBuildGroup < n_mt ? g0 + kBuildGroup : n_mt;
    const int nt_first = (int)(((int64_t)g0 * bm / v) * v / bn);
    for (int nt = nt_first; nt < n_nt; ++nt)
      for (int mt = g0; mt < g1; ++mt) {
        const int64_t arel = (int64_t)mt * bm / v;
        if (nt < arel * v / bn) break;   // nt_min grows with mt
        tiles.push_back(mt);
        tiles.push_back(nt);
      }
  }
}

// The upper-triangle build of one step (see EpiBuildSym): row tiles over the packed pairs
// (a, c >= a) of a in [a0, a1), column tiles over the packed pairs (b <= d) of b >= a0,
// ordered by b. Columns with b >= a start at a v - a (a - 1) / 2 of that order, so a row
// tile whose first virtual is a needs only the column tiles from there on. Launch order
// as in build_tile_table (groups of row tiles walked column tile by column tile).
void build_tile_table_sym(int tile, int v, int a0, int a1, std::vector<int>& tiles, int& n_mt, int& n_nt) {
  constexpr int kBuildGroup = PPL_BUILD_GROUP;
  int bm, bn;
  build_tile_dims(tile, &bm, &bn);
  const int64_t pr0 = pair_plus(a0, a0, v);
  const int64_t pr1 = a1 >= v ? npairs_plus(v) : pair_plus(a1, a1, v);
  const int64_t M = pr1 - pr0, W = v - a0, N = W * (W + 1) / 2;
  n_mt = (int)((M + bm - 1) / bm);
  n_nt = (int)((N + bn - 1) / bn);
  auto sfx = [&](int64_t a) { return a * v - a * (a - 1) / 2; };
  std::vector<int> nt_first(n_mt);
  int a = a0;
  for (int mt = 0; mt < n_mt; ++mt) {
    const int64_t m = (int64_t)mt * bm + pr0;                 // first packed pair of the tile
    while (a + 1 < a1 && pair_plus(a + 1, a + 1, v) <= m) ++a;
    nt_first[mt] = (int)((sfx(a) - sfx(a0)) / bn);
  }
  tiles.clear();
  for (int g0 = 0; g0 < n_mt; g0 += kBuildGroup) {
    const int g1 = g0 + kBuildGroup < n_mt ? g0 + kBuildGroup : n_mt;
    for (int nt = nt_first[g0]; nt < n_nt; ++nt)
      for (int mt = g0; mt < g1; ++mt) {
        if (nt < nt_first[mt]) break;   // nt_first grows with mt
        tiles.push_back(mt);
        tiles.push_back(nt);
      }
  }
}

// Operand rows b * v + d of the packed pairs b <= d, ordered by b, then d.
void build_column_order(int v, std::vector<int>& cols) {
  cols.clear();
  cols.reserve((size_t)v * (v + 1) / 2);
  for (int b = 0; b < v; ++b)
    for (int d = b; d < v; ++d) cols.push_back(b * v + d);
}

// ------------------------------------------------------------------ launchers
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi, class Map>
static int launch(hipStream_t s, int64_t grid, int64_t M, int64_t N, int64_t Kpad, const T* A,
                  int64_t lda, const T* B, int64_t ldb, Epi epi, Map map) {
  if (grid <= 0) return PPL_OK;
  if (grid > 0x7fffffffLL) return fail(PPL_E_ARG, "GEMM grid too large (%lld tiles)", (long long)grid);
  if (Kpad % KC != 0) return fail(PPL_E_ARG, "K padding %lld not a multiple of %d", (long long)Kpad, KC);
  hipLaunchKernelGGL((gemm_nt_kernel<T, WM, WN, WAVES_M, WAVES_N, KC, Epi, Map>), dim3((unsigned)grid),
                     dim3(64 * WAVES_M * WAVES_N), 0, s, M, N, Kpad, A, lda, B, ldb, epi, map);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

template <int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi, class Map>
static int launch_bf3(hipStream_t s, int64_t grid, int64_t M, int64_t N, int64_t Kpad,
                      const __bf16* Ah, const __bf16* Al, int64_t lda, const __bf16* Bh,
                      const __bf16* Bl, int64_t ldb, Epi epi, Map map) {
  if (grid <= 0) return PPL_OK;
  if (grid > 0x7fffffffLL) return fail(PPL_E_ARG, "GEMM grid too large (%lld tiles)", (long long)grid);
  if (Kpad % KC != 0) return fail(PPL_E_ARG, "K padding %lld not a multiple of %d", (long long)Kpad, KC);
  hipLaunchKernelGGL((gemm_nt_bf16x3_kernel<WM, WN, WAVES_M, WAVES_N, KC, Epi, Map>),
                     dim3((unsigned)grid), dim3(64 * WAVES_M * WAVES_N), 0, s, M, N, Kpad, Ah, Al,
                     lda, Bh, Bl, ldb, epi, map);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

template <int WM, int WN, int WAVES_M, int WAVES_N, class Epi, class Map>
static int launch_bf6(hipStream_t s, int64_t grid, int64_t M, int64_t N, int64_t Kpad, const __bf16* Ah,
                      const __bf16* Am, int64_t lda, const __bf16* Bh, const __bf16* Bm, int64_t ldb, Epi epi,
                      Map map) {
  if (grid <= 0) return PPL_OK;
  if (grid > 0x7fffffffLL) return fail(PPL_E_ARG, "GEMM grid too large (%lld tiles)", (long long)grid);
  if (Kpad % kKcBf6 != 0) return fail(PPL_E_ARG, "K padding %lld not a multiple of %d", (long long)Kpad, kKcBf6);
  if (!Am || !Bm) return fail(PPL_E_ARG, "BF16x6 operands need their mid planes");
  hipLaunchKernelGGL((gemm_nt_bf16x6_kernel<WM, WN, WAVES_M, WAVES_N, Epi, Map>), dim3((unsigned)grid),
                     dim3(64 * WAVES_M * WAVES_N), 0, s, M, N, Ah, Am, lda, Bh, Bm, ldb, epi, map);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

// sum of the split-K slices in slice order: C[m][c_col0 + n] = sum_s P[s][m][n]
template <class Tc>
__global__ void splitk_reduce_kernel(const Tc* __restrict__ P, int splits, int64_t split_stride,
                                     int64_t M, int64_t N, int64_t ldp_, Tc* C, int64_t ldc,
                                     int64_t c_col0) {
  const int64_t total = M * N;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const int64_t m = x / N, n = x - m * N;
    Tc acc = P[m * ldp_ + n];
    for (int sp = 1; sp < splits; ++sp) acc += P[sp * split_stride + m * ldp_ + n];
    C[m * ldc + c_col0 + n] = acc;
  }
}

// ------------------------------------------------------------------ stream-K
// The (tile, K chunk) iterations of one GEMM, tiles in row-tile-fastest order, are cut
// into G contiguous ranges of equal length, one per workgroup, with G the number of
// workgroups the device holds at once: the launch is one full wave of workgroups with
// no tail. A workgroup stores a tile that lies wholly inside its range straight into C.
// A tile shared by several workgroups is written by each into its own partial slot
// (slot 0: the first tile of its range, slot 1: the last one) and summed in workgroup
// order by streamk_fixup_kernel, so a given G gives bitwise reproducible results.
struct StreamK {
  int64_t n_mt, nk, iters, G;
  __host__ __device__ int64_t start(int64_t w) const { return w * iters / G; }
};

template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) __attribute__((amdgpu_waves_per_eu(2)))
gemm_streamk_kernel(int64_t M, int64_t N, const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                    int64_t ldb, T* C, int64_t ldc, int64_t c_col0, T* part, StreamK sk) {
  using G = TileGeom<T, WM, WN, WAVES_M, WAVES_N, KC>;
  __shared__ __attribute__((aligned(16))) T sA0[G::BUF_A];
  __shared__ __attribute__((aligned(16))) T sA1[G::BUF_A];
  __shared__ __attribute__((aligned(16))) T sB0[G::BUF_B];
  __shared__ __attribute__((aligned(16))) T sB1[G::BUF_B];
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t begin = sk.start(w), end = sk.start(w + 1);
  const int64_t first_tile = begin / sk.nk;
  for (int64_t it = begin; it < end;) {
    const int64_t tile = it / sk.nk, t0 = tile * sk.nk;
    const int64_t k0 = it - t0, k1 = end - t0 < sk.nk ? end - t0 : sk.nk;
    TileJob job{(tile % sk.n_mt) * G::BM, (tile / sk.n_mt) * G::BN, k0, k1, 0};
    const bool whole = k0 == 0 && k1 == sk.nk;
    EpiSK<T> epi{C, ldc, c_col0, M, N,
                 part + (w * 2 + (tile == first_tile ? 0 : 1)) * (int64_t)(G::BM * G::BN),
                 job.m0, job.n0, G::BN, !whole};
    tile_body<T, WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, A, lda, B, ldb, epi, sA0, sA1, sB0, sB1);
    it = t0 + k1;
    __syncthreads();   // the next tile refills the LDS buffers
  }
}

template <int WM, int WN, int WAVES_M, int WAVES_N, int KC>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
gemm_streamk_bf16x3_kernel(int64_t M, int64_t N, const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al,
                           int64_t lda, const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl, int64_t ldb,
                           float* C, int64_t ldc, int64_t c_col0, float* part, StreamK sk) {
  using G = Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>;
  constexpr int SA = kBf3Direct ? G::STAGE : G::LDS_A, SB = kBf3Direct ? G::STAGE : G::LDS_B;
  __shared__ __attribute__((aligned(16))) __bf16 sAh[SA];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[SA];
  __shared__ __attribute__((aligned(16))) __bf16 sBh[SB];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[kBf3Direct ? 8 : G::LDS_B];
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t begin = sk.start(w), end = sk.start(w + 1);
  const int64_t first_tile = begin / sk.nk;
  for (int64_t it = begin; it < end;) {
    const int64_t tile = it / sk.nk, t0 = tile * sk.nk;
    const int64_t k0 = it - t0, k1 = end - t0 < sk.nk ? end - t0 : sk.nk;
    TileJob job{(tile % sk.n_mt) * G::BM, (tile / sk.n_mt) * G::BN, k0, k1, 0};
    const bool whole = k0 == 0 && k1 == sk.nk;
    EpiSK<float> epi{C, ldc, c_col0, M, N,
                     part + (w * 2 + (tile == first_tile ? 0 : 1)) * (int64_t)(G::BM * G::BN),
                     job.m0, job.n0, G::BN, !whole};
    if constexpr (kBf3Direct)   // the first three arrays serve as the three stages
      bf3_tile_body_direct<WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, Ah, Al, lda, Bh, Bl, ldb, epi, sAh, sAl, sBh);
    else
      bf3_tile_body<WM, WN, WAVES_M, WAVES_N, KC>(job, M, N, Ah, Al, lda, Bh, Bl, ldb, epi, sAh, sAl, sBh, sBl);
    it = t0 + k1;
    __syncthreads();   // the next tile refills the LDS buffers
  }
}

template <int WM, int WN, int WAVES_M, int WAVES_N>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
gemm_streamk_bf16x6_kernel(int64_t M, int64_t N, const __bf16* Ah, const __bf16* Am, int64_t lda, const __bf16* Bh,
                           const __bf16* Bm, int64_t ldb, float* C, int64_t ldc, int64_t c_col0, float* part,
                           StreamK sk) {
  using G = Bf6Geom<WM, WN, WAVES_M, WAVES_N>;
  // (the direct body takes the two arrays as its two stages: 2 STAGE = LDS_A + LDS_B)
  __shared__ __attribute__((aligned(16))) __bf16 sA[kBf6Direct ? G::STAGE : G::LDS_A];
  __shared__ __attribute__((aligned(16))) __bf16 sB[kBf6Direct ? G::STAGE : G::LDS_B];
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t begin = sk.start(w), end = sk.start(w + 1);
  const int64_t first_tile = begin / sk.nk;
  for (int64_t it = begin; it < end;) {
    const int64_t tile = it / sk.nk, t0 = tile * sk.nk;
    const int64_t k0 = it - t0, k1 = end - t0 < sk.nk ? end - t0 : sk.nk;
    TileJob job{(tile % sk.n_mt) * G::BM, (tile / sk.n_mt) * G::BN, k0, k1, 0};
    const bool whole = k0 == 0 && k1 == sk.nk;
    EpiSK<float> epi{C, ldc, c_col0, M, N,
                     part + (w * 2 + (tile == first_tile ? 0 : 1)) * (int64_t)(G::BM * G::BN),
                     job.m0, job.n0, G::BN, !whole};
    if constexpr (kBf6Direct)
      bf6_tile_body_direct<WM, WN, WAVES_M, WAVES_N>(job, M, N, Ah, Am, lda, Bh, Bm, ldb, epi, sA, sB);
    else
      bf6_tile_body<WM, WN, WAVES_M, WAVES_N>(job, M, N, Ah, Am, lda, Bh, Bm, ldb, epi, sA, sB);
    it = t0 + k1;
    __syncthreads();   // the next tile refills the LDS buffers
  }
}

// C tile `blockIdx.x` = sum of the partial slots of the workgroups that shared it
template <class T>
__global__ void __launch_bounds__(256)
streamk_fixup_kernel(const T* __restrict__ part, T* C, int64_t ldc, int64_t c_col0, int64_t M, int64_t N,
                     int bm, int bn, StreamK sk) {
  const int64_t tile = blockIdx.x;
  const int64_t a = tile * sk.nk, b = a + sk.nk;
  int64_t wlo = a * sk.G / sk.iters;          // start(wlo) <= a; step up to the last such
  while (wlo + 1 < sk.G && sk.start(wlo + 1) <= a) ++wlo;
  int64_t whi = (b - 1) * sk.G / sk.iters;
  while (whi + 1 < sk.G && sk.start(whi + 1) <= b - 1) ++whi;
  if (wlo == whi) return;                    // one workgroup held the whole tile
  const int64_t m0 = (tile % sk.n_mt) * bm, n0 = (tile / sk.n_mt) * bn;
  const int64_t slot_elems = (int64_t)bm * bn;
  for (int e = threadIdx.x; e < bm * bn; e += blockDim.x) {
    const int r = e / bn, c = e - r * bn;
    if (m0 + r >= M || n0 + c >= N) continue;
    T acc = 0;
    bool first = true;
    for (int64_t w = wlo; w <= whi; ++w) {
      const int64_t s0 = sk.start(w);
      if (sk.start(w + 1) <= s0) continue;    // empty range
      const T x = part[(w * 2 + (s0 / sk.nk == tile ? 0 : 1)) * slot_elems + e];
      acc = first ? x : acc + x;
      first = false;
    }
    C[(m0 + r) * ldc + c_col0 + n0 + c] = acc;
  }
}

// workgroups of `kernel` resident on the current device at once (cached per device)
template <class K>
static int64_t resident_workgroups(K kernel, int threads) {
  static int64_t cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int cus = 0, nb = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess) return 0;
    cache[dev] = (int64_t)cus * (nb > 0 ? nb : 1);
  }
  return cache[dev];
}

// workgroups of a stream-K launch: all resident ones, at most kStreamKMaxGrid, and
// few enough that each gets at least kStreamKMinChunks K chunks
static int64_t streamk_grid(int64_t resident, int64_t iters) {
  int64_t g = resident < kStreamKMaxGrid ? resident : kStreamKMaxGrid;
  const int64_t cap = iters / kStreamKMinChunks;
  if (g > cap) g = cap;
  return g > 1 ? g : 1;
}

// K elements per staged chunk of a precision on a tile of bm x bn
static int kc_of(int prec, int bm, int bn) {
  return prec == PPL_BF16X3 ? bf3_kc(bm, bn) : (prec == PPL_BF16X6 ? kKcBf6 : kc_of_prec(prec));
}

uint64_t streamk_part_bytes(int tile, int prec, int64_t Nrows, int64_t Prows, int64_t Kpad) {
  const TileCfg& c = kContract[tile];
  const int KC = kc_of(prec, c.bm(), c.bn());
  const int64_t iters = ((Nrows + c.bm() - 1) / c.bm()) * ((Prows + c.bn() - 1) / c.bn()) * (Kpad / KC);
  return (uint64_t)streamk_grid(kStreamKMaxGrid, iters) * 2 * c.bm() * c.bn() * (prec == PPL_FP64 ? 8 : 4);
}

// grid of a stream-K launch: G workgroups over the (tile, chunk) iterations, with a
// check that the partial buffer holds G x 2 slots of BM x BN elements
static int streamk_setup(int64_t resident, int64_t M, int64_t N, int64_t nk, int bm, int bn, size_t elem,
                         const void* part, uint64_t part_bytes, StreamK& sk, int64_t& n_tiles) {
  if (resident <= 0) return fail(PPL_E_HIP, "occupancy query for the stream-K kernel failed");
  sk = StreamK{(M + bm - 1) / bm, nk, 0, 0};
  n_tiles = sk.n_mt * ((N + bn - 1) / bn);
  sk.iters = n_tiles * nk;
  if (sk.iters <= 0) return PPL_OK;
  sk.G = streamk_grid(resident, sk.iters);
  const uint64_t need = (uint64_t)sk.G * 2 * bm * bn * elem;
  if (!part || need > part_bytes)
    return fail(PPL_E_STATE, "stream-K partial buffer holds %llu bytes, needs %llu",
                (unsigned long long)part_bytes, (unsigned long long)need);
  if (n_tiles > 0x7fffffffLL) return fail(PPL_E_ARG, "GEMM grid too large (%lld tiles)", (long long)n_tiles);
  return PPL_OK;
}

template <int WM, int WN, int WAVES_M, int WAVES_N, int KC>
static int launch_streamk_bf3(hipStream_t s, int64_t M, int64_t N, int64_t Kpad, const __bf16* Ah,
                              const __bf16* Al, int64_t lda, const __bf16* Bh, const __bf16* Bl, int64_t ldb,
                              float* C, int64_t ldc, int64_t c_col0, void* part, uint64_t part_bytes) {
  using G = Bf3Geom<WM, WN, WAVES_M, WAVES_N, KC>;
  if (Kpad % KC != 0) return fail(PPL_E_ARG, "K padding %lld not a multiple of %d", (long long)Kpad, KC);
  auto kern = gemm_streamk_bf16x3_kernel<WM, WN, WAVES_M, WAVES_N, KC>;
  StreamK sk;
  int64_t n_tiles = 0;
  PPL_TRY(streamk_setup(resident_workgroups(kern, G::NT), M, N, Kpad / KC, G::BM, G::BN, sizeof(float), part,
                        part_bytes, sk, n_tiles));
  if (sk.iters <= 0) return PPL_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)sk.G), dim3(G::NT), 0, s, M, N, Ah, Al, lda, Bh, Bl, ldb, C, ldc,
                     c_col0, (float*)part, sk);
  PPL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(streamk_fixup_kernel<float>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const float*)part,
                     C, ldc, c_col0, M, N, G::BM, G::BN, sk);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

template <int WM, int WN, int WAVES_M, int WAVES_N>
static int launch_streamk_bf6(hipStream_t s, int64_t M, int64_t N, int64_t Kpad, const __bf16* Ah,
                              const __bf16* Am, int64_t lda, const __bf16* Bh, const __bf16* Bm, int64_t ldb,
                              float* C, int64_t ldc, int64_t c_col0, void* part, uint64_t part_bytes) {
  using G = Bf6Geom<WM, WN, WAVES_M, WAVES_N>;
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  if (Kpad % kKcBf6 != 0) return fail(PPL_E_ARG, "K padding %lld not a multiple of %d", (long long)Kpad, kKcBf6);
  if (!Am || !Bm) return fail(PPL_E_ARG, "BF16x6 operands need their mid planes");
  auto kern = gemm_streamk_bf16x6_kernel<WM, WN, WAVES_M, WAVES_N>;
  StreamK sk;
  int64_t n_tiles = 0;
  PPL_TRY(streamk_setup(resident_workgroups(kern, NT), M, N, Kpad / kKcBf6, G::BM, G::BN, sizeof(float), part,
                        part_bytes, sk, n_tiles));
  if (sk.iters <= 0) return PPL_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)sk.G), dim3(NT), 0, s, M, N, Ah, Am, lda, Bh, Bm, ldb, C, ldc, c_col0,
                     (float*)part, sk);
  PPL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(streamk_fixup_kernel<float>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const float*)part,
                     C, ldc, c_col0, M, N, G::BM, G::BN, sk);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC>
static int launch_streamk(hipStream_t s, int64_t M, int64_t N, int64_t Kpad, const T* A, int64_t lda,
                          const T* B, int64_t ldb, T* C, int64_t ldc, int64_t c_col0, void* part,
                          uint64_t part_bytes) {
  using G = TileGeom<T, WM, WN, WAVES_M, WAVES_N, KC>;
  if (Kpad % KC != 0) return fail(PPL_E_ARG, "K padding %lld not a multiple of %d", (long long)Kpad, KC);
  auto kern = gemm_streamk_kernel<T, WM, WN, WAVES_M, WAVES_N, KC>;
  StreamK sk;
  int64_t n_tiles = 0;
  PPL_TRY(streamk_setup(resident_workgroups(kern, G::NT), M, N, Kpad / KC, G::BM, G::BN, sizeof(T), part,
                        part_bytes, sk, n_tiles));
  if (sk.iters <= 0) return PPL_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)sk.G), dim3(G::NT), 0, s, M, N, A, lda, B, ldb, C, ldc, c_col0,
                     (T*)part, sk);
  PPL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(streamk_fixup_kernel<T>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const T*)part, C, ldc,
                     c_col0, M, N, G::BM, G::BN, sk);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

// dispatch of one precision over the contraction tiles
template <int WM, int WN, int WAVES_M, int WAVES_N>
static int contract_cfg(hipStream_t s, int prec, int64_t Nrows, int64_t Prows, int64_t Kpad,
                        const void* S, const void* S_lo, int64_t lds_, const void* V,
                        const void* V_lo, int64_t ldv, void* C, int64_t ldc, int64_t c_col0,
                        int splits, void* partial, int64_t partial_ld, uint64_t partial_bytes,
                        bool accumulate) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  if (accumulate && splits != 1) return fail(PPL_E_ARG, "an accumulating contraction runs one K slice");
  const double cbeta = accumulate ? 1.0 : 0.0;
  if (splits == 0) {   // stream-K
    if (prec == PPL_FP64)
      return launch_streamk<double, WM, WN, WAVES_M, WAVES_N, kKcF64>(
          s, Nrows, Prows, Kpad, (const double*)S, lds_, (const double*)V, ldv, (double*)C, ldc, c_col0, partial,
          partial_bytes);
    if (prec == PPL_FP32)
      return launch_streamk<float, WM, WN, WAVES_M, WAVES_N, kKcF32>(
          s, Nrows, Prows, Kpad, (const float*)S, lds_, (const float*)V, ldv, (float*)C, ldc, c_col0, partial,
          partial_bytes);
    if (prec == PPL_BF16X3)
      return launch_streamk_bf3<WM, WN, WAVES_M, WAVES_N, bf3_kc(BM, BN)>(
          s, Nrows, Prows, Kpad, (const __bf16*)S, (const __bf16*)S_lo, lds_, (const __bf16*)V,
          (const __bf16*)V_lo, ldv, (float*)C, ldc, c_col0, partial, partial_bytes);
    if (prec == PPL_BF16X6)
      return launch_streamk_bf6<WM, WN, WAVES_M, WAVES_N>(s, Nrows, Prows, Kpad, (const __bf16*)S,
                                                          (const __bf16*)S_lo, lds_, (const __bf16*)V,
                                                          (const __bf16*)V_lo, ldv, (float*)C, ldc, c_col0, partial,
                                                          partial_bytes);
    return fail(PPL_E_ARG, "unknown precision %d", prec);
  }
  const int KC = kc_of(prec, BM, BN);
  const int64_t nk = Kpad / KC;
  if (splits < 1) splits = 1;
  if (splits > nk) splits = (int)nk;
  const int64_t kps = (nk + splits - 1) / splits;
  splits = (int)((nk + kps - 1) / kps);                 // no empty slice
  const bool direct = splits == 1;
  if (!direct && (!partial || (uint64_t)splits * Nrows * partial_ld * (prec == PPL_FP64 ? 8 : 4) > partial_bytes))
    return fail(PPL_E_STATE, "split-K partial buffer too small for %d slices", splits);
  MapGrid map{(Nrows + BM - 1) / BM, (Prows + BN - 1) / BN, BM, BN, splits, nk, kps};
  const int64_t grid = map.n_mt * map.n_nt * splits;
  const int64_t pstride = Nrows * partial_ld;
  int rc = PPL_OK;
  if (prec == PPL_FP64) {
    EpiStore<double> epi = direct ? EpiStore<double>{(double*)C, ldc, c_col0, Nrows, Prows, 1.0, cbeta, 0}
                                  : EpiStore<double>{(double*)partial, partial_ld, 0, Nrows, Prows, 1.0, 0.0, pstride};
    rc = launch<double, WM, WN, WAVES_M, WAVES_N, kKcF64>(s, grid, Nrows, Prows, Kpad, (const double*)S, lds_,
                                                      (const double*)V, ldv, epi, map);
  } else if (prec == PPL_FP32) {
    EpiStore<float> epi = direct ? EpiStore<float>{(float*)C, ldc, c_col0, Nrows, Prows, 1.0, cbeta, 0}
                                 : EpiStore<float>{(float*)partial, partial_ld, 0, Nrows, Prows, 1.0, 0.0, pstride};
    rc = launch<float, WM, WN, WAVES_M, WAVES_N, kKcF32>(s, grid, Nrows, Prows, Kpad, (const float*)S, lds_,
                                                     (const float*)V, ldv, epi, map);
  } else if (prec == PPL_BF16X3) {
    EpiStore<float> epi = direct ? EpiStore<float>{(float*)C, ldc, c_col0, Nrows, Prows, 1.0, cbeta, 0}
                                 : EpiStore<float>{(float*)partial, partial_ld, 0, Nrows, Prows, 1.0, 0.0, pstride};
    rc = launch_bf3<WM, WN, WAVES_M, WAVES_N, bf3_kc(BM, BN)>(s, grid, Nrows, Prows, Kpad, (const __bf16*)S,
                                                  (const __bf16*)S_lo, lds_, (const __bf16*)V,
                                                  (const __bf16*)V_lo, ldv, epi, map);
  } else if (prec == PPL_BF16X6) {
    EpiStore<float> epi = direct ? EpiStore<float>{(float*)C, ldc, c_col0, Nrows, Prows, 1.0, cbeta, 0}
                                 : EpiStore<float>{(float*)partial, partial_ld, 0, Nrows, Prows, 1.0, 0.0, pstride};
    rc = launch_bf6<WM, WN, WAVES_M, WAVES_N>(s, grid, Nrows, Prows, Kpad, (const __bf16*)S, (const __bf16*)S_lo,
                                              lds_, (const __bf16*)V, (const __bf16*)V_lo, ldv, epi, map);
  } else {
    return fail(PPL_E_ARG, "unknown precision %d", prec);
  }
  if (rc != PPL_OK || direct) return rc;
  const int64_t total = Nrows * Prows;
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (prec == PPL_FP64)
    hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3((unsigned)g), dim3(256), 0, s, (const double*)partial,
                       splits, pstride, Nrows, Prows, partial_ld, (double*)C, ldc, c_col0);
  else
    hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3((unsigned)g), dim3(256), 0, s, (const float*)partial,
                       splits, pstride, Nrows, Prows, partial_ld, (float*)C, ldc, c_col0);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

int gemm_contract(hipStream_t s, int prec, int tile, int64_t Nrows, int64_t Prows, int64_t Kpad,
                  const void* S, const void* S_lo, int64_t lds_, const void* V, const void* V_lo,
                  int64_t ldv, void* C, int64_t ldc, int64_t c_col0, int splits, void* partial,
                  int64_t partial_ld, uint64_t partial_bytes, bool accumulate) {
  if (Nrows <= 0 || Prows <= 0) return PPL_OK;
#define PPL_CFG(id, a, b, c, d)                                                                  \
  case id:                                                                                       \
    return contract_cfg<a, b, c, d>(s, prec, Nrows, Prows, Kpad, S, S_lo, lds_, V, V_lo, ldv, C,  \
                                    ldc, c_col0, splits, partial, partial_ld, partial_bytes, accumulate);
  switch (tile) {
    PPL_CFG(0, 7, 2, 1, 4)
    PPL_CFG(1, 4, 4, 2, 2)
    PPL_CFG(2, 13, 1, 1, 4)
    PPL_CFG(3, 2, 4, 1, 4)
    PPL_CFG(4, 3, 4, 1, 4)
    PPL_CFG(5, 6, 2, 1, 4)
    PPL_CFG(6, 2, 2, 1, 4)
    PPL_CFG(7, 3, 2, 1, 4)
    PPL_CFG(8, 4, 2, 1, 4)
    PPL_CFG(9, 7, 2, 2, 4)
    PPL_CFG(10, 7, 1, 2, 4)
    default:
      return fail(PPL_E_ARG, "unknown contraction tile %d", tile);
  }
#undef PPL_CFG
}

// Workgroups of one contraction launch for a (tile, splits) choice.
int64_t contract_jobs(int tile, int prec, int64_t Nrows, int64_t Prows, int64_t Kpad, int splits) {
  const TileCfg& c = kContract[tile];
  const int KC = kc_of(prec, c.bm(), c.bn());
  const int64_t nk = Kpad / KC;
  if (splits > nk) splits = (int)nk;
  const int64_t kps = (nk + splits - 1) / splits;
  splits = (int)((nk + kps - 1) / kps);
  return ((Nrows + c.bm() - 1) / c.bm()) * ((Prows + c.bn() - 1) / c.bn()) * splits;
}

// Relative per-tile throughput on large problems, measured with HIP events on
// gfx950, per padded flop; 1.0 = best tile of the precision. FP64 and FP32
// (three-stage direct loads): best over 1, 2 and 4 K slices, averaged over R+ and R-
// at (30, 300, 900) and (40, 400, 1200) (FP32 at the first only; at (40, 400, 1200)
// FP32 ranks tiles 9, 8 and 0 the same way). BF16x3
// (three-stage direct loads): R+ and R- at (40, 400, 1200), best of 1 and 2 slices, per
// padded flop. BF16x6 (two-stage direct loads): R+ and R- at (40, 400, 1200) in the 7
// slices its error bound asks for there, per padded flop.
static const double kTileEff[4][11] = {
    /* FP64   */ {0.90, 0.91, 0.85, 0.83, 0.85, 0.91, 0.90, 0.95, 0.97, 0.98, 1.00},
    /* FP32   */ {0.94, 0.96, 0.87, 0.82, 0.90, 0.92, 0.92, 0.95, 0.97, 1.00, 0.93},
    /* BF16x3 */ {0.71, 0.79, 0.61, 0.39, 0.53, 0.68, 0.46, 0.42, 0.51, 1.00, 0.68},
    /* BF16x6 */ {0.84, 0.88, 0.63, 0.48, 0.66, 0.82, 0.53, 0.60, 0.69, 1.00, 0.68}};
static_assert(sizeof(kTileEff[0]) / sizeof(double) == kNumContract, "one efficiency per tile");

// BF16x6 products carry FP32's 24 bits, so its error is set by the length of each FP32
// accumulation: a K slice spans at most kBf6SliceK elements. Measured at (40,400,1200)
// (K = 80256, HIP path against FP64): one R lies 1.8e-6 from FP64 with one slice, then
// 1.3e-6, 9.5e-7 and 7.0e-7 with 2, 4 and 8 (the error goes as the square root of the
// slice length); 12288 gives 7 slices there, below 1e-6.
constexpr int64_t kBf6SliceK = 12288;
int contract_min_splits(int prec, int64_t Kpad) {
  if (prec != PPL_BF16X6) return 1;
  const int64_t sp = (Kpad + kBf6SliceK - 1) / kBf6SliceK;
  return (int)(sp < 1 ? 1 : (sp > kMaxSplits ? kMaxSplits : sp));
}

// Model choice of (tile, splits): useful work over the work of the padded tiles,
// times the fill of the last round of workgroups over 256 CUs, times the
// measured relative throughput of the tile.
void contract_choose(int prec, int64_t Nrows, int64_t Prows, int64_t Kpad, int max_splits, int* tile_out,
                     int* splits_out) {
  double best = -1.0;
  int bt = 0, bs = 1;
  const int fixed = *tile_out;
  for (int t = 0; t < kNumContract; ++t) {
    if (fixed >= 0 && t != fixed) continue;
    const TileCfg& c = kContract[t];
    const int64_t mp = (Nrows + c.bm() - 1) / c.bm() * c.bm(), np = (Prows + c.bn() - 1) / c.bn() * c.bn();
    const double pad = (double)Nrows * Prows / ((double)mp * np);
    const int sp_min = std::min(contract_min_splits(prec, Kpad), std::max(max_splits, 1));
    for (int sp = sp_min; sp <= max_splits; ++sp) {
      const int64_t jobs = contract_jobs(t, prec, Nrows, Prows, Kpad, sp);
      const double rounds = (double)jobs / 256.0;
      const double fill = rounds / std::ceil(rounds);
      // small penalty per extra slice (partial traffic, reduction launch)
      const int pi = prec == PPL_FP64 ? 0 : (prec == PPL_FP32 ? 1 : (prec == PPL_BF16X3 ? 2 : 3));
      const double score = pad * fill * (1.0 - 0.01 * (sp - 1)) * kTileEff[pi][t];
      if (score > best + 1e-9) {
        best = score;
        bt = t;
        bs = sp;
      }
    }
  }
  *tile_out = bt;
  *splits_out = bs;
}

template <int WM, int WN, int WAVES_M, int WAVES_N>
static int build_cfg(hipStream_t s, int prec, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                     const void* Xt_lo, int64_t ldx, void* G, const int* tile_list, int64_t n_valid_tiles) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  const int64_t M = (int64_t)(a1 - a0) * v, N = (int64_t)(v - a0) * v;
  MapBuild map{tile_list, n_valid_tiles, BM, BN, 0};
  map.nk = Kpad / kc_of(prec, BM, BN);
  if (prec == PPL_FP64) {
    const double* X = (const double*)Xt + (int64_t)a0 * v * ldx;
    EpiBuild<double> epi{(double*)G, M, N, v, a0};
    return launch<double, WM, WN, WAVES_M, WAVES_N, kKcF64>(s, n_valid_tiles, M, N, Kpad, X, ldx, X, ldx,
                                                            epi, map);
  }
  if (prec == PPL_FP32) {
    const float* X = (const float*)Xt + (int64_t)a0 * v * ldx;
    EpiBuild<float> epi{(float*)G, M, N, v, a0};
    return launch<float, WM, WN, WAVES_M, WAVES_N, kKcF32>(s, n_valid_tiles, M, N, Kpad, X, ldx, X, ldx,
                                                           epi, map);
  }
  if (prec == PPL_BF16X3) {
    const __bf16* Xh = (const __bf16*)Xt + (int64_t)a0 * v * ldx;
    const __bf16* Xl = (const __bf16*)Xt_lo + (int64_t)a0 * v * ldx;
    EpiBuild<float> epi{(float*)G, M, N, v, a0};
    return launch_bf3<WM, WN, WAVES_M, WAVES_N, bf3_kc(BM, BN)>(s, n_valid_tiles, M, N, Kpad, Xh, Xl, ldx, Xh,
                                                        Xl, ldx, epi, map);
  }
  if (prec == PPL_BF16X6) {
    const __bf16* Xh = (const __bf16*)Xt + (int64_t)a0 * v * ldx;
    const __bf16* Xm = (const __bf16*)Xt_lo + (int64_t)a0 * v * ldx;
    EpiBuild<float> epi{(float*)G, M, N, v, a0};
    return launch_bf6<WM, WN, WAVES_M, WAVES_N>(s, n_valid_tiles, M, N, Kpad, Xh, Xm, ldx, Xh, Xm, ldx, epi, map);
  }
  return fail(PPL_E_ARG, "unknown precision %d", prec);
}

// epilogue of the upper-triangle build: G blocks (EpiBuildSym) or the natural layout (EpiBuildT)
template <class Tg, bool NAT>
static auto build_sym_epi(void* G, int64_t M, int64_t N, int v, int a0, int W, int64_t pr0, const int* tab_vp,
                          const int* cstep) {
  if constexpr (NAT) return EpiBuildT<Tg>{(Tg*)G, M, N, N, v, pr0, tab_vp, cstep};
  else return EpiBuildSym<Tg>{(Tg*)G, M, N, v, a0, W, pr0, tab_vp, cstep};
}

template <int WM, int WN, int WAVES_M, int WAVES_N, bool NAT>
static int build_sym_cfg(hipStream_t s, int prec, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                         const void* Xt_lo, int64_t ldx, void* G, const int* tile_list, int64_t n_valid_tiles,
                         const int* tab_vp, const int* cols) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  const int64_t pr0 = pair_plus(a0, a0, v);
  const int64_t pr1 = a1 >= v ? npairs_plus(v) : pair_plus(a1, a1, v);
  const int W = v - a0;
  const int64_t M = pr1 - pr0, N = (int64_t)W * (W + 1) / 2;
  const int* cstep = cols + (npairs_plus(v) - N);       // first column with b = a0
  MapBuild map{tile_list, n_valid_tiles, BM, BN, 0};
  map.nk = Kpad / kc_of(prec, BM, BN);
  if (prec == PPL_FP64) {
    auto epi = build_sym_epi<double, NAT>(G, M, N, v, a0, W, pr0, tab_vp, cstep);
    return launch<double, WM, WN, WAVES_M, WAVES_N, kKcF64>(s, n_valid_tiles, M, N, Kpad, (const double*)Xt, ldx,
                                                            (const double*)Xt, ldx, epi, map);
  }
  if (prec == PPL_FP32) {
    auto epi = build_sym_epi<float, NAT>(G, M, N, v, a0, W, pr0, tab_vp, cstep);
    return launch<float, WM, WN, WAVES_M, WAVES_N, kKcF32>(s, n_valid_tiles, M, N, Kpad, (const float*)Xt, ldx,
                                                           (const float*)Xt, ldx, epi, map);
  }
  if (prec == PPL_BF16X3) {
    auto epi = build_sym_epi<float, NAT>(G, M, N, v, a0, W, pr0, tab_vp, cstep);
    return launch_bf3<WM, WN, WAVES_M, WAVES_N, bf3_kc(BM, BN)>(s, n_valid_tiles, M, N, Kpad, (const __bf16*)Xt,
                                                                (const __bf16*)Xt_lo, ldx, (const __bf16*)Xt,
                                                                (const __bf16*)Xt_lo, ldx, epi, map);
  }
  if (prec == PPL_BF16X6) {
    auto epi = build_sym_epi<float, NAT>(G, M, N, v, a0, W, pr0, tab_vp, cstep);
    return launch_bf6<WM, WN, WAVES_M, WAVES_N>(s, n_valid_tiles, M, N, Kpad, (const __bf16*)Xt,
                                                (const __bf16*)Xt_lo, ldx, (const __bf16*)Xt, (const __bf16*)Xt_lo,
                                                ldx, epi, map);
  }
  return fail(PPL_E_ARG, "unknown precision %d", prec);
}

template <bool NAT>
static int build_sym_tile(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                          const void* Xt_lo, int64_t ldx, void* G, const int* tl, int64_t nv, const int* tab_vp,
                          const int* cols) {
  switch (tile) {
    case 0: return build_sym_cfg<7, 2, 1, 4, NAT>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tl, nv, tab_vp, cols);
    case 1: return build_sym_cfg<4, 4, 2, 2, NAT>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tl, nv, tab_vp, cols);
    case 5: return build_sym_cfg<6, 2, 1, 4, NAT>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tl, nv, tab_vp, cols);
    case 8: return build_sym_cfg<4, 2, 1, 4, NAT>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tl, nv, tab_vp, cols);
    case 9: return build_sym_cfg<7, 2, 2, 4, NAT>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tl, nv, tab_vp, cols);
    case 10: return build_sym_cfg<7, 1, 2, 4, NAT>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tl, nv, tab_vp, cols);
    default: return fail(PPL_E_ARG, "tile %d is not a build tile", tile);
  }
}

int gemm_build_sym(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                   const void* Xt_lo, int64_t ldx, void* G, const int* tile_list, int64_t n_valid_tiles,
                   const int* tab_vp, const int* cols) {
  return build_sym_tile<false>(s, prec, tile, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles, tab_vp,
                               cols);
}

int gemm_build_natural(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad, const void* Xt,
                       const void* Xt_lo, int64_t ldx, void* T, const int* tile_list, int64_t n_valid_tiles,
                       const int* tab_vp, const int* cols) {
  return build_sym_tile<true>(s, prec, tile, v, a0, a1, Kpad, Xt, Xt_lo, ldx, T, tile_list, n_valid_tiles, tab_vp,
                              cols);
}

int gemm_build(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad,
               const void* Xt, const void* Xt_lo, int64_t ldx, void* G, const int* tile_list,
               int64_t n_valid_tiles) {
  switch (tile) {
    case 0: return build_cfg<7, 2, 1, 4>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles);
    case 1: return build_cfg<4, 4, 2, 2>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles);
    case 5: return build_cfg<6, 2, 1, 4>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles);
    case 8: return build_cfg<4, 2, 1, 4>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles);
    case 9: return build_cfg<7, 2, 2, 4>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles);
    case 10: return build_cfg<7, 1, 2, 4>(s, prec, v, a0, a1, Kpad, Xt, Xt_lo, ldx, G, tile_list, n_valid_tiles);
    default: return fail(PPL_E_ARG, "tile %d is not a build tile", tile);
  }
}

int gemm_store_f64(hipStream_t s, int64_t M, int64_t N, int64_t Kpad, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc) {
  constexpr int WM = 4, WN = 4, WAVES_M = 2, WAVES_N = 2;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  MapGrid map{(M + BM - 1) / BM, (N + BN - 1) / BN, BM, BN, 1, Kpad / kKcF64, Kpad / kKcF64};
  EpiStore<double> epi{C, ldc, 0, M, N, 1.0, 0.0, 0};
  return launch<double, WM, WN, WAVES_M, WAVES_N, kKcF64>(s, map.n_mt * map.n_nt, M, N, Kpad, A, lda, B,
                                                      ldb, epi, map);
}

// ------------------------------------------------------------------ grouped persistent contraction
// Many independent contraction GEMMs (instances x {R+, R-}) in one launch: a
// fixed grid of workgroups pulls (group, row tile, column tile) items from a
// queue sorted longest-first; each group carries its own tile shape. Every
// workgroup leaves the loop once the queue counter passes the item count.
bool grouped_tile_ok(int tile) { return (tile >= 0 && tile <= 2) || (tile >= 5 && tile <= 8); }

// the model's choice among the grouped tiles: the batch fills the device, so only the
// padding of the occupied-pair rows and the measured per-tile throughput count
int grouped_choose_tile(int prec, int64_t rows) {
  const int pi = prec == PPL_FP64 ? 0 : (prec == PPL_FP32 ? 1 : 2);
  int best = 5;
  double best_score = -1.0;
  for (int t = 0; t < kNumContract; ++t) {
    if (!grouped_tile_ok(t)) continue;
    const int bm = kContract[t].bm();
    const double score = (double)rows / (double)((rows + bm - 1) / bm * bm) * kTileEff[pi][t];
    if (score > best_score + 1e-9) {
      best_score = score;
      best = t;
    }
  }
  return best;
}

typedef __attribute__((address_space(1))) char global_char_t;

template <class T>
struct GroupedLds {       // LDS of the largest allowed tile (208 x 64 rows staged, 272 in all)
  static constexpr int KC = sizeof(T) == 8 ? kKcF64 : kKcF32;
  static constexpr int bytes = TileGeom<T, 13, 1, 1, 4, KC>::LDS_BYTES;
  static constexpr int stage = 272 * KC;   // elements of one direct-load stage of that tile
};

// The same item with the three-stage direct loads: the stages are three distinct LDS
// arrays of the kernel (so that the compiler tells the loads into one stage from the
// reads of another), and the function is inlined into it for the same reason.
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC>
__device__ __forceinline__ void grouped_tile_direct(const GroupDesc& g, int m0, int n0, T* st0, T* st1, T* st2,
                                                    global_char_t* base) {
  static_assert((16 * WM * WAVES_M + 16 * WN * WAVES_N) * KC <= GroupedLds<T>::stage, "tile exceeds the stages");
  static_assert(64 * WAVES_M * WAVES_N == 256, "grouped tiles use 256 threads");
  TileJob job{m0, n0, 0, g.nk, 0};
  const T* A = (const T*)(base + g.a_off);
  const T* B = (const T*)(base + g.b_off);
  EpiStore<T> epi{(T*)(base + g.c_off), g.ldc, 0, g.M, g.N, 1.0, 0.0, 0};
  tile_body_direct3<T, WM, WN, WAVES_M, WAVES_N, KC>(job, g.M, g.N, A, g.lda, B, g.ldb, epi, st0, st1, st2);
}

template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC>
__device__ __noinline__ void grouped_tile(const GroupDesc& g, int m0, int n0, char* smem, global_char_t* base) {
  using G = TileGeom<T, WM, WN, WAVES_M, WAVES_N, KC>;
  static_assert(G::LDS_BYTES <= GroupedLds<T>::bytes, "tile does not fit the grouped LDS buffer");
  static_assert(G::NT == 256, "grouped tiles use 256 threads");
  TileJob job{m0, n0, 0, g.nk, 0};
  // operands addressed from a base pointer typed as global memory: generic pointers
  // (loaded from memory, or passed to a function that is not inlined) give flat loads,
  // which also count against the LDS wait counter and serialize the chunk pipeline
  const T* A = (const T*)(base + g.a_off);
  const T* B = (const T*)(base + g.b_off);
  EpiStore<T> epi{(T*)(base + g.c_off), g.ldc, 0, g.M, g.N, 1.0, 0.0, 0};
  T* s = reinterpret_cast<T*>(smem);
  tile_body<T, WM, WN, WAVES_M, WAVES_N, KC>(job, g.M, g.N, A, g.lda, B, g.ldb, epi,
                                             s, s + G::BUF_A, s + 2 * G::BUF_A, s + 2 * G::BUF_A + G::BUF_B);
}

template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFpDirect3 && PPL_GROUPED_DIRECT3 ? 1 : 2)))
gemm_grouped_kernel(char* base, const GroupDesc* __restrict__ groups, const int4* __restrict__ items,
                    const int* __restrict__ q_begin, int* counters) {
  constexpr int KC = GroupedLds<T>::KC;
  constexpr bool kDirect = kFpDirect3 && PPL_GROUPED_DIRECT3;
  __shared__ __attribute__((aligned(16))) char smem[kDirect ? 16 : GroupedLds<T>::bytes];
  __shared__ __attribute__((aligned(16))) T st0[kDirect ? GroupedLds<T>::stage : 2];
  __shared__ __attribute__((aligned(16))) T st1[kDirect ? GroupedLds<T>::stage : 2];
  __shared__ __attribute__((aligned(16))) T st2[kDirect ? GroupedLds<T>::stage : 2];
  __shared__ int s_item;
  global_char_t* const gbase = (global_char_t*)base;
  // queue q holds items [q_begin[q], q_begin[q + 1]); a workgroup drains the queue of
  // its own XCD first, then helps the others in turn, and leaves once all are empty
  const int x0 = (int)(blockIdx.x % kGroupedQueues);
  for (int qi = 0; qi < kGroupedQueues; ++qi) {
    const int q = (x0 + qi) % kGroupedQueues;
    const int b = q_begin[q], e = q_begin[q + 1];
    for (;;) {
      if (threadIdx.x == 0) s_item = b + atomicAdd(&counters[q], 1);
      __syncthreads();
      const int it = s_item;
      __syncthreads();
      if (it >= e) break;
      const int4 w = items[it];
      const GroupDesc g = groups[w.x];
      if constexpr (kDirect) {
        switch (g.cfg) {
          case 0: grouped_tile_direct<T, 7, 2, 1, 4, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
          case 1: grouped_tile_direct<T, 4, 4, 2, 2, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
          case 2: grouped_tile_direct<T, 13, 1, 1, 4, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
          case 5: grouped_tile_direct<T, 6, 2, 1, 4, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
          case 6: grouped_tile_direct<T, 2, 2, 1, 4, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
          case 7: grouped_tile_direct<T, 3, 2, 1, 4, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
          default: grouped_tile_direct<T, 4, 2, 1, 4, KC>(g, w.y, w.z, st0, st1, st2, gbase); break;
        }
        continue;
      }
      switch (g.cfg) {
        case 0: grouped_tile<T, 7, 2, 1, 4, KC>(g, w.y, w.z, smem, gbase); break;
        case 1: grouped_tile<T, 4, 4, 2, 2, KC>(g, w.y, w.z, smem, gbase); break;
        case 2: grouped_tile<T, 13, 1, 1, 4, KC>(g, w.y, w.z, smem, gbase); break;
        case 5: grouped_tile<T, 6, 2, 1, 4, KC>(g, w.y, w.z, smem, gbase); break;
        case 6: grouped_tile<T, 2, 2, 1, 4, KC>(g, w.y, w.z, smem, gbase); break;
        case 7: grouped_tile<T, 3, 2, 1, 4, KC>(g, w.y, w.z, smem, gbase); break;
        default: grouped_tile<T, 4, 2, 1, 4, KC>(g, w.y, w.z, smem, gbase); break;
      }
    }
  }
}

__global__ void reset_counters_kernel(int* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// tile sizes a grouped item of `tile` covers (must match grouped_tile above)
void grouped_tile_dims(int tile, int* bm, int* bn) {
  switch (tile) {
    case 0: *bm = 112; *bn = 128; break;
    case 1: *bm = 128; *bn = 128; break;
    case 2: *bm = 208; *bn = 64; break;
    case 5: *bm = 96; *bn = 128; break;
    case 6: *bm = 32; *bn = 128; break;
    case 7: *bm = 48; *bn = 128; break;
    default: *bm = 64; *bn = 128; break;
  }
}

int gemm_grouped(hipStream_t s, int prec, char* base, const GroupDesc* groups, const int4* items, int n_items,
                 const int* q_begin, int* counters, int grid) {
  if (n_items <= 0) return PPL_OK;
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, counters, kGroupedQueues);
  PPL_HIP_TRY(hipGetLastError());
  if (prec == PPL_FP64)
    hipLaunchKernelGGL(gemm_grouped_kernel<double>, dim3(grid), dim3(256), 0, s, base, groups, items, q_begin,
                       counters);
  else if (prec == PPL_FP32)
    hipLaunchKernelGGL(gemm_grouped_kernel<float>, dim3(grid), dim3(256), 0, s, base, groups, items, q_begin,
                       counters);
  else
    return fail(PPL_E_UNSUPPORTED, "grouped contraction supports FP64 and FP32");
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

}  // namespace ppl
