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
#include "ppl_internal.h"

namespace ppl {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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

// ------------------------------------------------------------------ tile maps
struct MapGrid {         // dense grid, logical order: row tile fastest (tiles sharing B rows adjacent)
  int64_t n_mt, n_nt;
  int bm, bn;
  __device__ bool operator()(int64_t bid, int64_t& m0, int64_t& n0) const {
    const int64_t t = xcd_remap(bid, n_mt * n_nt);
    m0 = (t % n_mt) * bm;
    n0 = (t / n_mt) * bn;
    return true;
  }
};

struct MapBuild {        // block-upper-triangle of the (a,c) x (b,d) grid: only tiles with some b >= a
  const int* prefix;     // prefix[mt] = valid tiles in row tiles < mt (n_mt + 1 entries)
  int n_mt;
  int64_t total;
  int v, bm, bn;
  __device__ bool operator()(int64_t bid, int64_t& m0, int64_t& n0) const {
    const int64_t t = xcd_remap(bid, total);
    int lo = 0, hi = n_mt - 1;              // largest mt with prefix[mt] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int mt = lo;
    const int64_t arel = (int64_t)mt * bm / v;          // first a of the row tile, relative to a0
    const int64_t nt_min = arel * v / bn;
    m0 = (int64_t)mt * bm;
    n0 = (nt_min + (t - prefix[mt])) * bn;
    return true;
  }
};

// ------------------------------------------------------------------ epilogues
template <class Tc>
struct EpiStore {        // C[m][c_col0 + n] = alpha * acc + beta * C (beta == 0: no read)
  Tc* C;
  int64_t ldc, c_col0, M, N;
  double alpha, beta;
  __device__ void row(int64_t m, int64_t& base, bool& ok) const {
    ok = m < M;
    base = m * ldc + c_col0;
  }
  __device__ void put(int64_t base, bool ok, int64_t n, typename AccOf<Tc>::type x) const {
    if (!ok || n >= N) return;
    Tc* p = C + base + n;
    if (beta == 0.0) *p = (Tc)(alpha * x);
    else *p = (Tc)(alpha * x + beta * (double)*p);
  }
};

template <class Tg>
struct EpiBuild {        // G[pair(a,b) - pair(a0,a0)][c][d] for b >= a
  Tg* G;
  int64_t M, N;
  int v, a0;
  // per-row: a, c; per-col: b, d
  __device__ void row(int64_t m, int64_t& base, bool& ok) const {
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

// ------------------------------------------------------------------ the kernel (FP64 / FP32)
template <class T, int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi, class Map>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
gemm_nt_kernel(int64_t M, int64_t N, int64_t Kpad, const T* __restrict__ A, int64_t lda,
               const T* __restrict__ B, int64_t ldb, Epi epi, Map map) {
  using accv = typename AccOf<T>::vec;
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int VEC = 16 / sizeof(T);             // elements per 16-byte load
  constexpr int PAD = 16 / sizeof(T);             // keeps 16-byte alignment and spreads banks
  constexpr int LDSR = KC + PAD;
  constexpr int VPR = KC / VEC;                   // 16-byte vectors per staged row
  constexpr int NLA = (BM * VPR + NT - 1) / NT;
  constexpr int NLB = (BN * VPR + NT - 1) / NT;
  static_assert(KC % 4 == 0 && KC % VEC == 0, "bad KC");
  __shared__ __attribute__((aligned(16))) T sA[2][BM * LDSR];
  __shared__ __attribute__((aligned(16))) T sB[2][BN * LDSR];

  int64_t m0, n0;
  if (!map(blockIdx.x, m0, n0)) return;
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
    pa[i] = A + gr * lda + kv * VEC;
    oa[i] = r * LDSR + kv * VEC;
  }
#pragma unroll
  for (int i = 0; i < NLB; ++i) {
    int idx = tid + i * NT;
    if (idx >= BN * VPR) idx = BN * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = n0 + r;
    if (gr > N - 1) gr = N - 1;
    pb[i] = B + gr * ldb + kv * VEC;
    ob[i] = r * LDSR + kv * VEC;
  }

  uint4 ra[NLA], rb[NLB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < NLA; ++i) ra[i] = *reinterpret_cast<const uint4*>(pa[i] + k0);
#pragma unroll
    for (int i = 0; i < NLB; ++i) rb[i] = *reinterpret_cast<const uint4*>(pb[i] + k0);
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NLA; ++i) *reinterpret_cast<uint4*>(&sA[buf][oa[i]]) = ra[i];
#pragma unroll
    for (int i = 0; i < NLB; ++i) *reinterpret_cast<uint4*>(&sB[buf][ob[i]]) = rb[i];
  };

  accv acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = accv{0, 0, 0, 0};

  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR + (lane >> 4);
  const int brow = (wn * WN * 16 + (lane & 15)) * LDSR + (lane >> 4);
  const int64_t nk = Kpad / KC;

  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) gload((kt + 1) * KC);
    const T* As = sA[buf];
    const T* Bs = sB[buf];
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = As[arow + i * 16 * LDSR + kk];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Bs[brow + j * 16 * LDSR + kk];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM * 16 + i * 16 + AccOf<T>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r]);
      }
    }
  }
}

// ------------------------------------------------------------------ the kernel (BF16 x 3)
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi); x*y ~ hi*hi + hi*lo + lo*hi,
// the two small cross products accumulated in their own FP32 register set and
// added to the hi*hi set once at the end.
template <int WM, int WN, int WAVES_M, int WAVES_N, int KC, class Epi, class Map>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N)
gemm_nt_bf16x3_kernel(int64_t M, int64_t N, int64_t Kpad, const __bf16* __restrict__ Ah,
                      const __bf16* __restrict__ Al, int64_t lda, const __bf16* __restrict__ Bh,
                      const __bf16* __restrict__ Bl, int64_t ldb, Epi epi, Map map) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int VEC = 8;                           // bf16 per 16-byte load
  constexpr int LDSR = KC + 8;
  constexpr int VPR = KC / VEC;
  constexpr int NLA = (BM * VPR + NT - 1) / NT;
  constexpr int NLB = (BN * VPR + NT - 1) / NT;
  static_assert(KC % 32 == 0, "bad KC");
  __shared__ __attribute__((aligned(16))) __bf16 sAh[2][BM * LDSR];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[2][BM * LDSR];
  __shared__ __attribute__((aligned(16))) __bf16 sBh[2][BN * LDSR];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[2][BN * LDSR];

  int64_t m0, n0;
  if (!map(blockIdx.x, m0, n0)) return;
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
    ga[i] = gr * lda + kv * VEC;
    oa[i] = r * LDSR + kv * VEC;
  }
#pragma unroll
  for (int i = 0; i < NLB; ++i) {
    int idx = tid + i * NT;
    if (idx >= BN * VPR) idx = BN * VPR - 1;
    const int r = idx / VPR, kv = idx % VPR;
    int64_t gr = n0 + r;
    if (gr > N - 1) gr = N - 1;
    gb[i] = gr * ldb + kv * VEC;
    ob[i] = r * LDSR + kv * VEC;
  }
  uint4 rah[NLA], ral[NLA], rbh[NLB], rbl[NLB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < NLA; ++i) {
      rah[i] = *reinterpret_cast<const uint4*>(Ah + ga[i] + k0);
      ral[i] = *reinterpret_cast<const uint4*>(Al + ga[i] + k0);
    }
#pragma unroll
    for (int i = 0; i < NLB; ++i) {
      rbh[i] = *reinterpret_cast<const uint4*>(Bh + gb[i] + k0);
      rbl[i] = *reinterpret_cast<const uint4*>(Bl + gb[i] + k0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NLA; ++i) {
      *reinterpret_cast<uint4*>(&sAh[buf][oa[i]]) = rah[i];
      *reinterpret_cast<uint4*>(&sAl[buf][oa[i]]) = ral[i];
    }
#pragma unroll
    for (int i = 0; i < NLB; ++i) {
      *reinterpret_cast<uint4*>(&sBh[buf][ob[i]]) = rbh[i];
      *reinterpret_cast<uint4*>(&sBl[buf][ob[i]]) = rbl[i];
    }
  };

  f4 acc[WM][WN], accx[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc[i][j] = f4{0, 0, 0, 0};
      accx[i][j] = f4{0, 0, 0, 0};
    }

  const int arow = (wm * WM * 16 + (lane & 15)) * LDSR + 8 * (lane >> 4);
  const int brow = (wn * WN * 16 + (lane & 15)) * LDSR + 8 * (lane >> 4);
  const int64_t nk = Kpad / KC;

  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) gload((kt + 1) * KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 32) {
      bf8 ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ah[i] = *reinterpret_cast<const bf8*>(&sAh[buf][arow + i * 16 * LDSR + kk]);
        al[i] = *reinterpret_cast<const bf8*>(&sAl[buf][arow + i * 16 * LDSR + kk]);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        bh[j] = *reinterpret_cast<const bf8*>(&sBh[buf][brow + j * 16 * LDSR + kk]);
        bl[j] = *reinterpret_cast<const bf8*>(&sBl[buf][brow + j * 16 * LDSR + kk]);
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
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * WM * 16 + i * 16 + AccOf<__bf16>::row(lane, r);
      int64_t base;
      bool ok;
      epi.row(m, base, ok);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = n0 + wn * WN * 16 + j * 16 + (lane & 15);
        epi.put(base, ok, n, acc[i][j][r] + accx[i][j][r]);
      }
    }
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
};
static const int kNumContract = sizeof(kContract) / sizeof(kContract[0]);
static const TileCfg kBuild = {4, 4, 2, 2};   // 128 x 128

int contract_tile_count() { return kNumContract; }

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

int build_tile_dims(int tile, int* bm, int* bn) {
  (void)tile;
  *bm = kBuild.bm();
  *bn = kBuild.bn();
  return PPL_OK;
}

void build_tile_table(int tile, int v, int a0, int a1, std::vector<int>& prefix, int& n_mt,
                      int& n_nt) {
  int bm, bn;
  build_tile_dims(tile, &bm, &bn);
  const int64_t M = (int64_t)(a1 - a0) * v, N = (int64_t)(v - a0) * v;
  n_mt = (int)((M + bm - 1) / bm);
  n_nt = (int)((N + bn - 1) / bn);
  prefix.assign(n_mt + 1, 0);
  for (int mt = 0; mt < n_mt; ++mt) {
    const int64_t arel = (int64_t)mt * bm / v;
    const int64_t nt_min = arel * v / bn;
    prefix[mt + 1] = prefix[mt] + (int)(n_nt - nt_min);
  }
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

// dispatch of one precision over the contraction tiles
template <int WM, int WN, int WAVES_M, int WAVES_N>
static int contract_cfg(hipStream_t s, int prec, int64_t Nrows, int64_t Prows, int64_t Kpad,
                        const void* S, const void* S_lo, int64_t lds_, const void* V,
                        const void* V_lo, int64_t ldv, void* C, int64_t ldc, int64_t c_col0) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  MapGrid map{(Nrows + BM - 1) / BM, (Prows + BN - 1) / BN, BM, BN};
  const int64_t grid = map.n_mt * map.n_nt;
  if (prec == PPL_FP64) {
    EpiStore<double> epi{(double*)C, ldc, c_col0, Nrows, Prows, 1.0, 0.0};
    return launch<double, WM, WN, WAVES_M, WAVES_N, 16>(s, grid, Nrows, Prows, Kpad, (const double*)S,
                                                        lds_, (const double*)V, ldv, epi, map);
  }
  if (prec == PPL_FP32) {
    EpiStore<float> epi{(float*)C, ldc, c_col0, Nrows, Prows, 1.0, 0.0};
    return launch<float, WM, WN, WAVES_M, WAVES_N, 32>(s, grid, Nrows, Prows, Kpad, (const float*)S,
                                                       lds_, (const float*)V, ldv, epi, map);
  }
  if (prec == PPL_BF16X3) {
    EpiStore<float> epi{(float*)C, ldc, c_col0, Nrows, Prows, 1.0, 0.0};
    return launch_bf3<WM, WN, WAVES_M, WAVES_N, 32>(s, grid, Nrows, Prows, Kpad, (const __bf16*)S,
                                                    (const __bf16*)S_lo, lds_, (const __bf16*)V,
                                                    (const __bf16*)V_lo, ldv, epi, map);
  }
  return fail(PPL_E_ARG, "unknown precision %d", prec);
}

int gemm_contract(hipStream_t s, int prec, int tile, int64_t Nrows, int64_t Prows, int64_t Kpad,
                  const void* S, const void* S_lo, int64_t lds_, const void* V, const void* V_lo,
                  int64_t ldv, void* C, int64_t ldc, int64_t c_col0) {
  if (Nrows <= 0 || Prows <= 0) return PPL_OK;
#define PPL_CFG(id, a, b, c, d)                                                               \
  case id:                                                                                    \
    return contract_cfg<a, b, c, d>(s, prec, Nrows, Prows, Kpad, S, S_lo, lds_, V, V_lo, ldv, C, \
                                    ldc, c_col0);
  switch (tile) {
    PPL_CFG(0, 7, 2, 1, 4)
    PPL_CFG(1, 4, 4, 2, 2)
    PPL_CFG(2, 13, 1, 1, 4)
    PPL_CFG(3, 2, 4, 1, 4)
    PPL_CFG(4, 3, 4, 1, 4)
    PPL_CFG(5, 6, 2, 1, 4)
    default:
      return fail(PPL_E_ARG, "unknown contraction tile %d", tile);
  }
#undef PPL_CFG
}

int gemm_build(hipStream_t s, int prec, int tile, int v, int a0, int a1, int64_t Kpad,
               const void* Xt, const void* Xt_lo, int64_t ldx, void* G, const int* tile_prefix,
               int n_mtiles, int n_ntiles, int64_t n_valid_tiles) {
  (void)tile;
  (void)n_ntiles;
  constexpr int WM = 4, WN = 4, WAVES_M = 2, WAVES_N = 2;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  const int64_t M = (int64_t)(a1 - a0) * v, N = (int64_t)(v - a0) * v;
  MapBuild map{tile_prefix, n_mtiles, n_valid_tiles, v, BM, BN};
  if (prec == PPL_FP64) {
    const double* X = (const double*)Xt + (int64_t)a0 * v * ldx;
    EpiBuild<double> epi{(double*)G, M, N, v, a0};
    return launch<double, WM, WN, WAVES_M, WAVES_N, 16>(s, n_valid_tiles, M, N, Kpad, X, ldx, X, ldx,
                                                        epi, map);
  }
  if (prec == PPL_FP32) {
    const float* X = (const float*)Xt + (int64_t)a0 * v * ldx;
    EpiBuild<float> epi{(float*)G, M, N, v, a0};
    return launch<float, WM, WN, WAVES_M, WAVES_N, 32>(s, n_valid_tiles, M, N, Kpad, X, ldx, X, ldx,
                                                       epi, map);
  }
  if (prec == PPL_BF16X3) {
    const __bf16* Xh = (const __bf16*)Xt + (int64_t)a0 * v * ldx;
    const __bf16* Xl = (const __bf16*)Xt_lo + (int64_t)a0 * v * ldx;
    EpiBuild<float> epi{(float*)G, M, N, v, a0};
    return launch_bf3<WM, WN, WAVES_M, WAVES_N, 32>(s, n_valid_tiles, M, N, Kpad, Xh, Xl, ldx, Xh,
                                                    Xl, ldx, epi, map);
  }
  return fail(PPL_E_ARG, "unknown precision %d", prec);
}

int gemm_store_f64(hipStream_t s, int64_t M, int64_t N, int64_t Kpad, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc) {
  constexpr int WM = 4, WN = 4, WAVES_M = 2, WAVES_N = 2;
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  MapGrid map{(M + BM - 1) / BM, (N + BN - 1) / BN, BM, BN};
  EpiStore<double> epi{C, ldc, 0, M, N, 1.0, 0.0};
  return launch<double, WM, WN, WAVES_M, WAVES_N, 16>(s, map.n_mt * map.n_nt, M, N, Kpad, A, lda, B,
                                                      ldb, epi, map);
}

}  // namespace ppl
