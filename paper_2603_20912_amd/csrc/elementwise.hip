// Memory-bound kernels around the MFMA GEMMs: staging of the Cholesky blocks,
// packing into the symmetric/antisymmetric pair layout, unpacking of results,
// the packed Jacobi update with its FP64 residual/energy reductions.
//
// Pair layout (i<=j / a<=b, "+"; i<j / a<b, "-"), for pair-symmetric t
// (t_ij^ab = t_ji^ba, eq. (2)):
//   s_ij^ab = (t_ij^ab + t_ij^ba)/2 is symmetric in (a,b) and in (i,j),
//   a_ij^ab = (t_ij^ab - t_ij^ba)/2 is antisymmetric in both,
// and the ladder term of eq. (vfunction-chol) splits into
//   R+ = V+ S',  S'[(ij)][(cd)] = (2 - delta_cd) s_ij^cd,
//   R- = V- A',  A'[(ij)][(cd)] = 2 a_ij^cd,
// with V+-[(ab)][(cd)] = ((ac|bd) +- (ad|bc))/2, and R = R+ + R- on the
// (i<=j, a<=b) half, the rest following from the two (anti)symmetries.
// The Fock denominator D_ij^ab = e_i + e_j - e_a - e_b is symmetric in (a,b) and
// (i,j), so the update t <- (V + R)/D acts on each part separately.
#include "ppl_internal.h"
#include "pack_cubes.h"

namespace ppl {

static inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

#define PPL_LAUNCH_CHECK() PPL_HIP_TRY(hipGetLastError())

// ------------------------------------------------------------------ fill / tables
__global__ void zero_kernel(uint4* p, int64_t n16) {
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += st)
    p[i] = uint4{0, 0, 0, 0};
}

int zero_bytes(hipStream_t s, void* p, uint64_t bytes) {
  if (bytes == 0) return PPL_OK;
  if (bytes % 16 != 0 || ((uintptr_t)p) % 16 != 0)
    return fail(PPL_E_ARG, "zero_bytes: unaligned range");
  const int64_t n16 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n16, 256, 8192)), dim3(256), 0, s, (uint4*)p, n16);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

__global__ void tables_kernel(int n, int* plus, int* minus) {
  const int64_t total = (int64_t)n * n;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const int a = (int)(x / n), b = (int)(x % n);
    if (a <= b) plus[pair_plus(a, b, n)] = (a << 16) | b;
    if (a < b) minus[pair_minus(a, b, n)] = (a << 16) | b;
  }
}

int fill_tables(hipStream_t s, int o, int v, int* tab_vp, int* tab_vm, int* tab_op, int* tab_om) {
  hipLaunchKernelGGL(tables_kernel, dim3(grid_for((int64_t)v * v, 256)), dim3(256), 0, s, v, tab_vp, tab_vm);
  PPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(tables_kernel, dim3(grid_for((int64_t)o * o, 256)), dim3(256), 0, s, o, tab_op, tab_om);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// ------------------------------------------------------------------ precision helpers
template <int PREC> struct Store;
template <> struct Store<PPL_FP64> {
  __device__ static void put(void* hi, void*, int64_t i, double x) { ((double*)hi)[i] = x; }
};
template <> struct Store<PPL_FP32> {
  __device__ static void put(void* hi, void*, int64_t i, double x) { ((float*)hi)[i] = (float)x; }
};
template <> struct Store<PPL_BF16X3> {
  // x -> FP32 (round to nearest), hi = bf16(x32), lo = bf16(x32 - hi); both round to nearest even
  __device__ static void put(void* hi, void* lo, int64_t i, double x) {
    const float xf = (float)x;
    const __bf16 h = (__bf16)xf;
    const __bf16 l = (__bf16)(xf - (float)h);
    ((__bf16*)hi)[i] = h;
    ((__bf16*)lo)[i] = l;
  }
};
template <> struct Store<PPL_BF16X6> {
  // x -> FP32 (round to nearest), hi = bf16(x32), mid = bf16(x32 - hi), lo = bf16(x32 - hi - mid),
  // each rounded to nearest even (both differences are exact in FP32). The three planes lie
  // equally far apart: hi at h, mid at m, lo at m + (m - h).
  __device__ static void put(void* hi, void* mid, int64_t i, double x) {
    const float xf = (float)x;
    const __bf16 h = (__bf16)xf;
    const float r1 = xf - (float)h;
    const __bf16 m = (__bf16)r1;
    const __bf16 l = (__bf16)(r1 - (float)m);
    __bf16* ph = (__bf16*)hi;
    __bf16* pm = (__bf16*)mid;
    ph[i] = h;
    pm[i] = m;
    (pm + (pm - ph))[i] = l;
  }
};

// ------------------------------------------------------------------ staging (transposing copy)
// X[r1*R2 + r2][P] = L[P][r1_off + r1][r2_off + r2] for P < naux, 0 for naux <= P < ldx.
template <int PREC>
__global__ void __launch_bounds__(256)
stage_kernel(const double* __restrict__ L, int n, int naux, int r1_off, int r2_off, int R2,
             int64_t rows, int64_t ldx, void* xh, void* xl) {
  __shared__ double sh[32][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int P0 = blockIdx.y * 32;
  const int tid = threadIdx.x;
  {  // load: 64 consecutive rows for each of 32 vectors P
    const int rr = tid & 63;
    const int64_t r = r0 + rr;
    int64_t src = -1;
    if (r < rows) {
      const int64_t r1 = r / R2, r2 = r - r1 * R2;
      src = (r1_off + r1) * (int64_t)n + r2_off + r2;
    }
    for (int pp = tid >> 6; pp < 32; pp += 4) {
      const int P = P0 + pp;
      double x = 0.0;
      if (src >= 0 && P < naux) x = L[(int64_t)P * n * n + src];
      sh[pp][rr] = x;
    }
  }
  __syncthreads();
  {  // store: 32 consecutive P for each row
    const int pp = tid & 31;
    for (int rr = tid >> 5; rr < 64; rr += 8) {
      const int64_t r = r0 + rr;
      const int P = P0 + pp;
      if (r < rows && P < ldx) Store<PREC>::put(xh, xl, r * ldx + P, sh[pp][rr]);
    }
  }
}

template <int PREC>
static int stage_launch(hipStream_t s, const double* L, int n, int naux, int r1_off, int r2_off,
                        int R1, int R2, int64_t ldx, void* xh, void* xl) {
  const int64_t rows = (int64_t)R1 * R2;
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((ldx + 31) / 32));
  hipLaunchKernelGGL(stage_kernel<PREC>, grid, dim3(256), 0, s, L, n, naux, r1_off, r2_off, R2, rows,
                     ldx, xh, xl);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

int stage_vv(hipStream_t s, int prec, const double* L, int o, int v, int naux, int64_t ldx, void* xt,
             void* xt_lo) {
  const int n = o + v;
  if (prec == PPL_FP64) return stage_launch<PPL_FP64>(s, L, n, naux, o, o, v, v, ldx, xt, xt_lo);
  if (prec == PPL_FP32) return stage_launch<PPL_FP32>(s, L, n, naux, o, o, v, v, ldx, xt, xt_lo);
  if (prec == PPL_BF16X3) return stage_launch<PPL_BF16X3>(s, L, n, naux, o, o, v, v, ldx, xt, xt_lo);
  if (prec == PPL_BF16X6) return stage_launch<PPL_BF16X6>(s, L, n, naux, o, o, v, v, ldx, xt, xt_lo);
  return fail(PPL_E_ARG, "stage_vv: unknown precision %d", prec);
}

int stage_ov(hipStream_t s, const double* L, int o, int v, int naux, int64_t ldx, double* xov) {
  return stage_launch<PPL_FP64>(s, L, o + v, naux, 0, o, o, v, ldx, xov, nullptr);
}

// ------------------------------------------------------------------ G -> V+ / V- rows
// One block per pair (a,b) of the batch; 32 x 32 tiles (cB <= dB) of G_ab and
// of its transpose are staged through LDS so that both reads and the packed
// row writes are contiguous.
template <class Tg, int PREC>
__global__ void __launch_bounds__(256)
pack_vpm_kernel(int v, int64_t pair0, const Tg* __restrict__ G, const int* __restrict__ tab_vp,
                void* vp, void* vp_lo, int64_t ldp, int64_t vp_row0, void* vm, void* vm_lo,
                int64_t ldm, int64_t vm_row0, int64_t Pp, int64_t Pm) {
  __shared__ double t1[32][33], t2[32][33];
  const int64_t pr = pair0 + blockIdx.x;           // global V+ row of this block
  const int ab = tab_vp[pr];
  const int a = pair_first(ab), b = pair_second(ab);
  const Tg* g = G + (int64_t)blockIdx.x * v * v;
  const int64_t rowp = pr - vp_row0;
  const bool has_minus = a < b;
  const int64_t rowm = has_minus ? pair_minus(a, b, v) - vm_row0 : 0;
  const int tid = threadIdx.x;
  const int nt = (v + 31) / 32;
  for (int cb = 0; cb < nt; ++cb) {
    for (int db = cb; db < nt; ++db) {
      // t1[c][d] = G[cB+c][dB+d], t2[c][d] = G[dB+d][cB+c]
      for (int e = tid; e < 1024; e += 256) {
        const int r = e >> 5, q = e & 31;
        const int c1 = cb * 32 + r, d1 = db * 32 + q;
        t1[r][q] = (c1 < v && d1 < v) ? (double)g[(int64_t)c1 * v + d1] : 0.0;
        const int c2 = db * 32 + r, d2 = cb * 32 + q;   // row d, col c
        t2[q][r] = (c2 < v && d2 < v) ? (double)g[(int64_t)c2 * v + d2] : 0.0;
      }
      __syncthreads();
      for (int e = tid; e < 1024; e += 256) {
        const int r = e >> 5, q = e & 31;
        const int c = cb * 32 + r, d = db * 32 + q;
        if (c < v && d < v && c <= d) {
          const double gcd = t1[r][q], gdc = t2[r][q];
          Store<PREC>::put(vp, vp_lo, rowp * ldp + pair_plus(c, d, v), 0.5 * (gcd + gdc));
          if (has_minus && c < d)
            Store<PREC>::put(vm, vm_lo, rowm * ldm + pair_minus(c, d, v), 0.5 * (gcd - gdc));
        }
      }
      __syncthreads();
    }
  }
  // zero padding columns
  for (int64_t k = Pp + tid; k < ldp; k += 256) Store<PREC>::put(vp, vp_lo, rowp * ldp + k, 0.0);
  if (has_minus)
    for (int64_t k = Pm + tid; k < ldm; k += 256) Store<PREC>::put(vm, vm_lo, rowm * ldm + k, 0.0);
}

int pack_vpm(hipStream_t s, int prec, int v, int a0, int a1, const void* G, void* vp, void* vp_lo,
             int64_t ldp, int64_t vp_row0, void* vm, void* vm_lo, int64_t ldm, int64_t vm_row0,
             const int* tab_vp, const int* tab_vm) {
  (void)tab_vm;
  const int64_t p0 = pair_plus(a0, a0, v);
  const int64_t p1 = (a1 >= v) ? npairs_plus(v) : pair_plus(a1, a1, v);
  const int64_t npairs = p1 - p0;
  if (npairs <= 0) return PPL_OK;
  const int64_t Pp = npairs_plus(v), Pm = npairs_minus(v);
  dim3 grid((unsigned)npairs);
  if (prec == PPL_FP64)
    hipLaunchKernelGGL((pack_vpm_kernel<double, PPL_FP64>), grid, dim3(256), 0, s, v, p0,
                       (const double*)G, tab_vp, vp, vp_lo, ldp, vp_row0, vm, vm_lo, ldm, vm_row0, Pp, Pm);
  else if (prec == PPL_FP32)
    hipLaunchKernelGGL((pack_vpm_kernel<float, PPL_FP32>), grid, dim3(256), 0, s, v, p0,
                       (const float*)G, tab_vp, vp, vp_lo, ldp, vp_row0, vm, vm_lo, ldm, vm_row0, Pp, Pm);
  else if (prec == PPL_BF16X3)
    hipLaunchKernelGGL((pack_vpm_kernel<float, PPL_BF16X3>), grid, dim3(256), 0, s, v, p0,
                       (const float*)G, tab_vp, vp, vp_lo, ldp, vp_row0, vm, vm_lo, ldm, vm_row0, Pp, Pm);
  else if (prec == PPL_BF16X6)
    hipLaunchKernelGGL((pack_vpm_kernel<float, PPL_BF16X6>), grid, dim3(256), 0, s, v, p0,
                       (const float*)G, tab_vp, vp, vp_lo, ldp, vp_row0, vm, vm_lo, ldm, vm_row0, Pp, Pm);
  else
    return fail(PPL_E_ARG, "pack_vpm: unknown precision %d", prec);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// Upper triangle of V+- rows from an upper-triangle build step: G holds
// G_ab[c - a0][d - a0] = (ac|bd) for c, d >= a (W x W per pair, pairs from pair0); the
// block of pair (a, b) writes V+[ab][cd] and V-[ab][cd] for the columns (cd) >= (ab) in
// packed order (c > a, or c == a and d >= b), which need only c, d >= a. The columns
// before (ab) are the mirror image of earlier rows (mirror_lower) and are left alone.
// Streaming form (half_diag): rows are stored from vp_row0 / vm_row0 on, the diagonal
// entry is halved (V = U + U^T) and the columns [zp, own) and [zm, own) before the row's
// own pair are zeroed, so that a K range starting at zp (zm) sees U exactly.
template <class Tg, int PREC>
__global__ void __launch_bounds__(256)
pack_vpm_sym_kernel(int v, int a0, int64_t pair0, const Tg* __restrict__ G, const int* __restrict__ tab_vp,
                    void* vp, void* vp_lo, int64_t ldp, void* vm, void* vm_lo, int64_t ldm, int64_t Pp,
                    int64_t Pm, int64_t vp_row0, int64_t vm_row0, int half_diag, int64_t zp, int64_t zm) {
  __shared__ double t1[32][33], t2[32][33];
  const int W = v - a0;
  const int64_t pr = pair0 + blockIdx.x;
  const int ab = tab_vp[pr];
  const int a = pair_first(ab), b = pair_second(ab);
  const Tg* g = G + (int64_t)blockIdx.x * W * W;
  const bool has_minus = a < b;
  const int64_t qr = has_minus ? pair_minus(a, b, v) : 0;
  const int64_t rowp = pr - vp_row0, rowm = qr - vm_row0;
  const double dscale = half_diag ? 0.25 : 0.5;
  const int tid = threadIdx.x;
  const int nt = (v - a + 31) / 32;            // 32-wide tiles of c and d, starting at a
  // the tile pairs (ci, di >= ci) in turn; the G values of the next pair are fetched into
  // registers before the current pair is written, so that their latency overlaps it
  double n1[4], n2[4];
  auto fetch = [&](int ci, int di) __attribute__((always_inline)) {
    const int cB = a + ci * 32, dB = a + di * 32;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + 256 * k, r = e >> 5, q = e & 31;
      const int c1 = cB + r, d1 = dB + q;
      n1[k] = (c1 < v && d1 < v) ? (double)g[(int64_t)(c1 - a0) * W + (d1 - a0)] : 0.0;
      const int c2 = dB + r, d2 = cB + q;     // row d, col c
      n2[k] = (c2 < v && d2 < v) ? (double)g[(int64_t)(c2 - a0) * W + (d2 - a0)] : 0.0;
    }
  };
  int ci = 0, di = 0;
  fetch(ci, di);
  while (ci < nt) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + 256 * k, r = e >> 5, q = e & 31;
      t1[r][q] = n1[k];
      t2[q][r] = n2[k];
    }
    __syncthreads();
    const int cB = a + ci * 32, dB = a + di * 32;
    if (++di == nt) di = ++ci;                 // the next pair
    if (ci < nt) fetch(ci, di);
    for (int e = tid; e < 1024; e += 256) {
      const int r = e >> 5, q = e & 31;
      const int c = cB + r, d = dB + q;
      if (c < v && d < v && c <= d && (c > a || d >= b)) {
        const double gcd = t1[r][q], gdc = t2[r][q];
        const bool diag = c == a && d == b;
        Store<PREC>::put(vp, vp_lo, rowp * ldp + pair_plus(c, d, v), (diag ? dscale : 0.5) * (gcd + gdc));
        if (has_minus && c < d)
          Store<PREC>::put(vm, vm_lo, rowm * ldm + pair_minus(c, d, v), (diag ? dscale : 0.5) * (gcd - gdc));
      }
    }
    __syncthreads();
  }
  for (int64_t k = Pp + tid; k < ldp; k += 256) Store<PREC>::put(vp, vp_lo, rowp * ldp + k, 0.0);
  if (has_minus)
    for (int64_t k = Pm + tid; k < ldm; k += 256) Store<PREC>::put(vm, vm_lo, rowm * ldm + k, 0.0);
  if (half_diag) {
    for (int64_t k = zp + tid; k < pr; k += 256) Store<PREC>::put(vp, vp_lo, rowp * ldp + k, 0.0);
    if (has_minus)
      for (int64_t k = zm + tid; k < qr; k += 256) Store<PREC>::put(vm, vm_lo, rowm * ldm + k, 0.0);
  }
}

int pack_vpm_sym(hipStream_t s, int prec, int v, int a0, int a1, const void* G, void* vp, void* vp_lo,
                 int64_t ldp, void* vm, void* vm_lo, int64_t ldm, const int* tab_vp, int64_t vp_row0,
                 int64_t vm_row0, int half_diag, int64_t zp, int64_t zm) {
  const int64_t p0 = pair_plus(a0, a0, v);
  const int64_t p1 = (a1 >= v) ? npairs_plus(v) : pair_plus(a1, a1, v);
  const int64_t npairs = p1 - p0;
  if (npairs <= 0) return PPL_OK;
  const int64_t Pp = npairs_plus(v), Pm = npairs_minus(v);
  dim3 grid((unsigned)npairs);
  if (prec == PPL_FP64)
    hipLaunchKernelGGL((pack_vpm_sym_kernel<double, PPL_FP64>), grid, dim3(256), 0, s, v, a0, p0, (const double*)G,
                       tab_vp, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm, vp_row0, vm_row0, half_diag, zp, zm);
  else if (prec == PPL_FP32)
    hipLaunchKernelGGL((pack_vpm_sym_kernel<float, PPL_FP32>), grid, dim3(256), 0, s, v, a0, p0, (const float*)G,
                       tab_vp, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm, vp_row0, vm_row0, half_diag, zp, zm);
  else if (prec == PPL_BF16X3)
    hipLaunchKernelGGL((pack_vpm_sym_kernel<float, PPL_BF16X3>), grid, dim3(256), 0, s, v, a0, p0,
                       (const float*)G, tab_vp, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm, vp_row0, vm_row0, half_diag,
                       zp, zm);
  else if (prec == PPL_BF16X6)
    hipLaunchKernelGGL((pack_vpm_sym_kernel<float, PPL_BF16X6>), grid, dim3(256), 0, s, v, a0, p0,
                       (const float*)G, tab_vp, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm, vp_row0, vm_row0, half_diag,
                       zp, zm);
  else
    return fail(PPL_E_ARG, "pack_vpm_sym: unknown precision %d", prec);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// threads of one cube-packing workgroup (divides the 4096 elements of a cube)
#ifndef PPL_PACK_THREADS
#define PPL_PACK_THREADS 256
#endif
constexpr int kPackThreads = PPL_PACK_THREADS;
static_assert(kCube * kCube * kCube % PPL_PACK_THREADS == 0, "threads must divide a cube");
static_assert(kCube == 16, "the cube packing splits an element index into 4-bit fields");

// Whole V+- rows of a resident build step from the natural build output T, with no separate
// mirror pass: T[(pair(a, r) - pr0) * ldt + pair(x, y) - pr0] = (ar|xy) for the step's virtuals
// a in [a0, a1), r >= a and a <= x <= y (pr0 = pair(a0, a0)); T is symmetric in (x, y) since the
// Cholesky vectors are. For the entry of row (ab), column (cd) with (cd) >= (ab) in packed order
//   V+[ab][cd] = ((ac|bd) + (ad|bc)) / 2,   V-[ab][cd] = ((ac|bd) - (ad|bc)) / 2  (a < b, c < d),
// and the same value goes to the mirror entry [cd][ab], so every entry of V+- is written once
// (pack_cubes.h). One workgroup per cube of 16 x 16 x 16 indices (b, c, d): it stages
// (ac|bd) as s1[c][b][d] and (ad|bc) as s2[d][b][c] (each read from T along its contiguous
// index), then writes the rows (ab) along d and the mirror rows (cd) along b. The cube with
// ci == di == 0 also zeroes the padding columns of the rows (ab).
template <class Tg, int PREC>
__global__ void __launch_bounds__(kPackThreads)
pack_vpm_cubes_kernel(int v, int a0, int a1, const Tg* __restrict__ T, int64_t ldt, const int64_t* __restrict__ off,
                      int64_t g0, int64_t ncubes, void* vp, void* vp_lo, int64_t ldp, void* vm, void* vm_lo,
                      int64_t ldm, int64_t Pp, int64_t Pm) {
  constexpr int C = kCube, CP = kCube + 1;
  __shared__ Tg s1[C][CP][CP], s2[C][CP][CP];
  const int64_t g = g0 + cube_of_slot(blockIdx.x, ncubes);
  const int a = cube_virtual(off, a0, a1, g);
  const int nt = cube_blocks(v, a);
  int bi, ci, di;
  cube_decode(g - off[a], nt, bi, ci, di);
  const int b0 = a + C * bi, c0 = a + C * ci, d0 = a + C * di;
  const int64_t pr0 = pair_plus(a0, a0, v);
  const int tid = threadIdx.x;
  // s[rl][bl][yl] = (a r | b y) for r = r0 + rl, b = b0 + bl, y = y0 + yl (zero outside v);
  // element e = tid + kPackThreads k of the cube, read along its contiguous index. All reads of a
  // thread are issued before its first LDS store, so their latencies overlap.
  constexpr int K = C * C * C / kPackThreads;
  auto slot = [&](int k, bool bfast, int& rl, int& bl, int& yl) __attribute__((always_inline)) {
    const int e = tid + kPackThreads * k, m = (e >> 4) & 15, f = e & 15;
    rl = e >> 8;
    bl = bfast ? f : m;
    yl = bfast ? m : f;
  };
  auto fetch = [&](Tg (&x)[K], int r0, int y0) __attribute__((always_inline)) {
    const bool bfast = b0 > y0;              // pairs (y, b): contiguous along b
#pragma unroll
    for (int k = 0; k < K; ++k) {
      int rl, bl, yl;
      slot(k, bfast, rl, bl, yl);
      const int r = r0 + rl, b = b0 + bl, y = y0 + yl;
      const int lo = b < y ? b : y, hi = b < y ? y : b;
      x[k] = (r < v && b < v && y < v) ? T[(pair_plus(a, r, v) - pr0) * ldt + (pair_plus(lo, hi, v) - pr0)] : Tg(0);
    }
  };
  auto keep = [&](Tg (*s)[CP][CP], const Tg (&x)[K], int y0) __attribute__((always_inline)) {
    const bool bfast = b0 > y0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      int rl, bl, yl;
      slot(k, bfast, rl, bl, yl);
      s[rl][bl][yl] = x[k];
    }
  };
  Tg x1[K], x2[K];
  fetch(x1, c0, d0);
  if (ci != di) fetch(x2, d0, c0);
  keep(s1, x1, d0);
  if (ci != di) keep(s2, x2, c0);
  __syncthreads();
  const Tg (*t2)[CP][CP] = ci != di ? s2 : s1;   // (ad|bc) = t2[d][b][c]
  // rows (ab), along d
  for (int e = tid; e < C * C * C; e += kPackThreads) {
    const int bl = e >> 8, cl = (e >> 4) & 15, dl = e & 15;
    const int b = b0 + bl, c = c0 + cl, d = d0 + dl;
    if (b >= v || d >= v || c > d || (c == a && d < b)) continue;
    const double gcd = (double)s1[cl][bl][dl], gdc = (double)t2[dl][bl][cl];
    Store<PREC>::put(vp, vp_lo, pair_plus(a, b, v) * ldp + pair_plus(c, d, v), 0.5 * (gcd + gdc));
    if (a < b && c < d) Store<PREC>::put(vm, vm_lo, pair_minus(a, b, v) * ldm + pair_minus(c, d, v), 0.5 * (gcd - gdc));
  }
  // mirror rows (cd), along b
  for (int e = tid; e < C * C * C; e += kPackThreads) {
    const int cl = e >> 8, dl = (e >> 4) & 15, bl = e & 15;
    const int b = b0 + bl, c = c0 + cl, d = d0 + dl;
    if (b >= v || d >= v || c > d || (c == a && d <= b)) continue;
    const double gcd = (double)s1[cl][bl][dl], gdc = (double)t2[dl][bl][cl];
    Store<PREC>::put(vp, vp_lo, pair_plus(c, d, v) * ldp + pair_plus(a, b, v), 0.5 * (gcd + gdc));
    if (a < b && c < d) Store<PREC>::put(vm, vm_lo, pair_minus(c, d, v) * ldm + pair_minus(a, b, v), 0.5 * (gcd - gdc));
  }
  if (ci == 0 && di == 0) {
    const int64_t padp = ldp - Pp, padm = ldm - Pm;
    for (int e = tid; e < C * padp; e += kPackThreads) {
      const int b = b0 + (int)(e / padp);
      if (b < v) Store<PREC>::put(vp, vp_lo, pair_plus(a, b, v) * ldp + Pp + e % padp, 0.0);
    }
    for (int e = tid; e < C * padm; e += kPackThreads) {
      const int b = b0 + (int)(e / padm);
      if (b < v && a < b) Store<PREC>::put(vm, vm_lo, pair_minus(a, b, v) * ldm + Pm + e % padm, 0.0);
    }
  }
}

int pack_vpm_cubes(hipStream_t s, int prec, int v, int a0, int a1, const void* T, int64_t ldt, const int64_t* off,
                   void* vp, void* vp_lo, int64_t ldp, void* vm, void* vm_lo, int64_t ldm) {
  int64_t g0 = 0, n = 0;
  for (int a = 0; a < a1; ++a) (a < a0 ? g0 : n) += cubes_of(v, a);
  if (n <= 0) return PPL_OK;
  if (n > 0x7fffffffLL) return fail(PPL_E_ARG, "pack_vpm_cubes: %lld cubes", (long long)n);
  const int64_t Pp = npairs_plus(v), Pm = npairs_minus(v);
  const dim3 grid((unsigned)n);
  if (prec == PPL_FP64)
    hipLaunchKernelGGL((pack_vpm_cubes_kernel<double, PPL_FP64>), grid, dim3(kPackThreads), 0, s, v, a0, a1, (const double*)T,
                       ldt, off, g0, n, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm);
  else if (prec == PPL_FP32)
    hipLaunchKernelGGL((pack_vpm_cubes_kernel<float, PPL_FP32>), grid, dim3(kPackThreads), 0, s, v, a0, a1, (const float*)T,
                       ldt, off, g0, n, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm);
  else if (prec == PPL_BF16X3)
    hipLaunchKernelGGL((pack_vpm_cubes_kernel<float, PPL_BF16X3>), grid, dim3(kPackThreads), 0, s, v, a0, a1,
                       (const float*)T, ldt, off, g0, n, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm);
  else if (prec == PPL_BF16X6)
    hipLaunchKernelGGL((pack_vpm_cubes_kernel<float, PPL_BF16X6>), grid, dim3(kPackThreads), 0, s, v, a0, a1,
                       (const float*)T, ldt, off, g0, n, vp, vp_lo, ldp, vm, vm_lo, ldm, Pp, Pm);
  else
    return fail(PPL_E_ARG, "pack_vpm_cubes: unknown precision %d", prec);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// Ut[r][k] = U[k0 + k - u0][c0 + r] for rows u0 <= k0 + k < u1 of the block U (row length
// ldu, its first row is global row u0), zero for the other k; r < nr, k < nk (row length
// ldt). A bit copy of elements of type E through 64 x 64 LDS tiles.
template <class E>
__global__ void __launch_bounds__(256)
transpose_block_kernel(const E* __restrict__ U, int64_t ldu, int64_t u0, int64_t u1, int64_t c0, int64_t k0,
                       E* __restrict__ Ut, int64_t ldt, int64_t nr, int64_t nk, int64_t tiles_k) {
  __shared__ E sh[64][65];
  const int64_t tr = blockIdx.x / tiles_k, tk = blockIdx.x % tiles_k;
  const int64_t r0 = tr * 64, kb = tk * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int kl = e >> 6, rl = e & 63;                   // read U row k0 + kb + kl, column c0 + r0 + rl
    const int64_t gk = k0 + kb + kl, r = r0 + rl;
    E x = E(0);
    if (gk >= u0 && gk < u1 && r < nr) x = U[(gk - u0) * ldu + c0 + r];
    sh[kl][rl] = x;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rl = e >> 6, kl = e & 63;                   // write Ut row r0 + rl, column kb + kl
    const int64_t r = r0 + rl, k = kb + kl;
    if (r < nr && k < nk) Ut[r * ldt + k] = sh[kl][rl];
  }
}

int transpose_block(hipStream_t s, int elem_bytes, const void* U, int64_t ldu, int64_t u0, int64_t u1, int64_t c0,
                    int64_t k0, void* Ut, int64_t ldt, int64_t nr, int64_t nk) {
  if (nr <= 0 || nk <= 0) return PPL_OK;
  const int64_t tr = (nr + 63) / 64, tk = (nk + 63) / 64;
  if (tr * tk > 0x7fffffffLL) return fail(PPL_E_ARG, "transpose of %lld x %lld too large", (long long)nr, (long long)nk);
  const dim3 grid((unsigned)(tr * tk));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(transpose_block_kernel<uint64_t>, grid, dim3(256), 0, s, (const uint64_t*)U, ldu, u0, u1, c0,
                       k0, (uint64_t*)Ut, ldt, nr, nk, tk);
  else if (elem_bytes == 4)
    hipLaunchKernelGGL(transpose_block_kernel<uint32_t>, grid, dim3(256), 0, s, (const uint32_t*)U, ldu, u0, u1, c0,
                       k0, (uint32_t*)Ut, ldt, nr, nk, tk);
  else if (elem_bytes == 2)
    hipLaunchKernelGGL(transpose_block_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)U, ldu, u0, u1, c0,
                       k0, (uint16_t*)Ut, ldt, nr, nk, tk);
  else
    return fail(PPL_E_ARG, "transpose of %d-byte elements", elem_bytes);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// Y[p][q] = w X[q][p] for q < nq, p < np, and Y[p][q] = 0 for nq <= q < ldy (rows of X
// hold ldx, rows of Y ldy doubles). scaled: w = (2 - d_kl) / (2 - d_ab) with (k, l) =
// tab_q[q] and (a, b) = tab_p[p] (S' rows to the transposed symmetric operand of the
// hole-hole ladder); otherwise w = 1.
__global__ void __launch_bounds__(256)
transpose_pm_kernel(const double* __restrict__ X, int64_t ldx, double* __restrict__ Y, int64_t ldy, int64_t nq,
                    int64_t np, const int* __restrict__ tab_q, const int* __restrict__ tab_p, int scaled,
                    int64_t qwrite, int64_t tiles_q) {
  __shared__ double sh[64][65];
  const int64_t tp = blockIdx.x / tiles_q, tq = blockIdx.x % tiles_q;
  const int64_t p0 = tp * 64, q0 = tq * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int ql = e >> 6, pl = e & 63;                   // read X row q0 + ql, column p0 + pl
    const int64_t q = q0 + ql, p = p0 + pl;
    double x = 0.0;
    if (q < nq && p < np) {
      x = X[q * ldx + p];
      if (scaled) {
        const int kl = tab_q[q], ab = tab_p[p];
        const double wq = pair_first(kl) == pair_second(kl) ? 1.0 : 2.0;
        const double wp = pair_first(ab) == pair_second(ab) ? 1.0 : 2.0;
        x *= wq / wp;
      }
    }
    sh[ql][pl] = x;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int pl = e >> 6, ql = e & 63;                   // write Y row p0 + pl, column q0 + ql
    const int64_t p = p0 + pl, q = q0 + ql;
    if (p < np && q < qwrite) Y[p * ldy + q] = sh[ql][pl];
  }
}

int transpose_pm(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t nq, int64_t np,
                 const int* tab_q, const int* tab_p, int scaled, int pad) {
  if (np <= 0 || ldy <= 0) return PPL_OK;
  const int64_t qwrite = pad ? ldy : nq;          // columns written per row of Y
  const int64_t tq = (qwrite + 63) / 64, tp = (np + 63) / 64;
  if (tq * tp > 0x7fffffffLL) return fail(PPL_E_ARG, "transpose of %lld x %lld too large", (long long)np,
                                          (long long)ldy);
  hipLaunchKernelGGL(transpose_pm_kernel, dim3((unsigned)(tq * tp)), dim3(256), 0, s, X, ldx, Y, ldy, nq, np, tab_q,
                     tab_p, scaled, qwrite, tq);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// C[q][p] += T[p][q] for q < nq, p < np (C rows of ldc, T rows of ldt), 64 x 64 LDS tiles.
template <class Tc>
__global__ void __launch_bounds__(256)
add_transposed_kernel(Tc* __restrict__ C, int64_t ldc, const double* __restrict__ T, int64_t ldt, int64_t nq,
                      int64_t np, int64_t tiles_p) {
  __shared__ double sh[64][65];
  const int64_t tq = blockIdx.x / tiles_p, tp = blockIdx.x % tiles_p;
  const int64_t q0 = tq * 64, p0 = tp * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int pl = e >> 6, ql = e & 63;                   // read T row p0 + pl, column q0 + ql
    const int64_t pp = p0 + pl, q = q0 + ql;
    sh[pl][ql] = (pp < np && q < nq) ? T[pp * ldt + q] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int ql = e >> 6, pl = e & 63;                   // update C row q0 + ql, column p0 + pl
    const int64_t q = q0 + ql, pp = p0 + pl;
    if (q < nq && pp < np) C[q * ldc + pp] = (Tc)((double)C[q * ldc + pp] + sh[pl][ql]);
  }
}

int add_transposed(hipStream_t s, int c_prec, void* C, int64_t ldc, const double* T, int64_t ldt, int64_t nq,
                   int64_t np) {
  if (nq <= 0 || np <= 0) return PPL_OK;
  const int64_t tq = (nq + 63) / 64, tp = (np + 63) / 64;
  if (tq * tp > 0x7fffffffLL) return fail(PPL_E_ARG, "transposed add of %lld x %lld too large", (long long)nq,
                                          (long long)np);
  if (c_prec == PPL_FP64)
    hipLaunchKernelGGL(add_transposed_kernel<double>, dim3((unsigned)(tq * tp)), dim3(256), 0, s, (double*)C, ldc, T,
                       ldt, nq, np, tp);
  else
    hipLaunchKernelGGL(add_transposed_kernel<float>, dim3((unsigned)(tq * tp)), dim3(256), 0, s, (float*)C, ldc, T,
                       ldt, nq, np, tp);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// Strictly lower triangle of an n x n symmetric matrix (row length ld) from its upper
// triangle: V[r][q] = V[q][r] for q < r, as a bit copy of elements of type E. One 64 x 64
// block pair per workgroup: block (I, J), I >= J, reads rows J and columns I (upper) through
// LDS and writes rows I and columns J (lower), both along contiguous rows.
template <class E>
__global__ void __launch_bounds__(256) mirror_lower_kernel(E* V, int64_t n, int64_t ld, int vec_ok) {
  __shared__ E sh[64][65];
  const int64_t t = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int64_t J = t - I * (I + 1) / 2;
  const int tid = threadIdx.x;
  const int64_t r0 = I * 64, q0 = J * 64;
  if (vec_ok && I > J && r0 + 64 <= n) {
    // a whole block below the diagonal: 16-byte vectors along both rows (rows 16-byte
    // aligned, checked on the host), the transposition in LDS element by element
    constexpr int VE = 16 / (int)sizeof(E), VR = 64 / VE;
    union Vec { uint4 u; E e[VE]; };
    for (int x = tid; x < 64 * VR; x += 256) {
      const int ql = x / VR, vv = x % VR;
      Vec y;
      y.u = *reinterpret_cast<const uint4*>(&V[(q0 + ql) * ld + r0 + vv * VE]);
#pragma unroll
      for (int k = 0; k < VE; ++k) sh[ql][vv * VE + k] = y.e[k];
    }
    __syncthreads();
    for (int x = tid; x < 64 * VR; x += 256) {
      const int rl = x / VR, vv = x % VR;
      Vec y;
#pragma unroll
      for (int k = 0; k < VE; ++k) y.e[k] = sh[vv * VE + k][rl];
      *reinterpret_cast<uint4*>(&V[(r0 + rl) * ld + q0 + vv * VE]) = y.u;
    }
    return;
  }
  for (int e = tid; e < 64 * 64; e += 256) {
    const int ql = e >> 6, rl = e & 63;                  // read row q0 + ql, column r0 + rl
    const int64_t q = q0 + ql, r = r0 + rl;
    if (q < n && r < n && q < r) sh[ql][rl] = V[q * ld + r];
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rl = e >> 6, ql = e & 63;                  // write row r0 + rl, column q0 + ql
    const int64_t r = r0 + rl, q = q0 + ql;
    if (q < n && r < n && q < r) V[r * ld + q] = sh[ql][rl];
  }
}

int mirror_lower(hipStream_t s, int elem_bytes, void* V, int64_t n, int64_t ld) {
  if (n <= 1) return PPL_OK;
  const int64_t T = (n + 63) / 64, blocks = T * (T + 1) / 2;
  if (blocks > 0x7fffffffLL) return fail(PPL_E_ARG, "mirror of %lld rows too large", (long long)n);
  // 16-byte vectors need every row and every 64-element block start 16-byte aligned
  const int vec_ok = ((uintptr_t)V % 16 == 0) && ((uint64_t)ld * elem_bytes % 16 == 0);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(mirror_lower_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint64_t*)V, n, ld,
                       vec_ok);
  else if (elem_bytes == 4)
    hipLaunchKernelGGL(mirror_lower_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)V, n, ld,
                       vec_ok);
  else if (elem_bytes == 2)
    hipLaunchKernelGGL(mirror_lower_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint16_t*)V, n, ld,
                       vec_ok);
  else
    return fail(PPL_E_ARG, "mirror of %d-byte elements", elem_bytes);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// ------------------------------------------------------------------ generic (i,j,a,b) -> +/- packing
// With t1 ([i][a], row length v1) the packed tensor is X_ij^ab + t1_i^a t1_j^b.
__global__ void pack_plus_kernel(const double* __restrict__ X, int64_t si, int64_t sj, int64_t sa,
                                 int64_t sb, double s_off, double s_diag, double* plus, int64_t Np,
                                 int64_t Pp, int64_t ldp, const int* __restrict__ tab_op,
                                 const int* __restrict__ tab_vp, const double* __restrict__ t1, int64_t v1) {
  const int64_t total = Np * ldp;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const int64_t q = x / ldp, p = x - q * ldp;
    double val = 0.0;
    if (p < Pp) {
      const int ij = tab_op[q], ab = tab_vp[p];
      const int i = pair_first(ij), j = pair_second(ij), a = pair_first(ab), b = pair_second(ab);
      const int64_t base = i * si + j * sj;
      double xab = X[base + a * sa + b * sb], xba = X[base + b * sa + a * sb];
      if (t1) {
        xab += t1[i * v1 + a] * t1[j * v1 + b];
        xba += t1[i * v1 + b] * t1[j * v1 + a];
      }
      val = (a == b ? s_diag : s_off) * (xab + xba);
    }
    plus[x] = val;
  }
}

__global__ void pack_minus_kernel(const double* __restrict__ X, int64_t si, int64_t sj, int64_t sa,
                                  int64_t sb, double am, double* minus, int64_t Nm, int64_t Pm,
                                  int64_t ldm, const int* __restrict__ tab_om,
                                  const int* __restrict__ tab_vm, const double* __restrict__ t1, int64_t v1) {
  const int64_t total = Nm * ldm;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const int64_t q = x / ldm, p = x - q * ldm;
    double val = 0.0;
    if (p < Pm) {
      const int ij = tab_om[q], ab = tab_vm[p];
      const int i = pair_first(ij), j = pair_second(ij), a = pair_first(ab), b = pair_second(ab);
      const int64_t base = i * si + j * sj;
      double xab = X[base + a * sa + b * sb], xba = X[base + b * sa + a * sb];
      if (t1) {
        xab += t1[i * v1 + a] * t1[j * v1 + b];
        xba += t1[i * v1 + b] * t1[j * v1 + a];
      }
      val = am * (xab - xba);
    }
    minus[x] = val;
  }
}

int pack_pm(hipStream_t s, int o, int v, const double* X, int64_t si, int64_t sj, int64_t sa,
            int64_t sb, double sp_off, double sp_diag, double am, double* plus, int64_t ldp,
            double* minus, int64_t ldm, const int* tab_op, const int* tab_om, const int* tab_vp,
            const int* tab_vm, const double* t1) {
  const int64_t Np = npairs_plus(o), Nm = npairs_minus(o), Pp = npairs_plus(v), Pm = npairs_minus(v);
  hipLaunchKernelGGL(pack_plus_kernel, dim3(grid_for(Np * ldp, 256)), dim3(256), 0, s, X, si, sj, sa,
                     sb, sp_off, sp_diag, plus, Np, Pp, ldp, tab_op, tab_vp, t1, (int64_t)v);
  PPL_LAUNCH_CHECK();
  if (Nm > 0 && Pm > 0) {
    hipLaunchKernelGGL(pack_minus_kernel, dim3(grid_for(Nm * ldm, 256)), dim3(256), 0, s, X, si, sj,
                       sa, sb, am, minus, Nm, Pm, ldm, tab_om, tab_vm, t1, (int64_t)v);
    PPL_LAUNCH_CHECK();
  }
  return PPL_OK;
}

int stage_oo(hipStream_t s, const double* L, int o, int v, int naux, int64_t ldx, double* xoo) {
  return stage_launch<PPL_FP64>(s, L, o + v, naux, 0, 0, o, o, ldx, xoo, nullptr);
}

// ------------------------------------------------------------------ FP64 rows -> operand precision
template <int PREC>
__global__ void convert_kernel(const double* __restrict__ src, int64_t n, void* dh, void* dl) {
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += st)
    Store<PREC>::put(dh, dl, x, src[x]);
}

int convert_rows(hipStream_t s, int prec, const double* src, int64_t rows, int64_t cols, int64_t ld,
                 void* dst, void* dst_lo) {
  (void)cols;
  const int64_t n = rows * ld;
  if (n <= 0) return PPL_OK;
  if (prec == PPL_FP32)
    hipLaunchKernelGGL(convert_kernel<PPL_FP32>, dim3(grid_for(n, 256)), dim3(256), 0, s, src, n, dst, dst_lo);
  else if (prec == PPL_BF16X3)
    hipLaunchKernelGGL(convert_kernel<PPL_BF16X3>, dim3(grid_for(n, 256)), dim3(256), 0, s, src, n, dst, dst_lo);
  else if (prec == PPL_BF16X6)
    hipLaunchKernelGGL(convert_kernel<PPL_BF16X6>, dim3(grid_for(n, 256)), dim3(256), 0, s, src, n, dst, dst_lo);
  else if (prec == PPL_FP64)
    hipLaunchKernelGGL(convert_kernel<PPL_FP64>, dim3(grid_for(n, 256)), dim3(256), 0, s, src, n, dst, dst_lo);
  else
    return fail(PPL_E_ARG, "convert_rows: unknown precision %d", prec);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// ------------------------------------------------------------------ unpack R and t
// Both unpackings over tiles: a work item is one occupied pair (i0 <= j0) and one 32 x 32
// block pair (A <= B) of virtual indices. The packed values of (a, b), a <= b, are read
// along their rows once and give the four entries (i0 j0 a b), (i0 j0 b a), (j0 i0 a b) and
// (j0 i0 b a); the (b a) entries are written from an LDS transpose, so that reads and
// writes both run along contiguous rows. MODE 0 unpacks R (R = alpha r + beta R), MODE 1
// the amplitudes (s = S' / (2 - delta_ab), a = A' / 2).
template <class Tr, int MODE>
__global__ void __launch_bounds__(256)
unpack_tiled_kernel(int o, int v, const Tr* __restrict__ xp, int64_t ldp, const Tr* __restrict__ xm, int64_t ldm,
                    double* out, double alpha, double beta) {
  __shared__ double sp_[32][33], sm_[32][33];
  const int nb = (v + 31) / 32;
  const int64_t per = (int64_t)nb * (nb + 1) / 2;
  const int64_t items = npairs_plus(o) * per;
  const int tid = threadIdx.x;
  auto put = [&](int64_t x, double val) __attribute__((always_inline)) {
    out[x] = (MODE == 1 || beta == 0.0) ? alpha * val : alpha * val + beta * out[x];
  };
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t pr = it / per;
    int k = (int)(it % per), A = 0;
    while (k >= nb - A) k -= nb - A++;          // block pair (A, B = A + k)
    const int B = A + k;
    int i0 = 0;                                 // occupied pair pr = (i0, j0), i0 <= j0
    while (pair_plus(i0 + 1, i0 + 1, o) <= pr) ++i0;
    const int j0 = i0 + (int)(pr - pair_plus(i0, i0, o));
    const bool offd = i0 < j0;
    const int64_t qr = offd ? pair_minus(i0, j0, o) : 0;
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
      const int e = tid + 256 * e4, r = e >> 5, c = e & 31;
      const int a = A * 32 + r, b = B * 32 + c;
      const bool ok = a < v && b < v && a <= b;
      double pv = ok ? (double)xp[pr * ldp + pair_plus(a, b, v)] : 0.0;
      double mv = (ok && offd && a < b) ? (double)xm[qr * ldm + pair_minus(a, b, v)] : 0.0;
      if (MODE == 1) {
        if (a != b) pv *= 0.5;
        mv *= 0.5;
      }
      sp_[r][c] = pv;
      sm_[r][c] = mv;
    }
    __syncthreads();
    const int64_t row_ij = ((int64_t)i0 * o + j0) * v, row_ji = ((int64_t)j0 * o + i0) * v;
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {            // entries (a, b), a <= b
      const int e = tid + 256 * e4, r = e >> 5, c = e & 31;
      const int a = A * 32 + r, b = B * 32 + c;
      if (a < v && b < v && a <= b) {
        const double pv = sp_[r][c], mv = sm_[r][c];
        put((row_ij + a) * v + b, pv + mv);
        if (offd) put((row_ji + a) * v + b, pv - mv);
      }
    }
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {            // entries (b, a), a < b, from the transpose
      const int e = tid + 256 * e4, rb = e >> 5, ca = e & 31;
      const int b = B * 32 + rb, a = A * 32 + ca;
      if (b < v && a < b) {
        const double pv = sp_[ca][rb], mv = sm_[ca][rb];
        put((row_ij + b) * v + a, pv - mv);
        if (offd) put((row_ji + b) * v + a, pv + mv);
      }
    }
    __syncthreads();
  }
}

static int64_t unpack_grid(int o, int v) {
  const int64_t nb = (v + 31) / 32, items = npairs_plus(o) * (nb * (nb + 1) / 2);
  return items < 8192 ? items : 8192;
}

int unpack_r(hipStream_t s, int acc_prec, int o, int v, const void* rp, int64_t ldp, const void* rm,
             int64_t ldm, double* R, double alpha, double beta) {
  if (o <= 0 || v <= 0) return PPL_OK;
  const unsigned g = (unsigned)unpack_grid(o, v);
  if (acc_prec == PPL_FP64)
    hipLaunchKernelGGL((unpack_tiled_kernel<double, 0>), dim3(g), dim3(256), 0, s, o, v, (const double*)rp, ldp,
                       (const double*)rm, ldm, R, alpha, beta);
  else
    hipLaunchKernelGGL((unpack_tiled_kernel<float, 0>), dim3(g), dim3(256), 0, s, o, v, (const float*)rp, ldp,
                       (const float*)rm, ldm, R, alpha, beta);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

int unpack_t(hipStream_t s, int o, int v, const double* sp, int64_t ldp, const double* am,
             int64_t ldm, double* t2) {
  if (o <= 0 || v <= 0) return PPL_OK;
  hipLaunchKernelGGL((unpack_tiled_kernel<double, 1>), dim3((unsigned)unpack_grid(o, v)), dim3(256), 0, s, o, v,
                     sp, ldp, am, ldm, t2, 1.0, 0.0);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// ------------------------------------------------------------------ reductions
// Fixed grid (kReduceBlocks x kReduceThreads), grid-stride loops and a fixed
// tree order: the sums are bitwise reproducible for a given problem size.
template <int NV>
__device__ inline void block_reduce_store(double (&vals)[NV], double* partials) {
  __shared__ double sh[NV][kReduceThreads];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k][tid] = vals[k];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int k = 0; k < NV; ++k) sh[k][tid] += sh[k][tid + w];
    __syncthreads();
  }
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[blockIdx.x * 4 + k] = sh[k][0];
}

__global__ void final_reduce_kernel(const double* __restrict__ partials, int nblocks, double* out) {
  __shared__ double sh[4][kReduceThreads];
  const int tid = threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  for (int b = tid; b < nblocks; b += kReduceThreads)
    for (int k = 0; k < 4; ++k) acc[k] += partials[b * 4 + k];
  for (int k = 0; k < 4; ++k) sh[k][tid] = acc[k];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < 4; ++k) sh[k][tid] += sh[k][tid + w];
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < 4; ++k) out[k] = sh[k][0];
}

struct PairGeom {
  int o, v;
  int64_t Np, Nm, Pp, Pm, ldp, ldm;
  const int *tab_op, *tab_om, *tab_vp, *tab_vm;
};

// q = x / d, p = x - q d for x >= 0, d > 0; in 32 bits when the caller knows x < 2^31
// (the quotient is the same, the instruction sequence much shorter)
__device__ inline void row_col(int64_t x, int64_t d, bool narrow, int64_t& q, int64_t& p) {
  if (narrow) {
    const uint32_t q32 = (uint32_t)x / (uint32_t)d;
    q = q32;
  } else {
    q = x / d;
  }
  p = x - q * d;
}

// Denominator of a packed element
__device__ inline double denom(const double* e_occ, const double* e_vir, int ij, int ab) {
  return e_occ[pair_first(ij)] + e_occ[pair_second(ij)] - e_vir[pair_first(ab)] - e_vir[pair_second(ab)];
}

// mode 0: MP2 start   S' = (2-d_ab) VS / D, A' = 2 VA / D, energy of the result
// mode 1: Jacobi update from R+- (type Tr); residual^2, energy, non-finite count
// mode 2: energy of the current S'/A' only
// SAVE (mode 1 only): also write the new amplitudes and the error (new - old), both
// in the packed S'/A' scaling, to one DIIS slot each (plus part, then minus part at
// offset Np * ldp); padding columns of the slots are not written.
template <int MODE, class Tr, bool SAVE = false>
__global__ void __launch_bounds__(kReduceThreads)
sweep_kernel(PairGeom g, const double* __restrict__ e_occ, const double* __restrict__ e_vir,
             const double* __restrict__ vs, const double* __restrict__ va, const Tr* __restrict__ rp,
             const Tr* __restrict__ rm, double* sp, double* am, double* partials,
             double* __restrict__ tslot = nullptr, double* __restrict__ eslot = nullptr) {
  double r2 = 0.0, en = 0.0, bad = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // "+" part: weights (2 - d_ij)(2 - d_ab) turn packed sums into full-tensor sums
  const int64_t totp = g.Np * g.ldp, totm = g.Nm * g.ldm;
  const bool narrow = totp < 0x7fffffffLL && totm < 0x7fffffffLL;
  for (int64_t x = tid0; x < totp; x += st) {
    int64_t q, p;
    row_col(x, g.ldp, narrow, q, p);
    if (p >= g.Pp) continue;
    const int ij = g.tab_op[q], ab = g.tab_vp[p];
    const bool dij = pair_first(ij) == pair_second(ij), dab = pair_first(ab) == pair_second(ab);
    const double w = (dij ? 1.0 : 2.0) * (dab ? 1.0 : 2.0);
    const double wab = dab ? 1.0 : 2.0;             // S' = wab * s
    const double vsx = vs[x];
    double snew;
    if (MODE == 0) {
      snew = vsx / denom(e_occ, e_vir, ij, ab);
      sp[x] = wab * snew;
    } else if (MODE == 1) {
      snew = (vsx + (double)rp[x]) / denom(e_occ, e_vir, ij, ab);
      const double sold = sp[x] / wab;
      const double ds = snew - sold;
      r2 += w * ds * ds;
      sp[x] = wab * snew;
      if (SAVE) {
        tslot[x] = wab * snew;
        eslot[x] = wab * ds;
      }
    } else {
      snew = sp[x] / wab;
    }
    if (!isfinite(snew)) bad += 1.0;
    en += w * vsx * snew;
  }
  // "-" part: every packed (i<j, a<b) entry stands for 4 full-tensor entries
  for (int64_t x = tid0; x < totm; x += st) {
    int64_t q, p;
    row_col(x, g.ldm, narrow, q, p);
    if (p >= g.Pm) continue;
    const int ij = g.tab_om[q], ab = g.tab_vm[p];
    const double vax = va[x];
    double anew;
    if (MODE == 0) {
      anew = vax / denom(e_occ, e_vir, ij, ab);
      am[x] = 2.0 * anew;
    } else if (MODE == 1) {
      anew = (vax + (double)rm[x]) / denom(e_occ, e_vir, ij, ab);
      const double da = anew - 0.5 * am[x];
      r2 += 4.0 * da * da;
      am[x] = 2.0 * anew;
      if (SAVE) {
        tslot[totp + x] = 2.0 * anew;
        eslot[totp + x] = 2.0 * da;
      }
    } else {
      anew = 0.5 * am[x];
    }
    if (!isfinite(anew)) bad += 1.0;
    en += 12.0 * vax * anew;                        // E = sum V^S s + 3 sum V^A a (full tensor)
  }
  double vals[3] = {r2, en, bad};
  block_reduce_store<3>(vals, partials);
}

template <int MODE, class Tr>
static int sweep_launch(hipStream_t s, const PairGeom& g, const double* e_occ, const double* e_vir,
                        const double* vs, const double* va, const void* rp, const void* rm,
                        double* sp, double* am, double* partials, double* red_out) {
  hipLaunchKernelGGL((sweep_kernel<MODE, Tr>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, g,
                     e_occ, e_vir, vs, va, (const Tr*)rp, (const Tr*)rm, sp, am, partials);
  PPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials,
                     kReduceBlocks, red_out);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

static PairGeom geom(int o, int v, int64_t ldp, int64_t ldm, const int* tab_op, const int* tab_om,
                     const int* tab_vp, const int* tab_vm) {
  return PairGeom{o, v, npairs_plus(o), npairs_minus(o), npairs_plus(v), npairs_minus(v), ldp, ldm,
                  tab_op, tab_om, tab_vp, tab_vm};
}

int mp2_start(hipStream_t s, int o, int v, const double* e_occ, const double* e_vir, const double* vs,
              const double* va, int64_t ldp, int64_t ldm, double* sp, double* am, const int* tab_op,
              const int* tab_om, const int* tab_vp, const int* tab_vm, double* partials,
              double* red_out) {
  PairGeom g = geom(o, v, ldp, ldm, tab_op, tab_om, tab_vp, tab_vm);
  return sweep_launch<0, double>(s, g, e_occ, e_vir, vs, va, nullptr, nullptr, sp, am, partials, red_out);
}

int update_sweep(hipStream_t s, int acc_prec, int o, int v, const double* e_occ, const double* e_vir,
                 const double* vs, const double* va, const void* rp, const void* rm, int64_t ldp,
                 int64_t ldm, double* sp, double* am, const int* tab_op, const int* tab_om,
                 const int* tab_vp, const int* tab_vm, double* partials, double* red_out,
                 double* tslot, double* eslot) {
  PairGeom g = geom(o, v, ldp, ldm, tab_op, tab_om, tab_vp, tab_vm);
  if (tslot && eslot) {
    if (acc_prec == PPL_FP64)
      hipLaunchKernelGGL((sweep_kernel<1, double, true>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, g,
                         e_occ, e_vir, vs, va, (const double*)rp, (const double*)rm, sp, am, partials, tslot,
                         eslot);
    else
      hipLaunchKernelGGL((sweep_kernel<1, float, true>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, g,
                         e_occ, e_vir, vs, va, (const float*)rp, (const float*)rm, sp, am, partials, tslot,
                         eslot);
    PPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials, kReduceBlocks,
                       red_out);
    PPL_LAUNCH_CHECK();
    return PPL_OK;
  }
  if (acc_prec == PPL_FP64)
    return sweep_launch<1, double>(s, g, e_occ, e_vir, vs, va, rp, rm, sp, am, partials, red_out);
  return sweep_launch<1, float>(s, g, e_occ, e_vir, vs, va, rp, rm, sp, am, partials, red_out);
}

// ------------------------------------------------------------------ DIIS subspace
// Inner products <e_new, e_i> over the full o x o x v x v tensors, from the packed
// slots: a "+" entry of S' scaling carries weight (2 - d_ij) / (2 - d_ab) (its
// full-tensor multiplicity over the square of its packing factor), a "-" entry of A'
// scaling weight 1 (four entries, each half of A').
__global__ void __launch_bounds__(kReduceThreads)
diis_dots_kernel(PairGeom g, const double* __restrict__ E, int64_t slot_n, DiisSet set, int knew,
                 double* partials) {
  double acc[kDiisMax];
#pragma unroll
  for (int i = 0; i < kDiisMax; ++i) acc[i] = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double* en = E + knew * slot_n;
  const int64_t totp = g.Np * g.ldp, totm = g.Nm * g.ldm;
  const bool narrow = totp < 0x7fffffffLL && totm < 0x7fffffffLL;
  for (int64_t x = tid0; x < totp; x += st) {
    int64_t q, p;
    row_col(x, g.ldp, narrow, q, p);
    if (p >= g.Pp) continue;
    const int ij = g.tab_op[q], ab = g.tab_vp[p];
    const double w = (pair_first(ij) == pair_second(ij) ? 1.0 : 2.0) /
                     (pair_first(ab) == pair_second(ab) ? 1.0 : 2.0);
    const double a = w * en[x];
#pragma unroll
    for (int i = 0; i < kDiisMax; ++i)
      if (i < set.n) acc[i] += a * E[set.id[i] * slot_n + x];
  }
  for (int64_t x = tid0; x < totm; x += st) {
    int64_t q, p;
    row_col(x, g.ldm, narrow, q, p);
    if (p >= g.Pm) continue;
    const double a = en[totp + x];
#pragma unroll
    for (int i = 0; i < kDiisMax; ++i)
      if (i < set.n) acc[i] += a * E[set.id[i] * slot_n + totp + x];
  }
  __shared__ double sh[kDiisMax][kReduceThreads];
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kDiisMax; ++i) sh[i][tid] = acc[i];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int i = 0; i < kDiisMax; ++i) sh[i][tid] += sh[i][tid + w];
    __syncthreads();
  }
  if (tid < kDiisMax) partials[blockIdx.x * kDiisMax + tid] = sh[tid][0];
}

__global__ void diis_final_kernel(const double* __restrict__ partials, int nblocks, double* out) {
  __shared__ double sh[kDiisMax][kReduceThreads];
  const int tid = threadIdx.x;
  double acc[kDiisMax];
  for (int i = 0; i < kDiisMax; ++i) acc[i] = 0.0;
  for (int b = tid; b < nblocks; b += kReduceThreads)
    for (int i = 0; i < kDiisMax; ++i) acc[i] += partials[b * kDiisMax + i];
  for (int i = 0; i < kDiisMax; ++i) sh[i][tid] = acc[i];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int i = 0; i < kDiisMax; ++i) sh[i][tid] += sh[i][tid + w];
    __syncthreads();
  }
  if (tid < kDiisMax) out[tid] = sh[tid][0];
}

int diis_dots(hipStream_t s, int o, int v, int64_t ldp, int64_t ldm, const int* tab_op, const int* tab_om,
              const int* tab_vp, const int* tab_vm, const double* E, int64_t slot_n, const DiisSet& set,
              int knew, double* partials, double* out) {
  if (set.n < 1 || set.n > kDiisMax) return fail(PPL_E_ARG, "DIIS set of %d vectors", set.n);
  PairGeom g = geom(o, v, ldp, ldm, tab_op, tab_om, tab_vp, tab_vm);
  hipLaunchKernelGGL(diis_dots_kernel, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, g, E, slot_n, set, knew,
                     partials);
  PPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(diis_final_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials, kReduceBlocks, out);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// S'/A' = sum_i c_i T_i over the slots of the set; padding columns set to zero.
__global__ void diis_combine_kernel(PairGeom g, const double* __restrict__ T, int64_t slot_n, DiisSet set,
                                    double* sp, double* am) {
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t totp = g.Np * g.ldp, totm = g.Nm * g.ldm;
  const bool narrow = totp < 0x7fffffffLL && totm < 0x7fffffffLL;
  for (int64_t x = tid0; x < totp; x += st) {
    int64_t q, p;
    row_col(x, g.ldp, narrow, q, p);
    double y = 0.0;
    if (p < g.Pp)
      for (int i = 0; i < set.n; ++i) y += set.c[i] * T[set.id[i] * slot_n + x];
    sp[x] = y;
  }
  for (int64_t x = tid0; x < totm; x += st) {
    int64_t q, p;
    row_col(x, g.ldm, narrow, q, p);
    double y = 0.0;
    if (p < g.Pm)
      for (int i = 0; i < set.n; ++i) y += set.c[i] * T[set.id[i] * slot_n + totp + x];
    am[x] = y;
  }
}

int diis_combine(hipStream_t s, int o, int v, int64_t ldp, int64_t ldm, const double* T, int64_t slot_n,
                 const DiisSet& set, double* sp, double* am) {
  if (set.n < 1 || set.n > kDiisMax) return fail(PPL_E_ARG, "DIIS set of %d vectors", set.n);
  PairGeom g = geom(o, v, ldp, ldm, nullptr, nullptr, nullptr, nullptr);
  const int64_t total = std::max(g.Np * ldp, g.Nm * ldm);
  hipLaunchKernelGGL(diis_combine_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g, T, slot_n, set, sp, am);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

int energy_only(hipStream_t s, int o, int v, const double* vs, const double* va, const double* sp,
                const double* am, int64_t ldp, int64_t ldm, const int* tab_op, const int* tab_om,
                const int* tab_vp, const int* tab_vm, double* partials, double* red_out) {
  PairGeom g = geom(o, v, ldp, ldm, tab_op, tab_om, tab_vp, tab_vm);
  return sweep_launch<2, double>(s, g, nullptr, nullptr, vs, va, nullptr, nullptr, (double*)sp,
                                 (double*)am, partials, red_out);
}

// Sums of (L^P_ac - L^P_ca)^2 and (L^P_ac)^2 + (L^P_ca)^2 over the virtual block, a < c
// (red_out[0], red_out[1]): the relative asymmetry of the Cholesky vectors. Work items are
// 32 x 32 block pairs (P, A <= C): block (A, C) and block (C, A) are both read along rows
// and the second is transposed through LDS, so that every read is coalesced.
__global__ void __launch_bounds__(kReduceThreads)
asym_kernel(const double* __restrict__ L, int n, int o, int v, int naux, double* partials) {
  static_assert(kReduceThreads == 256, "four elements of a 32 x 32 block per thread");
  __shared__ double tr[32][33];
  double d2 = 0.0, l2 = 0.0;
  const int nb = (v + 31) / 32;
  const int64_t per_p = (int64_t)nb * (nb + 1) / 2;
  const int64_t items = (int64_t)naux * per_p;
  const int tid = threadIdx.x;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t P = it / per_p;
    int k = (int)(it % per_p), A = 0;
    while (k >= nb - A) k -= nb - A++;           // block pair (A, C = A + k)
    const int C = A + k;
    const double* Lp = L + P * n * n;
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {             // block (C, A) by rows, stored transposed
      const int e = tid + 256 * e4, r = e >> 5, q = e & 31;
      const int c = C * 32 + r, a = A * 32 + q;
      tr[q][r] = (c < v && a < v) ? Lp[(int64_t)(o + c) * n + o + a] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {             // block (A, C) by rows, against it
      const int e = tid + 256 * e4, r = e >> 5, q = e & 31;
      const int a = A * 32 + r, c = C * 32 + q;
      if (a < c && c < v) {
        const double lac = Lp[(int64_t)(o + a) * n + o + c], lca = tr[r][q];
        d2 += (lac - lca) * (lac - lca);
        l2 += lac * lac + lca * lca;
      }
    }
    __syncthreads();
  }
  double vals[3] = {d2, l2, 0.0};
  block_reduce_store<3>(vals, partials);
}

int asymmetry_vv(hipStream_t s, const double* L, int o, int v, int naux, double* partials, double* red_out) {
  hipLaunchKernelGGL(asym_kernel, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, L, o + v, o, v, naux, partials);
  PPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials, kReduceBlocks, red_out);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

__global__ void __launch_bounds__(kReduceThreads)
nonfinite_kernel(const double* __restrict__ x, int64_t n, double* partials) {
  double bad = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += st)
    if (!isfinite(x[i])) bad += 1.0;
  double vals[3] = {0.0, 0.0, bad};
  block_reduce_store<3>(vals, partials);
}

int count_nonfinite(hipStream_t s, const double* x, int64_t n, double* partials, double* red_out) {
  hipLaunchKernelGGL(nonfinite_kernel, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, x, n, partials);
  PPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials,
                     kReduceBlocks, red_out);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}


// ------------------------------------------------------------------ ring terms
// Operands of the ring terms as (o v) x (o v) matrices over the pairs (i,a) and (k,c),
// rows of ld elements (columns from o v on zero), stored in the operand precision PREC
// (FP64, FP32, or bf16 planes: the second pointer of each is its lo / mid plane):
//   Xa[(i,a)][(k,c)] = 2 t_ik^ac - t_ik^ca,  An[(i,a)][(k,c)] = -t_ik^ac,  B[(i,a)][(k,c)] = t_ik^ca.
template <int PREC>
__global__ void __launch_bounds__(256)
ring_pack_kernel(int o, int v, const double* __restrict__ t, int64_t ld, void* Xa, void* Xa_lo, void* An,
                 void* An_lo, void* B, void* B_lo) {
  const int64_t ov = (int64_t)o * v, total = ov * ld;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const int64_t row = x / ld, col = x - row * ld;
    double xa = 0.0, an = 0.0, b = 0.0;
    if (col < ov) {
      const int64_t i = row / v, a = row - i * v, k = col / v, c = col - k * v;
      const int64_t base = (i * o + k) * v * v;
      const double tac = t[base + a * v + c], tca = t[base + c * v + a];
      xa = 2.0 * tac - tca;
      an = -tac;
      b = tca;
    }
    Store<PREC>::put(Xa, Xa_lo, x, xa);
    Store<PREC>::put(An, An_lo, x, an);
    Store<PREC>::put(B, B_lo, x, b);
  }
}

int ring_pack(hipStream_t s, int o, int v, const double* t, int64_t ld, double* Xa, double* An, double* B) {
  return ring_pack_lp(s, PPL_FP64, o, v, t, ld, Xa, nullptr, An, nullptr, B, nullptr);
}

int ring_pack_lp(hipStream_t s, int prec, int o, int v, const double* t, int64_t ld, void* Xa, void* Xa_lo,
                 void* An, void* An_lo, void* B, void* B_lo) {
  const int64_t n = (int64_t)o * v * ld;
  if (n <= 0) return PPL_OK;
  const dim3 grid(grid_for(n, 256));
  if (prec == PPL_FP64)
    hipLaunchKernelGGL(ring_pack_kernel<PPL_FP64>, grid, dim3(256), 0, s, o, v, t, ld, Xa, Xa_lo, An, An_lo, B, B_lo);
  else if (prec == PPL_FP32)
    hipLaunchKernelGGL(ring_pack_kernel<PPL_FP32>, grid, dim3(256), 0, s, o, v, t, ld, Xa, Xa_lo, An, An_lo, B, B_lo);
  else if (prec == PPL_BF16X3)
    hipLaunchKernelGGL(ring_pack_kernel<PPL_BF16X3>, grid, dim3(256), 0, s, o, v, t, ld, Xa, Xa_lo, An, An_lo, B,
                       B_lo);
  else if (prec == PPL_BF16X6)
    hipLaunchKernelGGL(ring_pack_kernel<PPL_BF16X6>, grid, dim3(256), 0, s, o, v, t, ld, Xa, Xa_lo, An, An_lo, B,
                       B_lo);
  else
    return fail(PPL_E_ARG, "ring_pack: unknown precision %d", prec);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// K[(k,c)][(j,b)] = (kj|bc) = G[(k,j)][(b,c)] (G rows of ldg elements); columns from o v on zero
__global__ void __launch_bounds__(256)
ring_exchange_kernel(int o, int v, const double* __restrict__ G, int64_t ldg, double* K, int64_t ld) {
  const int64_t ov = (int64_t)o * v, total = ov * ld;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const int64_t row = x / ld, col = x - row * ld;
    double y = 0.0;
    if (col < ov) {
      const int64_t k = row / v, c = row - k * v, j = col / v, b = col - j * v;
      y = G[(k * o + j) * ldg + b * v + c];
    }
    K[x] = y;
  }
}

int ring_exchange(hipStream_t s, int o, int v, const double* G, int64_t ldg, double* K, int64_t ld) {
  const int64_t n = (int64_t)o * v * ld;
  if (n <= 0) return PPL_OK;
  hipLaunchKernelGGL(ring_exchange_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, o, v, G, ldg, K, ld);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// R_ij^ab = beta R_ij^ab + alpha (Y_ij^ab + Y_ji^ba) with Y_ij^ab = C1[(i,a)][(j,b)] - C2[(i,b)][(j,a)]
// (C1, C2 in the accumulator type Tc of the ring GEMMs)
template <class Tc>
__global__ void __launch_bounds__(256)
ring_unpack_kernel(int o, int v, const Tc* __restrict__ C1, const Tc* __restrict__ C2, int64_t ld, double* R,
                   double alpha, double beta) {
  const int64_t total = (int64_t)o * o * v * v;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    int64_t r = x;
    const int64_t b = r % v; r /= v;
    const int64_t a = r % v; r /= v;
    const int64_t j = r % o, i = r / o;
    const double y1 = (double)C1[(i * v + a) * ld + j * v + b] - (double)C2[(i * v + b) * ld + j * v + a];
    const double y2 = (double)C1[(j * v + b) * ld + i * v + a] - (double)C2[(j * v + a) * ld + i * v + b];
    const double y = alpha * (y1 + y2);
    R[x] = beta == 0.0 ? y : beta * R[x] + y;
  }
}

int ring_unpack(hipStream_t s, int o, int v, const double* C1, const double* C2, int64_t ld, double* R, double alpha,
                double beta) {
  const int64_t n = (int64_t)o * o * v * v;
  if (n <= 0) return PPL_OK;
  hipLaunchKernelGGL(ring_unpack_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, o, v, C1, C2, ld, R, alpha,
                     beta);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

int ring_unpack_f32(hipStream_t s, int o, int v, const float* C1, const float* C2, int64_t ld, double* R, double alpha,
                    double beta) {
  const int64_t n = (int64_t)o * o * v * v;
  if (n <= 0) return PPL_OK;
  hipLaunchKernelGGL(ring_unpack_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, o, v, C1, C2, ld, R, alpha,
                     beta);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

// R+- += the pair parts of a pair-symmetric full tensor (the inverse of unpack_r)
template <class Tc>
__global__ void __launch_bounds__(256)
add_pm_kernel(int o, int v, const double* __restrict__ R, Tc* rp, int64_t ldp, Tc* rm, int64_t ldm, int64_t Np,
              int64_t Pp, int64_t Nm, int64_t Pm, const int* __restrict__ tab_op, const int* __restrict__ tab_om,
              const int* __restrict__ tab_vp, const int* __restrict__ tab_vm) {
  const int64_t np = Np * Pp, total = np + Nm * Pm;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += st) {
    const bool plus = x < np;
    const int64_t y = plus ? x : x - np;
    const int64_t P = plus ? Pp : Pm;
    const int64_t q = y / P, c = y - q * P;
    const int ij = plus ? tab_op[q] : tab_om[q];
    const int ab = plus ? tab_vp[c] : tab_vm[c];
    const int64_t i = pair_first(ij), j = pair_second(ij), a = pair_first(ab), b = pair_second(ab);
    const double r1 = R[((i * o + j) * v + a) * v + b], r2 = R[((i * o + j) * v + b) * v + a];
    if (plus) {
      Tc* d = rp + q * ldp + c;
      *d = (Tc)((double)*d + 0.5 * (r1 + r2));
    } else {
      Tc* d = rm + q * ldm + c;
      *d = (Tc)((double)*d + 0.5 * (r1 - r2));
    }
  }
}

int add_pm(hipStream_t s, int c_prec, int o, int v, const double* R, void* rp, int64_t ldp, void* rm, int64_t ldm,
           const int* tab_op, const int* tab_om, const int* tab_vp, const int* tab_vm) {
  const int64_t Np = npairs_plus(o), Nm = npairs_minus(o), Pp = npairs_plus(v), Pm = npairs_minus(v);
  const int64_t n = Np * Pp + Nm * Pm;
  if (n <= 0) return PPL_OK;
  if (c_prec == PPL_FP64)
    hipLaunchKernelGGL(add_pm_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, o, v, R, (double*)rp, ldp,
                       (double*)rm, ldm, Np, Pp, Nm, Pm, tab_op, tab_om, tab_vp, tab_vm);
  else
    hipLaunchKernelGGL(add_pm_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, o, v, R, (float*)rp, ldp,
                       (float*)rm, ldm, Np, Pp, Nm, Pm, tab_op, tab_om, tab_vp, tab_vm);
  PPL_LAUNCH_CHECK();
  return PPL_OK;
}

}  // namespace ppl
