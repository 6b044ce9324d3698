// Learned start of the amplitude iteration: a 4 -> 128 -> 128 -> 1 SiLU network
// that maps per-element features of the first-order amplitudes,
//     x = (t_MP2 / sigma, D_ij^ab, e_i + e_j, e_a + e_b),
// to a correction f(x), giving the guess t = t_MP2 + sigma * f(x).
// Every feature is invariant under (i,j,a,b) -> (j,i,b,a), so the guess keeps
// the amplitudes' pair symmetry (eq. (2)).
//
// Training (FP32): one fused kernel per minibatch computes the forward pass,
// the mean-squared-error loss and the full backward pass for a block of rows,
// and writes per-workgroup gradient partials; a second kernel sums them in a
// fixed order (bitwise reproducible), a third applies Adam.
// Inference: the 128 x 128 hidden layer runs on the BF16 matrix cores
// (16x16x32, FP32 accumulation); the small layers stay in FP32.
//
// Flat parameter order: W1 [128][4], b1 [128], W2 [128][128], b2 [128], W3 [128], b3 [1].
#include "ppl_internal.h"

namespace ppl {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kH = 128;
constexpr int kOffW1 = 0, kOffB1 = kH * 4, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kNParams = kOffB3 + 1;
constexpr int kTrainRows = 32;     // rows per training workgroup
constexpr int kInferRows = 64;     // rows per inference workgroup (4 waves x 16)

int mlp_param_count() { return kNParams; }
int mlp_train_rows() { return kTrainRows; }

__device__ inline float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------------ training
// grid = ceil(n / kTrainRows) workgroups of 256 threads
__global__ void __launch_bounds__(256)
mlp_train_kernel(const float* __restrict__ prm, const float* __restrict__ X, const float* __restrict__ Y,
                 int64_t n, float inv_n, float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ float sW2[kH][kH + 1];
  __shared__ float sW1[kH][4], sb1[kH], sb2[kH], sW3[kH];
  __shared__ float sX[kTrainRows][4], sY[kTrainRows], sdy[kTrainRows];
  __shared__ float sH1[kTrainRows][kH], sD1[kTrainRows][kH], sT[kTrainRows][kH];
  __shared__ float sdW3[2][kH], sdb2[2][kH];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kTrainRows;
  for (int e = tid; e < kH * kH; e += 256) sW2[e / kH][e % kH] = prm[kOffW2 + e];
  for (int e = tid; e < kH * 4; e += 256) sW1[e / 4][e % 4] = prm[kOffW1 + e];
  if (tid < kH) {
    sb1[tid] = prm[kOffB1 + tid];
    sb2[tid] = prm[kOffB2 + tid];
    sW3[tid] = prm[kOffW3 + tid];
  }
  const float b3 = prm[kOffB3];
  if (tid < kTrainRows * 4) {
    const int r = tid / 4, c = tid % 4;
    sX[r][c] = (r0 + r < n) ? X[(r0 + r) * 4 + c] : 0.0f;
  }
  if (tid < kTrainRows) sY[tid] = (r0 + tid < n) ? Y[r0 + tid] : 0.0f;
  __syncthreads();
  // layer 1
  for (int e = tid; e < kTrainRows * kH; e += 256) {
    const int r = e / kH, h = e % kH;
    float z = sb1[h];
#pragma unroll
    for (int c = 0; c < 4; ++c) z += sW1[h][c] * sX[r][c];
    sH1[r][h] = silu_f(z);
    sD1[r][h] = dsilu_f(z);
  }
  __syncthreads();
  // layer 2: thread owns hidden unit h for 16 rows
  const int h = tid % kH, rg = tid / kH;
  float h2[16], d2[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = rg * 16 + q;
    float z = sb2[h];
    for (int k = 0; k < kH; ++k) z += sW2[h][k] * sH1[r][k];
    h2[q] = silu_f(z);
    d2[q] = dsilu_f(z);
    sT[r][h] = sW3[h] * h2[q];
  }
  __syncthreads();
  // output and loss (one thread per row, fixed order over h)
  float lsum = 0.0f;
  if (tid < kTrainRows) {
    float y = b3;
    for (int k = 0; k < kH; ++k) y += sT[tid][k];
    const bool valid = r0 + tid < n;
    const float diff = valid ? (y - sY[tid]) : 0.0f;
    sdy[tid] = 2.0f * diff * inv_n;
    lsum = diff * diff;
  }
  __syncthreads();
  // dZ2, dW3, db2 partials
  float dw3 = 0.0f, db2 = 0.0f;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = rg * 16 + q;
    const float dy = sdy[r];
    dw3 += dy * h2[q];
    const float dz = dy * sW3[h] * d2[q];
    db2 += dz;
    sT[r][h] = dz;                 // sT now holds dZ2
  }
  sdW3[rg][h] = dw3;
  sdb2[rg][h] = db2;
  __syncthreads();
  float* gp = gpart + (int64_t)blockIdx.x * kNParams;
  // dW2[h][k] = sum_r dZ2[r][h] H1[r][k]: thread owns h2_ = tid/2, 64 columns
  {
    const int hh = tid / 2, k0 = (tid % 2) * 64;
    float acc[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) acc[k] = 0.0f;
    for (int r = 0; r < kTrainRows; ++r) {
      const float dz = sT[r][hh];
#pragma unroll
      for (int k = 0; k < 64; ++k) acc[k] += dz * sH1[r][k0 + k];
    }
#pragma unroll
    for (int k = 0; k < 64; ++k) gp[kOffW2 + hh * kH + k0 + k] = acc[k];
  }
  // dH1 -> dZ1 (into sD1), thread owns column k for 16 rows
  {
    const int k = tid % kH;
    float dz1[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = rg * 16 + q;
      float s = 0.0f;
      for (int hh = 0; hh < kH; ++hh) s += sW2[hh][k] * sT[r][hh];
      dz1[q] = s * sD1[r][k];
    }
    __syncthreads();               // every read of sD1 by other threads is done
#pragma unroll
    for (int q = 0; q < 16; ++q) sD1[rg * 16 + q][k] = dz1[q];
  }
  __syncthreads();
  // dW1, db1, dW3, db2, b3 and the loss partial
  for (int e = tid; e < kH * 4; e += 256) {
    const int hh = e / 4, c = e % 4;
    float s = 0.0f;
    for (int r = 0; r < kTrainRows; ++r) s += sD1[r][hh] * sX[r][c];
    gp[kOffW1 + e] = s;
  }
  if (tid < kH) {
    float s = 0.0f;
    for (int r = 0; r < kTrainRows; ++r) s += sD1[r][tid];
    gp[kOffB1 + tid] = s;
    gp[kOffW3 + tid] = sdW3[0][tid] + sdW3[1][tid];
    gp[kOffB2 + tid] = sdb2[0][tid] + sdb2[1][tid];
  }
  if (tid == 0) {
    float s = 0.0f;
    for (int r = 0; r < kTrainRows; ++r) s += sdy[r];
    gp[kOffB3] = s;
  }
  // loss partial: fixed-order sum over the 32 row losses (threads 0..31 hold them)
  __shared__ float sl[kTrainRows];
  if (tid < kTrainRows) sl[tid] = lsum;
  __syncthreads();
  if (tid == 0) {
    float s = 0.0f;
    for (int r = 0; r < kTrainRows; ++r) s += sl[r];
    lpart[blockIdx.x] = s;
  }
}

// grad[p] = sum_w gpart[w][p] (workgroup order); loss = sum_w lpart[w] * inv_n
__global__ void mlp_grad_reduce_kernel(const float* __restrict__ gpart, const float* __restrict__ lpart,
                                       int nwg, float inv_n, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNParams) {
    float s = 0.0f;
    for (int w = 0; w < nwg; ++w) s += gpart[(int64_t)w * kNParams + p];
    grad[p] = s;
  }
  if (p == 0) {
    float s = 0.0f;
    for (int w = 0; w < nwg; ++w) s += lpart[w];
    *loss = s * inv_n;
  }
}

__global__ void mlp_adam_kernel(float* prm, const float* __restrict__ grad, float* m, float* v, float lr,
                                float b1, float b2, float bc1, float bc2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParams) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  prm[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

int mlp_train_launch(hipStream_t s, const float* prm, const float* X, const float* Y, int64_t n,
                     float* gpart, float* lpart, float* grad, float* loss) {
  const int64_t nwg = (n + kTrainRows - 1) / kTrainRows;
  const float inv_n = 1.0f / (float)n;
  hipLaunchKernelGGL(mlp_train_kernel, dim3((unsigned)nwg), dim3(256), 0, s, prm, X, Y, n, inv_n, gpart,
                     lpart);
  PPL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, gpart, lpart,
                     (int)nwg, inv_n, grad, loss);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

int mlp_adam_launch(hipStream_t s, float* prm, const float* grad, float* m, float* v, float lr, int step,
                    float beta1, float beta2, float eps) {
  const float bc1 = 1.0f - powf(beta1, (float)step), bc2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, prm, grad, m, v, lr,
                     beta1, beta2, bc1, bc2, eps);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

// ------------------------------------------------------------------ features, samples, sigma
__device__ inline void element_ijab(int64_t x, int o, int v, int& i, int& j, int& a, int& b) {
  b = (int)(x % v);
  const int64_t y = x / v;
  a = (int)(y % v);
  const int64_t z = y / v;
  j = (int)(z % o);
  i = (int)(z / o);
}

__global__ void mlp_samples_kernel(int o, int v, const double* __restrict__ tm, const double* __restrict__ ts,
                                   const double* __restrict__ e_occ, const double* __restrict__ e_vir,
                                   double sigma, const int64_t* __restrict__ idx, int64_t n, float* X,
                                   float* Y) {
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += st) {
    const int64_t x = idx[k];
    int i, j, a, b;
    element_ijab(x, o, v, i, j, a, b);
    const double eij = e_occ[i] + e_occ[j], eab = e_vir[a] + e_vir[b];
    X[k * 4 + 0] = (float)(tm[x] / sigma);
    X[k * 4 + 1] = (float)(e_occ[i] + e_occ[j] - e_vir[a] - e_vir[b]);
    X[k * 4 + 2] = (float)eij;
    X[k * 4 + 3] = (float)eab;
    if (Y) Y[k] = (float)((ts[x] - tm[x]) / sigma);
  }
}

int mlp_samples_launch(hipStream_t s, int o, int v, const double* tm, const double* ts, const double* e_occ,
                       const double* e_vir, double sigma, const int64_t* idx, int64_t n, float* X, float* Y) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(mlp_samples_kernel, dim3((unsigned)g), dim3(256), 0, s, o, v, tm, ts, e_occ, e_vir,
                     sigma, idx, n, X, Y);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

// ------------------------------------------------------------------ inference (BF16 MFMA hidden layer)
// Rows enumerate (i<j, all a, b) followed by (i=j, a<=b); each row writes the
// guess at (i,j,a,b) and at its pair partner (j,i,b,a), so no entry is written twice.
__global__ void __launch_bounds__(256)
mlp_infer_kernel(const float* __restrict__ prm, int o, int v, const double* __restrict__ tm,
                 const double* __restrict__ e_occ, const double* __restrict__ e_vir, double sigma,
                 const int* __restrict__ tab_om, const int* __restrict__ tab_vp, int64_t n_first,
                 int64_t n_total, double* __restrict__ tout) {
  constexpr int LDH = kH + 8;      // bf16 row stride (keeps 16-byte alignment)
  __shared__ __attribute__((aligned(16))) __bf16 sW2[kH * LDH];
  __shared__ __attribute__((aligned(16))) __bf16 sH1[kInferRows * LDH];
  __shared__ float sW1[kH][4], sb1[kH], sb2[kH], sW3[kH];
  __shared__ float sX[kInferRows][4];
  __shared__ int64_t sA[kInferRows], sB[kInferRows];   // output offsets (row and partner)
  __shared__ double sT[kInferRows];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kH * kH; e += 256) sW2[(e / kH) * LDH + (e % kH)] = (__bf16)prm[kOffW2 + e];
  for (int e = tid; e < kH * 4; e += 256) sW1[e / 4][e % 4] = prm[kOffW1 + e];
  if (tid < kH) {
    sb1[tid] = prm[kOffB1 + tid];
    sb2[tid] = prm[kOffB2 + tid];
    sW3[tid] = prm[kOffW3 + tid];
  }
  const float b3 = prm[kOffB3];
  const int64_t row0 = (int64_t)blockIdx.x * kInferRows;
  const int64_t vv = (int64_t)v * v;
  if (tid < kInferRows) {
    const int64_t e = row0 + tid;
    int i = 0, j = 0, a = 0, b = 0;
    bool ok = e < n_total;
    if (ok) {
      if (e < n_first) {
        const int ij = tab_om[e / vv];
        const int64_t rem = e % vv;
        i = pair_first(ij);
        j = pair_second(ij);
        a = (int)(rem / v);
        b = (int)(rem % v);
      } else {
        const int64_t e2 = e - n_first, Pp = npairs_plus(v);
        i = j = (int)(e2 / Pp);
        const int ab = tab_vp[e2 % Pp];
        a = pair_first(ab);
        b = pair_second(ab);
      }
    }
    const int64_t xa = (((int64_t)i * o + j) * v + a) * v + b;
    const int64_t xb = (((int64_t)j * o + i) * v + b) * v + a;
    const double t = ok ? tm[xa] : 0.0;
    sA[tid] = ok ? xa : -1;
    sB[tid] = ok ? xb : -1;
    sT[tid] = t;
    sX[tid][0] = (float)(t / sigma);
    sX[tid][1] = ok ? (float)(e_occ[i] + e_occ[j] - e_vir[a] - e_vir[b]) : 0.0f;
    sX[tid][2] = ok ? (float)(e_occ[i] + e_occ[j]) : 0.0f;
    sX[tid][3] = ok ? (float)(e_vir[a] + e_vir[b]) : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < kInferRows * kH; e += 256) {
    const int r = e / kH, h = e % kH;
    float z = sb1[h];
#pragma unroll
    for (int c = 0; c < 4; ++c) z += sW1[h][c] * sX[r][c];
    sH1[r * LDH + h] = (__bf16)silu_f(z);
  }
  __syncthreads();
  // Z2 rows [16*wave, 16*wave+16) x all 128 hidden units: A = H1 (rows x k), B[k][n] = W2[n][k]
  f4 acc[kH / 16];
#pragma unroll
  for (int jb = 0; jb < kH / 16; ++jb) acc[jb] = f4{0, 0, 0, 0};
  const int arow = (wave * 16 + (lane & 15)) * LDH + 8 * (lane >> 4);
#pragma unroll
  for (int kk = 0; kk < kH; kk += 32) {
    const bf8 a = *reinterpret_cast<const bf8*>(&sH1[arow + kk]);
#pragma unroll
    for (int jb = 0; jb < kH / 16; ++jb) {
      const bf8 bw = *reinterpret_cast<const bf8*>(&sW2[(jb * 16 + (lane & 15)) * LDH + 8 * (lane >> 4) + kk]);
      acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[jb], 0, 0, 0);
    }
  }
  // lane holds rows 4*(lane/16)+r of its wave's 16, columns 16*jb + lane%16
  float part[4] = {0, 0, 0, 0};
#pragma unroll
  for (int jb = 0; jb < kH / 16; ++jb) {
    const int hcol = jb * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) part[r] += sW3[hcol] * silu_f(acc[jb][r] + sb2[hcol]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) part[r] += __shfl_xor(part[r], off, 64);
  }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = wave * 16 + 4 * (lane >> 4) + r;
      if (sA[row] >= 0) {
        const double guess = sT[row] + sigma * (double)(part[r] + b3);
        tout[sA[row]] = guess;
        tout[sB[row]] = guess;
      }
    }
  }
}

int mlp_infer_launch(hipStream_t s, const float* prm, int o, int v, const double* tm, const double* e_occ,
                     const double* e_vir, double sigma, const int* tab_om, const int* tab_vp, double* tout) {
  const int64_t n_first = npairs_minus(o) * (int64_t)v * v;
  const int64_t n_total = n_first + (int64_t)o * npairs_plus(v);
  const int64_t g = (n_total + kInferRows - 1) / kInferRows;
  if (g > 0x7fffffffLL) return fail(PPL_E_ARG, "inference grid too large");
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)g), dim3(256), 0, s, prm, o, v, tm, e_occ, e_vir, sigma,
                     tab_om, tab_vp, n_first, n_total, tout);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

// sum of squares of a tensor (red_out[0]) with the fixed-order reduction of the sweep kernels
__global__ void __launch_bounds__(kReduceThreads)
sumsq_kernel(const double* __restrict__ x, int64_t n, double* partials) {
  __shared__ double sh[kReduceThreads];
  double s = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += st) s += x[i] * x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = sh[0];
    partials[blockIdx.x * 4 + 1] = 0.0;
    partials[blockIdx.x * 4 + 2] = 0.0;
    partials[blockIdx.x * 4 + 3] = 0.0;
  }
}

__global__ void final_reduce_kernel2(const double* __restrict__ partials, int nblocks, double* out) {
  __shared__ double sh[kReduceThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kReduceThreads) acc += partials[b * 4];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

int sumsq_launch(hipStream_t s, const double* x, int64_t n, double* partials, double* red_out) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, x, n, partials);
  PPL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(final_reduce_kernel2, dim3(1), dim3(kReduceThreads), 0, s, partials, kReduceBlocks,
                     red_out);
  PPL_HIP_TRY(hipGetLastError());
  return PPL_OK;
}

}  // namespace ppl
