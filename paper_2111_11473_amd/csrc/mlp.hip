// Kernels of the learned-guess network: a per-rank-index MLP n_in -> w -> w -> n_out with SiLU
// hidden activations, trained in FP32 (forward, backward, Adam) and run for inference in BF16 on
// MFMA with FP32 accumulation.
//
// Training pieces:
//   sgemm        C = op(A) op(B) on 64 x 64 tiles (FP32 VALU, LDS-staged), with fused epilogues:
//                bias + SiLU (keeps the pre-activation for the backward pass, or not in a pass
//                that is only a forward one), bias only, or a product with SiLU'(Z) (the backward
//                pass through an activation)
//   normalize    x_n = (x - mu) / sd per input column
//   mse_grad     dY = 2 (y_n - (t - mu) / sd) / (rows n_out) and per-block partial loss sums
//   colsum       bias gradients
//   adam         bias-corrected Adam update (Kingma and Ba, 2015)
//   init         Glorot-uniform weights from a counter-based generator (SplitMix64 of the index)
// Inference: one kernel per 64 rows evaluates all three layers with v_mfma_f32_16x16x16_bf16,
// keeping the activations in LDS.
// Parameter layout (FP32, one flat vector): W1 [n_in][w], b1 [w], W2 [w][w], b2 [w], W3 [w][n_out],
// b3 [n_out].
#include <mutex>

#include "internal.h"

namespace thc {
namespace {

constexpr int TPB = 256;

__device__ inline float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

constexpr int BM = 64, BN = 64, BK = 16;

// C[M][N] = op(A) op(B) (+ epilogue).  A is [M][K] (or [K][M] if TA), B is [K][N] (or [N][K] if TB).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(TPB) void sgemm_kernel(int64_t M, int64_t N, int64_t K, const float* __restrict__ A,
                                                    int64_t lda, const float* __restrict__ B, int64_t ldb,
                                                    float* __restrict__ C, int64_t ldc, const float* __restrict__ bias,
                                                    float* __restrict__ Z, int64_t ldz) {
  __shared__ float As[BK][BM + 1];
  __shared__ float Bs[BK][BN + 1];
  const int t = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int tr = t / 16, tc = t % 16;  // thread owns rows tr + 16 i, cols tc + 16 j
  float acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int q = 0; q < (BM * BK) / TPB; ++q) {
      const int e = t + TPB * q;
      int mm, kk;
      if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
      const int64_t m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? (TA ? A[k * lda + m] : A[m * lda + k]) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < (BN * BK) / TPB; ++q) {
      const int e = t + TPB * q;
      int nn, kk;
      if (TB) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
      const int64_t n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < N && k < K) ? (TB ? B[n * ldb + k] : B[k * ldb + n]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t m = m0 + tr + 16 * i, n = n0 + tc + 16 * j;
      if (m >= M || n >= N) continue;
      float x = acc[i][j];
      if (EPI == 1) {  // bias + SiLU; the pre-activation goes to Z
        x += bias[n];
        Z[m * ldz + n] = x;
        x = silu_f(x);
      } else if (EPI == 4) {  // bias + SiLU, pre-activation not kept (forward pass only)
        x = silu_f(x + bias[n]);
      } else if (EPI == 2) {  // bias only
        x += bias[n];
      } else if (EPI == 3) {  // times SiLU'(Z)
        x *= silu_grad_f(Z[m * ldz + n]);
      }
      C[m * ldc + n] = x;
    }
}

__global__ void normalize_kernel(int64_t rows, int64_t cols, const float* __restrict__ X, const float* __restrict__ mu,
                                 const float* __restrict__ sd, float* __restrict__ Xn) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % cols;
    Xn[e] = (X[e] - mu[c]) / sd[c];
  }
}

__global__ void denorm_kernel(int64_t rows, int64_t cols, const float* __restrict__ Yn, const float* __restrict__ mu,
                              const float* __restrict__ sd, float* __restrict__ Y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % cols;
    Y[e] = Yn[e] * sd[c] + mu[c];
  }
}

// dY = 2 (y_n - t_n) / (rows cols), t_n = (t - mu) / sd; part[block] = sum of (y_n - t_n)^2 over the block
__global__ void mse_grad_kernel(int64_t rows, int64_t cols, const float* __restrict__ Yn, const float* __restrict__ T,
                                const float* __restrict__ mu, const float* __restrict__ sd, float* __restrict__ dY,
                                double* __restrict__ part) {
  __shared__ double red[TPB];
  const int64_t n = rows * cols;
  const float scale = 2.0f / (float)n;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % cols;
    const float d = Yn[e] - (T[e] - mu[c]) / sd[c];
    dY[e] = scale * d;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_parts_kernel(int64_t nparts, const double* __restrict__ part, double denom, float* __restrict__ out) {
  __shared__ double red[TPB];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(red[0] / denom);
}

// out[n] = sum_r D[r][n]  (one workgroup per column)
__global__ void colsum_kernel(int64_t rows, int64_t cols, const float* __restrict__ D, float* __restrict__ out) {
  __shared__ float red[TPB];
  const int64_t n = blockIdx.x;
  float s = 0.0f;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) s += D[r * cols + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

// Per column of D[rows][cols]: mean and standard deviation (FP64 sums); a column whose spread is
// below 1e-6 of its scale gets sd = 1, so constant inputs standardize to zero.
__global__ void colstats_kernel(int64_t rows, int64_t cols, const float* __restrict__ D, float* __restrict__ mu,
                                float* __restrict__ sd) {
  __shared__ double r1[TPB], r2[TPB];
  const int64_t n = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    const double x = D[r * cols + n];
    s1 += x;
    s2 += x * x;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = r1[0] / (double)rows;
    const double var = fmax(r2[0] / (double)rows - m * m, 0.0);
    const double d = sqrt(var);
    mu[n] = (float)m;
    sd[n] = (float)(d > 1e-6 * fmax(1.0, fabs(m)) ? d : 1.0);
  }
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// weights of layer l: U(-a, a), a = sqrt(6 / (fan_in + fan_out)); biases zero
__global__ void init_kernel(int64_t n_in, int64_t w, int64_t n_out, uint64_t seed, float* __restrict__ p) {
  const int64_t s1 = n_in * w, s2 = s1 + w, s3 = s2 + w * w, s4 = s3 + w, s5 = s4 + w * n_out, total = s5 + n_out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    float a = 0.0f;
    if (e < s1) a = sqrtf(6.0f / (float)(n_in + w));
    else if (e >= s2 && e < s3) a = sqrtf(6.0f / (float)(2 * w));
    else if (e >= s4 && e < s5) a = sqrtf(6.0f / (float)(w + n_out));
    const double u = (double)(splitmix64(seed * 0x100000001B3ull + (uint64_t)e) >> 11) * (1.0 / 9007199254740992.0);
    p[e] = a == 0.0f ? 0.0f : a * (float)(2.0 * u - 1.0);
  }
}

// ---------------------------------------------------------------------------------------------
// BF16 inference: 64 rows per workgroup (16 per wave), all three layers, activations in LDS.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float x) {  // round to nearest even
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (short)(r >> 16);
}

constexpr int IW = 256;  // hidden width of the inference kernel
constexpr int KIN = 16;  // padded input width
constexpr int NOUT = 16; // padded output width

// Wb: bf16 weights [KIN][IW] | [IW][IW] | [IW][NOUT] (zero padded); bias fp32 [IW] | [IW] | [NOUT]
__global__ __launch_bounds__(TPB) void infer_kernel(int64_t rows, int64_t n_in, int64_t n_out,
                                                   const float* __restrict__ X, const float* __restrict__ mu_in,
                                                   const float* __restrict__ sd_in, const short* __restrict__ Wb,
                                                   const float* __restrict__ bias, const float* __restrict__ mu_out,
                                                   const float* __restrict__ sd_out, float* __restrict__ Y) {
  __shared__ short act[4][16][IW + 8];  // per wave: 16 rows of activations (bf16), padded rows
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + 16 * w;
  const short* W1 = Wb;
  const short* W2 = W1 + KIN * IW;
  const short* W3 = W2 + IW * IW;
  const float* b1 = bias;
  const float* b2 = b1 + IW;
  const float* b3 = b2 + IW;

  // A fragment of the normalized input: row lr, k = 4 lk .. 4 lk + 3
  bf16x4 xa;
  {
    const int64_t r = r0 + lr;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * lk + j;
      float x = 0.0f;
      if (r < rows && k < n_in) x = (X[r * n_in + k] - mu_in[k]) / sd_in[k];
      xa[j] = to_bf16(x);
    }
  }
  // layer 1: 16 column blocks, one k-step
#pragma unroll 4
  for (int nb = 0; nb < IW / 16; ++nb) {
    bf16x4 wbf;
#pragma unroll
    for (int j = 0; j < 4; ++j) wbf[j] = W1[(4 * lk + j) * IW + 16 * nb + lr];
    f4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xa, wbf, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) act[w][4 * lk + j][16 * nb + lr] = to_bf16(silu_f(acc[j] + b1[16 * nb + lr]));
  }
  __syncthreads();
  // layer 2: 16 column blocks x 16 k-steps; the result overwrites the activations after a barrier
  f4 acc2[IW / 16];
#pragma unroll
  for (int nb = 0; nb < IW / 16; ++nb) acc2[nb] = f4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < IW / 16; ++ks) {
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = act[w][lr][16 * ks + 4 * lk + j];
#pragma unroll
    for (int nb = 0; nb < IW / 16; ++nb) {
      bf16x4 wbf;
#pragma unroll
      for (int j = 0; j < 4; ++j) wbf[j] = W2[(16 * ks + 4 * lk + j) * IW + 16 * nb + lr];
      acc2[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wbf, acc2[nb], 0, 0, 0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < IW / 16; ++nb)
#pragma unroll
    for (int j = 0; j < 4; ++j) act[w][4 * lk + j][16 * nb + lr] = to_bf16(silu_f(acc2[nb][j] + b2[16 * nb + lr]));
  __syncthreads();
  // layer 3: one column block (n_out <= 16), 16 k-steps
  f4 acc3 = f4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < IW / 16; ++ks) {
    bf16x4 a, wbf;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = act[w][lr][16 * ks + 4 * lk + j];
      wbf[j] = W3[(16 * ks + 4 * lk + j) * NOUT + lr];
    }
    acc3 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wbf, acc3, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t r = r0 + 4 * lk + j;
    const int n = lr;
    if (r < rows && n < n_out) Y[r * n_out + n] = (acc3[j] + b3[n]) * sd_out[n] + mu_out[n];
  }
}

// bf16 copy of the weights in the inference kernel's padded layout, fp32 biases alongside
__global__ void pack_bf16_kernel(int64_t n_in, int64_t n_out, const float* __restrict__ p, short* __restrict__ Wb,
                                 float* __restrict__ bias) {
  const int64_t s1 = n_in * IW, s2 = s1 + IW, s3 = s2 + IW * IW, s4 = s3 + IW;
  const int64_t total = KIN * IW + IW * IW + IW * NOUT;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    float x = 0.0f;
    if (e < KIN * IW) {
      const int64_t k = e / IW, n = e % IW;
      if (k < n_in) x = p[k * IW + n];
    } else if (e < KIN * IW + IW * IW) {
      x = p[s2 + (e - KIN * IW)];
    } else {
      const int64_t f = e - KIN * IW - IW * IW, k = f / NOUT, n = f % NOUT;
      if (n < n_out) x = p[s4 + k * n_out + n];
    }
    Wb[e] = to_bf16(x);
  }
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * IW + NOUT; e += (int64_t)gridDim.x * blockDim.x) {
    float x = 0.0f;
    if (e < IW) x = p[s1 + e];
    else if (e < 2 * IW) x = p[s3 + (e - IW)];
    else if (e - 2 * IW < n_out) x = p[s4 + IW * n_out + (e - 2 * IW)];
    bias[e] = x;
  }
}

unsigned nblk(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (unsigned)b;
}

}  // namespace

// Scratch of the allocation-free FP32 forward pass: the activations of one call live in this
// file-scope device array (MLP_SCRATCH_FLOATS floats, 32 MiB), which every GPU the library runs on
// holds until the process ends.  In host code `scratch` is only a stand-in for the symbol, not a
// device address: kernels get the address that mlp_scratch_resolve looked up for the device.
static __device__ __align__(256) float scratch[MLP_SCRATCH_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float* scratch_at[MAX_DEVICES] = {};  // device address of `scratch` per device id, once resolved
}  // namespace

hipError_t mlp_scratch_resolve(float** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_at[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_at[dev] = static_cast<float*>(p);
  }
  *out = scratch_at[dev];
  return hipSuccess;
}

hipError_t mlp_sgemm(bool tA, bool tB, int epi, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                     const float* B, int64_t ldb, float* C, int64_t ldc, const float* bias, float* Z, int64_t ldz,
                     hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if ((M + BM - 1) / BM > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM));
#define SG(TA, TB, E) hipLaunchKernelGGL((sgemm_kernel<TA, TB, E>), grid, dim3(TPB), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, Z, ldz)
  if (!tA && !tB) {
    if (epi == 1) SG(false, false, 1); else if (epi == 2) SG(false, false, 2); else if (epi == 4) SG(false, false, 4);
    else SG(false, false, 0);
  } else if (tA && !tB) {
    SG(true, false, 0);
  } else if (!tA && tB) {
    if (epi == 3) SG(false, true, 3); else SG(false, true, 0);
  } else {
    return hipErrorInvalidValue;
  }
#undef SG
  return hipGetLastError();
}

hipError_t mlp_normalize(int64_t rows, int64_t cols, const float* X, const float* mu, const float* sd, float* Xn,
                         hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3(nblk(rows * cols)), dim3(TPB), 0, s, rows, cols, X, mu, sd, Xn);
  return hipGetLastError();
}

hipError_t mlp_denorm(int64_t rows, int64_t cols, const float* Yn, const float* mu, const float* sd, float* Y,
                      hipStream_t s) {
  hipLaunchKernelGGL(denorm_kernel, dim3(nblk(rows * cols)), dim3(TPB), 0, s, rows, cols, Yn, mu, sd, Y);
  return hipGetLastError();
}

hipError_t mlp_mse_grad(int64_t rows, int64_t cols, const float* Yn, const float* T, const float* mu, const float* sd,
                        float* dY, double* part, int64_t nparts, float* loss, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>(nparts, nblk(rows * cols));
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(TPB), 0, s, rows, cols, Yn, T, mu, sd, dY, part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(TPB), 0, s, (int64_t)nb, part, (double)(rows * cols), loss);
  return hipGetLastError();
}

hipError_t mlp_colsum(int64_t rows, int64_t cols, const float* D, float* out, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)cols), dim3(TPB), 0, s, rows, cols, D, out);
  return hipGetLastError();
}

hipError_t mlp_colstats(int64_t rows, int64_t cols, const float* D, float* mu, float* sd, hipStream_t s) {
  if (cols <= 0 || rows <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(colstats_kernel, dim3((unsigned)cols), dim3(TPB), 0, s, rows, cols, D, mu, sd);
  return hipGetLastError();
}

hipError_t mlp_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    int64_t step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(nblk(n)), dim3(TPB), 0, s, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_init(int64_t n_in, int64_t w, int64_t n_out, uint64_t seed, float* p, hipStream_t s) {
  const int64_t total = n_in * w + w + w * w + w + w * n_out + n_out;
  hipLaunchKernelGGL(init_kernel, dim3(nblk(total)), dim3(TPB), 0, s, n_in, w, n_out, seed, p);
  return hipGetLastError();
}

bool mlp_infer_supported(int64_t n_in, int64_t w, int64_t n_out) {
  return w == IW && n_in >= 1 && n_in <= KIN && n_out >= 1 && n_out <= NOUT;
}
int64_t mlp_bf16_weights(int64_t) { return KIN * IW + IW * IW + IW * NOUT; }
int64_t mlp_bf16_biases() { return 2 * IW + NOUT; }

hipError_t mlp_pack_bf16(int64_t n_in, int64_t n_out, const float* p, short* Wb, float* bias, hipStream_t s) {
  hipLaunchKernelGGL(pack_bf16_kernel, dim3(nblk(KIN * IW + IW * IW + IW * NOUT)), dim3(TPB), 0, s, n_in, n_out, p, Wb,
                     bias);
  return hipGetLastError();
}

hipError_t mlp_infer_bf16(int64_t rows, int64_t n_in, int64_t n_out, const float* X, const float* mu_in,
                          const float* sd_in, const short* Wb, const float* bias, const float* mu_out,
                          const float* sd_out, float* Y, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t nb = (rows + 63) / 64;
  if (nb > 2147483647LL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(infer_kernel, dim3((unsigned)nb), dim3(TPB), 0, s, rows, n_in, n_out, X, mu_in, sd_in, Wb, bias,
                     mu_out, sd_out, Y);
  return hipGetLastError();
}

}  // namespace thc
