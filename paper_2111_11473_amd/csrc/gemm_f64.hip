// FP64 batched GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// Every dense rank-index contraction of the THC-CCSD residual (the Khatri-Rao panel
// products, the C T C^T chains, the ERI-core contractions) is a call of this kernel with a
// fused prologue (k-indexed scaling of either operand: the Hadamard "Form" steps whose
// factor depends on the contracted index) and a fused epilogue (elementwise product with a
// third matrix, alpha/beta accumulation).
//
// Tiling: a 256-thread workgroup (4 wave64s in a 2x2 grid) owns a BM x BN tile of C and
// walks K in steps of 16 through LDS.  Each wave owns a (BM/2) x (BN/2) sub-tile held as
// (BM/32) x (BN/32) MFMA accumulators of 16x16 doubles.  The next K-slab is prefetched into
// registers while the current one is multiplied.  Ragged M, N, K are handled by
// zero-filled loads and masked stores, so no operand needs padding.
#include <type_traits>

#include "internal.h"

namespace thc {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BK = 16;
constexpr int PAD = 1;  // odd LDS row pitch: conflict-free transposing stores

// F32: operands rounded to FP32 on their way into LDS, v_mfma_f32_16x16x4f32 with FP32
// accumulation (the mixed-precision path); otherwise FP64 throughout.
template <int BM, int BN, bool TA, bool TB, bool F32>
__global__ __launch_bounds__(256) void dgemm_kernel(const Gemm g, const int64_t kchunk) {
  using TL = typename std::conditional<F32, float, double>::type;
  using ACC = typename std::conditional<F32, flt4, dbl4>::type;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TI = WM / 16, TJ = WN / 16;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  __shared__ TL As[BK][BM + PAD];
  __shared__ TL Bs[BK][BN + PAD];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t bz = blockIdx.z;
  const int64_t b = bz / g.ksplit;
  const int split = (int)(bz % g.ksplit);
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = (kbeg + kchunk < g.K) ? kbeg + kchunk : g.K;

  const double* __restrict__ A = g.A + b * g.sA;
  const double* __restrict__ B = g.B + b * g.sB;
  const double* __restrict__ sa = g.kscaleA ? g.kscaleA + b * g.sksA : nullptr;
  const double* __restrict__ sb = g.kscaleB ? g.kscaleB + b * g.sksB : nullptr;

  double ra[NA], rb[NB];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      int mm, kk;
      if (TA) { mm = t % BM; kk = t / BM + (256 / BM) * r; }
      else    { kk = t % BK; mm = t / BK + 16 * r; }
      const int64_t m = m0 + mm, k = k0 + kk;
      double x = 0.0;
      if (m < g.M && k < kend) {
        x = TA ? A[k * g.lda + m] : A[m * g.lda + k];
        if (sa) x *= sa[k * g.ksA];
      }
      ra[r] = x;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      int nn, kk;
      if (TB) { kk = t % BK; nn = t / BK + 16 * r; }
      else    { nn = t % BN; kk = t / BN + (256 / BN) * r; }
      const int64_t n = n0 + nn, k = k0 + kk;
      double x = 0.0;
      if (n < g.N && k < kend) {
        x = TB ? B[n * g.ldb + k] : B[k * g.ldb + n];
        if (sb) x *= sb[k * g.ksB];
      }
      rb[r] = x;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      int mm, kk;
      if (TA) { mm = t % BM; kk = t / BM + (256 / BM) * r; }
      else    { kk = t % BK; mm = t / BK + 16 * r; }
      As[kk][mm] = (TL)ra[r];
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      int nn, kk;
      if (TB) { kk = t % BK; nn = t / BK + 16 * r; }
      else    { nn = t % BN; kk = t / BN + (256 / BN) * r; }
      Bs[kk][nn] = (TL)rb[r];
    }
  };

  ACC acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = ACC{0, 0, 0, 0};

  const int lr = lane & 15, lk = lane >> 4;
  if (kbeg < kend) load(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TL af[TI], bf[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) af[i] = As[kk + lk][wm * WM + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bf[j] = Bs[kk + lk][wn * WN + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          if constexpr (F32)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  double* __restrict__ C = g.C ? g.C + b * g.sC + (int64_t)split * g.sSplit : nullptr;
  float* __restrict__ Cf = g.Cf ? g.Cf + b * g.sC + (int64_t)split * g.sSplit : nullptr;
  const double* __restrict__ H = g.hmul ? g.hmul + b * g.sH : nullptr;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // output element r of a lane: FP64 MFMA row lk + 4 r, FP32 MFMA row 4 lk + r; column lr
        const int64_t m = m0 + wm * WM + i * 16 + (F32 ? 4 * lk + r : lk + 4 * r);
        const int64_t n = n0 + wn * WN + j * 16 + lr;
        if (m < g.M && n < g.N) {
          double x = g.alpha * (double)acc[i][j][r];
          if (H) x *= H[m * g.ldh + n];
          const int64_t off = g.pair_rows ? ((m >> 1) * g.ldc + n) * 2 + (m & 1) : m * g.ldc + n;
          if (Cf) {
            Cf[off] = (float)x;  // FP32 output (beta is zero for it)
          } else {
            if (g.beta != 0.0) x += g.beta * C[off];
            C[off] = x;
          }
        }
      }
}

template <int BM, int BN, bool F32>
hipError_t launch_tile(const Gemm& g, int64_t kchunk, hipStream_t s) {
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM),
            (unsigned)(g.batch * g.ksplit));
  if (!g.transA && !g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, false, false, F32>), grid, dim3(256), 0, s, g, kchunk);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, true, false, F32>), grid, dim3(256), 0, s, g, kchunk);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, false, true, F32>), grid, dim3(256), 0, s, g, kchunk);
  else hipLaunchKernelGGL((dgemm_kernel<BM, BN, true, true, F32>), grid, dim3(256), 0, s, g, kchunk);
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_f64(const Gemm& g0, hipStream_t s) {
  Gemm g = g0;
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.batch * g.ksplit > 65535) return hipErrorInvalidValue;
  if (g.K <= 0) {
    // C = beta * C (or zero): run with an empty K range so the epilogue still applies.
    g.K = 0;
  }
  int64_t kchunk = (g.K + g.ksplit - 1) / g.ksplit;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk == 0) kchunk = BK;
  const int64_t t128 = ((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch * g.ksplit;
  if ((g.C == nullptr) == (g.Cf == nullptr)) return hipErrorInvalidValue;  // exactly one output
  if (g.Cf && (g.beta != 0.0 || !g.f32)) return hipErrorInvalidValue;
  const bool big = g.M >= 96 && g.N >= 96 && t128 >= 480;
  if (big && (g.M + 127) / 128 > 65535) return hipErrorInvalidValue;
  if (!big && (g.M + 63) / 64 > 65535) return hipErrorInvalidValue;
  if (g.f32) return big ? launch_tile<128, 128, true>(g, kchunk, s) : launch_tile<64, 64, true>(g, kchunk, s);
  return big ? launch_tile<128, 128, false>(g, kchunk, s) : launch_tile<64, 64, false>(g, kchunk, s);
}

}  // namespace thc
