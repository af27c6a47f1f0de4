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
// zero-filled LDS tiles and masked stores, so no operand needs padding.
#include <type_traits>

#include "internal.h"

namespace thc {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BK = 16;
__device__ const double kOne = 1.0;
constexpr int RSRC_W3 = 0x00020000;  // raw 32-bit buffer access

// A buffer of 2 GiB from base (uniform across the wave): byte offsets at or beyond 2^31 read
// as zero.
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const double* base) {
  const uint64_t a = (uint64_t)base;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(hi << 32 | lo), (short)0, (int)0x80000000u, RSRC_W3);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0u, 0));
}

// F32: operands rounded to FP32 on their way into LDS, v_mfma_f32_16x16x4f32 with FP32
// accumulation (the mixed-precision path); otherwise FP64 throughout.
//
// Loads are branch-free: an element outside the matrix is read from the tile origin (always
// inside) and replaced by zero when it is written to LDS, and the k-indexed scaling is applied
// there too, so the global loads of the next slab are all in flight while the current slab is
// multiplied.  Two LDS buffers: one barrier per slab.  Per-thread offsets are 32-bit, relative
// to a per-tile base pointer.
template <int BM, int BN, bool TA, bool TB, bool F32, int OCC>
__global__ __launch_bounds__(256, OCC) void dgemm_kernel(const Gemm g, const int64_t kchunk) {
  using TL = typename std::conditional<F32, float, double>::type;
  using ACC = typename std::conditional<F32, flt4, dbl4>::type;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TI = WM / 16, TJ = WN / 16;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  // LDS row pitch: an operand stored k-fastest is transposed on its way in (odd pitch: the 16
  // k-rows a wave writes fall on distinct banks); one stored m- or n-fastest is copied row by
  // row (pitch of 32 banks mod 64: consecutive k-rows on opposite halves of the banks)
  constexpr int PA = BM + (TA ? 16 : 1), PB = BN + (TB ? 1 : 16);
  __shared__ TL As[2][BK][PA];
  __shared__ TL Bs[2][BK][PB];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t bz = blockIdx.z;
  const int64_t b = bz / g.ksplit;
  const int split = (int)(bz % g.ksplit);
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = (kbeg + kchunk < g.K) ? kbeg + kchunk : g.K;

  // tile origins (row m0 / column n0, k = 0)
  const double* __restrict__ A = g.A + b * g.sA + (TA ? m0 : m0 * g.lda);
  const double* __restrict__ B = g.B + b * g.sB + (TB ? n0 * g.ldb : n0);
  // an absent k-scaling reads the constant 1 with stride 0, so the slab code has no branches
  const double* __restrict__ sa = g.kscaleA ? g.kscaleA + b * g.sksA : &kOne;
  const double* __restrict__ sb = g.kscaleB ? g.kscaleB + b * g.sksB : &kOne;
  const int64_t ksa = g.kscaleA ? g.ksA : 0, ksb = g.kscaleB ? g.ksB : 0;
  const uint32_t lda = (uint32_t)g.lda, ldb = (uint32_t)g.ldb;
  const int mlim = (int)((g.M - m0 < BM) ? g.M - m0 : BM);  // rows / columns of this tile inside C
  const int nlim = (int)((g.N - n0 < BN) ? g.N - n0 : BN);

  // This thread's share of a slab: one k (ka, kb) and NA rows mm = ma + sma r of the A tile,
  // NB columns nn = nb + snb r of the B tile; consecutive lanes read consecutive addresses.
  const int ka = TA ? t >> 4 : t & 15, ma = TA ? t & 15 : t >> 4;
  const int kb = TB ? t & 15 : t >> 4, nb = TB ? t >> 4 : t & 15;
  constexpr int SMA = 16, SNB = 16;

  // Operand elements come through buffer loads from the slab origin: an element outside the
  // matrix gets an offset beyond the buffer's range, which the hardware reads as zero.
  constexpr uint32_t OOB = 0x80000000u;
  const uint32_t aoff = 8u * (TA ? (uint32_t)ka * lda + (uint32_t)ma : (uint32_t)ma * lda + (uint32_t)ka);
  const uint32_t boff = 8u * (TB ? (uint32_t)nb * ldb + (uint32_t)kb : (uint32_t)kb * ldb + (uint32_t)nb);
  const uint32_t astep = 8u * SMA * (TA ? 1u : lda), bstep = 8u * SNB * (TB ? ldb : 1u);

  double ra[NA], rb[NB], rsa, rsb;

  auto load = [&](int64_t k0) {
    const int kl = (int)(kend - k0);  // valid k within this slab: k < kl
    const __amdgpu_buffer_rsrc_t rA = rsrc(A + (TA ? k0 * g.lda : k0));
    const __amdgpu_buffer_rsrc_t rB = rsrc(B + (TB ? k0 : k0 * g.ldb));
#pragma unroll
    for (int r = 0; r < NA; ++r)
      ra[r] = bload(rA, (ka < kl && ma + SMA * r < mlim) ? aoff + astep * r : OOB);
#pragma unroll
    for (int r = 0; r < NB; ++r)
      rb[r] = bload(rB, (kb < kl && nb + SNB * r < nlim) ? boff + bstep * r : OOB);
    rsa = sa[(k0 + (ka < kl ? ka : 0)) * ksa];
    rsb = sb[(k0 + (kb < kl ? kb : 0)) * ksb];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NA; ++r) As[buf][ka][ma + SMA * r] = (TL)(ra[r] * rsa);
#pragma unroll
    for (int r = 0; r < NB; ++r) Bs[buf][kb][nb + SNB * r] = (TL)(rb[r] * rsb);
  };

  ACC acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = ACC{0, 0, 0, 0};

  const int lr = lane & 15, lk = lane >> 4;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TL af[TI], bf[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) af[i] = As[buf][kk + lk][wm * WM + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bf[j] = Bs[buf][kk + lk][wn * WN + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          if constexpr (F32)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  };
  const int nslab = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
  if (nslab > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  int64_t k0 = kbeg;
  for (int sl = 1; sl < nslab; ++sl) {  // slab sl - 1 is multiplied while slab sl is fetched
    load(k0 + BK);
    compute(buf);
    store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    k0 += BK;
  }
  if (nslab > 0) compute(buf);

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
  constexpr int OCC = 2;  // two workgroups per CU: one multiplies while the other loads
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM),
            (unsigned)(g.batch * g.ksplit));
  // byte offsets within a slab stay below 2^31 (the buffer range)
  const int64_t la = 8 * (BM + BK) * g.lda, lb = 8 * (BN + BK) * g.ldb;
  if (la >= (int64_t(1) << 31) || lb >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  if (!g.transA && !g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, false, false, F32, OCC>), grid, dim3(256), 0, s, g, kchunk);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, true, false, F32, OCC>), grid, dim3(256), 0, s, g, kchunk);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, false, true, F32, OCC>), grid, dim3(256), 0, s, g, kchunk);
  else hipLaunchKernelGGL((dgemm_kernel<BM, BN, true, true, F32, OCC>), grid, dim3(256), 0, s, g, kchunk);
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
