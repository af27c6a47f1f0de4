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

// Position of C element (m, n) of one batch in the output layout of g.
__device__ inline int64_t c_offset(const Gemm& g, int64_t m, int64_t n) {
  if (g.cblk > 0)
    return ((m >> 4) * (g.ldc / g.cblk) + n / g.cblk) * 16 * g.cblk + (m & 15) * g.cblk + n % g.cblk;
  if (g.pair_rows)
    return g.xtile ? ((((n >> 6) * g.ldc + (m >> 1)) << 6) + (n & 63)) * 2 + (m & 1)
                   : ((m >> 1) * g.ldc + n) * 2 + (m & 1);
  return m * g.ldc + n;
}
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
  // XCD-aware tile order: workgroups are dispatched round-robin to the 8 XCDs (dispatch id
  // mod 8), so the dispatch id is remapped to give each XCD a contiguous range of tiles -- whole
  // rows of tiles, splits and batches, whose shared A and B panels then meet in one L2.
  const uint32_t nx = gridDim.x, nxy = gridDim.x * gridDim.y, total = nxy * gridDim.z;
  const uint32_t hw = blockIdx.x + nx * blockIdx.y + nxy * blockIdx.z;
  const uint32_t t8 = total & ~7u;
  const uint32_t lid = hw < t8 ? (hw & 7u) * (t8 >> 3) + (hw >> 3) : hw;
  const int64_t bz = lid / nxy;
  const int64_t b = bz / g.ksplit;
  const int split = (int)(bz % g.ksplit);
  int64_t m0 = (int64_t)((lid % nxy) / nx) * BM, n0 = (int64_t)(lid % nx) * BN;
  if (g.upper) {  // the grid enumerates the tiles (r, c) with r <= c only, row by row
    const int nt = (int)((g.N + BN - 1) / BN);
    int tr = (int)(lid % nxy), r = 0;
    while (tr >= nt - r) { tr -= nt - r; ++r; }
    m0 = (int64_t)r * BM;
    n0 = (int64_t)(r + tr) * BN;
  }
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
  const bool rd = C && g.beta != 0.0;
  // Epilogue by blocks of 16 rows: every load (C for beta, the Hadamard factor) of a block is
  // issued before its stores, so the loads overlap instead of waiting one by one behind stores
  // to possibly the same addresses.  Output element r of a lane: FP64 MFMA row lk + 4 r, FP32
  // MFMA row 4 lk + r; column lr.
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    int64_t off[TJ][4];
    double x[TJ][4];
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * WM + i * 16 + (F32 ? 4 * lk + r : lk + 4 * r);
        const int64_t n = n0 + wn * WN + j * 16 + lr;
        const bool ok = m < g.M && n < g.N;
        off[j][r] = ok ? c_offset(g, m, n) : -1;
        x[j][r] = g.alpha * (double)acc[i][j][r];
        if (H && ok) x[j][r] *= H[m * g.ldh + n];
        if (rd && ok) x[j][r] += g.beta * C[off[j][r]];
      }
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (off[j][r] < 0) continue;
        if (Cf) Cf[off[j][r]] = (float)x[j][r];  // FP32 output (beta is zero for it)
        else C[off[j][r]] = x[j][r];
      }
  }
}

// C = alpha sum_s W_s (times the Hadamard factor) + beta C for a product computed as ksplit
// partial products W_s (each batch x M x N, rows of N) in the workspace.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const Gemm g, const double* __restrict__ ws, int ns) {
  const int64_t MN = g.M * g.N, total = g.batch * MN;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int64_t b = idx / MN, r = idx - b * MN, m = r / g.N, n = r - m * g.N;
    double x = 0.0;
    for (int k = 0; k < ns; ++k) x += ws[k * total + idx];
    x *= g.alpha;
    if (g.hmul) x *= g.hmul[b * g.sH + m * g.ldh + n];
    const int64_t off = b * g.sC + c_offset(g, m, n);
    if (g.Cf) {
      g.Cf[off] = (float)x;
    } else {
      if (g.beta != 0.0) x += g.beta * g.C[off];
      g.C[off] = x;
    }
  }
}

template <int BM, int BN, bool F32>
hipError_t launch_tile(const Gemm& g, int64_t kchunk, hipStream_t s) {
  constexpr int OCC = 2;  // two workgroups per CU: one multiplies while the other loads
  static_assert(BM == BN, "square tiles (the upper mode walks a triangle of them)");
  const int64_t ntn = (g.N + BN - 1) / BN;
  dim3 grid((unsigned)(g.upper ? ntn * (ntn + 1) / 2 : ntn), (unsigned)(g.upper ? 1 : (g.M + BM - 1) / BM),
            (unsigned)(g.batch * g.ksplit));
  if ((uint64_t)grid.x * grid.y * grid.z >= (uint64_t(1) << 32)) return hipErrorInvalidValue;  // 32-bit tile ids
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
  // A batch that shares B and whose A, C (and Hadamard factor) blocks follow each other row by
  // row is one product with batch * M rows: fold it, so that it gets the large tiles.
  if (g.batch > 1 && g.sB == 0 && !g.transA && !g.upper && g.sA == g.M * g.lda && g.sC == g.M * g.ldc &&
      (!g.kscaleA || g.sksA == 0) && (!g.kscaleB || g.sksB == 0) && (!g.hmul || g.sH == g.M * g.ldh) &&
      (!g.pair_rows || g.M % 2 == 0) && !g.xtile && g.cblk == 0 && g.ksplit == 1) {
    g.M *= g.batch;
    g.batch = 1;
    g.sA = g.sC = g.sH = 0;
  }
  // Batches interleaved row by row (row m of batch b at m * batch + b) fold the same way.
  if (g.batch > 1 && g.sB == 0 && !g.transA && !g.pair_rows && !g.upper && g.cblk == 0 && g.ksplit == 1 &&
      g.sA >= g.K &&
      g.sC >= g.N &&
      g.lda == g.batch * g.sA && g.ldc == g.batch * g.sC && (!g.kscaleA || g.sksA == 0) &&
      (!g.kscaleB || g.sksB == 0) && (!g.hmul || (g.sH >= g.N && g.ldh == g.batch * g.sH))) {
    g.M *= g.batch;
    g.lda = g.sA;
    g.ldc = g.sC;
    if (g.hmul) g.ldh = g.sH;
    g.batch = 1;
    g.sA = g.sC = g.sH = 0;
  }
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.K <= 0) {
    // C = beta * C (or zero): run with an empty K range so the epilogue still applies.
    g.K = 0;
  }
  if ((g.C == nullptr) == (g.Cf == nullptr)) return hipErrorInvalidValue;  // exactly one output
  if ((g.xtile && !g.pair_rows) || g.cblk < 0 || (g.cblk > 0 && (g.pair_rows || g.ldc % g.cblk != 0)) ||
      (g.upper && g.M != g.N))
    return hipErrorInvalidValue;
  if (g.Cf && (g.beta != 0.0 || !g.f32)) return hipErrorInvalidValue;
  // Few output tiles and a long K: split K over more workgroups (about three per CU), partial
  // products in the workspace, then one reduction that applies the epilogue.
  if (g.ksplit == 1 && g.ws && g.K >= 256 && !g.upper) {
    const int64_t t64 = ((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch;
    if (t64 < 384) {
      const int64_t ns = std::min<int64_t>(std::min<int64_t>(g.K / 128, (768 + t64 - 1) / t64), 32);
      if (ns >= 2 && ns * g.batch * g.M * g.N <= g.ws_len && g.batch * ns <= 65535) {
        Gemm h = g;
        h.C = g.ws; h.ldc = g.N; h.sC = g.M * g.N; h.sSplit = g.batch * g.M * g.N;
        h.alpha = 1.0; h.beta = 0.0; h.hmul = nullptr; h.pair_rows = false; h.xtile = false; h.cblk = 0;
        h.Cf = nullptr;
        h.ksplit = (int)ns; h.ws = nullptr;
        hipError_t e = gemm_f64(h, s);
        if (e != hipSuccess) return e;
        const int64_t total = g.batch * g.M * g.N;
        const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, g, (const double*)g.ws, (int)ns);
        return hipGetLastError();
      }
    }
  }
  if (g.batch * g.ksplit > 65535) return hipErrorInvalidValue;
  int64_t kchunk = (g.K + g.ksplit - 1) / g.ksplit;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk == 0) kchunk = BK;
  const int64_t t128 = ((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch * g.ksplit;
  // 128 x 128 tiles need enough of them and a K long enough to amortize their prologue and
  // epilogue; short-K products run on 64 x 64 tiles, up to eight workgroups per CU
  const bool big = g.M >= 96 && g.N >= 96 && t128 >= 480 && kchunk > 64;
  if (big && (g.M + 127) / 128 > 65535) return hipErrorInvalidValue;
  if (!big && (g.M + 63) / 64 > 65535) return hipErrorInvalidValue;
  if (g.f32) return big ? launch_tile<128, 128, true>(g, kchunk, s) : launch_tile<64, 64, true>(g, kchunk, s);
  return big ? launch_tile<128, 128, false>(g, kchunk, s) : launch_tile<64, 64, false>(g, kchunk, s);
}

}  // namespace thc
