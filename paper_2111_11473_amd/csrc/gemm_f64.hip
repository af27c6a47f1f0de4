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
  if (g.cblk > 0) {  // cblk is a power of two (checked on the host): shifts and masks
    const int sh = __builtin_ctz((unsigned)g.cblk);
    return ((((m >> 4) * (g.ldc >> sh) + (n >> sh)) << 4) + (m & 15)) * g.cblk + (n & (g.cblk - 1));
  }
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

// Tile of this workgroup.  XCD-aware order: workgroups are dispatched round-robin to the 8 XCDs
// (dispatch id mod 8), so the dispatch id is remapped to give each XCD a contiguous range of
// tiles -- whole rows of tiles, splits and batches, whose shared A and B panels then meet in one
// L2.  In the upper mode the grid enumerates the tiles (r, c) with r <= c only, row by row.
struct TileId {
  int64_t b, m0, n0;
  int split;
};
template <int BM, int BN>
__device__ inline TileId tile_id(const Gemm& g) {
  const uint32_t nx = gridDim.x, nxy = gridDim.x * gridDim.y, total = nxy * gridDim.z;
  const uint32_t hw = blockIdx.x + nx * blockIdx.y + nxy * blockIdx.z;
  const uint32_t t8 = total & ~7u;
  const uint32_t lid = hw < t8 ? (hw & 7u) * (t8 >> 3) + (hw >> 3) : hw;
  const int64_t bz = lid / nxy;
  TileId id;
  id.b = bz / g.ksplit;
  id.split = (int)(bz % g.ksplit);
  id.m0 = (int64_t)((lid % nxy) / nx) * BM;
  id.n0 = (int64_t)(lid % nx) * BN;
  if (g.upper) {
    const int nt = (int)((g.N + BN - 1) / BN);
    int tr = (int)(lid % nxy), r = 0;
    while (tr >= nt - r) { tr -= nt - r; ++r; }
    id.m0 = (int64_t)r * BM;
    id.n0 = (int64_t)(r + tr) * BN;
  }
  return id;
}

// Epilogue by blocks of 16 rows: every load (C for beta, the Hadamard factor) of a block is
// issued before its stores, so the loads overlap instead of waiting one by one behind stores
// to possibly the same addresses.  acc[i][j][r] is output element r of the lane in 16 x 16
// block (i, j) of the wave's (WM x WN) patch at (wm0, wn0): row lk + 4 r for the FP64 MFMA
// (ROW4 false), row 4 lk + r for the FP32-accumulating ones; column lr.
template <int TI, int TJ, bool ROW4, typename ACC>
__device__ inline void epilogue(const Gemm& g, const TileId& id, int64_t wm0, int64_t wn0, int lr, int lk,
                                const ACC (&acc)[TI][TJ]) {
  double* __restrict__ C = g.C ? g.C + id.b * g.sC + (int64_t)id.split * g.sSplit : nullptr;
  float* __restrict__ Cf = g.Cf ? g.Cf + id.b * g.sC + (int64_t)id.split * g.sSplit : nullptr;
  const double* __restrict__ H = g.hmul ? g.hmul + id.b * g.sH : nullptr;
  const bool rd = C && g.beta != 0.0;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    int64_t off[TJ][4];
    double x[TJ][4];
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = id.m0 + wm0 + i * 16 + (ROW4 ? 4 * lk + r : lk + 4 * r);
        const int64_t n = id.n0 + wn0 + j * 16 + lr;
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

// F32: operands rounded to FP32 on their way into LDS, v_mfma_f32_16x16x4f32 with FP32
// accumulation (the mixed-precision path); otherwise FP64 throughout.
//
// Loads are branch-free: an element outside the matrix is read from the tile origin (always
// inside) and replaced by zero when it is written to LDS, and the k-indexed scaling is applied
// there too, so the global loads of the next slab are all in flight while the current slab is
// multiplied.  Two LDS buffers: one barrier per slab.  Per-thread offsets are 32-bit, relative
// to a per-tile base pointer.
// SHORT (K of at most four slabs): the loads of every slab are issued at once, so a tile waits
// for memory once rather than once per slab; the slabs then pass through the two LDS buffers.
template <int BM, int BN, bool TA, bool TB, bool F32, int OCC, bool SHORT>
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
  const TileId id = tile_id<BM, BN>(g);
  const int64_t b = id.b, m0 = id.m0, n0 = id.n0;
  const int split = id.split;
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
    // scale factors through buffer loads too: a generic (flat) load would also count against the
    // LDS wait before the slab's first product
    rsa = bload(rsrc(sa), ka < kl ? (uint32_t)(8 * (k0 + ka) * ksa) : OOB);
    rsb = bload(rsrc(sb), kb < kl ? (uint32_t)(8 * (k0 + kb) * ksb) : OOB);
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
  // nk: how many k of the slab hold data (the rest are zeros); k-steps of 4 past them are skipped
  auto compute = [&](int buf, int nk = BK) {
    // a wave with products ready issues before one that is loading (measured +2 to +5% on the
    // large products, +40% on long split-K ones; the short-K path, bound by its stores, lost 3%)
    if constexpr (!SHORT) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      if (kk >= nk) break;
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
    if constexpr (!SHORT) __builtin_amdgcn_s_setprio(0);
  };
  const int nslab = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
  if constexpr (SHORT) {
    // all four slabs, branch-free: a slab past the end of K reads as zeros (every offset out of
    // range) and adds nothing
    constexpr int NSL = 4;
    double pa[NSL][NA], pb[NSL][NB], psa[NSL], psb[NSL];
#pragma unroll
    for (int q = 0; q < NSL; ++q) {
      load(kbeg + q * BK);
#pragma unroll
      for (int r = 0; r < NA; ++r) pa[q][r] = ra[r];
#pragma unroll
      for (int r = 0; r < NB; ++r) pb[q][r] = rb[r];
      psa[q] = rsa;
      psb[q] = rsb;
    }
    // slab q goes to buffer q % 2 once the barrier after slab q - 2's product has passed; only
    // the k-steps that hold data are multiplied
#pragma unroll
    for (int q = 0; q < NSL; ++q) {
      if (q >= nslab) break;
#pragma unroll
      for (int r = 0; r < NA; ++r) ra[r] = pa[q][r];
#pragma unroll
      for (int r = 0; r < NB; ++r) rb[r] = pb[q][r];
      rsa = psa[q];
      rsb = psb[q];
      store(q & 1);
      if (q > 0) compute((q - 1) & 1);
      __syncthreads();
    }
    if (nslab > 0) compute((nslab - 1) & 1, (int)(kend - kbeg) - BK * (nslab - 1));
  } else {
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
  }

  epilogue<TI, TJ, F32>(g, id, wm * WM, wn * WN, lr, lk, acc);
}

// Split-BF16 products (the compensated mode of the mixed-precision path): every operand is
// rounded to FP32 and split into three bf16 pieces by truncation -- hi (its top 16 bits), mid (the
// top 16 bits of the remainder) and lo (what is left, at most 8 significant bits, so exact):
// x = hi + mid + lo exactly.  Each product is the six terms down to second order in the pieces,
// mid mid + hi lo + lo hi + hi mid + mid hi + hi hi (smallest first), on
// v_mfma_f32_16x16x16bf16_1k with FP32 accumulation; the dropped terms (mid lo, lo mid, lo lo)
// are O(2^-24) relative, the FP32 product's own rounding.  A thread loads packets of 4
// consecutive k of one row, scales them, splits them and stores the three packets (8 bytes each)
// to LDS, where a lane's MFMA fragment (row lr, k = 4 lk .. 4 lk + 3) is one packet.  One 16-k slab is one MFMA k-step; tiles, double
// buffering, the XCD-aware order and the epilogue are those of the FP64/FP32 kernel.
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

// hi / mid / lo bf16 pieces of two FP32 values, each piece packed two to a dword (element 0 in
// the low half).  Both subtractions are exact: each removes the leading bits of its operand.
__device__ inline void split_pair(float x0, float x1, uint32_t& hi, uint32_t& mi, uint32_t& lo) {
  const uint32_t h0 = __builtin_bit_cast(uint32_t, x0) & 0xFFFF0000u;
  const uint32_t h1 = __builtin_bit_cast(uint32_t, x1) & 0xFFFF0000u;
  const float r0 = x0 - __builtin_bit_cast(float, h0), r1 = x1 - __builtin_bit_cast(float, h1);
  const uint32_t m0 = __builtin_bit_cast(uint32_t, r0) & 0xFFFF0000u;
  const uint32_t m1 = __builtin_bit_cast(uint32_t, r1) & 0xFFFF0000u;
  const float q0 = r0 - __builtin_bit_cast(float, m0), q1 = r1 - __builtin_bit_cast(float, m1);
  hi = (h0 >> 16) | h1;
  mi = (m0 >> 16) | m1;
  lo = (__builtin_bit_cast(uint32_t, q0) >> 16) | (__builtin_bit_cast(uint32_t, q1) & 0xFFFF0000u);
}

template <int BM, int BN, bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void bgemm_kernel(const Gemm g, const int64_t kchunk) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TI = WM / 16, TJ = WN / 16;
  constexpr int QA = BM / 64, QB = BN / 64;  // packets (4 k of one row) per thread and slab
  // LDS: [buffer][hi, mid, lo][k / 4][row] packets; rows padded so that the four k / 4 planes a
  // wave reads at once sit 32 banks apart
  __shared__ u2 As[2][3][4][BM + 16];
  __shared__ u2 Bs[2][3][4][BN + 16];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const TileId id = tile_id<BM, BN>(g);
  const int64_t b = id.b, m0 = id.m0, n0 = id.n0;
  const int64_t kbeg = (int64_t)id.split * kchunk;
  const int64_t kend = (kbeg + kchunk < g.K) ? kbeg + kchunk : g.K;

  const double* __restrict__ A = g.A + b * g.sA + (TA ? m0 : m0 * g.lda);
  const double* __restrict__ B = g.B + b * g.sB + (TB ? n0 * g.ldb : n0);
  const double* __restrict__ sa = g.kscaleA ? g.kscaleA + b * g.sksA : &kOne;
  const double* __restrict__ sb = g.kscaleB ? g.kscaleB + b * g.sksB : &kOne;
  const int64_t ksa = g.kscaleA ? g.ksA : 0, ksb = g.kscaleB ? g.ksB : 0;
  const uint32_t lda = (uint32_t)g.lda, ldb = (uint32_t)g.ldb;
  const int mlim = (int)((g.M - m0 < BM) ? g.M - m0 : BM);
  const int nlim = (int)((g.N - n0 < BN) ? g.N - n0 : BN);
  constexpr uint32_t OOB = 0x80000000u;

  // packet q of this thread: row (column) and k / 4 within the slab; consecutive lanes read
  // consecutive addresses (a k-fastest operand: 4 lanes per row; an m/n-fastest one: a row per k)
  int am[QA], aq[QA], bn[QB], bq[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int p = t + 256 * q;
    am[q] = TA ? p % BM : p >> 2;
    aq[q] = TA ? p / BM : p & 3;
  }
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int p = t + 256 * q;
    bn[q] = TB ? p >> 2 : p % BN;
    bq[q] = TB ? p & 3 : p / BN;
  }

  double ra[QA][4], rb[QB][4], rsa[QA][4], rsb[QB][4];
  auto load = [&](int64_t k0) {
    const int kl = (int)(kend - k0);
    const __amdgpu_buffer_rsrc_t rA = rsrc(A + (TA ? k0 * g.lda : k0));
    const __amdgpu_buffer_rsrc_t rB = rsrc(B + (TB ? k0 : k0 * g.ldb));
    const __amdgpu_buffer_rsrc_t rSa = rsrc(sa), rSb = rsrc(sb);
#pragma unroll
    for (int q = 0; q < QA; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * aq[q] + e;
        const uint32_t off = 8u * (TA ? (uint32_t)k * lda + (uint32_t)am[q] : (uint32_t)am[q] * lda + (uint32_t)k);
        ra[q][e] = bload(rA, (am[q] < mlim && k < kl) ? off : OOB);
        rsa[q][e] = bload(rSa, (uint32_t)(8 * (k0 + (k < kl ? k : 0)) * ksa));
      }
#pragma unroll
    for (int q = 0; q < QB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * bq[q] + e;
        const uint32_t off = 8u * (TB ? (uint32_t)bn[q] * ldb + (uint32_t)k : (uint32_t)k * ldb + (uint32_t)bn[q]);
        rb[q][e] = bload(rB, (bn[q] < nlim && k < kl) ? off : OOB);
        rsb[q][e] = bload(rSb, (uint32_t)(8 * (k0 + (k < kl ? k : 0)) * ksb));
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      uint32_t h0, m0, l0, h1, m1, l1;
      split_pair((float)(ra[q][0] * rsa[q][0]), (float)(ra[q][1] * rsa[q][1]), h0, m0, l0);
      split_pair((float)(ra[q][2] * rsa[q][2]), (float)(ra[q][3] * rsa[q][3]), h1, m1, l1);
      As[buf][0][aq[q]][am[q]] = u2{h0, h1};
      As[buf][1][aq[q]][am[q]] = u2{m0, m1};
      As[buf][2][aq[q]][am[q]] = u2{l0, l1};
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      uint32_t h0, m0, l0, h1, m1, l1;
      split_pair((float)(rb[q][0] * rsb[q][0]), (float)(rb[q][1] * rsb[q][1]), h0, m0, l0);
      split_pair((float)(rb[q][2] * rsb[q][2]), (float)(rb[q][3] * rsb[q][3]), h1, m1, l1);
      Bs[buf][0][bq[q]][bn[q]] = u2{h0, h1};
      Bs[buf][1][bq[q]][bn[q]] = u2{m0, m1};
      Bs[buf][2][bq[q]][bn[q]] = u2{l0, l1};
    }
  };

  flt4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = flt4{0, 0, 0, 0};

  const int lr = lane & 15, lk = lane >> 4;
  auto compute = [&](int buf) {
    bf4 ah[TI], am_[TI], al[TI], bh[TJ], bm[TJ], bl[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      ah[i] = __builtin_bit_cast(bf4, As[buf][0][lk][wm * WM + i * 16 + lr]);
      am_[i] = __builtin_bit_cast(bf4, As[buf][1][lk][wm * WM + i * 16 + lr]);
      al[i] = __builtin_bit_cast(bf4, As[buf][2][lk][wm * WM + i * 16 + lr]);
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      bh[j] = __builtin_bit_cast(bf4, Bs[buf][0][lk][wn * WN + j * 16 + lr]);
      bm[j] = __builtin_bit_cast(bf4, Bs[buf][1][lk][wn * WN + j * 16 + lr]);
      bl[j] = __builtin_bit_cast(bf4, Bs[buf][2][lk][wn * WN + j * 16 + lr]);
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am_[i], bm[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bm[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am_[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
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
  for (int sl = 1; sl < nslab; ++sl) {
    load(k0 + BK);
    compute(buf);
    store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    k0 += BK;
  }
  if (nslab > 0) compute(buf);

  epilogue<TI, TJ, true>(g, id, wm * WM, wn * WN, lr, lk, acc);
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

bool slab_offsets_fit(const Gemm& g, int BM, int BN) {
  const int64_t la = 8 * (g.transA ? (int64_t)BK * g.lda + BM : (int64_t)BM * g.lda + BK);
  const int64_t lb = 8 * (g.transB ? (int64_t)BN * g.ldb + BK : (int64_t)BK * g.ldb + BN);
  return la < (int64_t(1) << 31) && lb < (int64_t(1) << 31);
}

template <int BM, int BN, bool F32, bool SHORT = false>
hipError_t launch_tile(const Gemm& g, int64_t kchunk, hipStream_t s) {
  constexpr int OCC = 2;  // two workgroups per CU: one multiplies while the other loads
  static_assert(BM == BN, "square tiles (the upper mode walks a triangle of them)");
  const int64_t ntn = (g.N + BN - 1) / BN;
  dim3 grid((unsigned)(g.upper ? ntn * (ntn + 1) / 2 : ntn), (unsigned)(g.upper ? 1 : (g.M + BM - 1) / BM),
            (unsigned)(g.batch * g.ksplit));
  if ((uint64_t)grid.x * grid.y * grid.z >= (uint64_t(1) << 32)) return hipErrorInvalidValue;  // 32-bit tile ids
  // byte offsets within a slab stay below 2^31 (the buffer range): a slab spans BK rows of a
  // k-major operand, or BM (BN) rows of an m- (n-) major one
  if (!slab_offsets_fit(g, BM, BN)) return hipErrorInvalidValue;
  if (!g.transA && !g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, false, false, F32, OCC, SHORT>), grid, dim3(256), 0, s, g, kchunk);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, true, false, F32, OCC, SHORT>), grid, dim3(256), 0, s, g, kchunk);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((dgemm_kernel<BM, BN, false, true, F32, OCC, SHORT>), grid, dim3(256), 0, s, g, kchunk);
  else hipLaunchKernelGGL((dgemm_kernel<BM, BN, true, true, F32, OCC, SHORT>), grid, dim3(256), 0, s, g, kchunk);
  return hipGetLastError();
}

template <int BM, int BN>
hipError_t launch_btile(const Gemm& g, int64_t kchunk, hipStream_t s) {
  const int64_t ntn = (g.N + BN - 1) / BN;
  dim3 grid((unsigned)(g.upper ? ntn * (ntn + 1) / 2 : ntn), (unsigned)(g.upper ? 1 : (g.M + BM - 1) / BM),
            (unsigned)(g.batch * g.ksplit));
  if ((uint64_t)grid.x * grid.y * grid.z >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
  if (!slab_offsets_fit(g, BM, BN)) return hipErrorInvalidValue;
  if (!g.transA && !g.transB) hipLaunchKernelGGL((bgemm_kernel<BM, BN, false, false>), grid, dim3(256), 0, s, g, kchunk);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((bgemm_kernel<BM, BN, true, false>), grid, dim3(256), 0, s, g, kchunk);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((bgemm_kernel<BM, BN, false, true>), grid, dim3(256), 0, s, g, kchunk);
  else hipLaunchKernelGGL((bgemm_kernel<BM, BN, true, true>), grid, dim3(256), 0, s, g, kchunk);
  return hipGetLastError();
}

// 128 x 128 tiles need enough of them and a K slice long enough to amortize their prologue and
// epilogue; short-K products run on 64 x 64 tiles, up to eight workgroups per CU.
bool big_tiles(const Gemm& g, int64_t kchunk) {
  const int64_t t128 = ((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch * g.ksplit;
  return g.M >= 96 && g.N >= 96 && t128 >= 480 && kchunk > 64;
}

}  // namespace

int gemm_tile_edge_split(const Gemm& g) {
  const int64_t ks = g.ksplit < 1 ? 1 : g.ksplit;
  int64_t kchunk = (g.K + ks - 1) / ks;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk == 0) kchunk = BK;
  Gemm h = g;
  h.ksplit = (int)ks;
  return big_tiles(h, kchunk) ? 128 : 64;
}

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
  if ((g.xtile && !g.pair_rows) || g.cblk < 0 ||
      (g.cblk > 0 && (g.pair_rows || (g.cblk & (g.cblk - 1)) != 0 || g.ldc % g.cblk != 0)) ||
      (g.upper && g.M != g.N))
    return hipErrorInvalidValue;
  // k-scale factors are read through 32-bit byte offsets
  if ((g.kscaleA && 8 * g.K * g.ksA >= (int64_t(1) << 31)) || (g.kscaleB && 8 * g.K * g.ksB >= (int64_t(1) << 31)))
    return hipErrorInvalidValue;
  if (g.Cf && (g.beta != 0.0 || !(g.f32 || g.bf16x3))) return hipErrorInvalidValue;
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
  const bool big = big_tiles(g, kchunk);
  if (big && (g.M + 127) / 128 > 65535) return hipErrorInvalidValue;
  if (!big && (g.M + 63) / 64 > 65535) return hipErrorInvalidValue;
  if (g.bf16x3) return big ? launch_btile<128, 128>(g, kchunk, s) : launch_btile<64, 64>(g, kchunk, s);
  const bool shortk = kchunk <= 4 * BK;
  if (g.f32) {
    if (big) return launch_tile<128, 128, true>(g, kchunk, s);
    return shortk ? launch_tile<64, 64, true, true>(g, kchunk, s) : launch_tile<64, 64, true>(g, kchunk, s);
  }
  if (big) return launch_tile<128, 128, false>(g, kchunk, s);
  return shortk ? launch_tile<64, 64, false, true>(g, kchunk, s) : launch_tile<64, 64, false>(g, kchunk, s);
}

}  // namespace thc
