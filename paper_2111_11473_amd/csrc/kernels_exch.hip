// Exchange contraction of the T2^2 ring algorithm (paper Alg. 7, Eq. 37 exchange part), fused:
//   Gt^X[i][I] = sum_J xo[i][J] z[I][J] sum_k xo[k][I] Rx^X[k][J]
// for every X of a block.  Written as two products it materialises the Q x Q matrix
// F^X = z o (xo^T Rx^X) for each X; here F never leaves the chip.
//
// A workgroup (4 waves) owns one X and a tile of 64 I (16 per wave) and walks J in blocks of 16.
// Per J block each wave forms the transposed block Ft[J][I] = sum_k Rx[k][J] xo[k][I] with FP64
// MFMA (16x16x4, K = o), scales it by z[I][J] in registers, and feeds it directly as the B
// operand of the second product Gt[i][I] += sum_J xo[i][J] Ft[J][I]: in the MFMA register
// layout, output element r of a lane (row lane/16 + 4 r, column lane % 16) is exactly the lane's
// B element of k-step r (row lane/16, column lane % 16 of rows 4 r .. 4 r + 3).  The o x 16
// slices of Rx^X and xo and the 64 x 16 slice of z for the next J block are prefetched into
// registers while the current one is used from LDS.
// The slices are fetched with buffer loads whose out-of-range lanes read zero (k >= o, J >= Q,
// I >= Q), so the padded k-steps that remain multiply zeros and the loop has no branches; two LDS
// buffers, one barrier per J block.
// Layouts (row-major): xo [o][Q]; z [Q][Q]; Rx, Gt [X][o][Q].  Requires o <= 16 OB; instantiated
// up to OB = 13 with 50 first-product k-steps (o <= 200), where the FP64 accumulators and operands
// fill the 512 registers a lane has at one wave per SIMD and the two LDS buffers take 123 KB.
//
// F32 (the mixed-precision path): the slices are rounded to FP32 on their way into LDS and both
// products run on v_mfma_f32_16x16x4f32 with FP32 accumulation.  There output element r of a
// lane is row 4 (lane / 16) + r, so lane (lk = lane / 16) holds Ft rows J = 4 lk + r and k-step r
// of the second product takes J in that order (row lk of the step is J = 4 lk + r); the A operand,
// xo[i][J], is read in the same order.  The FP32 LDS rows are padded so that the four lane groups of a read
// fall on distinct banks.
#include <type_traits>

#include "internal.h"

namespace thc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BI = 64, BJ = 16, NT = 256;
constexpr int RSRC_W3 = 0x00020000;  // raw 32-bit buffer access
constexpr uint32_t OOB = 0x80000000u;

// A buffer of 2 GiB from base (uniform across the wave): offsets at or beyond 2^31 read as zero.
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const double* base) {
  const uint64_t a = (uint64_t)base;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(hi << 32 | lo), (short)0, (int)OOB, RSRC_W3);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0u, 0));
}

// KST: k-steps of 4 in the first product (o rounded up to 4, at most 4 OB): the steps that would
// multiply only the zero padding of o are not issued.
template <int OB, int KST, bool F32>
__global__ __launch_bounds__(NT, OB <= 4 ? 3 : 1) void exch_kernel(int64_t o, int64_t Q, const double* __restrict__ xo,
                                                  const double* __restrict__ z, const double* __restrict__ Rx,
                                                  double* __restrict__ Gt) {
  using T = typename std::conditional<F32, float, double>::type;
  using V4 = typename std::conditional<F32, f4, d4>::type;
  static_assert(KST >= 1 && KST <= 4 * OB, "k-steps within the padded o");
  constexpr int OP = 16 * OB;             // padded o
  constexpr int NRX = (OP * BJ) / NT;     // Rx / xo slice elements per thread
  constexpr int NZ = (BI * BJ) / NT;      // z slice elements per thread
  static_assert((OP * BJ) % NT == 0, "whole slices per thread");
  // row pitches (elements) of the LDS slices; the transposed stores of xo and z go to rows of an
  // odd FP64 pitch, so the 16 rows a wave's consecutive lanes write fall on distinct banks
  constexpr int PR = F32 ? BJ + 4 : BJ, PJ = F32 ? OP + 4 : OP + 1, PZ = F32 ? BI + 4 : BI + 1;
  __shared__ T rx_s[2][OP * PR];  // [k][j]
  __shared__ T xj_s[2][BJ * PJ];  // [j][i]
  __shared__ T z_s[2][BJ * PZ];   // [j][I]

  const int64_t X = blockIdx.y;
  const int64_t I0 = (int64_t)blockIdx.x * BI;
  const double* __restrict__ R = Rx + X * o * Q;
  double* __restrict__ out = Gt + X * o * Q;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t Iw = I0 + 16 * w + lr;    // this lane's I (B operand column, output column)

  // B operand of the first product: xo[4 s + lk][Iw], held for the whole J walk
  T xb[4 * OB];
#pragma unroll
  for (int s = 0; s < 4 * OB; ++s) {
    const int64_t k = 4 * s + lk;
    xb[s] = (T)((k < o && Iw < Q) ? xo[k * Q + Iw] : 0.0);
  }

  // element q of this thread's share of a J block: Rx / xo row k, column jr; z row I0 + iz, column jz
  const int jr = t % BJ, jz = t % BJ;
  uint32_t roff[NRX], zoff[NZ];
  bool rok[NRX], zok[NZ];
#pragma unroll
  for (int q = 0; q < NRX; ++q) {
    const int k = (t + NT * q) / BJ;
    roff[q] = 8u * ((uint32_t)k * (uint32_t)Q + (uint32_t)jr);
    rok[q] = k < o;
  }
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    const int iz = (t + NT * q) / BJ;
    zoff[q] = 8u * ((uint32_t)iz * (uint32_t)Q + (uint32_t)jz);
    zok[q] = I0 + iz < Q;
  }

  double prx[NRX], pxj[NRX], pz[NZ];
  auto load = [&](int64_t J0) {
    const bool jok = J0 + jr < Q;  // jr == jz
    const __amdgpu_buffer_rsrc_t rr = rsrc(R + J0), rx = rsrc(xo + J0), rz = rsrc(z + I0 * Q + J0);
#pragma unroll
    for (int q = 0; q < NRX; ++q) {
      const uint32_t off = rok[q] && jok ? roff[q] : OOB;
      prx[q] = bload(rr, off);
      pxj[q] = bload(rx, off);
    }
#pragma unroll
    for (int q = 0; q < NZ; ++q) pz[q] = bload(rz, zok[q] && jok ? zoff[q] : OOB);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NRX; ++q) {
      const int e = t + NT * q;
      rx_s[buf][PR == BJ ? e : (e / BJ) * PR + e % BJ] = (T)prx[q];
      xj_s[buf][(e % BJ) * PJ + e / BJ] = (T)pxj[q];
    }
#pragma unroll
    for (int q = 0; q < NZ; ++q) {
      const int e = t + NT * q;
      z_s[buf][(e % BJ) * PZ + e / BJ] = (T)pz[q];
    }
  };

  V4 acc[OB];
#pragma unroll
  for (int b = 0; b < OB; ++b) acc[b] = V4{0, 0, 0, 0};
  auto mfma = [](T a, T b, V4 c) {
    if constexpr (F32) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  };
  // Ft row of output element r of this lane (and so the J of k-step r's row lk)
  auto jrow = [&](int r) { return F32 ? 4 * lk + r : lk + 4 * r; };

  auto compute = [&](int buf) {
    // Ft[J][I] for J in this block (rows), this wave's 16 I (columns)
    V4 ft = V4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KST; ++s) ft = mfma(rx_s[buf][(4 * s + lk) * PR + lr], xb[s], ft);
    // scale by z[I][J]: element r is (J = jrow(r), I = 16 w + lr)
#pragma unroll
    for (int r = 0; r < 4; ++r) ft[r] *= z_s[buf][jrow(r) * PZ + 16 * w + lr];
    // Gt[i][I] += sum_J xo[i][J] Ft[J][I]; k-step r uses ft[r] as its B element
#pragma unroll
    for (int b = 0; b < OB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[b] = mfma(xj_s[buf][jrow(r) * PJ + 16 * b + lr], ft[r], acc[b]);
  };

  const int64_t nb = (Q + BJ - 1) / BJ;
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t jb = 1; jb < nb; ++jb) {  // block jb - 1 is multiplied while block jb is fetched
    load(jb * BJ);
    compute(buf);
    store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  compute(buf);

  // output element r of block b: i = 16 b + jrow(r), I = Iw
  if (Iw < Q) {
#pragma unroll
    for (int b = 0; b < OB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = 16 * b + jrow(r);
        if (i < o) out[i * Q + Iw] = (double)acc[b][r];
      }
  }
}

template <int OB, int KST, bool F32>
hipError_t launch_k(int64_t o, int64_t Q, int64_t nx, const double* xo, const double* z, const double* Rx, double* Gt,
                    hipStream_t s) {
  const int64_t ti = (Q + BI - 1) / BI;
  // byte offsets within a J block stay below 2^31 (the buffer range)
  if (ti > 2147483647LL || nx > 65535 || 8 * (BI + 1) * Q >= (int64_t(1) << 31) || 8 * (16 * OB + 1) * Q >= (int64_t(1) << 31))
    return hipErrorInvalidValue;
  if (4 * KST < o) return hipErrorInvalidValue;
  hipLaunchKernelGGL((exch_kernel<OB, KST, F32>), dim3((unsigned)ti, (unsigned)nx), dim3(NT), 0, s, o, Q, xo, z, Rx,
                     Gt);
  return hipGetLastError();
}
template <int OB, int KST = 4 * OB>
hipError_t launch(bool f32, int64_t o, int64_t Q, int64_t nx, const double* xo, const double* z, const double* Rx,
                  double* Gt, hipStream_t s) {
  return f32 ? launch_k<OB, KST, true>(o, Q, nx, xo, z, Rx, Gt, s) : launch_k<OB, KST, false>(o, Q, nx, xo, z, Rx, Gt, s);
}

}  // namespace

bool exch_supported(int64_t o) { return o >= 1 && o <= 200; }

hipError_t exch_fused(int64_t o, int64_t Q, int64_t nx, const double* xo, const double* z, const double* Rx,
                      double* Gt, bool f32, hipStream_t s) {
  if (nx <= 0 || Q <= 0) return hipSuccess;
  if (o <= 16) return launch<1>(f32, o, Q, nx, xo, z, Rx, Gt, s);
  if (o <= 32) return launch<2>(f32, o, Q, nx, xo, z, Rx, Gt, s);
  if (o <= 64) {  // the k-step count of the first product fitted to o in steps of 8
    if (o <= 40) return launch<4, 10>(f32, o, Q, nx, xo, z, Rx, Gt, s);
    if (o <= 48) return launch<4, 12>(f32, o, Q, nx, xo, z, Rx, Gt, s);
    if (o <= 56) return launch<4, 14>(f32, o, Q, nx, xo, z, Rx, Gt, s);
    return launch<4>(f32, o, Q, nx, xo, z, Rx, Gt, s);
  }
  if (o <= 128) return launch<8>(f32, o, Q, nx, xo, z, Rx, Gt, s);
  // 13 row blocks: 52 accumulators and up to 52 first-product operands per lane, held in the
  // combined vector and accumulation registers at one wave per SIMD (FP64: 467 of 512)
  if (o <= 200) return launch<13, 50>(f32, o, Q, nx, xo, z, Rx, Gt, s);
  return hipErrorInvalidValue;
}

}  // namespace thc
