// The three-way product of the quartic T2^2 algorithm (paper Alg. 6, line 11):
//   H^XYZ += sum_I ( E_I^XY F_I^XZ + E_I^XZ F_I^XY ) G_I^YZ
// It is not a matrix product (all three factors carry two of the three output indices), so it
// runs on the vector ALUs: 5 flops (one multiply, two FMAs) per (X, Y, Z, I).
//
// Work decomposition: a workgroup of 4 wave64s owns an 8 x 32 x 64 (X, Y, Z) block of H held
// in registers for the whole I range.  Lane = Z (coalesced loads of E_I^XZ, F_I^XZ, G_I^YZ and
// of H), wave = a group of 8 Y, and the 8 X are the same for the whole workgroup, so E_I^XY and
// F_I^XY are wave-uniform and are read once per wave into scalar registers.  Each thread
// keeps 64 accumulators (8 X by 8 Y at its Z).
// Layouts (row-major, rank padded with zeros to Pp, a multiple of 64; X restricted to a block of
// Xb ranks so that H fits in memory): E, F: [I][Xb][Pp]; G: [I][Pp][Pp]; H: [Xb][Pp][Pp].
#include "internal.h"

namespace thc {
namespace {

constexpr int HX = 8, HYW = 8, HW = 4, HZ = 64;

__global__ __launch_bounds__(256) void h_kernel(int Pp, int Xb, int64_t nI, const double* __restrict__ E,
                                                const double* __restrict__ F, const double* __restrict__ G,
                                                double* __restrict__ H) {
  // Pp is a multiple of 64 and every operand is zero-padded to Pp, so there are no bounds checks.
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int z = blockIdx.x * HZ + lane;
  const unsigned zu = (unsigned)z;
  const int y0 = blockIdx.y * (HYW * HW) + wave * HYW;
  const int x0 = blockIdx.z * HX;
  const int64_t PP = (int64_t)Pp * Pp;    // per-I stride of G
  const int64_t XP = (int64_t)Xb * Pp;    // per-I stride of E and F

  double acc[HX][HYW];
  double* __restrict__ Hb = H + ((int64_t)x0 * Pp + y0) * Pp + z;
#pragma unroll
  for (int xi = 0; xi < HX; ++xi)
#pragma unroll
    for (int yi = 0; yi < HYW; ++yi) acc[xi][yi] = Hb[((int64_t)xi * Pp + yi) * Pp];

  const double* __restrict__ EI = E;
  const double* __restrict__ FI = F;
  const double* __restrict__ GI = G;
  for (int64_t I = 0; I < nI; ++I, EI += XP, FI += XP, GI += PP) {
    double ez[HX], fz[HX], gz[HYW];
#pragma unroll
    for (int xi = 0; xi < HX; ++xi) {
      const double* __restrict__ er = EI + (int64_t)(x0 + xi) * Pp;  // uniform row base
      const double* __restrict__ fr = FI + (int64_t)(x0 + xi) * Pp;
      ez[xi] = er[zu];
      fz[xi] = fr[zu];
    }
#pragma unroll
    for (int yi = 0; yi < HYW; ++yi) {
      const double* __restrict__ gr = GI + (int64_t)(y0 + yi) * Pp;
      gz[yi] = gr[zu];
    }
#pragma unroll
    for (int xi = 0; xi < HX; ++xi) {
      const double* __restrict__ ex = EI + (x0 + xi) * Pp + y0;  // wave-uniform row segment
      const double* __restrict__ fx = FI + (x0 + xi) * Pp + y0;
#pragma unroll
      for (int yi = 0; yi < HYW; ++yi) {
        const double t = ex[yi] * fz[xi] + fx[yi] * ez[xi];
        acc[xi][yi] += t * gz[yi];
      }
    }
  }

#pragma unroll
  for (int xi = 0; xi < HX; ++xi)
#pragma unroll
    for (int yi = 0; yi < HYW; ++yi) Hb[((int64_t)xi * Pp + yi) * Pp] = acc[xi][yi];
}

}  // namespace

hipError_t h_accumulate(int64_t Pp, int64_t Xb, int64_t nI, const double* E, const double* F, const double* G,
                        double* H, hipStream_t s) {
  if (Pp % 64 != 0 || Pp > 32768 || Xb % HX != 0 || Xb > Pp || Xb <= 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(Pp / HZ), (unsigned)(Pp / (HYW * HW)), (unsigned)(Xb / HX));
  hipLaunchKernelGGL(h_kernel, grid, dim3(256), 0, s, (int)Pp, (int)Xb, nI, E, F, G, H);
  return hipGetLastError();
}

}  // namespace thc
