// The three-way product of the quartic T2^2 algorithm (paper Alg. 6):
//   H^XYZ += sum_I ( E_I^XY F_I^XZ + E_I^XZ F_I^XY ) G_I^YZ
// It is not a matrix product (each factor carries two of the three output indices), so it
// runs on the vector ALUs: 5 flops (one multiply, two FMAs) per (X, Y, Z, I).
//
// Work decomposition.  A 256-thread workgroup (4 wave64s) owns an 8 x 32 x 64 (X, Y, Z) tile of
// H held in registers for the whole I range: lane = Z, wave = 8 Y, and the 8 X are shared by the
// workgroup, so each thread keeps 64 accumulators (8 X by 8 Y at its Z).  E_I^XZ, F_I^XZ and
// G_I^YZ are per-lane coalesced buffer loads (a descriptor per operand row block in SGPRs, one
// 32-bit lane offset in a VGPR, the row offset in an SGPR, so no 64-bit per-lane addresses);
// E_I^XY and F_I^XY are wave-uniform and are read with scalar loads into SGPRs.
// Tiles are grouped 4 (X) x 2 (Y) x 4 (Z) and each group of 32 tiles goes to one XCD
// (workgroup id mod 8 selects the XCD), so the workgroups resident on an XCD at the same time
// share their E, F and G slices through that XCD's L2.
// Layouts (row-major, rank zero-padded to Pp, a multiple of 64; X restricted to a block of Xb
// ranks, a multiple of 8): E, F: [I][Xb][Pp]; G: [I][Pp][Pp]; H: [Xb][Pp][Pp].
#include "internal.h"

namespace thc {
namespace {

constexpr int HX = 8, HYW = 8, HW = 4, HZ = 64;
constexpr int TY = HYW * HW;                                   // 32 Y per workgroup
constexpr int GX = 4, GY = 2, GZ = 4, GT = GX * GY * GZ;       // tiles per XCD group
constexpr int RSRC_W3 = 0x00020000;                            // raw 32-bit buffer access

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const double* base, int64_t ndoubles) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(ndoubles * 8), RSRC_W3);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ inline void bstore(double x, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}

__global__ __launch_bounds__(256) void h_kernel(int Pp, int Xb, int64_t nI, const double* __restrict__ E,
                                                const double* __restrict__ F, const double* __restrict__ G,
                                                double* __restrict__ H, int ntx, int nty, int ntz, int gx,
                                                int gy) {
  // XCD-contiguous numbering of the tiles (the grid is a multiple of 8; workgroup b runs on XCD b % 8)
  const int nblk = gridDim.x, b = blockIdx.x;
  const int tix = (b & 7) * (nblk >> 3) + (b >> 3);
  const int gid = tix / GT, in = tix % GT;
  const int tx = (gid % gx) * GX + in % GX;
  const int ty = ((gid / gx) % gy) * GY + (in / GX) % GY;
  const int tz = (gid / (gx * gy)) * GZ + in / (GX * GY);
  if (tx >= ntx || ty >= nty || tz >= ntz) return;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = tx * HX, y0 = ty * TY + wave * HYW, z0 = tz * HZ;
  const int64_t PP = (int64_t)Pp * Pp;    // per-I stride of G
  const int64_t XP = (int64_t)Xb * Pp;    // per-I stride of E and F

  // H tile rows: (x0 + xi, y0 + yi, z0 + lane), relative to the tile origin
  const double* Hb = H + ((int64_t)x0 * Pp + y0) * Pp + z0;
  const __amdgpu_buffer_rsrc_t rh = rsrc(Hb, ((int64_t)(HX - 1) * Pp + HYW) * Pp);
  const unsigned lo = (unsigned)lane * 8u;
  const unsigned rowb = (unsigned)Pp * 8u;  // bytes per rank row
  double acc[HX][HYW];
#pragma unroll
  for (int xi = 0; xi < HX; ++xi)
#pragma unroll
    for (int yi = 0; yi < HYW; ++yi) acc[xi][yi] = bload(rh, lo, (unsigned)(xi * Pp + yi) * rowb);

  const double* EI = E + (int64_t)x0 * Pp;
  const double* FI = F + (int64_t)x0 * Pp;
  const double* GI = G + (int64_t)y0 * Pp;
  const unsigned zo = (unsigned)(z0 + lane) * 8u;
  for (int64_t I = 0; I < nI; ++I, EI += XP, FI += XP, GI += PP) {
    const __amdgpu_buffer_rsrc_t re = rsrc(EI, (int64_t)HX * Pp);
    const __amdgpu_buffer_rsrc_t rf = rsrc(FI, (int64_t)HX * Pp);
    const __amdgpu_buffer_rsrc_t rg = rsrc(GI, (int64_t)HYW * Pp);
    double ez[HX], fz[HX], gz[HYW];
#pragma unroll
    for (int xi = 0; xi < HX; ++xi) {
      ez[xi] = bload(re, zo, (unsigned)xi * rowb);
      fz[xi] = bload(rf, zo, (unsigned)xi * rowb);
    }
#pragma unroll
    for (int yi = 0; yi < HYW; ++yi) gz[yi] = bload(rg, zo, (unsigned)yi * rowb);
#pragma unroll
    for (int xi = 0; xi < HX; ++xi) {
      const double* __restrict__ ex = EI + xi * Pp + y0;  // wave-uniform row segment
      const double* __restrict__ fx = FI + xi * Pp + y0;
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
    for (int yi = 0; yi < HYW; ++yi) bstore(acc[xi][yi], rh, lo, (unsigned)(xi * Pp + yi) * rowb);
}

}  // namespace

hipError_t h_accumulate(int64_t Pp, int64_t Xb, int64_t nI, const double* E, const double* F, const double* G,
                        double* H, hipStream_t s) {
  if (Pp % 64 != 0 || Pp > 8192 || Xb % HX != 0 || Xb > Pp || Xb <= 0) return hipErrorInvalidValue;
  const int ntx = (int)(Xb / HX), nty = (int)(Pp / TY), ntz = (int)(Pp / HZ);
  const int gx = (ntx + GX - 1) / GX, gy = (nty + GY - 1) / GY, gz = (ntz + GZ - 1) / GZ;
  const int64_t nblk = (int64_t)gx * gy * gz * GT;  // a multiple of 8
  if (nblk > 2147483647LL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(h_kernel, dim3((unsigned)nblk), dim3(256), 0, s, (int)Pp, (int)Xb, nI, E, F, G, H, ntx, nty,
                     ntz, gx, gy);
  return hipGetLastError();
}

}  // namespace thc
