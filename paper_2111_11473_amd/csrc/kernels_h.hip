// The three-way product of the quartic T2^2 algorithm (paper Alg. 6):
//   H^XYZ += sum_I ( E_I^XY F_I^XZ + E_I^XZ F_I^XY ) G_I^YZ
// Each factor carries two of the three output indices, so this is not a matrix product; it
// runs on the FP64 vector ALUs.
//
// Symmetry.  The bracket t_I(X; Y, Z) = E^XY F^XZ + E^XZ F^XY is symmetric in Y <-> Z, so for
// Y != Z one t serves both H^XYZ (times G^YZ) and H^XZY (times G^ZY): 7 flops and 4 VALU
// instructions for two outputs instead of 10 flops and 6 instructions.
//
// Work decomposition.  Lanes run over X (64 per wave).  Y and Z are cut into blocks of 16; a
// workgroup owns one X tile, one Y block and a BZ = 4 NWZ wide slice of one Z block with
// Yb <= Zb.  For Yb < Zb it accumulates both H^XYZ and its mirror H^XZY; a diagonal block
// (Yb == Zb) covers every ordered pair inside itself directly and keeps no mirror.  Wave
// (wy, wz) holds an 8 (Y) x 4 (Z) patch: 32 accumulators plus 32 mirror accumulators per lane.
//
// Operand staging.  E and F are stored with pairs of rows interleaved ([Y/2][X][2]), so one
// 16-byte LDS read gives a lane both rows of a pair at its X (16-byte reads have about twice the
// LDS bandwidth of 8-byte ones).  They are stored X tile by X tile and grid point by grid point
// ([X/64][I][Y/2][64][2]): a tile's row pairs at one I are contiguous 1 KB pieces of one block,
// and consecutive I are adjacent.  G is stored in 16 x 8 blocks, so a tile's G^YZ is one
// contiguous 1 KB block and its G^ZY two 512-byte pieces.  Per I the workgroup's rows -- E^XY,
// F^XY for its 16 Y, E^XZ, F^XZ for its Z slice -- and its two G blocks are copied by buffer
// loads straight into LDS, NS stages deep (NS - 1 values of I in flight), and each wave waits
// only for its own copies of the next stage before the barrier.  The only factor that is
// uniform across the lanes, G, is held 16 values to a VGPR pair (lane l holds value l % 16) and
// broadcast into the FMA by the DPP row_newbcast source modifier, so the inner loop has no
// scalar loads.
// Tile order comes from a host-built table: runs of `slots` tiles (the workgroups resident on one
// XCD) that share an X tile and a compact patch of (Y, Z) blocks are placed at workgroup ids b with
// b % 8 = that XCD, so tiles sharing operand rows run on one XCD at about the same time and share
// them through its L2.  The table is launched one generation (8 runs, every slot of the device)
// at a time, so the workgroups of a run start together and cannot drift apart by more than one
// tile's lifetime; consecutive generations walk the grid points in opposite directions, so a
// generation starts on the points its predecessor read last (still in the last-level cache).
// One workgroup per tile measured faster than a persistent grid walking the table.
// Layouts (Y, Z ranks zero-padded to Pp, a multiple of 16; X restricted to a block of Xb ranks, a
// multiple of 64 and at most Pp rounded up to 64):
//   E, F: [Xb/64][ldi][Pp/2][64][2] (E_I^XY at [X/64][I][Y/2][X%64][Y%2]);
//   G: [I][Pp/16][Pp/8][16][8] (G_I^YZ at [I][Y/16][Z/8][Y%16][Z%8]);
//   H: [Pp][Pp][Xb] (H^XYZ at [Y][Z][X]).
#include <algorithm>
#include <utility>
#include <vector>

#include "internal.h"

namespace thc {
namespace {

constexpr int LANES = 64;                  // X per wave and per workgroup
constexpr int BY = 16;                     // Y (and Z) block edge
constexpr int WY = 8, WZ = 4;              // per-wave patch
constexpr int RSRC_W3 = 0x00020000;        // raw 32-bit buffer access
constexpr uint32_t EMPTY = 0x80000000u;

// TE: storage type of E and F (the FP64 kernel instantiates double; G and H are FP64).
template <int NWZ, int NS, typename TE>
struct Geo {
  static constexpr int NW = (BY / WY) * NWZ;        // waves per workgroup
  static constexpr int NTHREADS = NW * LANES;
  static constexpr int BZ = WZ * NWZ;               // Z slice per workgroup
  static constexpr int NZS = BY / BZ;               // Z slices per block
  // stage layout (bytes): row pairs of 64 X (128 values each) -- E^Y, F^Y (BY/2 pairs each),
  // E^Z, F^Z (BZ/2 pairs each) -- then the FP64 G blocks G^YZ [BY][BZ] and G^ZY [BZ][BY]
  static constexpr int ESZ = (int)sizeof(TE);
  static constexpr int PAIR_B = 128 * ESZ;
  static constexpr int NPAIRS = BY + BZ;
  static constexpr int EY = 0, FY = BY / 2, EZ = BY, FZ = BY + BZ / 2;  // in pairs
  static constexpr int G_B = NPAIRS * PAIR_B;
  static constexpr int GM_B = G_B + BY * BZ * 8;
  static constexpr int STAGE_B = GM_B + BZ * BY * 8;
  static constexpr int PPC = 1024 / PAIR_B;         // row pairs per 1 KB DMA chunk
  static constexpr int CH_ROWS = NPAIRS / PPC;      // row chunks per stage
  static constexpr int CH_G = BY * BZ * 8 / 1024;   // 1 KB chunks per G block
  static constexpr int QROWS = CH_ROWS / NW;        // row chunks issued by every wave
  static_assert(CH_ROWS % NW == 0 && (BY / 2) % PPC == 0 && (BZ / 2) % PPC == 0, "row chunks split evenly");
  static_assert(2 * CH_G <= NW && (BY * BZ * 8) % 1024 == 0, "one round of G chunks");
  static_assert(NS >= 2 && NS * STAGE_B <= 160 * 1024, "stages must fit in LDS");
  static_assert(BZ == H_GBLK, "a Z slice is one column block of G");
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

__device__ inline d2 pair_at(const char* p) { return *(const d2*)p; }
__device__ inline d2 pair_at_f(const char* p) {
  const f2 v = *(const f2*)p;
  return d2{(double)v.x, (double)v.y};
}

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, int64_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(uint32_t)nbytes, RSRC_W3);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ inline void bstore(double x, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}
// 16 bytes per lane from a buffer straight into LDS at lds + 16 * lane (no VGPR destination)
__device__ inline void bload_lds(__amdgpu_buffer_rsrc_t r, void* lds, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, voff, soff, 0, 0);
}

// Waits until at most n of this wave's vector-memory operations are outstanding (n is
// wave-uniform) and its LDS operations are complete, then joins the workgroup barrier.  Written
// as one block so that neither the wait nor the barrier picks up the compiler's conservative
// vmcnt(0).
template <int N>
__device__ inline void wait_bar() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}
// Wait for stage I + 1 with `later` further stages (0 <= later < 3) of Q or Q + 1 copies each
// (extra: this wave also copies a G chunk) still allowed in flight, then the barrier.
template <int Q>
__device__ inline void wait_pipe(int later, bool extra) {
  if (later >= 2) {
    if (extra) wait_bar<2 * (Q + 1)>(); else wait_bar<2 * Q>();
  } else if (later == 1) {
    if (extra) wait_bar<Q + 1>(); else wait_bar<Q>();
  } else {
    wait_bar<0>();
  }
}

// One row j of the wave patch (four Z): t_k = ey fz_k + ez_k fy, then acc_k += G^YZ t_k and
// accm_k += G^ZY t_k with G broadcast from lane B + k of each row of 16 lanes (B = 4 (j % 4)).
// The instruction order keeps every DPP read at least two wait states after the VALU write of
// t_k, as the hardware requires (inline assembly is invisible to the compiler's hazard pass).
template <int B>
__device__ inline void h_row(double (&acc)[WZ], double (&accm)[WZ], double ey, double fy, const double (&ez)[WZ],
                             const double (&fz)[WZ], double g, double gm) {
  double t0, t1, t2, t3;
  asm("v_mul_f64 %[t0], %[ey], %[f0]\n\t"
      "v_mul_f64 %[t1], %[ey], %[f1]\n\t"
      "v_mul_f64 %[t2], %[ey], %[f2]\n\t"
      "v_mul_f64 %[t3], %[ey], %[f3]\n\t"
      "v_fma_f64 %[t0], %[e0], %[fy], %[t0]\n\t"
      "v_fma_f64 %[t1], %[e1], %[fy], %[t1]\n\t"
      "v_fma_f64 %[t2], %[e2], %[fy], %[t2]\n\t"
      "v_fma_f64 %[t3], %[e3], %[fy], %[t3]\n\t"
      "v_fmac_f64_dpp %[a0], %[g], %[t0] row_newbcast:%[b0]\n\t"
      "v_fmac_f64_dpp %[m0], %[gm], %[t0] row_newbcast:%[b0]\n\t"
      "v_fmac_f64_dpp %[a1], %[g], %[t1] row_newbcast:%[b1]\n\t"
      "v_fmac_f64_dpp %[m1], %[gm], %[t1] row_newbcast:%[b1]\n\t"
      "v_fmac_f64_dpp %[a2], %[g], %[t2] row_newbcast:%[b2]\n\t"
      "v_fmac_f64_dpp %[m2], %[gm], %[t2] row_newbcast:%[b2]\n\t"
      "v_fmac_f64_dpp %[a3], %[g], %[t3] row_newbcast:%[b3]\n\t"
      "v_fmac_f64_dpp %[m3], %[gm], %[t3] row_newbcast:%[b3]"
      : [a0] "+v"(acc[0]), [a1] "+v"(acc[1]), [a2] "+v"(acc[2]), [a3] "+v"(acc[3]), [m0] "+v"(accm[0]),
        [m1] "+v"(accm[1]), [m2] "+v"(accm[2]), [m3] "+v"(accm[3]), [t0] "=&v"(t0), [t1] "=&v"(t1),
        [t2] "=&v"(t2), [t3] "=&v"(t3)
      : [ey] "v"(ey), [fy] "v"(fy), [e0] "v"(ez[0]), [e1] "v"(ez[1]), [e2] "v"(ez[2]), [e3] "v"(ez[3]),
        [f0] "v"(fz[0]), [f1] "v"(fz[1]), [f2] "v"(fz[2]), [f3] "v"(fz[3]), [g] "v"(g), [gm] "v"(gm),
        [b0] "n"(B), [b1] "n"(B + 1), [b2] "n"(B + 2), [b3] "n"(B + 3));
}
static_assert(WZ == 4 && WY == 8, "h_row covers four Z; a patch is eight rows");

template <int NWZ, int NS, typename TE>
__global__ __launch_bounds__((Geo<NWZ, NS, TE>::NTHREADS)) void h_kernel(int Pp, int Xb, int64_t ldi, int64_t nI,
                                                                       const TE* __restrict__ E,
                                                                       const TE* __restrict__ F,
                                                                       const double* __restrict__ G,
                                                                       double* __restrict__ H,
                                                                       const uint32_t* __restrict__ tiles,
                                                                       int flags) {
  using C = Geo<NWZ, NS, TE>;
  __shared__ __attribute__((aligned(16))) char lds[NS * C::STAGE_B];
  const uint32_t tile = tiles[blockIdx.x];
  if (tile & EMPTY) return;  // whole workgroup, before any barrier
  const bool rev = flags & 1;    // walk the grid points backwards
  const bool fresh = flags & 2;  // first chunk: H starts from zero instead of being read
  const int Yb = tile & 511, Zb = (tile >> 9) & 511, zs = (tile >> 18) & 3, xt = (tile >> 20) & 1023;
  const bool mirror = Yb != Zb;
  const int y0 = Yb * BY, z0 = Zb * BY + zs * C::BZ, X0 = xt * LANES;

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __builtin_assume(w >= 0 && w < C::NW);
  const int ly0 = (w % (BY / WY)) * WY, lz0 = (w / (BY / WY)) * WZ;
  const unsigned xrow = (unsigned)Xb * 8u;  // bytes per (Y) row of H
  const unsigned lo = (unsigned)lane * 8u;

  // A diagonal block has no mirror: its G^ZY slots stay zero (the DMA never writes them), so the
  // mirror FMAs add nothing and the broadcast sources always come from LDS.
  if (!mirror)
    for (int i = threadIdx.x; i < C::BZ * BY; i += C::NTHREADS)
#pragma unroll
      for (int b = 0; b < NS; ++b) ((double*)(lds + b * C::STAGE_B + C::GM_B))[i] = 0.0;

  // accumulators: acc[j][k] = H[y0+ly0+j][z0+lz0+k][X0+lane], accm[j][k] = H[z0+lz0+k][y0+ly0+j][X0+lane]
  double acc[WY][WZ], accm[WY][WZ];
  const double* Hw = H + ((int64_t)(y0 + ly0) * Pp + z0 + lz0) * Xb + X0;
  const double* Hm = H + ((int64_t)(z0 + lz0) * Pp + y0 + ly0) * Xb + X0;
  const int64_t hw_bytes = ((int64_t)(WY - 1) * Pp + WZ) * Xb * 8;
  const int64_t hm_bytes = ((int64_t)(WZ - 1) * Pp + WY) * Xb * 8;
  if (fresh) {
#pragma unroll
    for (int j = 0; j < WY; ++j)
#pragma unroll
      for (int k = 0; k < WZ; ++k) acc[j][k] = accm[j][k] = 0.0;
  } else {
    const __amdgpu_buffer_rsrc_t rh = rsrc(Hw, hw_bytes);
    const __amdgpu_buffer_rsrc_t rm = rsrc(Hm, hm_bytes);
#pragma unroll
    for (int j = 0; j < WY; ++j)
#pragma unroll
      for (int k = 0; k < WZ; ++k) acc[j][k] = bload(rh, lo, (unsigned)(j * Pp + k) * xrow);
    if (mirror) {
#pragma unroll
      for (int j = 0; j < WY; ++j)
#pragma unroll
        for (int k = 0; k < WZ; ++k) accm[j][k] = bload(rm, lo, (unsigned)(k * Pp + j) * xrow);
    } else {
#pragma unroll
      for (int j = 0; j < WY; ++j)
#pragma unroll
        for (int k = 0; k < WZ; ++k) accm[j][k] = 0.0;
    }
  }

  // DMA plan of one stage: chunk c (1 KB) lands at stage + 1 KB c; wave w issues chunks w + NW q.
  // Row chunks first: chunk c holds PPC consecutive stage pairs starting at c PPC (E^Y, F^Y, E^Z,
  // F^Z in that order; lanes 64/PPC apart take consecutive pairs), then one round of FP64 G chunks,
  // c = CH_ROWS + w: G^YZ (the tile's 16 x 8 block, CH_G chunks) and, off the diagonal, G^ZY
  // (rows z0.. z0+7, columns y0.. y0+15: halves of two blocks, 8 rows of 16 per chunk).
  constexpr int LPP = 64 / C::PPC;                                    // lanes per row pair
  const unsigned voff_r = (unsigned)(lane / LPP) * C::PAIR_B + (unsigned)(lane % LPP) * 16u;
  const bool g_yz = w < C::CH_G, g_zy = !g_yz && w < 2 * C::CH_G && mirror;
  const int gs = g_yz ? w : w - C::CH_G;
  constexpr unsigned GBLK_B = 16u * C::BZ * 8u;                       // bytes of one G block
  const unsigned nbz = (unsigned)Pp / C::BZ;                          // G blocks per block row
  unsigned voff_g, so_g;
  // Both G blocks land in LDS swizzled (see gsw / gmsw below) so that the sixteen values a wave
  // broadcasts from either fall in distinct banks: lane l fills LDS granule l (16 bytes) with the
  // granule of the source block that the swizzle puts there.
  if (g_yz) {
    const int y = lane / 4, zp = (lane % 4) ^ (((y >> 1) & 1) << 1);  // storage row, source column pair
    voff_g = (unsigned)gs * 1024u + (unsigned)(y * 4 + zp) * 16u;
    so_g = ((unsigned)Yb * nbz + (unsigned)(z0 / C::BZ)) * GBLK_B;
  } else {
    const int r = gs * 8 + lane / 8;                     // destination row (Z)
    const int col = (2 * (lane % 8)) ^ (4 * (r & 3));    // source column (Y) of the storage pair
    voff_g = (unsigned)(col / C::BZ) * GBLK_B + ((unsigned)(zs * C::BZ + r) * C::BZ + (unsigned)(col % C::BZ)) * 8u;
    so_g = ((unsigned)Zb * nbz + (unsigned)(y0 / C::BZ)) * GBLK_B;
  }
  const bool extra = g_yz || g_zy;  // this wave copies QROWS + extra chunks per stage
  const int64_t PX = (int64_t)Pp * LANES;  // elements of E, F per (X tile, I)
  const int64_t PP = (int64_t)Pp * Pp;     // elements of G per I
  // Sources of the next stage to copy: a generation walks the grid points forwards or (rev)
  // backwards, so each stage moves the three row pointers by one grid point.
  const int64_t first = (rev && nI > 0) ? nI - 1 : 0;
  const TE* e_at = E + ((int64_t)xt * ldi + first) * PX;
  const TE* f_at = F + ((int64_t)xt * ldi + first) * PX;
  const double* g_at = G + first * PP;
  const int64_t dPX = rev ? -PX : PX, dPP = rev ? -PP : PP;
  auto stage_in = [&](int buf) {
    const __amdgpu_buffer_rsrc_t re = rsrc(e_at, PX * C::ESZ);
    const __amdgpu_buffer_rsrc_t rf = rsrc(f_at, PX * C::ESZ);
    char* sb = lds + buf * C::STAGE_B;
#pragma unroll
    for (int q = 0; q < C::QROWS; ++q) {
      const int c = w + C::NW * q;
      const int sp = c * C::PPC;  // first stage pair of the chunk (all its pairs share a region)
      const bool isF = (sp >= C::FY && sp < C::EZ) || sp >= C::FZ;
      const int pair = sp < C::FY ? y0 / 2 + sp : sp < C::EZ ? y0 / 2 + sp - C::FY
                                                : sp < C::FZ ? z0 / 2 + sp - C::EZ : z0 / 2 + sp - C::FZ;
      bload_lds(isF ? rf : re, sb + c * 1024, voff_r, (unsigned)pair * C::PAIR_B);
    }
    if (extra) bload_lds(rsrc(g_at, PP * 8), sb + C::G_B + w * 1024, voff_g, so_g);
    e_at += dPX;
    f_at += dPX;
    g_at += dPP;
  };

  // broadcast-register sources: lane l holds G^YZ[ly0 + 4 r + m / 4][lz0 + m % 4], m = l % 16.
  // LDS holds G^YZ (y, z) at y BZ + (z ^ 4 ((y >> 1) & 1)) and G^ZY (z, y) at z BY + (y ^ 4 (z & 3)):
  // the 4 x 4 values a read takes (32 banks of 4 bytes) then cover every bank once instead of
  // two (G^YZ: rows y and y + 2) or four (G^ZY: every row) times.
  const int m = lane & 15;
  const int goff0 = (ly0 + (m >> 2)) * C::BZ + ((lz0 + (m & 3)) ^ (((m >> 3) & 1) << 2));
  const int gmoff0 = (lz0 + (m & 3)) * BY + ((ly0 + (m >> 2)) ^ (4 * (m & 3)));

  constexpr int D = NS - 1;  // stages in flight ahead of the one being consumed
  static_assert(D <= 3, "wait_pipe allows at most two stages in flight behind the next one");
  auto next = [](int b) { return b + 1 == NS ? 0 : b + 1; };
  int64_t issued = 0;
  int sbuf = 0;  // buffer of the next stage to copy: (buf + D) % NS once the pipe is full
  for (; issued < D && issued < nI; ++issued) {
    stage_in(sbuf);
    sbuf = next(sbuf);
  }
  wait_pipe<C::QROWS>((int)(issued > 0 ? issued - 1 : 0), extra);  // stage 0 has landed everywhere
  int buf = 0;
  auto consume = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(1);  // the FMAs before another wave's copies when both are ready
    const char* __restrict__ st = lds + buf * C::STAGE_B;
    const double* __restrict__ sg = (const double*)(st + C::G_B);
    const double* __restrict__ sgm = (const double*)(st + C::GM_B);
    auto pair = [&](int sp) {  // this lane's X in stage pair sp, as two FP64 values
      const char* a = st + sp * C::PAIR_B + lane * 2 * C::ESZ;
      if constexpr (C::ESZ == 8) return pair_at(a); else return pair_at_f(a);
    };
    d2 ey[WY / 2], fy[WY / 2], ez[WZ / 2], fz[WZ / 2];
    double g[2], gm[2];
#pragma unroll
    for (int p = 0; p < WZ / 2; ++p) {
      ez[p] = pair(C::EZ + lz0 / 2 + p);
      fz[p] = pair(C::FZ + lz0 / 2 + p);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      g[r] = sg[goff0 + 4 * r * C::BZ];
      gm[r] = sgm[gmoff0 ^ (4 * r)];
    }
#pragma unroll
    for (int p = 0; p < WY / 2; ++p) {
      ey[p] = pair(C::EY + ly0 / 2 + p);
      fy[p] = pair(C::FY + ly0 / 2 + p);
    }
    const double ezs[WZ] = {ez[0].x, ez[0].y, ez[1].x, ez[1].y};
    const double fzs[WZ] = {fz[0].x, fz[0].y, fz[1].x, fz[1].y};
    h_row<0>(acc[0], accm[0], ey[0].x, fy[0].x, ezs, fzs, g[0], gm[0]);
    h_row<4>(acc[1], accm[1], ey[0].y, fy[0].y, ezs, fzs, g[0], gm[0]);
    h_row<8>(acc[2], accm[2], ey[1].x, fy[1].x, ezs, fzs, g[0], gm[0]);
    h_row<12>(acc[3], accm[3], ey[1].y, fy[1].y, ezs, fzs, g[0], gm[0]);
    h_row<0>(acc[4], accm[4], ey[2].x, fy[2].x, ezs, fzs, g[1], gm[1]);
    h_row<4>(acc[5], accm[5], ey[2].y, fy[2].y, ezs, fzs, g[1], gm[1]);
    h_row<8>(acc[6], accm[6], ey[3].x, fy[3].x, ezs, fzs, g[1], gm[1]);
    h_row<12>(acc[7], accm[7], ey[3].y, fy[3].y, ezs, fzs, g[1], gm[1]);
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
  };
  // Steady state: every grid point also issues the stage D ahead, and the stage after the next
  // one (D - 1 of them) may stay in flight.
  const int64_t steady = nI - D;
  for (int64_t I = 0; I < steady; ++I) {
    stage_in(sbuf);
    sbuf = next(sbuf);
    consume();
    wait_pipe<C::QROWS>(D - 1, extra);
    buf = next(buf);
  }
  // Drain: nothing more to issue; stage I + 1 must have landed, nI - I - 2 may be in flight.
  for (int64_t I = steady > 0 ? steady : 0; I < nI; ++I) {
    consume();
    const int64_t later = nI - I - 2;
    wait_pipe<C::QROWS>((int)(later > 0 ? later : 0), extra);
    buf = next(buf);
  }

  {
    const __amdgpu_buffer_rsrc_t rh = rsrc(Hw, hw_bytes);
    const __amdgpu_buffer_rsrc_t rm = rsrc(Hm, hm_bytes);
#pragma unroll
    for (int j = 0; j < WY; ++j)
#pragma unroll
      for (int k = 0; k < WZ; ++k) bstore(acc[j][k], rh, lo, (unsigned)(j * Pp + k) * xrow);
    if (mirror) {
#pragma unroll
      for (int j = 0; j < WY; ++j)
#pragma unroll
        for (int k = 0; k < WZ; ++k) bstore(accm[j][k], rm, lo, (unsigned)(k * Pp + j) * xrow);
    }
  }
}

// Position of cell (y, z) along the Hilbert curve that fills an n x n grid (n a power of two).
int64_t hilbert_index(int64_t n, int64_t y, int64_t z) {
  int64_t d = 0;
  for (int64_t s = n / 2; s > 0; s /= 2) {
    const int64_t ry = (y & s) ? 1 : 0, rz = (z & s) ? 1 : 0;
    d += s * s * ((3 * ry) ^ rz);
    if (rz == 0) {  // rotate the quadrant so the curve enters and leaves it at the right corners
      if (ry == 1) {
        y = n - 1 - y;
        z = n - 1 - z;
      }
      std::swap(y, z);
    }
  }
  return d;
}

template <int NZS>
std::vector<uint32_t> tiles_for(int64_t Pp, int64_t Xb, int64_t slots) {
  const int64_t nB = Pp / BY, nX = Xb / LANES;
  // Block pairs (Yb <= Zb) in Hilbert-curve order: any run of consecutive pairs covers a compact
  // patch of the (Y, Z) triangle, so the runs that share an XCD's L2 touch few distinct operand
  // rows and G blocks (about 20% fewer bytes per grid point than row-major groups of 4 x 8 blocks,
  // whose runs straddle two groups once the diagonal groups put them out of step).
  int64_t n = 1;
  while (n < nB) n *= 2;
  std::vector<std::pair<int64_t, uint32_t>> pairs;
  pairs.reserve((size_t)(nB * (nB + 1) / 2));
  for (int64_t yb = 0; yb < nB; ++yb)
    for (int64_t zb = yb; zb < nB; ++zb) pairs.push_back({hilbert_index(n, yb, zb), (uint32_t)(yb | (zb << 9))});
  std::sort(pairs.begin(), pairs.end());
  std::vector<uint32_t> lin;
  lin.reserve(pairs.size() * NZS * (size_t)nX);
  for (int64_t xt = 0; xt < nX; ++xt)
    for (const auto& p : pairs)
      for (int64_t s = 0; s < NZS; ++s) lin.push_back(p.second | (uint32_t)(s << 18) | (uint32_t)(xt << 20));
  const int64_t runs = ((int64_t)lin.size() + slots - 1) / slots;
  std::vector<uint32_t> out((size_t)(((runs + 7) / 8) * 8 * slots), EMPTY);
  for (size_t e = 0; e < lin.size(); ++e) {
    const int64_t c = (int64_t)e / slots, k = (int64_t)e % slots;
    out[(size_t)((c / 8) * 8 * slots + k * 8 + c % 8)] = lin[e];
  }
  return out;
}

template <int NWZ, int NS, typename TE>
hipError_t launch(int64_t Pp, int64_t Xb, int64_t ldi, int64_t nI, const TE* E, const TE* F,
                  const double* G, double* H, const uint32_t* tiles, int64_t ntiles, int64_t slots, bool fresh,
                  hipStream_t s) {
  if (Pp % BY != 0 || Pp <= 0 || Pp > 8192 || Xb % LANES != 0 || Xb > (Pp + LANES - 1) / LANES * LANES || Xb <= 0 || ntiles <= 0 || ntiles > 2147483647LL ||
      nI < 0 || ldi < nI || slots < 1 || ntiles % (8 * slots) != 0)
    return hipErrorInvalidValue;
  // One launch per generation of 8 slots tiles (every workgroup resident at once): the runs of
  // a generation start together, so the workgroups sharing operand rows through an L2 stay
  // within one tile's lifetime of each other.
  const int64_t gen = 8 * slots;
  for (int64_t t0 = 0; t0 < ntiles; t0 += gen) {
    hipLaunchKernelGGL((h_kernel<NWZ, NS, TE>), dim3((unsigned)gen), dim3(Geo<NWZ, NS, TE>::NTHREADS), 0, s,
                       (int)Pp, (int)Xb, ldi, nI, E, F, G, H, tiles + t0, (int)((t0 / gen) & 1) | (fresh ? 2 : 0));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------------
// FP32 instantiation for the mixed-precision path: E, F and G in FP32, FP32 arithmetic and FP32
// accumulation over one grid-point chunk, added into the FP64 H at its end.  With 4-byte
// accumulators a wave holds an 8 (Y) x 8 (Z) patch (64 + 64 mirror accumulators in 128 VGPRs),
// so a workgroup of four waves owns a whole 16 x 16 (Y, Z) block pair: per output a third of the
// LDS reads and half the copied bytes of the FP64 kernel.  G is stored in 16 x 16 blocks
// ([I][Pp/16][Pp/16][16][16]); the tile's G^YZ block (Yb, Zb) is copied as it is, its G^ZY block
// (Zb, Yb) with its 16-byte granules swizzled (row zz, granule g at position 4 zz + (g ^ ((zz / 2)
// % 4))), so that the column pieces a wave broadcasts from it fall on distinct LDS banks.  G is
// broadcast into the FMAs by DPP row_newbcast as in the FP64 kernel (16 values to a VGPR).
constexpr int W8 = 8;                           // patch edge (Y and Z) per wave
constexpr int S32_PAIR = 64 * 2 * 4;            // one row pair of 64 X (FP32): 512 bytes
constexpr int S32_EY = 0, S32_FY = 8 * S32_PAIR, S32_EZ = 16 * S32_PAIR, S32_FZ = 24 * S32_PAIR;
constexpr int S32_G = 32 * S32_PAIR, S32_GT = S32_G + 1024, S32_STAGE = S32_GT + 1024;  // 18 KB
constexpr int S32_NS = 4;
static_assert(S32_NS * S32_STAGE * 2 <= 160 * 1024, "two workgroups per CU");

// One row j of the wave patch (eight Z): t_k = ey fz_k + ez_k fy, then acc_k += G^YZ t_k and
// accm_k += G^ZY t_k, G broadcast from lane B + k of each row of 16 lanes (B = 8 (j % 2)).  Every
// DPP read comes at least two instructions after the VALU write of its t_k.
template <int B>
__device__ inline void h_row32(float (&acc)[W8], float (&accm)[W8], float ey, float fy, const float (&ez)[W8],
                               const float (&fz)[W8], float g, float gm) {
  float t0, t1, t2, t3, t4, t5, t6, t7;
  asm("v_mul_f32 %[t0], %[ey], %[f0]\n\t"
      "v_mul_f32 %[t1], %[ey], %[f1]\n\t"
      "v_mul_f32 %[t2], %[ey], %[f2]\n\t"
      "v_mul_f32 %[t3], %[ey], %[f3]\n\t"
      "v_mul_f32 %[t4], %[ey], %[f4]\n\t"
      "v_mul_f32 %[t5], %[ey], %[f5]\n\t"
      "v_mul_f32 %[t6], %[ey], %[f6]\n\t"
      "v_mul_f32 %[t7], %[ey], %[f7]\n\t"
      "v_fmac_f32 %[t0], %[e0], %[fy]\n\t"
      "v_fmac_f32 %[t1], %[e1], %[fy]\n\t"
      "v_fmac_f32 %[t2], %[e2], %[fy]\n\t"
      "v_fmac_f32 %[t3], %[e3], %[fy]\n\t"
      "v_fmac_f32 %[t4], %[e4], %[fy]\n\t"
      "v_fmac_f32 %[t5], %[e5], %[fy]\n\t"
      "v_fmac_f32 %[t6], %[e6], %[fy]\n\t"
      "v_fmac_f32 %[t7], %[e7], %[fy]\n\t"
      "v_fmac_f32_dpp %[a0], %[g], %[t0] row_newbcast:%[b0]\n\t"
      "v_fmac_f32_dpp %[m0], %[gm], %[t0] row_newbcast:%[b0]\n\t"
      "v_fmac_f32_dpp %[a1], %[g], %[t1] row_newbcast:%[b1]\n\t"
      "v_fmac_f32_dpp %[m1], %[gm], %[t1] row_newbcast:%[b1]\n\t"
      "v_fmac_f32_dpp %[a2], %[g], %[t2] row_newbcast:%[b2]\n\t"
      "v_fmac_f32_dpp %[m2], %[gm], %[t2] row_newbcast:%[b2]\n\t"
      "v_fmac_f32_dpp %[a3], %[g], %[t3] row_newbcast:%[b3]\n\t"
      "v_fmac_f32_dpp %[m3], %[gm], %[t3] row_newbcast:%[b3]\n\t"
      "v_fmac_f32_dpp %[a4], %[g], %[t4] row_newbcast:%[b4]\n\t"
      "v_fmac_f32_dpp %[m4], %[gm], %[t4] row_newbcast:%[b4]\n\t"
      "v_fmac_f32_dpp %[a5], %[g], %[t5] row_newbcast:%[b5]\n\t"
      "v_fmac_f32_dpp %[m5], %[gm], %[t5] row_newbcast:%[b5]\n\t"
      "v_fmac_f32_dpp %[a6], %[g], %[t6] row_newbcast:%[b6]\n\t"
      "v_fmac_f32_dpp %[m6], %[gm], %[t6] row_newbcast:%[b6]\n\t"
      "v_fmac_f32_dpp %[a7], %[g], %[t7] row_newbcast:%[b7]\n\t"
      "v_fmac_f32_dpp %[m7], %[gm], %[t7] row_newbcast:%[b7]"
      : [a0] "+v"(acc[0]), [a1] "+v"(acc[1]), [a2] "+v"(acc[2]), [a3] "+v"(acc[3]), [a4] "+v"(acc[4]),
        [a5] "+v"(acc[5]), [a6] "+v"(acc[6]), [a7] "+v"(acc[7]), [m0] "+v"(accm[0]), [m1] "+v"(accm[1]),
        [m2] "+v"(accm[2]), [m3] "+v"(accm[3]), [m4] "+v"(accm[4]), [m5] "+v"(accm[5]), [m6] "+v"(accm[6]),
        [m7] "+v"(accm[7]), [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3), [t4] "=&v"(t4),
        [t5] "=&v"(t5), [t6] "=&v"(t6), [t7] "=&v"(t7)
      : [ey] "v"(ey), [fy] "v"(fy), [e0] "v"(ez[0]), [e1] "v"(ez[1]), [e2] "v"(ez[2]), [e3] "v"(ez[3]),
        [e4] "v"(ez[4]), [e5] "v"(ez[5]), [e6] "v"(ez[6]), [e7] "v"(ez[7]), [f0] "v"(fz[0]), [f1] "v"(fz[1]),
        [f2] "v"(fz[2]), [f3] "v"(fz[3]), [f4] "v"(fz[4]), [f5] "v"(fz[5]), [f6] "v"(fz[6]), [f7] "v"(fz[7]),
        [g] "v"(g), [gm] "v"(gm), [b0] "n"(B), [b1] "n"(B + 1), [b2] "n"(B + 2), [b3] "n"(B + 3),
        [b4] "n"(B + 4), [b5] "n"(B + 5), [b6] "n"(B + 6), [b7] "n"(B + 7));
}

__global__ __launch_bounds__(256) void h32_kernel(int Pp, int Xb, int64_t ldi, int64_t nI, const float* __restrict__ E,
                                                  const float* __restrict__ F, const float* __restrict__ G,
                                                  double* __restrict__ H, const uint32_t* __restrict__ tiles,
                                                  int flags) {
  __shared__ __attribute__((aligned(16))) char lds[S32_NS * S32_STAGE];
  const uint32_t tile = tiles[blockIdx.x];
  if (tile & EMPTY) return;  // whole workgroup, before any barrier
  const bool rev = flags & 1;
  const bool fresh = flags & 2;
  const int Yb = tile & 511, Zb = (tile >> 9) & 511, xt = (tile >> 20) & 1023;
  const bool mirror = Yb != Zb;
  const int y0 = Yb * BY, z0 = Zb * BY, X0 = xt * LANES;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __builtin_assume(w >= 0 && w < 4);
  const int ly0 = (w & 1) * W8, lz0 = (w >> 1) * W8;

  // a diagonal block has no mirror: its G^ZY slots stay zero (never copied)
  if (!mirror)
    for (int i = threadIdx.x; i < 256; i += 256)
#pragma unroll
      for (int b = 0; b < S32_NS; ++b) ((float*)(lds + b * S32_STAGE + S32_GT))[i] = 0.0f;

  float acc[W8][W8], accm[W8][W8];
#pragma unroll
  for (int j = 0; j < W8; ++j)
#pragma unroll
    for (int k = 0; k < W8; ++k) acc[j][k] = accm[j][k] = 0.0f;

  // copies of one stage: wave w takes row chunks w, w + 4, w + 8, w + 12 (1 KB = two row pairs
  // each: E^Y, F^Y, E^Z, F^Z four chunks apiece); wave 0 also the G^YZ block, wave 1 (off the
  // diagonal) the G^ZY block, lane l fetching the source granule the swizzle puts at position l
  const unsigned voff_r = (unsigned)(lane >> 5) * S32_PAIR + (unsigned)(lane & 31) * 16u;
  const bool g_yz = w == 0, g_zy = w == 1 && mirror;
  const bool extra = g_yz || g_zy;
  const unsigned nb16 = (unsigned)Pp / 16u;
  const int gz_row = lane >> 2, gz_gran = (lane & 3) ^ ((gz_row >> 1) & 3);
  const unsigned voff_g = g_zy ? (unsigned)(gz_row * 16 + 4 * gz_gran) * 4u : (unsigned)lane * 16u;
  const unsigned so_g = (g_zy ? (unsigned)Zb * nb16 + (unsigned)Yb : (unsigned)Yb * nb16 + (unsigned)Zb) * 1024u;
  const int64_t PX = (int64_t)Pp * LANES;
  const int64_t PP = (int64_t)Pp * Pp;
  const int64_t first = (rev && nI > 0) ? nI - 1 : 0;
  const float* e_at = E + ((int64_t)xt * ldi + first) * PX;
  const float* f_at = F + ((int64_t)xt * ldi + first) * PX;
  const float* g_at = G + first * PP;
  const int64_t dPX = rev ? -PX : PX, dPP = rev ? -PP : PP;
  auto stage_in = [&](int buf) {
    const __amdgpu_buffer_rsrc_t re = rsrc(e_at, PX * 4);
    const __amdgpu_buffer_rsrc_t rf = rsrc(f_at, PX * 4);
    char* sb = lds + buf * S32_STAGE;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = w + 4 * q;      // chunk: region c / 4 (E^Y, F^Y, E^Z, F^Z), pairs 2 (c % 4), + 1
      const int reg = c >> 2;
      const int pair0 = (reg < 2 ? y0 : z0) / 2 + 2 * (c & 3);
      bload_lds((reg & 1) ? rf : re, sb + c * 1024, voff_r, (unsigned)pair0 * S32_PAIR);
    }
    if (extra) bload_lds(rsrc(g_at, PP * 4), sb + (g_yz ? S32_G : S32_GT), voff_g, so_g);
    e_at += dPX;
    f_at += dPX;
    g_at += dPP;
  };

  // broadcast sources: lane l holds G^YZ[ly0 + 2 r + m / 8][lz0 + m % 8] and G^ZY[lz0 + m % 8][ly0 +
  // 2 r + m / 8] (r = 0..3, m = l % 16); the G^ZY row zz = lz0 + m % 8 lies at granule position
  // 4 zz + (g ^ ((zz / 2) % 4)) for its column granule g
  const int m = lane & 15;
  const int goff = (ly0 + (m >> 3)) * 16 + lz0 + (m & 7);
  const int gzz = lz0 + (m & 7);
  int gmoff[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int yy = ly0 + 2 * r + (m >> 3);
    gmoff[r] = (gzz * 4 + ((yy >> 2) ^ ((gzz >> 1) & 3))) * 4 + (yy & 3);
  }

  constexpr int D = S32_NS - 1;
  auto next = [](int b) { return b + 1 == S32_NS ? 0 : b + 1; };
  int sbuf = 0;
  int64_t issued = 0;
  for (; issued < D && issued < nI; ++issued) {
    stage_in(sbuf);
    sbuf = next(sbuf);
  }
  wait_pipe<4>((int)(issued > 0 ? issued - 1 : 0), extra);
  int buf = 0;
  auto consume = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(1);
    const char* __restrict__ st = lds + buf * S32_STAGE;
    const float* __restrict__ sg = (const float*)(st + S32_G);
    const float* __restrict__ sgt = (const float*)(st + S32_GT);
    auto pair = [&](int off, int p) { return *(const f2*)(st + off + p * S32_PAIR + lane * 8); };
    float ez[W8], fz[W8];
#pragma unroll
    for (int q = 0; q < W8 / 2; ++q) {
      const f2 a = pair(S32_EZ, lz0 / 2 + q), b = pair(S32_FZ, lz0 / 2 + q);
      ez[2 * q] = a.x; ez[2 * q + 1] = a.y;
      fz[2 * q] = b.x; fz[2 * q + 1] = b.y;
    }
    float g[4], gm[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      g[r] = sg[goff + 32 * r];
      gm[r] = sgt[gmoff[r]];
    }
#pragma unroll
    for (int p = 0; p < W8 / 2; ++p) {
      const f2 ey = pair(S32_EY, ly0 / 2 + p), fy = pair(S32_FY, ly0 / 2 + p);
      h_row32<0>(acc[2 * p], accm[2 * p], ey.x, fy.x, ez, fz, g[p], gm[p]);
      h_row32<8>(acc[2 * p + 1], accm[2 * p + 1], ey.y, fy.y, ez, fz, g[p], gm[p]);
    }
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
  };
  const int64_t steady = nI - D;
  for (int64_t I = 0; I < steady; ++I) {
    stage_in(sbuf);
    sbuf = next(sbuf);
    consume();
    wait_pipe<4>(D - 1, extra);
    buf = next(buf);
  }
  for (int64_t I = steady > 0 ? steady : 0; I < nI; ++I) {
    consume();
    const int64_t later = nI - I - 2;
    wait_pipe<4>((int)(later > 0 ? later : 0), extra);
    buf = next(buf);
  }

  // H (FP64, [Pp][Pp][Xb]) = or += the chunk's sums
  const unsigned xrow = (unsigned)Xb * 8u;
  const unsigned lo = (unsigned)lane * 8u;
  const double* Hw = H + ((int64_t)(y0 + ly0) * Pp + z0 + lz0) * Xb + X0;
  const double* Hm = H + ((int64_t)(z0 + lz0) * Pp + y0 + ly0) * Xb + X0;
  const int64_t h_bytes = ((int64_t)(W8 - 1) * Pp + W8) * Xb * 8;
  const __amdgpu_buffer_rsrc_t rh = rsrc(Hw, h_bytes);
  const __amdgpu_buffer_rsrc_t rm = rsrc(Hm, h_bytes);
#pragma unroll
  for (int j = 0; j < W8; ++j)
#pragma unroll
    for (int k = 0; k < W8; ++k) {
      const unsigned o = (unsigned)(j * Pp + k) * xrow;
      const double v = fresh ? (double)acc[j][k] : bload(rh, lo, o) + (double)acc[j][k];
      bstore(v, rh, lo, o);
    }
  if (mirror) {
#pragma unroll
    for (int j = 0; j < W8; ++j)
#pragma unroll
      for (int k = 0; k < W8; ++k) {
        const unsigned o = (unsigned)(k * Pp + j) * xrow;
        const double v = fresh ? (double)accm[j][k] : bload(rm, lo, o) + (double)accm[j][k];
        bstore(v, rm, lo, o);
      }
  }
}

constexpr int H_NWZ = 2, H_NS = 3;    // 4 waves, 26 KB stages, three stages (two workgroups per CU)

}  // namespace

// Resident workgroups per XCD (8 XCDs; workgroup b runs on XCD b % 8): CUs per XCD times the
// workgroups of the FP64 kernel that fit on one CU.
int64_t h_slots_per_xcd() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, h_kernel<H_NWZ, H_NS, double>,
                                                   Geo<H_NWZ, H_NS, double>::NTHREADS, 0) != hipSuccess)
    return 0;
  return std::max<int64_t>(1, (int64_t)(cus / 8) * std::max(per_cu, 1));
}

// Tile table: every (X tile, Y block Yb, Z block Zb >= Yb, Z slice) once, in runs of `slots`
// tiles that share an X tile and a Hilbert-curve patch of block pairs; run c sits at workgroup ids
// b = 8 slots (c / 8) + 8 k + (c % 8), k < slots, so that it runs on one XCD.  Unused entries are
// EMPTY.
std::vector<uint32_t> h_tiles(int64_t Pp, int64_t Xb, int64_t slots) {
  return tiles_for<BY / (WZ * H_NWZ)>(Pp, Xb, slots);
}

hipError_t h_accumulate(int64_t Pp, int64_t Xb, int64_t ldi, int64_t nI, const double* E, const double* F,
                        const double* G, double* H, const uint32_t* tiles, int64_t ntiles, int64_t slots,
                        bool fresh, hipStream_t s) {
  return launch<H_NWZ, H_NS, double>(Pp, Xb, ldi, nI, E, F, G, H, tiles, ntiles, slots, fresh, s);
}

int64_t h32_slots_per_xcd() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, h32_kernel, 256, 0) != hipSuccess)
    return 0;
  return std::max<int64_t>(1, (int64_t)(cus / 8) * std::max(per_cu, 1));
}

std::vector<uint32_t> h32_tiles(int64_t Pp, int64_t Xb, int64_t slots) { return tiles_for<1>(Pp, Xb, slots); }

hipError_t h_accumulate_f32(int64_t Pp, int64_t Xb, int64_t ldi, int64_t nI, const float* E, const float* F,
                            const float* G, double* H, const uint32_t* tiles, int64_t ntiles, int64_t slots,
                            bool fresh, hipStream_t s) {
  if (Pp % BY != 0 || Pp <= 0 || Pp > 8192 || Xb % LANES != 0 || Xb > (Pp + LANES - 1) / LANES * LANES || Xb <= 0 ||
      ntiles <= 0 || ntiles > 2147483647LL || nI < 0 || ldi < nI || slots < 1 || ntiles % (8 * slots) != 0)
    return hipErrorInvalidValue;
  const int64_t gen = 8 * slots;
  for (int64_t t0 = 0; t0 < ntiles; t0 += gen) {
    hipLaunchKernelGGL(h32_kernel, dim3((unsigned)gen), dim3(256), 0, s, (int)Pp, (int)Xb, ldi, nI, E, F, G, H,
                       tiles + t0, (int)((t0 / gen) & 1) | (fresh ? 2 : 0));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace thc
