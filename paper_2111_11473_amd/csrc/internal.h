// Internal declarations of the THC-CCSD HIP library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "hostla.h"

namespace thc {

// Row-major batched GEMM descriptor:
//   C[b](m, n) = alpha * sum_k opA(m, k) opB(k, n) * hmul(m, n) + beta * C[b](m, n)
// opA(m, k) = transA ? A[k*lda + m] : A[m*lda + k], scaled by kscaleA[k*ksA + b*sksA] if given;
// opB(k, n) = transB ? B[n*ldb + k] : B[k*ldb + n], scaled by kscaleB[k*ksB + b*sksB] if given.
// hmul (optional) multiplies the product elementwise: hmul[m*ldh + n + b*sH].
// ksplit > 1 splits K into ksplit slices; slice s writes to C + s*sSplit (the caller reduces).
struct Gemm {
  int64_t M = 0, N = 0, K = 0;
  bool transA = false, transB = false;
  const double* A = nullptr; int64_t lda = 0, sA = 0;
  const double* B = nullptr; int64_t ldb = 0, sB = 0;
  double* C = nullptr; int64_t ldc = 0, sC = 0;
  double alpha = 1.0, beta = 0.0;
  const double* kscaleA = nullptr; int64_t ksA = 1, sksA = 0;
  const double* kscaleB = nullptr; int64_t ksB = 1, sksB = 0;
  const double* hmul = nullptr; int64_t ldh = 0, sH = 0;
  int64_t batch = 1;
  int ksplit = 1; int64_t sSplit = 0;
  bool pair_rows = false;  // C element (m, n) at C[((m / 2) ldc + n) 2 + m % 2]: rows interleaved in pairs
  // With pair_rows and xtile: columns cut into tiles of 64, each tile a [ldc][64][2] block of row
  // pairs: C[(((n / 64) ldc + m / 2) 64 + n % 64) 2 + m % 2].
  bool xtile = false;
  // cblk > 0: C cut into 16 x cblk blocks, block-row-major, each block row-major:
  // C[((m / 16) (ldc / cblk) + n / cblk) 16 cblk + (m % 16) cblk + n % cblk] (ldc % cblk == 0).
  int cblk = 0;
  // upper: only the tiles holding some element (m, n) with m <= n are computed (every such
  // element is); the others are left untouched.  For symmetric products (M == N).
  bool upper = false;
  bool f32 = false;        // FP32 MFMA (operands rounded to FP32, FP32 accumulation)
  bool bf16x3 = false;     // split-BF16 products (hi hi + hi lo + lo hi, FP32 accumulation)
  bool keep64 = false;     // stays FP64 in the mixed-precision path
  float* Cf = nullptr;     // FP32 output instead of C (requires f32 and beta = 0)
  // Workspace for an automatic split of K (products with few output tiles and a long K); the
  // partial products go here and a reduction applies the epilogue.  Optional.
  double* ws = nullptr; int64_t ws_len = 0;
};

hipError_t gemm_f64(const Gemm& g, hipStream_t s);
// Tile edge (128 or 64) that gemm_f64 runs a product on when its K split is given explicitly
// (g.ksplit; no batch folding or automatic split applies, as for the symmetric upper products).
int gemm_tile_edge_split(const Gemm& g);

// Elementwise / reduction kernels (kernels_misc.hip).
hipError_t k_form_C(int64_t P, int64_t nb, const double* Bvv, const double* Boo, const double* Go,
                    const double* Gv, double* Ccat, double* C3, hipStream_t s);
hipError_t k_colsum_rowscaled(int64_t nb, int64_t rows, int64_t P, const double* Y, const double* W,
                              int64_t sW, double* out, int64_t ldo, hipStream_t s);
hipError_t k_hadamard_energy(int64_t P, int64_t nb, const double* T, const double* MT, double* F,
                             double* epart, hipStream_t s);
hipError_t k_batch_sum(int64_t nb, int64_t len, const double* X, double alpha, double* out, hipStream_t s);
// out[i][j] += alpha sum_b X_b[min(i, j)][max(i, j)] (X: nb upper-triangle-valid P x P matrices).
hipError_t k_batch_sum_sym(int64_t nb, int64_t P, const double* X, double alpha, double* out, hipStream_t s);
hipError_t k_wsum(int64_t nb, int64_t len, const double* w, const double* X, int64_t sX, double alpha,
                  double* out, hipStream_t s);
hipError_t k_copy2d(int64_t batch, int64_t rows, int64_t cols, const double* src, int64_t lds, int64_t sbs,
                    double* dst, int64_t ldd, int64_t sbd, bool transpose, hipStream_t s);
hipError_t k_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t k_hadamard(int64_t n, const double* x, const double* y, double alpha, double beta, double* out,
                      hipStream_t s);
hipError_t k_sym_add(int64_t P, const double* Q, double alpha, double* out, hipStream_t s);
hipError_t k_dot_cols(int64_t P, int64_t nb, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                      double* out, hipStream_t s);
// y = A x for an M x K row-major A (one workgroup per row)
hipError_t k_gemv(int64_t M, int64_t K, const double* A, int64_t lda, const double* x, double* y, hipStream_t s);
hipError_t k_diag(int64_t P, const double* X, int64_t ldx, double* d, hipStream_t s);
hipError_t k_trace_sq(int64_t nb, int64_t o, const double* K, double* out, hipStream_t s);
hipError_t k_diag_eri(int64_t P, int64_t Q, int64_t o, const double* xo, const double* Rx, double* Cx,
                      hipStream_t s);
hipError_t k_dot(int64_t n, const double* x, const double* y, double* out, hipStream_t s);
hipError_t k_sum(int64_t n, const double* x, double* out, hipStream_t s);
hipError_t k_jacobi(int64_t P, int64_t o, int64_t v, const double* sh, const double* e, const double* delta, const double* s1,
                    const double* eps, double* Th, double* t1, double* dT, double* dt1, hipStream_t s);
hipError_t k_guess_features(int64_t P, int64_t o, int64_t v, const double* Th, const double* e, const double* eps,
                            const double* fro2, float* phi, hipStream_t s);
hipError_t k_guess_apply(int64_t P, const float* pred, int64_t ld, double* Th, double* delta, hipStream_t s);
hipError_t k_lincomb(int64_t n, int m, const double* coef, const double* const* vecs, double* out, hipStream_t s);
hipError_t k_kr(int64_t o, int64_t v, int64_t P, const double* Yo, const double* Yv, double* B, hipStream_t s);
hipError_t k_mp2_denom(int64_t rows0, int64_t rows, int64_t ov, int64_t v, const double* eps, int64_t o,
                       double* X, hipStream_t s);
hipError_t k_fill(int64_t n, double val, double* x, hipStream_t s);
hipError_t k_set_diag(int64_t n, const double* d, double* X, int64_t ld, hipStream_t s);

// Synthetic inputs on the device (synth_gen.hip; values bit-identical to the Python generator).
// out[i] = N(0,1) draw first + i of (seed, stream) / divisor.
hipError_t synth_normals(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, double divisor, double* out,
                         hipStream_t s);
// Rows [r0, r0 + nr) x columns [c0, c0 + nc) of Cholesky vectors K0 .. K0 + nK - 1 (n x n each),
// times gamma, into out[nK][nr][nc].
hipError_t synth_chol_block(uint64_t seed, int64_t n, int64_t K0, int64_t nK, int64_t r0, int64_t nr, int64_t c0,
                            int64_t nc, double decay, double gamma, double* out, hipStream_t s);
hipError_t synth_scale(int64_t n, double a, double* x, hipStream_t s);
// x = y / sqrt(*dot)
hipError_t synth_normalize(int64_t n, const double* y, const double* dot, double* x, hipStream_t s);
// Orbital energies (host): o occupied then v virtual, each sorted ascending.
void synth_energies(uint64_t seed, int64_t o, int64_t v, double* eps);

// Weighted CP-ALS pieces (cpals.hip).
hipError_t cp_weighted_rows(int64_t m, int64_t n, const double* w, const double* X, double* out, hipStream_t s);
hipError_t cp_mttkrp_reduce(int64_t I, int64_t J, int64_t n, const double* T, const double* V, bool over_j,
                            double* out, hipStream_t s);
int64_t cp_wnorm2_parts(int64_t I, int64_t J, int64_t K);
hipError_t cp_wnorm2(int64_t I, int64_t J, int64_t K, const double* A, const double* w1, const double* w2,
                     const double* w3, double* part, hipStream_t s);
hipError_t cp_col_dot(int64_t n, int64_t m, const double* A, const double* B, double* out, hipStream_t s);
hipError_t cp_cg_step(int64_t n, int64_t m, const double* rz, const double* pq, const double* P, const double* Q,
                      double* U, double* R, hipStream_t s);
hipError_t cp_cg_precond(int64_t n, int64_t m, const double* d, const double* R, double* Zr, hipStream_t s);
hipError_t cp_cg_dir(int64_t n, int64_t m, const double* rz_new, const double* rz_old, const double* Zr, double* P,
                     hipStream_t s);
hipError_t cp_diag(int64_t n, const double* S, double* d, hipStream_t s);

// Fused exchange contraction Gt^X = xo (z o (xo^T Rx^X))^T for X = 0..nx-1 (kernels_exch.hip);
// xo [o][Q], z [Q][Q], Rx and Gt [nx][o][Q].  Supported for 1 <= o <= 200.  f32: operands rounded
// to FP32, FP32 MFMA and accumulation (the mixed-precision path); else FP64 throughout.
bool exch_supported(int64_t o);
hipError_t exch_fused(int64_t o, int64_t Q, int64_t nx, const double* xo, const double* z, const double* Rx,
                      double* Gt, bool f32, hipStream_t s);

// Learned-guess network kernels (mlp.hip).  sgemm epilogues: 0 none, 1 bias + SiLU (pre-activation
// to Z), 2 bias, 3 times SiLU'(Z).
// Floats in the per-device scratch array of the allocation-free forward pass (32 MiB).
constexpr int64_t MLP_SCRATCH_FLOATS = int64_t(1) << 23;
// Device address of that array on the current device (looked up once per device, then cached).
hipError_t mlp_scratch_resolve(float** out);
// epi: 0 none, 1 bias + SiLU keeping the pre-activation in Z, 2 bias, 3 times SiLU'(Z),
// 4 bias + SiLU without Z
hipError_t mlp_sgemm(bool tA, bool tB, int epi, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                     const float* B, int64_t ldb, float* C, int64_t ldc, const float* bias, float* Z, int64_t ldz,
                     hipStream_t s);
hipError_t mlp_normalize(int64_t rows, int64_t cols, const float* X, const float* mu, const float* sd, float* Xn,
                         hipStream_t s);
hipError_t mlp_denorm(int64_t rows, int64_t cols, const float* Yn, const float* mu, const float* sd, float* Y,
                      hipStream_t s);
hipError_t mlp_mse_grad(int64_t rows, int64_t cols, const float* Yn, const float* T, const float* mu, const float* sd,
                        float* dY, double* part, int64_t nparts, float* loss, hipStream_t s);
hipError_t mlp_colsum(int64_t rows, int64_t cols, const float* D, float* out, hipStream_t s);
hipError_t mlp_colstats(int64_t rows, int64_t cols, const float* D, float* mu, float* sd, hipStream_t s);
hipError_t mlp_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    int64_t step, hipStream_t s);
hipError_t mlp_init(int64_t n_in, int64_t w, int64_t n_out, uint64_t seed, float* p, hipStream_t s);
bool mlp_infer_supported(int64_t n_in, int64_t w, int64_t n_out);
int64_t mlp_bf16_weights(int64_t n_in);
int64_t mlp_bf16_biases();
hipError_t mlp_pack_bf16(int64_t n_in, int64_t n_out, const float* p, short* Wb, float* bias, hipStream_t s);
hipError_t mlp_infer_bf16(int64_t rows, int64_t n_in, int64_t n_out, const float* X, const float* mu_in,
                          const float* sd_in, const short* Wb, const float* bias, const float* mu_out,
                          const float* sd_out, float* Y, hipStream_t s);

// VALU kernel for H^XYZ += sum_I (E^XY F^XZ + E^XZ F^XY) G^YZ (kernels_h.hip).
// E, F: [Xb/64][ldi][Pp/2][64][2] (X tile, grid point, row pair, X within the tile, row of the
// pair); G: [I][Pp/16][Pp/8][16][8] (16 x 8 blocks); H: [Pp][Pp][Xb]; tiles from
// h_tiles(Pp, Xb, slots).  ldi >= nI is the grid-point stride of one X tile of E and F.  fresh:
// H = the sum instead of H += (every element of H is written: the tiles cover all of it).
hipError_t h_accumulate(int64_t Pp, int64_t Xb, int64_t ldi, int64_t nI, const double* E, const double* F,
                        const double* G, double* H, const uint32_t* tiles, int64_t ntiles, int64_t slots,
                        bool fresh, hipStream_t s);
// FP32 kernel of the mixed-precision path: E, F as above in FP32; G in FP32 16 x 16 blocks,
// [I][Pp/16][Pp/16][16][16]; FP32 arithmetic and accumulation over the chunk, added into the FP64
// H (or written, fresh); tiles from h32_tiles (16 x 16 block pairs).
hipError_t h_accumulate_f32(int64_t Pp, int64_t Xb, int64_t ldi, int64_t nI, const float* E, const float* F,
                            const float* G, double* H, const uint32_t* tiles, int64_t ntiles, int64_t slots,
                            bool fresh, hipStream_t s);
std::vector<uint32_t> h32_tiles(int64_t Pp, int64_t Xb, int64_t slots);
int64_t h32_slots_per_xcd();
constexpr int H_GBLK = 8;  // column width of the G blocks
std::vector<uint32_t> h_tiles(int64_t Pp, int64_t Xb, int64_t slots);
int64_t h_slots_per_xcd();

}  // namespace thc
