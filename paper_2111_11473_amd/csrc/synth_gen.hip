// Device generation of the seeded synthetic inputs (the twin of the Python generator, through
// the shared synth_core.h): normals of a stream, the Cholesky vectors L^K_pq = gamma N(0,1)
// e^(-K/decay) (symmetric: element (p, q) is draw K n^2 + min(p,q) n + max(p,q)), written
// straight into the blocks the residual reads (oo, ov, vv) or as whole n x n matrices, and the
// power iteration that fixes the global scale gamma from lambda_max(L_ov L_ov^T).
// The generation is elementwise (one hash, a logarithm and a cosine series per value): a pure
// compute stream with one coalesced store per value.
#include <algorithm>

#include "internal.h"
#include "synth_core.h"

namespace thc {
namespace {

constexpr int TPB = 256;

unsigned grid_for(int64_t n) {
  const int64_t b = (n + TPB - 1) / TPB;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

__global__ __launch_bounds__(TPB) void normals_kernel(uint64_t key, uint64_t first, int64_t count, double divisor,
                                                      double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < count; i += (int64_t)gridDim.x * TPB)
    out[i] = thc_synth::normal(key, first + (uint64_t)i) / divisor;
}

// Value (p, q) of Cholesky vector K, scaled by gamma (gamma = 1: unscaled).
__device__ inline double chol_value(uint64_t key, int64_t n, int64_t K, int64_t p, int64_t q, double decay,
                                    double gamma) {
  const int64_t a = p < q ? p : q, b = p < q ? q : p;
  const double x = thc_synth::normal(key, (uint64_t)(K * n * n + a * n + b)) * thc_synth::decay_factor(K, decay);
  return x * gamma;
}

// One block of rows [r0, r0 + nr) x columns [c0, c0 + nc) of vectors K0 .. K0 + nK - 1 into
// out[K - K0][r - r0][c - c0] (row pitch nc, matrix pitch nr nc).
__global__ __launch_bounds__(TPB) void chol_block_kernel(uint64_t key, int64_t n, int64_t K0, int64_t nK, int64_t r0,
                                                         int64_t nr, int64_t c0, int64_t nc, double decay,
                                                         double gamma, double* __restrict__ out) {
  const int64_t per = nr * nc, total = nK * per;
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < total; e += (int64_t)gridDim.x * TPB) {
    const int64_t k = e / per, rc = e - k * per, r = rc / nc, c = rc - r * nc;
    out[e] = chol_value(key, n, K0 + k, r0 + r, c0 + c, decay, gamma);
  }
}

__global__ __launch_bounds__(TPB) void scale_kernel(int64_t n, double a, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) x[i] = x[i] * a;
}

// x = y / sqrt(dot) (the normalization step of the power iteration; dot = |y|^2 on the device)
__global__ __launch_bounds__(TPB) void normalize_kernel(int64_t n, const double* __restrict__ y,
                                                        const double* __restrict__ dot, double* __restrict__ x) {
  const double nrm = sqrt(*dot);
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) x[i] = y[i] / nrm;
}

}  // namespace

hipError_t synth_normals(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, double divisor, double* out,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(normals_kernel, dim3(grid_for(count)), dim3(TPB), 0, s, thc_synth::key(seed, stream), first,
                     count, divisor, out);
  return hipGetLastError();
}

hipError_t synth_chol_block(uint64_t seed, int64_t n, int64_t K0, int64_t nK, int64_t r0, int64_t nr, int64_t c0,
                            int64_t nc, double decay, double gamma, double* out, hipStream_t s) {
  if (nK <= 0 || nr <= 0 || nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_block_kernel, dim3(grid_for(nK * nr * nc)), dim3(TPB), 0, s,
                     thc_synth::key(seed, thc_synth::CHOL), n, K0, nK, r0, nr, c0, nc, decay, gamma, out);
  return hipGetLastError();
}

hipError_t synth_scale(int64_t n, double a, double* x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(TPB), 0, s, n, a, x);
  return hipGetLastError();
}

hipError_t synth_normalize(int64_t n, const double* y, const double* dot, double* x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(n)), dim3(TPB), 0, s, n, y, dot, x);
  return hipGetLastError();
}

void synth_energies(uint64_t seed, int64_t o, int64_t v, double* eps) {
  THC_NOCONTRACT
  const uint64_t ko = thc_synth::key(seed, thc_synth::EPS_O), kv = thc_synth::key(seed, thc_synth::EPS_V);
  for (int64_t i = 0; i < o; ++i) eps[i] = -1.5 + 1.2 * thc_synth::uniform(ko, (uint64_t)i);
  for (int64_t a = 0; a < v; ++a) eps[o + a] = 0.1 + 4.9 * thc_synth::uniform(kv, (uint64_t)a);
  std::sort(eps, eps + o);
  std::sort(eps + o, eps + o + v);
}

}  // namespace thc
