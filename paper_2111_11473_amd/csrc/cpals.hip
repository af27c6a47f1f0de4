// Kernels of the weighted CP-ALS (paper Sec. II.c-d, Appendix I): the reductions that finish the
// matricized-tensor-times-Khatri-Rao products after their matrix-product part, and the column-wise
// steps of the block preconditioned conjugate gradients that solve S U = B for every row of a
// factor at once (S the n x n Hadamard product of Gram matrices, preconditioned by its diagonal;
// U, B stored [n][m], column c one right-hand side).  All HBM-bound elementwise passes.
#include "internal.h"

namespace thc {
namespace {

constexpr int TPB = 256;

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 65536)); }

// out[r][c] = w[r]^2 X[r][c] (w null: a copy)
__global__ void weighted_rows_kernel(int64_t m, int64_t n, const double* __restrict__ w, const double* __restrict__ X,
                                     double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < m * n; e += (int64_t)gridDim.x * TPB) {
    const double s = w ? w[e / n] : 1.0;
    out[e] = s * s * X[e];
  }
}

// T[i][j][c] (I x J x n); over_j: out[c][i] = sum_j V[j][c] T[i][j][c]; else out[c][j] = sum_i V[i][c] T[i][j][c]
__global__ void mttkrp_reduce_kernel(int64_t I, int64_t J, int64_t n, const double* __restrict__ T,
                                     const double* __restrict__ V, bool over_j, double* __restrict__ out) {
  const int64_t rows = over_j ? I : J, len = over_j ? J : I;
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < rows * n; e += (int64_t)gridDim.x * TPB) {
    const int64_t r = e / n, c = e % n;
    double s = 0.0;
    if (over_j)
      for (int64_t j = 0; j < len; ++j) s += V[j * n + c] * T[(r * J + j) * n + c];
    else
      for (int64_t i = 0; i < len; ++i) s += V[i * n + c] * T[(i * J + r) * n + c];
    out[c * rows + r] = s;
  }
}

// sum of (w1_i w2_j w3_k A_ijk)^2, one partial per block
__global__ void wnorm2_kernel(int64_t I, int64_t J, int64_t K, const double* __restrict__ A,
                              const double* __restrict__ w1, const double* __restrict__ w2,
                              const double* __restrict__ w3, double* __restrict__ part) {
  __shared__ double red[TPB];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < I * J * K; e += (int64_t)gridDim.x * TPB) {
    const int64_t k = e % K, ij = e / K, j = ij % J, i = ij / J;
    const double w = (w1 ? w1[i] : 1.0) * (w2 ? w2[j] : 1.0) * (w3 ? w3[k] : 1.0);
    const double x = w * A[e];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[c] = sum_r A[r][c] B[r][c]  ([n][m])
__global__ void col_dot_kernel(int64_t n, int64_t m, const double* __restrict__ A, const double* __restrict__ B,
                               double* __restrict__ out) {
  for (int64_t c = (int64_t)blockIdx.x * TPB + threadIdx.x; c < m; c += (int64_t)gridDim.x * TPB) {
    double s = 0.0;
    for (int64_t r = 0; r < n; ++r) s += A[r * m + c] * B[r * m + c];
    out[c] = s;
  }
}

// alpha_c = rz_c / pq_c (0 where pq_c is 0);  U += alpha p;  R -= alpha q
__global__ void cg_step_kernel(int64_t n, int64_t m, const double* __restrict__ rz, const double* __restrict__ pq,
                               const double* __restrict__ P, const double* __restrict__ Qm, double* __restrict__ U,
                               double* __restrict__ R) {
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n * m; e += (int64_t)gridDim.x * TPB) {
    const int64_t c = e % m;
    const double a = pq[c] != 0.0 ? rz[c] / pq[c] : 0.0;
    U[e] += a * P[e];
    R[e] -= a * Qm[e];
  }
}

// Zr = R / d (row-wise diagonal preconditioner)
__global__ void cg_precond_kernel(int64_t n, int64_t m, const double* __restrict__ d, const double* __restrict__ R,
                                  double* __restrict__ Zr) {
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n * m; e += (int64_t)gridDim.x * TPB)
    Zr[e] = R[e] / d[e / m];
}

// P = Zr + (rz_new / rz_old) P  (beta 0 where rz_old is 0)
__global__ void cg_dir_kernel(int64_t n, int64_t m, const double* __restrict__ rz_new, const double* __restrict__ rz_old,
                              const double* __restrict__ Zr, double* __restrict__ P) {
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n * m; e += (int64_t)gridDim.x * TPB) {
    const int64_t c = e % m;
    const double b = rz_old[c] != 0.0 ? rz_new[c] / rz_old[c] : 0.0;
    P[e] = Zr[e] + b * P[e];
  }
}

__global__ void diag_kernel(int64_t n, const double* __restrict__ S, double* __restrict__ d) {
  for (int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x; r < n; r += (int64_t)gridDim.x * TPB) d[r] = S[r * n + r];
}

}  // namespace

#define CP_LAUNCH(kernel, n, ...)                                                      \
  do {                                                                                 \
    hipLaunchKernelGGL(kernel, dim3(grid_of(n)), dim3(TPB), 0, s, __VA_ARGS__);       \
    return hipGetLastError();                                                          \
  } while (0)

hipError_t cp_weighted_rows(int64_t m, int64_t n, const double* w, const double* X, double* out, hipStream_t s) {
  CP_LAUNCH(weighted_rows_kernel, m * n, m, n, w, X, out);
}
hipError_t cp_mttkrp_reduce(int64_t I, int64_t J, int64_t n, const double* T, const double* V, bool over_j,
                            double* out, hipStream_t s) {
  CP_LAUNCH(mttkrp_reduce_kernel, (over_j ? I : J) * n, I, J, n, T, V, over_j, out);
}
int64_t cp_wnorm2_parts(int64_t I, int64_t J, int64_t K) { return (int64_t)grid_of(I * J * K); }
hipError_t cp_wnorm2(int64_t I, int64_t J, int64_t K, const double* A, const double* w1, const double* w2,
                     const double* w3, double* part, hipStream_t s) {
  CP_LAUNCH(wnorm2_kernel, I * J * K, I, J, K, A, w1, w2, w3, part);
}
hipError_t cp_col_dot(int64_t n, int64_t m, const double* A, const double* B, double* out, hipStream_t s) {
  CP_LAUNCH(col_dot_kernel, m, n, m, A, B, out);
}
hipError_t cp_cg_step(int64_t n, int64_t m, const double* rz, const double* pq, const double* P, const double* Q,
                      double* U, double* R, hipStream_t s) {
  CP_LAUNCH(cg_step_kernel, n * m, n, m, rz, pq, P, Q, U, R);
}
hipError_t cp_cg_precond(int64_t n, int64_t m, const double* d, const double* R, double* Zr, hipStream_t s) {
  CP_LAUNCH(cg_precond_kernel, n * m, n, m, d, R, Zr);
}
hipError_t cp_cg_dir(int64_t n, int64_t m, const double* rz_new, const double* rz_old, const double* Zr, double* P,
                     hipStream_t s) {
  CP_LAUNCH(cg_dir_kernel, n * m, n, m, rz_new, rz_old, Zr, P);
}
hipError_t cp_diag(int64_t n, const double* S, double* d, hipStream_t s) { CP_LAUNCH(diag_kernel, n, n, S, d); }

}  // namespace thc
