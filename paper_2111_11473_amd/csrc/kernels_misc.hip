// Elementwise, Hadamard and reduction kernels of the THC-CCSD residual (FP64).
// All are HBM-streaming kernels: one pass over their operands, coalesced along the
// fastest (rank) index, fixed-order reductions so that results are reproducible.
#include "internal.h"

namespace thc {
namespace {

constexpr int TPB = 256;

inline unsigned nblocks(int64_t n, int per = TPB) {
  int64_t b = (n + per - 1) / per;
  if (b > 1048576) b = 1048576;
  return (unsigned)(b < 1 ? 1 : b);
}

// Block-wide sum of one double per thread (blockDim.x == TPB or 1024); result in thread 0.
template <int NT>
__device__ double block_sum(double x) {
  __shared__ double red[NT / 64];
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

// The Hadamard steps of Alg. 1 and Alg. 3 fused: for the nb Cholesky vectors of a block,
// C^A = Go o Bvv^A - Gv o Boo^A written in the [X][A][Y] layout that the C T C^T chain
// reads, and C3 += sum_A Boo^A o Bvv^A.
__global__ void form_C_kernel(int64_t P, int64_t nb, const double* __restrict__ Bvv,
                              const double* __restrict__ Boo, const double* __restrict__ Go,
                              const double* __restrict__ Gv, double* __restrict__ Ccat,
                              double* __restrict__ C3) {
  const int64_t PP = P * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < PP; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t X = e / P, Y = e % P;
    const double go = Go[e], gv = Gv[e];
    double c3 = 0.0;
    for (int64_t A = 0; A < nb; ++A) {
      const double bv = Bvv[A * PP + e], bo = Boo[A * PP + e];
      Ccat[X * nb * P + A * P + Y] = go * bv - gv * bo;
      c3 += bo * bv;
    }
    C3[e] += c3;
  }
}

// out[X * ldo + A] = sum_i Y[i][X] * W[A][i][X]   (a Khatri-Rao contraction of a panel)
__global__ void colsum_rowscaled_kernel(int64_t nb, int64_t rows, int64_t P, const double* __restrict__ Y,
                                        const double* __restrict__ W, int64_t sW, double* __restrict__ out,
                                        int64_t ldo) {
  const int64_t n = nb * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t A = e / P, X = e % P;
    const double* w = W + A * sW + X;
    double s = 0.0;
    for (int64_t i = 0; i < rows; ++i) s += Y[i * P + X] * w[i * P];
    out[X * ldo + A] = s;
  }
}

// F^A = T o (M^A)^T (given MT^A = (M^A)^T) and the exchange energy partial
// sum_YZ F^A_YZ MT^A_ZY = sum_YZ T_YZ M^A_YZ M^A_ZY, one partial per (A, block).
// F[A] = T o M[A] and the partial sums of sum_YZ T[Y][Z] M[A][Y][Z] M[A][Z][Y], by 32 x 32 tiles:
// the tile (Y-block, Z-block) and its transposed partner are both read coalesced (the partner
// through LDS).  Grid (64, nb): block b of matrix A takes tiles b, b + 64, ... and writes its
// sum to epart[A][b].
__global__ __launch_bounds__(TPB) void hadamard_energy_kernel(int64_t P, const double* __restrict__ T,
                                                              const double* __restrict__ MT, double* __restrict__ F,
                                                              double* __restrict__ epart) {
  constexpr int TS = 32;
  __shared__ double mt_s[TS][TS + 1];  // M[Z-block rows][Y-block columns], read transposed
  const int64_t PP = P * P, nt = (P + TS - 1) / TS;
  const int64_t A = blockIdx.y;
  const double* mt = MT + A * PP;
  double* f = F + A * PP;
  const int c = threadIdx.x % TS, r0 = threadIdx.x / TS;  // 8 rows per pass
  double s = 0.0;
  for (int64_t tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
    const int64_t by = tile / nt, bz = tile % nt;
    __syncthreads();  // the previous tile's reads of mt_s are done
#pragma unroll
    for (int k = 0; k < TS / 8; ++k) {
      const int r = r0 + 8 * k;
      const int64_t Zr = bz * TS + r, Yc = by * TS + c;
      mt_s[r][c] = (Zr < P && Yc < P) ? mt[Zr * P + Yc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TS / 8; ++k) {
      const int r = r0 + 8 * k;
      const int64_t Y = by * TS + r, Z = bz * TS + c;
      if (Y < P && Z < P) {
        const int64_t e = Y * P + Z;
        const double x = T[e] * mt[e];
        f[e] = x;
        s += x * mt_s[c][r];  // M[Z][Y]
      }
    }
  }
  s = block_sum<TPB>(s);
  if (threadIdx.x == 0) epart[A * gridDim.x + blockIdx.x] = s;
}

__global__ void batch_sum_kernel(int64_t nb, int64_t len, const double* __restrict__ X, double alpha,
                                 double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t A = 0; A < nb; ++A) s += X[A * len + e];
    out[e] += alpha * s;
  }
}

__global__ void batch_sum_sym_kernel(int64_t nb, int64_t P, const double* __restrict__ X, double alpha,
                                     double* __restrict__ out) {
  const int64_t PP = P * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < PP; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / P, j = e % P;
    const int64_t u = i <= j ? e : j * P + i;
    double s = 0.0;
    for (int64_t A = 0; A < nb; ++A) s += X[A * PP + u];
    out[e] += alpha * s;
  }
}

__global__ void wsum_kernel(int64_t nb, int64_t len, const double* __restrict__ w, const double* __restrict__ X,
                            int64_t sX, double alpha, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t A = 0; A < nb; ++A) s += w[A] * X[A * sX + e];
    out[e] += alpha * s;
  }
}

__global__ void copy2d_kernel(int64_t batch, int64_t rows, int64_t cols, const double* __restrict__ src,
                              int64_t lds, int64_t sbs, double* __restrict__ dst, int64_t ldd, int64_t sbd,
                              int transpose) {
  const int64_t n = batch * rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / (rows * cols), rc = e % (rows * cols);
    const int64_t r = rc / cols, c = rc % cols;
    const double x = transpose ? src[b * sbs + c * lds + r] : src[b * sbs + r * lds + c];
    dst[b * sbd + r * ldd + c] = x;
  }
}

__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + (b == 0.0 ? 0.0 : b * y[e]);
}

__global__ void hadamard_kernel(int64_t n, const double* __restrict__ x, const double* __restrict__ y, double alpha,
                                double beta, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = alpha * x[e] * y[e] + (beta == 0.0 ? 0.0 : beta * out[e]);
}

__global__ void sym_add_kernel(int64_t P, const double* __restrict__ Q, double alpha, double* __restrict__ out) {
  const int64_t n = P * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / P, j = e % P;
    out[e] += alpha * (Q[e] + Q[j * P + i]);
  }
}

__global__ void dot_cols_kernel(int64_t P, int64_t nb, const double* __restrict__ X, int64_t ldx,
                                const double* __restrict__ Y, int64_t ldy, double* __restrict__ out) {
  const int64_t A = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < P; r += blockDim.x) s += X[r * ldx + A] * Y[r * ldy + A];
  s = block_sum<TPB>(s);
  if (threadIdx.x == 0) out[A] = s;
}

// y[m] = sum_k A[m][k] x[k]: one workgroup per row (the row is the long dimension)
__global__ void gemv_kernel(int64_t K, const double* __restrict__ A, int64_t lda, const double* __restrict__ x,
                            double* __restrict__ y) {
  const int64_t m = blockIdx.x;
  const double* a = A + m * lda;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += blockDim.x) s += a[k] * x[k];
  s = block_sum<TPB>(s);
  if (threadIdx.x == 0) y[m] = s;
}

__global__ void diag_kernel(int64_t P, const double* __restrict__ X, int64_t ldx, double* __restrict__ d) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < P; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = X[e * ldx + e];
}

__global__ void trace_sq_kernel(int64_t o, const double* __restrict__ K, double* __restrict__ out) {
  const int64_t A = blockIdx.x;
  const double* k = K + A * o * o;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < o * o; e += blockDim.x) {
    const int64_t i = e / o, j = e % o;
    s += k[e] * k[j * o + i];
  }
  s = block_sum<TPB>(s);
  if (threadIdx.x == 0) out[A] = s;
}

// Cx[X][I] = sum_i xo[i][I] Rx[X][i][I]  (Alg. 7, from the half-transformed R)
__global__ void diag_eri_kernel(int64_t P, int64_t Q, int64_t o, const double* __restrict__ xo,
                                const double* __restrict__ Rx, double* __restrict__ Cx) {
  const int64_t n = P * Q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t X = e / Q, I = e % Q;
    const double* r = Rx + X * o * Q + I;
    double s = 0.0;
    for (int64_t i = 0; i < o; ++i) s += xo[i * Q + I] * r[i * Q];
    Cx[e] = s;
  }
}

__global__ void dot_kernel(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                           double* __restrict__ out) {
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) s += x[e] * (y ? y[e] : 1.0);
  s = block_sum<1024>(s);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void jacobi_kernel(int64_t P, int64_t o, int64_t v, const double* __restrict__ sh,
                              const double* __restrict__ e, const double* __restrict__ delta,
                              const double* __restrict__ s1,
                              const double* __restrict__ eps, double* __restrict__ Th, double* __restrict__ t1,
                              double* __restrict__ dT, double* __restrict__ dt1) {
  const int64_t n2 = P * P, n1 = o * v;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n2 + n1; k += (int64_t)gridDim.x * blockDim.x) {
    if (k < n2) {
      const int64_t p = k / P, q = k % P;
      const double base = e[p] + e[q];
      const double den = delta ? fmax(base + delta[p] + delta[q], 0.5 * base) : base;
      const double d = -sh[k] / den;
      dT[k] = d;
      Th[k] += d;
    } else if (s1) {
      const int64_t m = k - n2, i = m / v, a = m % v;
      const double d = -s1[m] / (eps[o + a] - eps[i]);
      dt1[m] = d;
      t1[m] += d;
    } else {
      dt1[k - n2] = 0.0;
    }
  }
}

// Learned-guess features per rank index P (FP32): [T_PP, e_P, T_PP e_P, eps_HOMO, eps_LUMO,
// mean eps_occ, mean eps_vir, N_P / o, ||T||_F / sqrt(N_P), sum_Q |T_PQ|]; fro2 = ||T||_F^2.
__global__ void guess_features_kernel(int64_t P, int64_t o, int64_t v, const double* __restrict__ Th,
                                      const double* __restrict__ e, const double* __restrict__ eps,
                                      const double* __restrict__ fro2, float* __restrict__ phi) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    double homo = eps[0], lumo = eps[o], so = 0.0, sv = 0.0, rs = 0.0;
    for (int64_t i = 0; i < o; ++i) { homo = fmax(homo, eps[i]); so += eps[i]; }
    for (int64_t a = 0; a < v; ++a) { lumo = fmin(lumo, eps[o + a]); sv += eps[o + a]; }
    for (int64_t q = 0; q < P; ++q) rs += fabs(Th[p * P + q]);
    const double d = Th[p * P + p];
    float* f = phi + p * 10;
    f[0] = (float)d;
    f[1] = (float)e[p];
    f[2] = (float)(d * e[p]);
    f[3] = (float)homo;
    f[4] = (float)lumo;
    f[5] = (float)(so / (double)o);
    f[6] = (float)(sv / (double)v);
    f[7] = (float)((double)P / (double)o);
    f[8] = (float)sqrt(fro2[0] / (double)P);
    f[9] = (float)rs;
  }
}

// T_PQ <- (1 + c_P) T_PQ (1 + c_Q), delta_P <- pred[P][1]; c_P = pred[P][0]
__global__ void guess_apply_kernel(int64_t P, const float* __restrict__ pred, int64_t ld, double* __restrict__ Th,
                                   double* __restrict__ delta) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P * P; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = k / P, q = k % P;
    Th[k] *= (1.0 + (double)pred[p * ld]) * (1.0 + (double)pred[q * ld]);
    if (q == 0 && delta) delta[p] = ld > 1 ? (double)pred[p * ld + 1] : 0.0;
  }
}

struct LinComb {
  const double* v[16];
  double c[16];
};

__global__ void lincomb_kernel(int64_t n, int m, LinComb lc, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += lc.c[k] * lc.v[k][e];
    out[e] = s;
  }
}

__global__ void kr_kernel(int64_t o, int64_t v, int64_t P, const double* __restrict__ Yo,
                          const double* __restrict__ Yv, double* __restrict__ B) {
  const int64_t n = o * v * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ia = e / P, X = e % P;
    const int64_t i = ia / v, a = ia % v;
    B[e] = Yo[i * P + X] * Yv[a * P + X];
  }
}

// X[r][c] <- -X[r][c] / (Delta_{r0+r} + Delta_c), Delta_{ia} = eps_a - eps_i, ia = i*v + a
__global__ void mp2_denom_kernel(int64_t r0, int64_t rows, int64_t ov, int64_t v, const double* __restrict__ eps,
                                 int64_t o, double* __restrict__ X) {
  const int64_t n = rows * ov;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = r0 + e / ov, c = e % ov;
    const double dr = eps[o + r % v] - eps[r / v];
    const double dc = eps[o + c % v] - eps[c / v];
    X[e] = -X[e] / (dr + dc);
  }
}

__global__ void fill_kernel(int64_t n, double val, double* __restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = val;
}

__global__ void set_diag_kernel(int64_t n, const double* __restrict__ d, double* __restrict__ X, int64_t ld) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    X[e * ld + e] += d[e];
}

}  // namespace

#define LAUNCH(kern, grid, block, ...)                                  \
  do {                                                                  \
    hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);           \
    return hipGetLastError();                                           \
  } while (0)

hipError_t k_form_C(int64_t P, int64_t nb, const double* Bvv, const double* Boo, const double* Go, const double* Gv,
                    double* Ccat, double* C3, hipStream_t s) {
  LAUNCH(form_C_kernel, dim3(nblocks(P * P)), dim3(TPB), P, nb, Bvv, Boo, Go, Gv, Ccat, C3);
}
hipError_t k_colsum_rowscaled(int64_t nb, int64_t rows, int64_t P, const double* Y, const double* W, int64_t sW,
                              double* out, int64_t ldo, hipStream_t s) {
  LAUNCH(colsum_rowscaled_kernel, dim3(nblocks(nb * P)), dim3(TPB), nb, rows, P, Y, W, sW, out, ldo);
}
hipError_t k_hadamard_energy(int64_t P, int64_t nb, const double* T, const double* MT, double* F, double* epart,
                             hipStream_t s) {
  // 64 partials per Cholesky vector; epart must hold nb * 64 doubles.
  LAUNCH(hadamard_energy_kernel, dim3(64, (unsigned)nb), dim3(TPB), P, T, MT, F, epart);
}
hipError_t k_batch_sum(int64_t nb, int64_t len, const double* X, double alpha, double* out, hipStream_t s) {
  LAUNCH(batch_sum_kernel, dim3(nblocks(len)), dim3(TPB), nb, len, X, alpha, out);
}
hipError_t k_batch_sum_sym(int64_t nb, int64_t P, const double* X, double alpha, double* out, hipStream_t s) {
  LAUNCH(batch_sum_sym_kernel, dim3(nblocks(P * P)), dim3(TPB), nb, P, X, alpha, out);
}
hipError_t k_wsum(int64_t nb, int64_t len, const double* w, const double* X, int64_t sX, double alpha, double* out,
                  hipStream_t s) {
  LAUNCH(wsum_kernel, dim3(nblocks(len)), dim3(TPB), nb, len, w, X, sX, alpha, out);
}
hipError_t k_copy2d(int64_t batch, int64_t rows, int64_t cols, const double* src, int64_t lds, int64_t sbs,
                    double* dst, int64_t ldd, int64_t sbd, bool transpose, hipStream_t s) {
  LAUNCH(copy2d_kernel, dim3(nblocks(batch * rows * cols)), dim3(TPB), batch, rows, cols, src, lds, sbs, dst, ldd,
         sbd, (int)transpose);
}
hipError_t k_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  LAUNCH(axpby_kernel, dim3(nblocks(n)), dim3(TPB), n, a, x, b, y);
}
hipError_t k_hadamard(int64_t n, const double* x, const double* y, double alpha, double beta, double* out,
                      hipStream_t s) {
  LAUNCH(hadamard_kernel, dim3(nblocks(n)), dim3(TPB), n, x, y, alpha, beta, out);
}
hipError_t k_sym_add(int64_t P, const double* Q, double alpha, double* out, hipStream_t s) {
  LAUNCH(sym_add_kernel, dim3(nblocks(P * P)), dim3(TPB), P, Q, alpha, out);
}
hipError_t k_dot_cols(int64_t P, int64_t nb, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                      double* out, hipStream_t s) {
  LAUNCH(dot_cols_kernel, dim3((unsigned)nb), dim3(TPB), P, nb, X, ldx, Y, ldy, out);
}
hipError_t k_gemv(int64_t M, int64_t K, const double* A, int64_t lda, const double* x, double* y, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (M > 2147483647LL) return hipErrorInvalidValue;
  LAUNCH(gemv_kernel, dim3((unsigned)M), dim3(TPB), K, A, lda, x, y);
}
hipError_t k_diag(int64_t P, const double* X, int64_t ldx, double* d, hipStream_t s) {
  LAUNCH(diag_kernel, dim3(nblocks(P)), dim3(TPB), P, X, ldx, d);
}
hipError_t k_trace_sq(int64_t nb, int64_t o, const double* K, double* out, hipStream_t s) {
  LAUNCH(trace_sq_kernel, dim3((unsigned)nb), dim3(TPB), o, K, out);
}
hipError_t k_diag_eri(int64_t P, int64_t Q, int64_t o, const double* xo, const double* Rx, double* Cx,
                      hipStream_t s) {
  LAUNCH(diag_eri_kernel, dim3(nblocks(P * Q)), dim3(TPB), P, Q, o, xo, Rx, Cx);
}
hipError_t k_dot(int64_t n, const double* x, const double* y, double* out, hipStream_t s) {
  LAUNCH(dot_kernel, dim3(1), dim3(1024), n, x, y, out);
}
hipError_t k_sum(int64_t n, const double* x, double* out, hipStream_t s) {
  LAUNCH(dot_kernel, dim3(1), dim3(1024), n, x, (const double*)nullptr, out);
}
hipError_t k_jacobi(int64_t P, int64_t o, int64_t v, const double* sh, const double* e, const double* delta, const double* s1,
                    const double* eps, double* Th, double* t1, double* dT, double* dt1, hipStream_t s) {
  LAUNCH(jacobi_kernel, dim3(nblocks(P * P + o * v)), dim3(TPB), P, o, v, sh, e, delta, s1, eps, Th, t1, dT, dt1);
}
hipError_t k_guess_features(int64_t P, int64_t o, int64_t v, const double* Th, const double* e, const double* eps,
                            const double* fro2, float* phi, hipStream_t s) {
  LAUNCH(guess_features_kernel, dim3(nblocks(P)), dim3(TPB), P, o, v, Th, e, eps, fro2, phi);
}
hipError_t k_guess_apply(int64_t P, const float* pred, int64_t ld, double* Th, double* delta, hipStream_t s) {
  LAUNCH(guess_apply_kernel, dim3(nblocks(P * P)), dim3(TPB), P, pred, ld, Th, delta);
}
hipError_t k_lincomb(int64_t n, int m, const double* coef, const double* const* vecs, double* out, hipStream_t s) {
  if (m > 16) return hipErrorInvalidValue;
  LinComb lc{};
  for (int k = 0; k < m; ++k) { lc.v[k] = vecs[k]; lc.c[k] = coef[k]; }
  LAUNCH(lincomb_kernel, dim3(nblocks(n)), dim3(TPB), n, m, lc, out);
}
hipError_t k_kr(int64_t o, int64_t v, int64_t P, const double* Yo, const double* Yv, double* B, hipStream_t s) {
  LAUNCH(kr_kernel, dim3(nblocks(o * v * P)), dim3(TPB), o, v, P, Yo, Yv, B);
}
hipError_t k_mp2_denom(int64_t r0, int64_t rows, int64_t ov, int64_t v, const double* eps, int64_t o, double* X,
                       hipStream_t s) {
  LAUNCH(mp2_denom_kernel, dim3(nblocks(rows * ov)), dim3(TPB), r0, rows, ov, v, eps, o, X);
}
hipError_t k_fill(int64_t n, double val, double* x, hipStream_t s) {
  LAUNCH(fill_kernel, dim3(nblocks(n)), dim3(TPB), n, val, x);
}
hipError_t k_set_diag(int64_t n, const double* d, double* X, int64_t ld, hipStream_t s) {
  LAUNCH(set_diag_kernel, dim3(nblocks(n)), dim3(TPB), n, d, X, ld);
}

}  // namespace thc
