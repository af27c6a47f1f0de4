// Host FP64 dense linear algebra used once at set-up (never in the iteration):
//  * Cholesky factorization of small diagonal blocks (the blocked GPU factorization
//    hands its 64x64 diagonal blocks here) and the inverse of a lower-triangular block;
//  * the symmetric eigenproblem of the (N_P x N_P) Fock operator in the orthonormalized
//    amplitude basis: Householder reduction to tridiagonal form followed by the implicit
//    QL iteration with Wilkinson-type shifts, with the orthogonal transformations
//    accumulated (Golub & Van Loan, Matrix Computations, Sec. 8.3).  The QL step sequence (shift
//    from the leading 2 x 2 block, rotations chased up the tridiagonal) is the published tql2
//    procedure of Bowdler, Martin, Reinsch & Wilkinson (Numer. Math. 11, 293-306, 1968).
// All matrices are row-major.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "hostla.h"

namespace thc {

int host_cholesky(int64_t n, double* A) {
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return 1;
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (int64_t i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
    for (int64_t k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
  }
  return 0;
}

void host_tri_inverse_lower(int64_t n, const double* L, double* X) {
  std::fill(X, X + n * n, 0.0);
  for (int64_t c = 0; c < n; ++c) {
    // solve L x = e_c by forward substitution, x stored in column c of X
    for (int64_t i = c; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int64_t k = c; k < i; ++k) s -= L[i * n + k] * X[k * n + c];
      X[i * n + c] = s / L[i * n + i];
    }
  }
}

namespace {

// Apply a function to rows [0, n) in parallel chunks.
// (Serial below min_n items, where starting threads costs more than it saves.)
template <class Fn>
void parallel_rows(int64_t n, Fn fn, int64_t min_n = 256) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 16) nt = 16;
  if (n < min_n || nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
    if (a < b) th.emplace_back(fn, a, b);
  }
  for (auto& x : th) x.join();
}

}  // namespace

// Eigen-decomposition of the symmetric matrix A (n x n, row-major).  On return w holds the
// eigenvalues in ascending order and column j of A the eigenvector of w[j].
int host_syev(int64_t n, double* A, double* w) {
  if (n == 1) { w[0] = A[0]; A[0] = 1.0; return 0; }
  std::vector<double> d(n), e(n, 0.0);
  std::vector<double> V((size_t)n * n);  // Householder vectors, row k holds v_k (entries k+1..n-1)
  std::vector<double> p(n), q(n);
  // --- Householder reduction: A <- H_k A H_k on the trailing block ---
  for (int64_t k = 0; k + 2 < n; ++k) {
    double* vk = &V[(size_t)k * n];
    double sig = 0.0;
    for (int64_t i = k + 1; i < n; ++i) sig += A[i * n + k] * A[i * n + k];
    const double xn = std::sqrt(sig);
    if (xn == 0.0) {
      d[k] = A[k * n + k];
      e[k] = 0.0;
      std::fill(vk, vk + n, 0.0);
      continue;
    }
    const double x0 = A[(k + 1) * n + k];
    const double alpha = x0 > 0 ? -xn : xn;
    for (int64_t i = 0; i <= k; ++i) vk[i] = 0.0;
    for (int64_t i = k + 1; i < n; ++i) vk[i] = A[i * n + k];
    vk[k + 1] -= alpha;
    double vn = 0.0;
    for (int64_t i = k + 1; i < n; ++i) vn += vk[i] * vk[i];
    vn = std::sqrt(vn);
    for (int64_t i = k + 1; i < n; ++i) vk[i] /= vn;
    // p = 2 A v on the trailing block
    parallel_rows(n - k - 1, [&](int64_t a, int64_t b) {
      for (int64_t r = a; r < b; ++r) {
        const int64_t i = k + 1 + r;
        const double* Ai = A + i * n;
        double s = 0.0;
        for (int64_t j = k + 1; j < n; ++j) s += Ai[j] * vk[j];
        p[i] = 2.0 * s;
      }
    });
    double K = 0.0;
    for (int64_t i = k + 1; i < n; ++i) K += vk[i] * p[i];
    for (int64_t i = k + 1; i < n; ++i) q[i] = p[i] - K * vk[i];
    parallel_rows(n - k - 1, [&](int64_t a, int64_t b) {
      for (int64_t r = a; r < b; ++r) {
        const int64_t i = k + 1 + r;
        double* Ai = A + i * n;
        const double vi = vk[i], qi = q[i];
        for (int64_t j = k + 1; j < n; ++j) Ai[j] -= vi * q[j] + qi * vk[j];
      }
    });
    d[k] = A[k * n + k];
    e[k] = alpha;  // sub-diagonal element between k and k+1
  }
  d[n - 2] = A[(n - 2) * n + n - 2];
  e[n - 2] = A[(n - 1) * n + n - 2];
  d[n - 1] = A[(n - 1) * n + n - 1];
  e[n - 1] = 0.0;
  // --- accumulate Q = H_0 ... H_{n-3}; stored transposed (row j of Zt = column j of Q) ---
  // Zt = Q^T = H_{n-3} ... H_0 applied from the right to the identity: Zt <- Zt H_k for
  // k = n-3 .. 0.  Rows of Zt are independent, so each thread takes blocks of 16 rows and applies
  // every reflector to them while they stay in its cache (the reflectors stream past once per
  // block instead of the whole matrix once per reflector).
  std::vector<double> Zt((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
  constexpr int64_t RB = 16;
  parallel_rows((n + RB - 1) / RB, [&](int64_t a, int64_t b) {
    for (int64_t blk = a; blk < b; ++blk) {
      const int64_t r0 = blk * RB, r1 = std::min(n, r0 + RB);
      for (int64_t k = n - 3; k >= 0; --k) {
        const double* vk = &V[(size_t)k * n];
        for (int64_t r = r0; r < r1; ++r) {
          double* z = &Zt[(size_t)r * n];
          double s = 0.0;
          for (int64_t j = k + 1; j < n; ++j) s += z[j] * vk[j];
          s *= 2.0;
          if (s != 0.0)
            for (int64_t j = k + 1; j < n; ++j) z[j] -= s * vk[j];
        }
      }
    }
  }, 2);
  // --- implicit QL on the tridiagonal (d, e): e[i] couples i and i+1 ---
  // The iteration itself needs only (d, e); its plane rotations (combining columns i, i+1 of Q,
  // i.e. rows i, i+1 of Zt) are recorded in order and applied afterwards, each thread taking
  // slices of 64 columns of Zt through the whole sequence (columns are independent, and a slice
  // of every row stays in cache while the sweeps run over it).
  struct Rot {
    int64_t i;
    double c, s;
  };
  std::vector<Rot> rots;
  rots.reserve((size_t)n * 8);
  for (int64_t l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int64_t m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      if (++iter > 80) return 2;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool underflow = false;
      for (int64_t i = m - 1; i >= l; --i) {
        const double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          underflow = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        rots.push_back({i, c, s});
      }
      if (underflow) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  constexpr int64_t CW = 64;
  parallel_rows((n + CW - 1) / CW, [&](int64_t a, int64_t b) {
    for (int64_t sl = a; sl < b; ++sl) {
      const int64_t k0 = sl * CW, kw = std::min(n, k0 + CW) - k0;
      for (const Rot& q : rots) {
        double* z0 = &Zt[(size_t)q.i * n + k0];
        double* z1 = z0 + n;
        for (int64_t k = 0; k < kw; ++k) {
          const double a0 = z0[k], a1 = z1[k];
          z1[k] = q.s * a0 + q.c * a1;
          z0[k] = q.c * a0 - q.s * a1;
        }
      }
    }
  }, 2);
  // sort ascending, write eigenvectors into the columns of A
  std::vector<int64_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
  for (int64_t j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    const double* z = &Zt[(size_t)idx[j] * n];
    for (int64_t i = 0; i < n; ++i) A[i * n + j] = z[i];
  }
  return 0;
}

}  // namespace thc
