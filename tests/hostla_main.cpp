// CPU driver for the library's host linear algebra (csrc/hostla.cpp), built by
// tests/test_host_sanitize.py with the address and undefined-behaviour sanitizers.
// Usage: hostla_main <kind> <n>   kind: random | diagonal | identity | rank1 | zero | clustered | spd
// Prints the relative errors of the decomposition it checks, one per line.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hostla.h"

namespace {
uint64_t state = 0x9e3779b97f4a7c15ull;
double next_uniform() {  // xorshift64*, mapped to [-1, 1)
  state ^= state >> 12;
  state ^= state << 25;
  state ^= state >> 27;
  return (double)((state * 2685821657736338717ull) >> 11) * 0x1.0p-52 - 1.0;
}
}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) return 64;
  const char* kind = argv[1];
  const int64_t n = std::atoll(argv[2]);
  if (n < 1) return 64;
  std::vector<double> A((size_t)(n * n), 0.0);
  std::vector<double> u(n);
  for (auto& x : u) x = next_uniform();
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      double a = 0.0;
      if (!std::strcmp(kind, "random") || !std::strcmp(kind, "spd")) a = next_uniform();
      else if (!std::strcmp(kind, "diagonal")) a = i == j ? (double)((i * 7) % 11) - 5.0 : 0.0;
      else if (!std::strcmp(kind, "identity")) a = i == j ? 1.0 : 0.0;
      else if (!std::strcmp(kind, "rank1")) a = u[i] * u[j] + (i == j ? 1.0 : 0.0);
      else if (!std::strcmp(kind, "clustered")) a = (i == j ? (double)(i % 3) : 0.0) + 1e-9 * next_uniform();
      else if (std::strcmp(kind, "zero")) return 64;
      A[i * n + j] = A[j * n + i] = a;
    }
  if (!std::strcmp(kind, "spd")) {  // A A^T + n I, then Cholesky and the triangular inverse
    std::vector<double> S((size_t)(n * n), 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        double s = i == j ? (double)n : 0.0;
        for (int64_t k = 0; k < n; ++k) s += A[i * n + k] * A[j * n + k];
        S[i * n + j] = s;
      }
    std::vector<double> L = S, Li((size_t)(n * n));
    if (thc::host_cholesky(n, L.data()) != 0) return 2;
    thc::host_tri_inverse_lower(n, L.data(), Li.data());
    double err = 0.0, nrm = 0.0, inv = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j <= i; ++j) {
        double s = 0.0, t = 0.0;
        for (int64_t k = 0; k <= j; ++k) s += L[i * n + k] * L[j * n + k];
        for (int64_t k = j; k <= i; ++k) t += L[i * n + k] * Li[k * n + j];
        err = std::fmax(err, std::fabs(s - S[i * n + j]));
        nrm = std::fmax(nrm, std::fabs(S[i * n + j]));
        inv = std::fmax(inv, std::fabs(t - (i == j ? 1.0 : 0.0)));
      }
    std::printf("%.3e\n%.3e\n", err / nrm, inv);
    return 0;
  }
  std::vector<double> V = A, w(n);
  if (thc::host_syev(n, V.data(), w.data()) != 0) return 3;
  double nrm = 0.0, res = 0.0, orth = 0.0;
  for (double x : A) nrm = std::fmax(nrm, std::fabs(x));
  for (int64_t j = 0; j < n; ++j) {
    if (j > 0 && w[j] < w[j - 1]) return 4;  // ascending order
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += A[i * n + k] * V[k * n + j];
      res = std::fmax(res, std::fabs(s - w[j] * V[i * n + j]));
    }
    for (int64_t l = 0; l <= j; ++l) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += V[k * n + l] * V[k * n + j];
      orth = std::fmax(orth, std::fabs(s - (l == j ? 1.0 : 0.0)));
    }
  }
  std::printf("%.3e\n%.3e\n", nrm > 0.0 ? res / nrm : res, orth);
  return 0;
}
