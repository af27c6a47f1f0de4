// Host FP64 dense linear algebra used at set-up only (no HIP dependency).
#pragma once
#include <cstdint>

namespace thc {
int host_cholesky(int64_t n, double* A);                     // lower factor in place; 0 on success
void host_tri_inverse_lower(int64_t n, const double* L, double* Linv);
int host_syev(int64_t n, double* A, double* w);              // eigenvectors in the columns of A
}  // namespace thc
