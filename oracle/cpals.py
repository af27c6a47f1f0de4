"""Weighted CANDECOMP/PARAFAC by alternating least squares (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition followed (Sec. II.c Eq. 15-16, Sec. II.d Eq. 21, Appendix I Eq. 43-46): a 3-index array
A[i, j, k] is approximated by sum_n X[i, n] Y[j, n] Z[k, n], minimizing
    O = sum_ijk (w1_i w2_j w3_k)^2 (A_ijk - sum_n X_in Y_jn Z_kn)^2
(Eq. 15: the projectors U_ia^P with the eigenvalues eps_P as the weights of the third index; Eq. 21:
the Cholesky vectors with occupation weights on the first two).  One sweep updates X, then Y, then
Z, each as the exact minimizer with the other two fixed.  For X the normal equations are
    sum_n' S_nn' X_in' = R_in,  S = (Y^T W2^2 Y) o (Z^T W3^2 Z),  R_in = sum_jk w2_j^2 w3_k^2 A_ijk Y_jn Z_kn
(Eq. 44-46 with the weights of Eq. 16; the weight of the updated index factors out of each row), and
likewise for Y and Z.  The systems are solved directly here.
"""
from __future__ import annotations

import numpy as np


def _w(w, size):
    return np.ones(size) if w is None else np.asarray(w, dtype=np.float64)


def objective(A, X, Y, Z, w1=None, w2=None, w3=None) -> float:
    I, J, K = A.shape
    W = (_w(w1, I)[:, None, None] * _w(w2, J)[None, :, None] * _w(w3, K)[None, None, :]) ** 2
    M = np.einsum("in,jn,kn->ijk", X, Y, Z)
    return float(np.sum(W * (A - M) ** 2))


def update(A, X, Y, Z, w1=None, w2=None, w3=None, mode=0):
    """The exact least-squares update of factor `mode` (0: X, 1: Y, 2: Z); returns the new factor."""
    I, J, K = A.shape
    a1, a2, a3 = _w(w1, I) ** 2, _w(w2, J) ** 2, _w(w3, K) ** 2
    if mode == 0:
        S = (Y.T @ (a2[:, None] * Y)) * (Z.T @ (a3[:, None] * Z))
        R = np.einsum("ijk,j,jn,k,kn->in", A, a2, Y, a3, Z)
    elif mode == 1:
        S = (X.T @ (a1[:, None] * X)) * (Z.T @ (a3[:, None] * Z))
        R = np.einsum("ijk,i,in,k,kn->jn", A, a1, X, a3, Z)
    else:
        S = (X.T @ (a1[:, None] * X)) * (Y.T @ (a2[:, None] * Y))
        R = np.einsum("ijk,i,in,j,jn->kn", A, a1, X, a2, Y)
    return np.linalg.solve(S, R.T).T


def cp_als(A, X, Y, Z, sweeps, w1=None, w2=None, w3=None):
    """`sweeps` ALS sweeps (X, Y, Z in turn) from the given factors; returns the factors and the
    objective before the first sweep and after each."""
    X, Y, Z = X.copy(), Y.copy(), Z.copy()
    obj = [objective(A, X, Y, Z, w1, w2, w3)]
    for _ in range(sweeps):
        X = update(A, X, Y, Z, w1, w2, w3, 0)
        Y = update(A, X, Y, Z, w1, w2, w3, 1)
        Z = update(A, X, Y, Z, w1, w2, w3, 2)
        obj.append(objective(A, X, Y, Z, w1, w2, w3))
    return X, Y, Z, obj
