"""MP2 one-particle density matrix from THC-factorized amplitudes, densely (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition followed: the unrelaxed closed-shell MP2 one-particle density of Appendix II,
  D_ij = -2 sum_kab t_ik^ab (2 t_jk^ab - t_jk^ba)        (Eq. 47)
  D_ab =  2 sum_ijc t_ij^ac (2 t_ij^bc - t_ji^bc)        (Eq. 48)
with t_ij^ab rebuilt densely from the factors and core (Eq. 22-23; Eq. 49-50 insert exactly this
form).  The factorized O(N^4) evaluation (Eq. 51-56) is what the GPU library implements; here the
two plain contractions of the definition are written out.
"""
from __future__ import annotations

import numpy as np

from .thc import amplitudes


def mp2_density(Xo: np.ndarray, Xv: np.ndarray, Z: np.ndarray):
    """(D_oo [o, o], D_vv [v, v]) of the amplitudes t = B Z B^T (Eq. 47, 48)."""
    t2 = amplitudes(Xo, Xv, Z)  # t2[i, j, a, b]
    # D_ij = -2 sum_kab t_ik^ab (2 t_jk^ab - t_jk^ba)
    Doo = -2.0 * (2.0 * np.einsum("ikab,jkab->ij", t2, t2) - np.einsum("ikab,jkba->ij", t2, t2))
    # D_ab = 2 sum_ijc t_ij^ac (2 t_ij^bc - t_ji^bc)
    Dvv = 2.0 * (2.0 * np.einsum("ijac,ijbc->ab", t2, t2) - np.einsum("ijac,jibc->ab", t2, t2))
    return Doo, Dvv
