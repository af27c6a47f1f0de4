"""FP64 CPU oracle for THC-factorized rank-reduced CCSD (Hohenstein, Fales, Parrish,
Martinez, "Rank-reduced coupled-cluster III", arXiv:2111.11473).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library may import, call or link this
package; only tests/, the smoke check and the benchmark's CPU-baseline leg use it.

The oracle is dense and slow on purpose: it rebuilds the full T1-dressed integrals, the
full amplitudes t_ij^ab from the THC factors, evaluates every term of the closed-shell
CCSD residual in the grouping of the paper's Eq. 28-42 with plain einsum contractions,
and only then projects onto the amplitude space (Eq. 6).  It shares no code with the HIP
path.  Index convention: t2[i, j, a, b] = t_ij^ab pairs (i, a) with (j, b), so that
t2[i, j, a, b] = t2[j, i, b, a].
"""
from .ccsd import (dress_cholesky, one_electron, dressed_fock, doubles_terms, singles_terms,
                   doubles_residual, singles_residual, energy, C_D)
from .thc import (khatri_rao, amplitudes, project, eri_fit, eri_thc_dense, metric, fock_operator,
                  pseudo_canonical, mp2_amplitudes, mp2_guess, thc_residual, solve, SolveResult,
                  driver_projection, energy_from_factors)
from .density import mp2_density
from . import cpals
