"""Singlet full CI of a two-electron closed-shell system, used only to pin CCSD results (CCSD is
exact for two electrons).  Built from the Cholesky vectors and orbital energies alone, with no
amplitude equations: it shares no code with the oracle or the library."""
import numpy as np


def two_electron_fci(eps, L):
    """Singlet full CI of one doubly occupied orbital's two electrons, built from the Cholesky
    vectors alone: the one-electron operator is the Fock matrix minus the closed-shell mean field
    of the occupied orbital, the Hamiltonian on spatial pair functions is h x 1 + 1 x h + (pr|qs),
    restricted to the symmetric (singlet) pairs.  Returns the correlation energy of the state
    dominated by the reference, and the MP2 energy for scale."""
    n = eps.size
    g = np.einsum("Apq,Ars->pqrs", L, L)
    h = np.diag(eps) - (2.0 * g[:, :, 0, 0] - g[:, 0, 0, :])
    rows = []
    for p in range(n):
        for q in range(p, n):
            c = np.zeros((n, n))
            c[p, q] = c[q, p] = 1.0 if p == q else 1.0 / np.sqrt(2.0)
            rows.append(c.ravel())
    C = np.array(rows)  # first row: the reference |0 0>
    H = np.kron(h, np.eye(n)) + np.kron(np.eye(n), h) + g.transpose(0, 2, 1, 3).reshape(n * n, n * n)
    Hs = C @ H @ C.T
    w, U = np.linalg.eigh(Hs)
    k = int(np.argmax(np.abs(U[0])))
    emp2 = sum((L[:, 0, a] @ L[:, 0, b]) ** 2 / (2 * eps[0] - eps[a] - eps[b])
               for a in range(1, n) for b in range(1, n))
    return w[k] - Hs[0, 0], emp2
