"""Independent textbook spin-orbital CCSD used only to pin the oracle.

This is the spin-orbital CCSD of Stanton, Gauss, Watts and Bartlett (J. Chem. Phys. 94,
4334 (1991)) in its standard intermediate form (F_ae, F_mi, F_me, W_mnij, W_abef,
W_mbej), with explicit T1 and antisymmetrized integrals <pq||rs>, built here from the
same spatial Cholesky vectors.  The diagonal Fock elements are kept inside F_ae and F_mi,
so the functions return the residuals <Phi|exp(-T) H exp(T)|0> themselves.  It shares no
code with the closed-shell oracle: it starts from spin orbitals, uses no T1 dressing and
no closed-shell spin adaptation.
"""
from __future__ import annotations

import numpy as np


def spin_orbital_system(eps: np.ndarray, L: np.ndarray, o: int):
    """Spin-orbital Fock matrix and <pq||rs> for a closed-shell system whose Fock matrix
    is diag(eps).  Ordering: occupied alpha, occupied beta, virtual alpha, virtual beta."""
    n = eps.size
    v = n - o
    spatial = np.concatenate([np.arange(o), np.arange(o), np.arange(o, n), np.arange(o, n)])
    spin = np.concatenate([np.zeros(o), np.ones(o), np.zeros(v), np.ones(v)]).astype(int)
    g = np.einsum("Apq,Ars->pqrs", L, L)  # chemist (pq|rs)
    gs = g[np.ix_(spatial, spatial, spatial, spatial)]
    same = (spin[:, None] == spin[None, :]).astype(float)
    # <pq|rs> = (pr|qs) delta(sp, sr) delta(sq, ss)
    phys = gs.transpose(0, 2, 1, 3) * same[:, None, :, None] * same[None, :, None, :]
    anti = phys - phys.transpose(0, 1, 3, 2)
    f = np.diag(eps[spatial])
    return f, anti, 2 * o


def residuals(f, anti, t1, t2, nocc):
    """Spin-orbital CCSD residuals R1[i, a], R2[i, j, a, b]."""
    o = slice(0, nocc)
    v = slice(nocc, f.shape[0])
    fov, foo, fvv = f[o, v], f[o, o], f[v, v]
    I = anti
    ein = lambda s, *a: np.einsum(s, *a, optimize=True)
    tau = t2 + ein("ia,jb->ijab", t1, t1) - ein("ib,ja->ijab", t1, t1)
    taut = t2 + 0.5 * (ein("ia,jb->ijab", t1, t1) - ein("ib,ja->ijab", t1, t1))

    Fae = (fvv - 0.5 * ein("me,ma->ae", fov, t1) + ein("mf,mafe->ae", t1, I[o, v, v, v])
           - 0.5 * ein("mnaf,mnef->ae", taut, I[o, o, v, v]))
    Fmi = (foo + 0.5 * ein("ie,me->mi", t1, fov) + ein("ne,mnie->mi", t1, I[o, o, o, v])
           + 0.5 * ein("inef,mnef->mi", taut, I[o, o, v, v]))
    Fme = fov + ein("nf,mnef->me", t1, I[o, o, v, v])

    Wmnij = I[o, o, o, o] + 0.25 * ein("ijef,mnef->mnij", tau, I[o, o, v, v])
    x = ein("je,mnie->mnij", t1, I[o, o, o, v])
    Wmnij = Wmnij + x - x.transpose(0, 1, 3, 2)
    Wabef = I[v, v, v, v] + 0.25 * ein("mnab,mnef->abef", tau, I[o, o, v, v])
    x = ein("mb,amef->abef", t1, I[v, o, v, v])
    Wabef = Wabef - (x - x.transpose(1, 0, 2, 3))
    Wmbej = (I[o, v, v, o] + ein("jf,mbef->mbej", t1, I[o, v, v, v])
             - ein("nb,mnej->mbej", t1, I[o, o, v, o])
             - ein("jnfb,mnef->mbej", 0.5 * t2 + ein("jf,nb->jnfb", t1, t1), I[o, o, v, v]))

    R1 = (fov + ein("ie,ae->ia", t1, Fae) - ein("ma,mi->ia", t1, Fmi) + ein("imae,me->ia", t2, Fme)
          - ein("nf,naif->ia", t1, I[o, v, o, v]) - 0.5 * ein("imef,maef->ia", t2, I[o, v, v, v])
          - 0.5 * ein("mnae,nmei->ia", t2, I[o, o, v, o]))

    R2 = I[o, o, v, v].copy()
    x = ein("ijae,be->ijab", t2, Fae - 0.5 * ein("mb,me->be", t1, Fme))
    R2 += x - x.transpose(0, 1, 3, 2)
    x = ein("imab,mj->ijab", t2, Fmi + 0.5 * ein("je,me->mj", t1, Fme))
    R2 -= x - x.transpose(1, 0, 2, 3)
    R2 += 0.5 * ein("mnab,mnij->ijab", tau, Wmnij)
    R2 += 0.5 * ein("ijef,abef->ijab", tau, Wabef)
    x = ein("imae,mbej->ijab", t2, Wmbej) - ein("ie,ma,mbej->ijab", t1, t1, I[o, v, v, o])
    R2 += x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
    x = ein("ie,abej->ijab", t1, I[v, v, v, o])
    R2 += x - x.transpose(1, 0, 2, 3)
    x = ein("ma,mbij->ijab", t1, I[o, v, o, o])
    R2 -= x - x.transpose(0, 1, 3, 2)
    return R1, R2


def energy(f, anti, t1, t2, nocc):
    o = slice(0, nocc)
    v = slice(nocc, f.shape[0])
    return float(np.einsum("ia,ia->", f[o, v], t1) + 0.25 * np.einsum("ijab,ijab->", anti[o, o, v, v], t2)
                 + 0.5 * np.einsum("ijab,ia,jb->", anti[o, o, v, v], t1, t1))


def spin_adapt(t1, t2, o, v):
    """Closed-shell (t_i^a, t_ij^ab) -> spin-orbital amplitudes (ordering as above)."""
    no, nv = 2 * o, 2 * v
    T1 = np.zeros((no, nv))
    T1[:o, :v] = t1
    T1[o:, v:] = t1
    T2 = np.zeros((no, no, nv, nv))
    A, Bb = slice(0, o), slice(o, 2 * o)
    a, b = slice(0, v), slice(v, 2 * v)
    tx = t2.transpose(0, 1, 3, 2)  # t_ij^ba
    T2[A, Bb, a, b] = t2
    T2[Bb, A, b, a] = t2
    T2[A, Bb, b, a] = -tx
    T2[Bb, A, a, b] = -tx
    T2[A, A, a, a] = t2 - tx
    T2[Bb, Bb, b, b] = t2 - tx
    return T1, T2


def solve(eps, L, o, tol=1e-11, maxit=200):
    """Plain spin-orbital CCSD by Jacobi steps with the textbook denominators and DIIS."""
    f, anti, no = spin_orbital_system(eps, L, o)
    n2 = f.shape[0]
    nv = n2 - no
    e = np.diag(f)
    D1 = e[:no, None] - e[None, no:]
    D2 = e[:no, None, None, None] + e[None, :no, None, None] - e[None, None, no:, None] - e[None, None, None, no:]
    t1 = np.zeros((no, nv))
    t2 = anti[:no, :no, no:, no:] / D2
    vecs, errs = [], []
    E_old = 0.0
    for it in range(maxit):
        R1, R2 = residuals(f, anti, t1, t2, no)
        d1, d2 = R1 / D1, R2 / D2
        t1, t2 = t1 + d1, t2 + d2
        vecs.append(np.concatenate([t1.ravel(), t2.ravel()]))
        errs.append(np.concatenate([d1.ravel(), d2.ravel()]))
        if len(vecs) > 8:
            vecs.pop(0); errs.pop(0)
        if len(vecs) >= 2:
            m = len(vecs)
            Bm = -np.ones((m + 1, m + 1)); Bm[-1, -1] = 0.0
            for i in range(m):
                for j in range(m):
                    Bm[i, j] = errs[i] @ errs[j]
            rhs = np.zeros(m + 1); rhs[-1] = -1.0
            c = np.linalg.solve(Bm, rhs)[:m]
            x = sum(ci * vi for ci, vi in zip(c, vecs))
            t1 = x[: t1.size].reshape(t1.shape)
            t2 = x[t1.size:].reshape(t2.shape)
        E = energy(f, anti, t1, t2, no)
        if abs(E - E_old) < tol and max(np.abs(d1).max(), np.abs(d2).max()) < tol:
            return E, t1, t2
        E_old = E
    raise RuntimeError("spin-orbital CCSD did not converge")


def mp3_energy(f, anti, nocc):
    """Third-order Møller–Plesset energy from antisymmetrized spin-orbital integrals and a
    diagonal Fock matrix, in the standard three-term closed form (Szabo & Ostlund, Modern
    Quantum Chemistry, Eq. 6.74): particle ladder, hole ladder and ring, each over two MP2
    denominators."""
    e = np.diag(f)
    eo, ev = e[:nocc], e[nocc:]
    D = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    t = anti[:nocc, :nocc, nocc:, nocc:] / D
    ladder_p = 0.125 * np.einsum("ijab,abcd,ijcd->", t, anti[nocc:, nocc:, nocc:, nocc:], t)
    ladder_h = 0.125 * np.einsum("ijab,klij,klab->", t, anti[:nocc, :nocc, :nocc, :nocc], t)
    ring = np.einsum("ijab,kbcj,ikac->", t, anti[:nocc, nocc:, nocc:, :nocc], t)
    return ladder_p + ladder_h + ring
