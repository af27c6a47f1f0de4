"""Dense closed-shell CCSD residual with the T1-transformed Hamiltonian (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every term below is the paper's dense expression, written out with einsum:
  T1 transformation ............ Sec. III, Eq. 24-27
  ladders (Alg. 1) ............. Eq. 28
  bare + Coulomb rings (Alg. 2)  Eq. 29
  remaining linear (Alg. 3) .... Eq. 31
  T2^2 ladder/exchange (Alg. 6)  Eq. 32 and Eq. 33
  T2^2 rings (Alg. 7) .......... Eq. 35-37
  Fock + xi (Alg. 8-9) ......... Eq. 39-41
  singles (Alg. 8, 10) ......... Eq. 38 and Eq. 42
Readings taken where the text is ambiguous (each also listed in the design notes):
  * Eq. 35 / Alg. 7 print a prefactor 1/4 and, in Eq. 35, (t - t') on the right; the
    contraction of Eq. 36-37 (R = 2t - t' on both sides) is used with prefactor C_D = 1/2,
    the value for which the sum of all terms equals textbook CCSD (checked in the tests
    against an independent spin-orbital CCSD and against closed-shell direct-ring CCD).
  * Eq. 41 prints (t_ij^ac + t_ji^ca), equal to 2 t_ij^ac; it is read as the pair
    permutation P_ij^ab, as Alg. 9 computes (sigma = E B^T + B E^T).
  * Eq. 31 has no hats; Alg. 3 dresses l_ij and l_ab, so the dressed integrals are used.
  * Dressed oo/vv blocks enter with the orientation of the equations ((ki^|lj) etc.);
    at t1 = 0 every orientation coincides.
  * The THC form of (ia|jb) (Eq. 17) is used only in the T2^2 terms Eq. 32, 33, 35, where
    the paper's algorithms contract it (Alg. 4-7); every other term, the xi intermediates
    (Alg. 8 uses l_ia) and the energy use the Cholesky integrals.
  * There is no one-electron Hamiltonian in the synthetic input: h = diag(eps) - G0[L] so
    that the undressed Fock matrix is exactly diag(eps) (Brillouin: F_ia = 0).
"""
from __future__ import annotations

import numpy as np

C_D = 0.5  # prefactor of the Eq. 35-37 ring contraction (see module docstring)


def _split(L, o):
    return L[:, :o, :o], L[:, :o, o:], L[:, o:, :o], L[:, o:, o:]


def dress_cholesky(L: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """Eq. 25-27 in the MO basis (C = 1): C^p = 1 - t1^T, C^h = 1 + t1 with t1 placed in
    the (virtual, occupied) block, L^_pq = sum_mn C^p_mp C^h_nq L_mn."""
    nL, n, _ = L.shape
    o = t1.shape[0]
    tau = np.zeros((n, n))
    tau[o:, :o] = t1.T  # tau[a, i] = t_i^a
    Cp = np.eye(n) - tau.T
    Ch = np.eye(n) + tau
    return np.einsum("mp,Amn,nq->Apq", Cp, L, Ch, optimize=True)


def one_electron(eps: np.ndarray, L: np.ndarray, o: int) -> np.ndarray:
    """h = diag(eps) - sum_k [2 (pq|kk) - (pk|kq)] with Cholesky (pq|rs) = sum_A L_pq L_rs."""
    J = np.einsum("Apq,Akk->pq", L, L[:, :o, :o])
    K = np.einsum("Apk,Akq->pq", L[:, :, :o], L[:, :o, :])
    return np.diag(eps) - (2.0 * J - K)


def dressed_fock(eps: np.ndarray, L: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """F^_pq = h^_pq + sum_k [2 (pq^|kk) - (pk^|kq)], h^ = C^pT h C^h (T1-transformed Fock)."""
    o = t1.shape[0]
    n = L.shape[1]
    h = one_electron(eps, L, o)
    tau = np.zeros((n, n))
    tau[o:, :o] = t1.T
    hh = (np.eye(n) - tau) @ h @ (np.eye(n) + tau)
    Lh = dress_cholesky(L, t1)
    J = np.einsum("Apq,Akk->pq", Lh, Lh[:, :o, :o])
    K = np.einsum("Apk,Akq->pq", Lh[:, :, :o], Lh[:, :o, :])
    return hh + 2.0 * J - K


def _g(La, Lb):
    """(pq|rs) = sum_A La_pq Lb_rs for two (nL, ., .) blocks."""
    return np.einsum("Apq,Ars->pqrs", La, Lb, optimize=True)


def _u(t2):
    """2 t_ik^ac - t_ik^ca as an array u[i, k, a, c]."""
    return 2.0 * t2 - t2.transpose(0, 1, 3, 2)


def doubles_terms(eps, L, t1, t2, V=None) -> dict:
    """Each grouped contribution R[i, j, a, b] (external pairs (i, a), (j, b)) of the
    doubles residual.  V is the ovov integral tensor V[i, a, j, b] = (ia|jb) used in the
    T2^2 terms (the THC form, Eq. 17); None means the Cholesky ovov block."""
    o = t2.shape[0]
    Lh = dress_cholesky(L, t1)
    Lh_oo, Lh_ov, Lh_vo, Lh_vv = _split(Lh, o)
    L_ov = L[:, :o, o:]
    g_ovov = _g(L_ov, L_ov)  # (ia|jb), T1-invariant
    if V is None:
        V = g_ovov
    t = t2
    u = _u(t2)
    terms = {}

    # Eq. 28: pp, hh and mixed particle-hole ladders (Alg. 1)
    g_vvvv = _g(Lh_vv, Lh_vv)   # (ac^|bd)
    g_oooo = _g(Lh_oo, Lh_oo)   # (ki^|lj)
    g_vvoo = _g(Lh_vv, Lh_oo)   # (ac^|lj)
    g_oovv = _g(Lh_oo, Lh_vv)   # (ki^|bd)
    terms["eq28"] = (np.einsum("ijcd,acbd->ijab", t, g_vvvv, optimize=True)
                     + np.einsum("klab,kilj->ijab", t, g_oooo, optimize=True)
                     - np.einsum("ilcb,aclj->ijab", t, g_vvoo, optimize=True)
                     - np.einsum("kjad,kibd->ijab", t, g_oovv, optimize=True))

    # Eq. 29: bare (ai^|bj) and the Coulomb rings (Alg. 2)
    g_vovo = _g(Lh_vo, Lh_vo)   # (ai^|bj)
    g_voov = _g(Lh_vo, L_ov)    # (bj^|kc)
    terms["eq29"] = (g_vovo.transpose(1, 3, 0, 2)
                     + np.einsum("ikac,bjkc->ijab", u, g_voov, optimize=True)
                     + np.einsum("jkbc,aikc->ijab", u, g_voov, optimize=True))

    # Eq. 31 (with the hats of Alg. 3): remaining terms linear in T2
    terms["eq31"] = -(np.einsum("ikac,kjbc->ijab", t, g_oovv, optimize=True)
                      + np.einsum("jkbc,kiac->ijab", t, g_oovv, optimize=True))

    # Eq. 32: sum_kcld t_ij^cd t_kl^ab (kc|ld)
    X = np.einsum("ijcd,kcld->klij", t, V, optimize=True)
    terms["eq32"] = np.einsum("klab,klij->ijab", t, X, optimize=True)

    # Eq. 33: sum_kcld t_ik^cb t_lj^ad (lc|kd)
    Y = np.einsum("ikcb,lckd->ibld", t, V, optimize=True)
    terms["eq33"] = np.einsum("ibld,ljad->ijab", Y, t, optimize=True)

    # Eq. 35-37: C_D [ sum u_ik^ac (2(kc|ld) - (kd|lc)) u_jl^bd + sum t_ik^ca (kd|lc) t_jl^db ]
    LV = 2.0 * V - V.transpose(0, 3, 2, 1)
    Z1 = np.einsum("ikac,kcld->iald", u, LV, optimize=True)
    part1 = np.einsum("iald,jlbd->ijab", Z1, u, optimize=True)
    Z2 = np.einsum("ikca,kdlc->iald", t, V, optimize=True)
    part2 = np.einsum("iald,jldb->ijab", Z2, t, optimize=True)
    terms["eq35"] = C_D * (part1 + part2)

    # Eq. 39-41: Fock and xi intermediates (Cholesky ovov), pair-permuted
    F = dressed_fock(eps, L, t1)
    xi_oo = (np.einsum("jmde,mekd->kj", t, 2.0 * g_ovov, optimize=True)
             - np.einsum("jmde,mdke->kj", t, g_ovov, optimize=True))
    xi_vv = -(np.einsum("lmdb,ldmc->bc", t, 2.0 * g_ovov, optimize=True)
              - np.einsum("lmdb,lcmd->bc", t, g_ovov, optimize=True))
    Xv = F[o:, o:] + xi_vv
    Xo = F[:o, :o] + xi_oo
    half = np.einsum("ijac,bc->ijab", t, Xv, optimize=True) - np.einsum("ikab,kj->ijab", t, Xo, optimize=True)
    terms["eq41"] = half + half.transpose(1, 0, 3, 2)
    return terms


def singles_terms(eps, L, t1, t2) -> dict:
    """Singles residual R[i, a] (Eq. 38 and Eq. 42)."""
    o = t2.shape[0]
    Lh = dress_cholesky(L, t1)
    Lh_oo, _, _, Lh_vv = _split(Lh, o)
    L_ov = L[:, :o, o:]
    t = t2
    u = _u(t2)
    g_ovvv = _g(L_ov, Lh_vv)  # (kd^|ac)
    g_ovoo = _g(L_ov, Lh_oo)  # (lc^|ki)
    g_ooov = _g(Lh_oo, L_ov)  # (li^|kc)
    eq38 = (np.einsum("ikcd,kdac->ia", t, 2.0 * g_ovvv, optimize=True)
            - np.einsum("ikcd,kcad->ia", t, g_ovvv, optimize=True)
            - np.einsum("klac,lcki->ia", t, 2.0 * g_ovoo, optimize=True)
            + np.einsum("klac,likc->ia", t, g_ooov, optimize=True))
    F = dressed_fock(eps, L, t1)
    eq42 = F[o:, :o].T + np.einsum("ikac,kc->ia", u, F[:o, o:], optimize=True)
    return {"eq38": eq38, "eq42": eq42}


def doubles_residual(eps, L, t1, t2, V=None) -> np.ndarray:
    return sum(doubles_terms(eps, L, t1, t2, V).values())


def singles_residual(eps, L, t1, t2) -> np.ndarray:
    return sum(singles_terms(eps, L, t1, t2).values())


def energy(L, t1, t2) -> float:
    """Closed-shell CCSD correlation energy, sum_iajb (t_ij^ab + t_i^a t_j^b)(2(ia|jb) - (ib|ja))
    with Cholesky integrals (the usual energy expression, unchanged by the rank reduction)."""
    o = t2.shape[0]
    L_ov = L[:, :o, o:]
    g = _g(L_ov, L_ov)
    tau = t2 + np.einsum("ia,jb->ijab", t1, t1)
    return float(2.0 * np.einsum("ijab,iajb->", tau, g) - np.einsum("ijab,ibja->", tau, g))
