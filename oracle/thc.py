"""THC layer of the oracle: amplitudes from the factors, projection, ERI fit, working
basis, MP2 guess and the Jacobi + DIIS solver (FP64, numpy/scipy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions followed:
  amplitudes  t_ij^ab = sum_WX y_i^W y_a^W T^WX y_j^X y_b^X          Eq. 22-23
  projection  sigma^WX = sum_ijab y_i^W y_a^W R_ij^ab y_j^X y_b^X     Eq. 6 with the
              CP projectors of Eq. 14 (raw collocation basis: the orthonormal form of
              Eq. 11-14 is the congruence W^T sigma W below)
  metric      S^WX = sum_ia y_i^W y_a^W y_i^X y_a^X                   Eq. 10
  ERI fit     xi^T = G^-1 C^T L, z = xi^T xi (unit weights)            Eq. 19-20
  energy      the usual CCSD expression (Sec. II.a)
Readings (no statement in the paper): the update is Jacobi in the generalized
eigenbasis of the Fock part, E_mat w = e S w, where the projected Fock operator is
exactly diagonal (denominators e_P + e_Q); DIIS is Pulay's with the preconditioned
residual as error vector, dropping its oldest vectors while their error overlap matrix has a
condition number above 1e12; convergence is ||(sigma^, sigma1)||_F < tol and |dE| < tol_e.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.linalg

from . import ccsd


def khatri_rao(Xo: np.ndarray, Xv: np.ndarray) -> np.ndarray:
    """B[(i, a), W] = Xo[i, W] * Xv[a, W], shape (o*v, nP)."""
    o, P = Xo.shape
    v = Xv.shape[0]
    return (Xo[:, None, :] * Xv[None, :, :]).reshape(o * v, P)


def amplitudes(Xo, Xv, Z) -> np.ndarray:
    """Dense t2[i, j, a, b] from the THC factors (Eq. 23)."""
    o, v = Xo.shape[0], Xv.shape[0]
    B = khatri_rao(Xo, Xv)
    return (B @ Z @ B.T).reshape(o, v, o, v).transpose(0, 2, 1, 3)


def project(R2, Xo, Xv) -> np.ndarray:
    """sigma = B^T R B with R viewed as an (ov x ov) matrix (Eq. 6)."""
    o, v = Xo.shape[0], Xv.shape[0]
    B = khatri_rao(Xo, Xv)
    Rm = R2.transpose(0, 2, 1, 3).reshape(o * v, o * v)
    return B.T @ Rm @ B


def eri_fit(L, o, xo, xv):
    """Least-squares THC of the ovov Cholesky block (Eq. 19-20, unit weights):
    for every A, min || L_ia^A - sum_I x_i^I x_a^I xi^AI ||, then z = xi^T xi."""
    Cq = khatri_rao(xo, xv)                       # (ov, nQ)
    Lm = L[:, :o, o:].reshape(L.shape[0], -1)     # (nL, ov)
    G = Cq.T @ Cq
    xiT = scipy.linalg.solve(G, Cq.T @ Lm.T, assume_a="pos")   # (nQ, nL)
    return xiT @ xiT.T, xiT


def eri_thc_dense(xo, xv, z) -> np.ndarray:
    """V[i, a, j, b] = sum_IJ x_i^I x_a^I z^IJ x_j^J x_b^J (Eq. 17)."""
    o, v = xo.shape[0], xv.shape[0]
    Cq = khatri_rao(xo, xv)
    return (Cq @ z @ Cq.T).reshape(o, v, o, v)


def metric(Xo, Xv) -> np.ndarray:
    B = khatri_rao(Xo, Xv)
    return B.T @ B


def fock_operator(Xo, Xv, eps) -> np.ndarray:
    """E_mat = B^T diag(eps_a - eps_i) B: the projected Fock part, so that
    B^T (Delta t) B = E_mat Z S + S Z E_mat for t = B Z B^T."""
    o = Xo.shape[0]
    d = (eps[o:][None, :] - eps[:o][:, None]).reshape(-1)
    B = khatri_rao(Xo, Xv)
    return B.T @ (d[:, None] * B)


def pseudo_canonical(Xo, Xv, eps):
    """Generalized eigenpairs E_mat w = e S w with W^T S W = 1."""
    S = metric(Xo, Xv)
    E = fock_operator(Xo, Xv, eps)
    e, W = scipy.linalg.eigh(E, S)
    return e, W


def mp2_amplitudes(eps, L, o) -> np.ndarray:
    """t_ij^ab = -(ia|jb) / (eps_a + eps_b - eps_i - eps_j) with Cholesky integrals."""
    L_ov = L[:, :o, o:]
    g = np.einsum("Aia,Ajb->iajb", L_ov, L_ov)
    d = eps[o:][None, :] - eps[:o][:, None]
    return -(g / (d[:, :, None, None] + d[None, None, :, :])).transpose(0, 2, 1, 3)


def mp2_guess(eps, L, Xo, Xv) -> np.ndarray:
    """Least-squares fit of the MP2 amplitudes by the THC form:
    Z0 = argmin || B Z B^T - t_MP2 ||_F = S^-1 B^T t_MP2 B S^-1."""
    o = Xo.shape[0]
    t = mp2_amplitudes(eps, L, o)
    M = project(t, Xo, Xv)
    S = metric(Xo, Xv)
    Y = scipy.linalg.solve(S, M, assume_a="pos")
    return scipy.linalg.solve(S, Y.T, assume_a="pos").T


def thc_residual(eps, L, Xo, Xv, Z, t1, V=None, terms=False):
    """Projected doubles residual sigma_raw (nP x nP) and singles residual (o x v) of the
    state (Z, t1); V is the ovov tensor for the T2^2 terms (THC, Eq. 17)."""
    t2 = amplitudes(Xo, Xv, Z)
    if terms:
        d = ccsd.doubles_terms(eps, L, t1, t2, V)
        s = ccsd.singles_terms(eps, L, t1, t2)
        return {k: project(r, Xo, Xv) for k, r in d.items()}, s
    R2 = ccsd.doubles_residual(eps, L, t1, t2, V)
    R1 = ccsd.singles_residual(eps, L, t1, t2)
    return project(R2, Xo, Xv), R1


def driver_projection(L, Xo, Xv) -> np.ndarray:
    """The projected residual at t1 = 0, t2 = 0, where every term but the driver (ia|jb)
    vanishes (Eq. 6 applied to R_ij^ab = (ia|jb)), contracted through the factors:
    sigma = M^T M with M[K, W] = sum_ia L_ia^K y_i^W y_a^W (Cholesky integrals)."""
    o = Xo.shape[0]
    M = L[:, :o, o:].reshape(L.shape[0], -1) @ khatri_rao(Xo, Xv)
    return M.T @ M


def energy_from_factors(L, Xo, Xv, Z) -> float:
    """The correlation energy at t1 = 0 of the THC amplitudes t = B Z B^T (the usual
    closed-shell expression, Sec. II.a), contracted through the factors one Cholesky vector
    at a time: Coulomb 2 sum_K m_K^T Z m_K with m_K[W] = sum_ia y_i^W L_ia^K y_a^W, exchange
    sum_K sum_WX Z^WX N_K[W, X] N_K[X, W] with N_K = Xo^T L_ov^K Xv."""
    o = Xo.shape[0]
    e = 0.0
    for K in range(L.shape[0]):
        Lk = L[K, :o, o:]
        LX = Lk @ Xv
        m = (Xo * LX).sum(axis=0)
        N = Xo.T @ LX
        e += 2.0 * (m @ Z @ m) - float(np.sum(Z * N * N.T))
    return float(e)


@dataclass
class SolveResult:
    energy: float
    Z: np.ndarray
    t1: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)


def _diis_condition(vecs, errs, limit=1e12):
    """Keeps the DIIS subspace well conditioned: drops the oldest vector (in place) while the
    error overlap matrix of those kept has a condition number above `limit`."""
    while len(vecs) >= 2:
        w = np.linalg.eigvalsh(np.array([[np.dot(a, b) for b in errs] for a in errs]))
        if w[0] > w[-1] / limit:
            return
        vecs.pop(0)
        errs.pop(0)


def _diis_extrapolate(vecs, errs):
    m = len(vecs)
    Bm = np.empty((m + 1, m + 1))
    Bm[-1, :] = -1.0
    Bm[:, -1] = -1.0
    Bm[-1, -1] = 0.0
    for i in range(m):
        for j in range(m):
            Bm[i, j] = np.dot(errs[i], errs[j])
    rhs = np.zeros(m + 1)
    rhs[-1] = -1.0
    c = np.linalg.solve(Bm, rhs)[:m]
    return sum(ci * vi for ci, vi in zip(c, vecs))


def solve(eps, L, Xo, Xv, xo=None, xv=None, Z0=None, singles=True, tol=1e-8, tol_e=1e-8,
          maxit=100, diis=8, V=None, scale=None, shift=None) -> SolveResult:
    """Jacobi + DIIS solution of sigma(Z, t1) = 0 in the pseudo-canonical basis.
    Each iteration: residual and energy at the current amplitudes, convergence test,
    T^ <- T^ - sigma^/D, t1 <- t1 - sigma1/(eps_a - eps_i), DIIS(diis), with D_PQ = e_P + e_Q.
    Learned-guess hooks: `scale` (c_P) starts from diag(1+c) T^0 diag(1+c); `shift` (delta_P)
    uses D_PQ = max(e_P + e_Q + delta_P + delta_Q, (e_P + e_Q) / 2)."""
    o, v = Xo.shape[0], Xv.shape[0]
    if V is None and xo is not None:
        z, _ = eri_fit(L, o, xo, xv)
        V = eri_thc_dense(xo, xv, z)
    e, W = pseudo_canonical(Xo, Xv, eps)
    S = metric(Xo, Xv)
    D2 = e[:, None] + e[None, :]
    if shift is not None:
        D2 = np.maximum(D2 + shift[:, None] + shift[None, :], 0.5 * D2)
    D1 = eps[o:][None, :] - eps[:o][:, None]
    if Z0 is None:
        Z0 = mp2_guess(eps, L, Xo, Xv)
    Th = W.T @ S @ Z0 @ S @ W
    if scale is not None:
        Th = (1.0 + scale)[:, None] * Th * (1.0 + scale)[None, :]
    t1 = np.zeros((o, v))
    vecs, errs, hist = [], [], []
    E_old = None
    for it in range(1, maxit + 1):
        Z = W @ Th @ W.T
        t2 = amplitudes(Xo, Xv, Z)
        R2 = ccsd.doubles_residual(eps, L, t1, t2, V)
        sig = project(R2, Xo, Xv)
        sig1 = ccsd.singles_residual(eps, L, t1, t2) if singles else np.zeros((o, v))
        E = ccsd.energy(L, t1, t2)
        sh = W.T @ sig @ W
        rn = float(np.sqrt(np.sum(sh * sh) + np.sum(sig1 * sig1)))
        hist.append((E, rn))
        if E_old is not None and rn < tol and abs(E - E_old) < tol_e:
            return SolveResult(E, Z, t1, it, True, hist)
        E_old = E
        dT = -sh / D2
        dt1 = -sig1 / D1
        Th = Th + dT
        t1 = t1 + dt1
        if diis > 0:
            vecs.append(np.concatenate([Th.ravel(), t1.ravel()]))
            errs.append(np.concatenate([dT.ravel(), dt1.ravel()]))
            if len(vecs) > diis:
                vecs.pop(0)
                errs.pop(0)
            _diis_condition(vecs, errs)
            if len(vecs) >= 2:
                x = _diis_extrapolate(vecs, errs)
                Th = x[: Th.size].reshape(Th.shape)
                t1 = x[Th.size:].reshape(t1.shape)
    Z = W @ Th @ W.T
    return SolveResult(E_old, Z, t1, maxit, False, hist)
