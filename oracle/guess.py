"""Learned starting guess: features, how a prediction is applied, training targets, and the
reference network (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The learned guess is not part of the paper; it is specified as follows.  Everything lives
in the pseudo-canonical working basis (E_mat w = e S w), where the MP2 guess is T^0 and the
Jacobi denominators are e_P + e_Q.
  features   phi_P = [T^0_PP, e_P, T^0_PP e_P, eps_HOMO, eps_LUMO, mean eps_occ,
             mean eps_vir, N_P / o, ||T^0||_F / sqrt(N_P), sum_Q |T^0_PQ|]
  prediction (c_P, delta_P) per rank index P
  start      T^init = diag(1 + c) T^0 diag(1 + c)
  shift      D_PQ = max(e_P + e_Q + delta_P + delta_Q, (e_P + e_Q) / 2)
  targets    c*: least-squares diagonal scaling of T^0 onto the converged T^*, by Gauss-Newton;
             delta*: least-squares secant fit  -sigma^0 ~= (e_P + e_Q + delta_P + delta_Q) (T^* - T^0)
             (the residual changes from sigma^0 at the guess to zero at convergence).
Network: x -> (x - mu_in) / sd_in -> W1, b1 -> SiLU -> W2, b2 -> SiLU -> W3, b3 -> y_n,
y = y_n sd_out + mu_out; loss = mean over rows and outputs of (y_n - (t - mu_out) / sd_out)^2;
SiLU(z) = z / (1 + exp(-z)).  Parameters are one flat vector [W1 (in x w), b1, W2 (w x w), b2,
W3 (w x out), b3], weights row-major with the input index first.  Training uses Adam
(Kingma and Ba, 2015) with bias-corrected moments.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 10
N_OUT = 2


def features(Th0: np.ndarray, e: np.ndarray, eps: np.ndarray, o: int) -> np.ndarray:
    """phi[P, :] as listed in the module docstring."""
    P = Th0.shape[0]
    d = np.diag(Th0)
    phi = np.empty((P, N_FEAT))
    phi[:, 0] = d
    phi[:, 1] = e
    phi[:, 2] = d * e
    phi[:, 3] = eps[:o].max()
    phi[:, 4] = eps[o:].min()
    phi[:, 5] = eps[:o].mean()
    phi[:, 6] = eps[o:].mean()
    phi[:, 7] = P / o
    phi[:, 8] = np.linalg.norm(Th0) / np.sqrt(P)
    phi[:, 9] = np.abs(Th0).sum(axis=1)
    return phi


def apply_scaling(Th0: np.ndarray, c: np.ndarray) -> np.ndarray:
    s = 1.0 + c
    return s[:, None] * Th0 * s[None, :]


def shifted_denominators(e: np.ndarray, delta: np.ndarray | None) -> np.ndarray:
    base = e[:, None] + e[None, :]
    if delta is None:
        return base
    return np.maximum(base + delta[:, None] + delta[None, :], 0.5 * base)


def fit_scaling(Th0: np.ndarray, Tstar: np.ndarray, iters: int = 30, ridge: float = 1e-12) -> np.ndarray:
    """argmin_c || diag(1+c) T^0 diag(1+c) - T^* ||_F by Gauss-Newton on s = 1 + c
    (normal matrix built from the residual's Jacobian, with a tiny ridge)."""
    P = Th0.shape[0]
    s = np.ones(P)
    T2 = Th0 * Th0
    for _ in range(iters):
        r = s[:, None] * Th0 * s[None, :] - Tstar
        # J[(p,q), k] = delta_pk s_q T0_pq + delta_qk s_p T0_pq
        JTJ = 2.0 * (s[:, None] * s[None, :]) * T2
        JTJ[np.diag_indices(P)] = 2.0 * (T2 @ (s * s)) + 2.0 * (s * s) * np.diag(T2)
        # (J^T r)_k = 2 sum_q r_kq s_q T0_kq ;  (J^T J)_kl = 2 delta_kl sum_q s_q^2 T0_kq^2 + 2 s_k s_l T0_kl^2
        JTr = 2.0 * ((r * Th0) @ s)
        scale = max(1.0, np.abs(np.diag(JTJ)).max())
        ds = np.linalg.solve(JTJ + ridge * scale * np.eye(P), -JTr)
        s = s + ds
        if np.abs(ds).max() < 1e-14:
            break
    return s - 1.0


def fit_shift(e: np.ndarray, Th0: np.ndarray, Tstar: np.ndarray, sig0: np.ndarray, ridge: float = 1e-10) -> np.ndarray:
    """argmin_delta sum_PQ ( -sigma^0_PQ - (e_P + e_Q + delta_P + delta_Q) dT_PQ )^2, dT = T^* - T^0."""
    dT = Tstar - Th0
    r = -sig0 - (e[:, None] + e[None, :]) * dT
    D2 = dT * dT
    A = np.diag(D2.sum(axis=1)) + D2
    b = (r * dT).sum(axis=1)
    scale = max(1e-300, np.abs(np.diag(A)).max())
    return np.linalg.solve(A + ridge * scale * np.eye(len(e)), b)


# ---------------------------------------------------------------------------------------------
# reference network

def n_params(n_in: int, width: int, n_out: int) -> int:
    return n_in * width + width + width * width + width + width * n_out + n_out


def unpack(p: np.ndarray, n_in: int, width: int, n_out: int):
    k = 0
    out = []
    for shape in ((n_in, width), (width,), (width, width), (width,), (width, n_out), (n_out,)):
        size = int(np.prod(shape))
        out.append(p[k:k + size].reshape(shape))
        k += size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, dims, X, norm):
    """Returns (y, y_n, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, *dims)
    mu_in, sd_in, mu_out, sd_out = norm
    xn = (X - mu_in) / sd_in
    z1 = xn @ W1 + b1
    h1 = silu(z1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    yn = h2 @ W3 + b3
    return yn * sd_out + mu_out, yn, (xn, z1, h1, z2, h2)


def loss_and_grad(p, dims, X, T, norm):
    W1, b1, W2, b2, W3, b3 = unpack(p, *dims)
    _, yn, (xn, z1, h1, z2, h2) = forward(p, dims, X, norm)
    tn = (T - norm[2]) / norm[3]
    diff = yn - tn
    loss = float(np.mean(diff * diff))
    dyn = 2.0 * diff / diff.size
    gW3 = h2.T @ dyn
    gb3 = dyn.sum(axis=0)
    dz2 = (dyn @ W3.T) * silu_prime(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * silu_prime(z1)
    gW1 = xn.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
