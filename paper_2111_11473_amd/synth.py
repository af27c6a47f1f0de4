"""Seeded synthetic THC-CCSD inputs (orbital energies, Cholesky vectors, collocation factors).

This module holds no arithmetic of the method itself: it only turns (seed, stream, index)
into numbers with the shapes and value distributions of the workloads, so that the CPU
oracle and the GPU library can be fed identical inputs.  Nothing here imports either side.

Generator: a counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  For a key k
derived from (seed, stream), draw i is the SplitMix64 output function applied to the
state k + (i+1)*0x9E3779B97F4A7C15.  Uniforms take the top 53 bits, normals come from the
Box-Muller transform of two consecutive uniforms (cosine branch only).  The logarithm, cosine
and exponential inside are evaluated here from fixed sequences of IEEE additions,
multiplications and divisions (exact range reductions, truncated series with the coefficients
as exact binary constants), not through a math library, so that the library's device twin of
this generator (csrc/synth_core.h, compiled without contraction into fused multiply-adds)
reproduces every value bit for bit.

Value distributions (paper Sec. II, Eq. 1 ordering N_o < N_v < N_CD ~ N_THC ~ N_aux):
  eps_o ~ U[-1.5, -0.3] Eh, eps_v ~ U[0.1, 5.0] Eh, each sorted ascending;
  L^K_pq = gamma * N(0,1) * exp(-K/decay), symmetric in pq (upper triangle drawn, mirrored);
  X_o, X_v ~ N(0,1)/sqrt(N_P) (amplitude collocation, the y factors of Eq. 22-23);
  x_o, x_v ~ N(0,1)/sqrt(N_Q) (ovov ERI collocation, the x factors of Eq. 17).
gamma is one global scale fixed so that gamma^2 * lambda_max(L_ov L_ov^T) = 0.2 * Delta_min,
Delta_min = 2 (min eps_v - max eps_o); without it the unit-variance vectors give amplitudes
of order 10 and no coupled-cluster iteration converges.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_EPS_O, STREAM_EPS_V, STREAM_L, STREAM_XO_AMP, STREAM_XV_AMP, STREAM_XO_ERI, STREAM_XV_ERI = range(7)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mix(np.array([stream], dtype=np.uint64) + _GOLDEN)
        k = _mix(np.array([seed], dtype=np.uint64) * _GOLDEN ^ s)
    return k[0]


def bits(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Raw 64-bit draws for counter values idx (any integer array)."""
    k = _key(seed, stream)
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(k + (idx + np.uint64(1)) * _GOLDEN)


def uniform(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Uniforms in the open interval (0, 1) from the top 53 bits."""
    b = bits(seed, stream, idx) >> np.uint64(11)
    return (b.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


_H = float.fromhex
_LN2 = _H("0x1.62e42fefa39efp-1")
_LN2_HI = _H("0x1.62e42fee00000p-1")     # top 32 bits of ln 2: n * _LN2_HI is exact for |n| < 2^21
_LN2_LO = _H("0x1.a39ef00000000p-33")    # ln 2 - _LN2_HI
_INV_LN2 = _H("0x1.71547652b82fep+0")
_SQRT_HALF = _H("0x1.6a09e667f3bcdp-1")
_TWO_PI = _H("0x1.921fb54442d18p+2")
# 1/(2k+1), k = 0..10 (atanh series of the logarithm)
_ATANH = [_H(c) for c in ("0x1.0000000000000p+0", "0x1.5555555555555p-2", "0x1.999999999999ap-3",
                          "0x1.2492492492492p-3", "0x1.c71c71c71c71cp-4", "0x1.745d1745d1746p-4",
                          "0x1.3b13b13b13b14p-4", "0x1.1111111111111p-4", "0x1.e1e1e1e1e1e1ep-5",
                          "0x1.af286bca1af28p-5", "0x1.8618618618618p-5")]
# (-1)^k/(2k)! and (-1)^k/(2k+1)!, k = 0..9 (cosine and sine series)
_COS = [_H(c) for c in ("0x1.0000000000000p+0", "-0x1.0000000000000p-1", "0x1.5555555555555p-5",
                        "-0x1.6c16c16c16c17p-10", "0x1.a01a01a01a01ap-16", "-0x1.27e4fb7789f5cp-22",
                        "0x1.1eed8eff8d898p-29", "-0x1.93974a8c07c9dp-37", "0x1.ae7f3e733b81fp-45",
                        "-0x1.6827863b97d97p-53")]
_SIN = [_H(c) for c in ("0x1.0000000000000p+0", "-0x1.5555555555555p-3", "0x1.1111111111111p-7",
                        "-0x1.a01a01a01a01ap-13", "0x1.71de3a556c734p-19", "-0x1.ae64567f544e4p-26",
                        "0x1.6124613a86d09p-33", "-0x1.ae7f3e733b81fp-41", "0x1.952c77030ad4ap-49",
                        "-0x1.2f49b46814157p-57")]
# 1/k!, k = 0..14 (exponential series)
_EXP = [_H(c) for c in ("0x1.0000000000000p+0", "0x1.0000000000000p+0", "0x1.0000000000000p-1",
                        "0x1.5555555555555p-3", "0x1.5555555555555p-5", "0x1.1111111111111p-7",
                        "0x1.6c16c16c16c17p-10", "0x1.a01a01a01a01ap-13", "0x1.a01a01a01a01ap-16",
                        "0x1.71de3a556c734p-19", "0x1.27e4fb7789f5cp-22", "0x1.ae64567f544e4p-26",
                        "0x1.1eed8eff8d898p-29", "0x1.6124613a86d09p-33", "0x1.93974a8c07c9dp-37")]


def _horner(coef, x):
    p = np.full_like(x, coef[-1])
    for c in coef[-2::-1]:
        p = p * x + c
    return p


def gen_log(u: np.ndarray) -> np.ndarray:
    """ln u for u > 0: u = m 2^e with m in [sqrt(1/2), sqrt(2)) (exact), then
    e ln 2 + 2 atanh((m - 1)/(m + 1)) by its series (|s| < 0.172, 11 terms)."""
    m, e = np.frexp(np.asarray(u, dtype=np.float64))
    small = m < _SQRT_HALF
    m = np.where(small, m * 2.0, m)
    e = (e - small.astype(e.dtype)).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    return e * _LN2 + 2.0 * (s * _horner(_ATANH, s * s))


def gen_cos_turns(t: np.ndarray) -> np.ndarray:
    """cos(2 pi t) for t in [0, 1): the reductions to a quarter of an eighth turn are exact
    (Sterbenz), then the cosine or sine series on |x| <= pi/4 (10 terms)."""
    t = np.asarray(t, dtype=np.float64)
    a = np.where(t >= 0.5, 1.0 - t, t)          # cos(2 pi t) = cos(2 pi (1 - t)), a in [0, 1/2]
    neg = a > 0.25
    a = np.where(neg, 0.5 - a, a)               # cos(2 pi a) = -cos(2 pi (1/2 - a)), a in [0, 1/4]
    use_sin = a > 0.125
    a = np.where(use_sin, 0.25 - a, a)          # cos(2 pi a) = sin(2 pi (1/4 - a)), a in [0, 1/8]
    x = a * _TWO_PI
    x2 = x * x
    c = _horner(_COS, x2)
    sn = x * _horner(_SIN, x2)
    r = np.where(use_sin, sn, c)
    return np.where(neg, -r, r)


def gen_exp(x: np.ndarray) -> np.ndarray:
    """e^x for moderate x: x = n ln 2 + r with n = floor(x / ln 2 + 1/2) (two-part ln 2), the
    series of e^r (|r| <= 0.35, 15 terms), scaled by 2^n exactly."""
    x = np.asarray(x, dtype=np.float64)
    n = np.floor(x * _INV_LN2 + 0.5)
    r = (x - n * _LN2_HI) - n * _LN2_LO
    return np.ldexp(_horner(_EXP, r), n.astype(np.int64))


def normal(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Standard normals; normal i consumes uniforms 2i and 2i+1 (Box-Muller, cosine branch)."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform(seed, stream, idx * np.uint64(2))
    u2 = uniform(seed, stream, idx * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * gen_log(u1)) * gen_cos_turns(u2)


def decay_factor(K, decay: float) -> np.ndarray:
    """e^(-K/decay) of Cholesky vector K."""
    return gen_exp(-np.asarray(K, dtype=np.float64) / float(decay))


@dataclass(frozen=True)
class Config:
    """Sizes of one synthetic system: occupied o, virtual v, Cholesky rank nL,
    amplitude THC rank nP, ERI THC grid nQ; Cholesky decay length; seed."""
    name: str
    o: int
    v: int
    nL: int
    nP: int
    nQ: int
    decay: float = 30.0
    seed: int = 1000
    gamma: float | None = None  # None: the lambda_max rule above
    coupling: float = 0.2       # the rule's fraction of the smallest pair gap

    @property
    def n(self) -> int:
        return self.o + self.v


# The workloads: tiny oracle scale, the plain FP64 GPU scale, the mixed-precision scale,
# the ~2500-basis-function single-GPU scale, and two extra parity sizes.
CONFIGS = {
    "tiny": Config("tiny", 10, 40, 150, 120, 300, 30.0, 1000),
    "fp64": Config("fp64", 50, 450, 1500, 1000, 2500, 150.0, 1001),
    "mixed": Config("mixed", 200, 1800, 6000, 4000, 10000, 600.0, 1002),
    "paper": Config("paper", 350, 2150, 10000, 7000, 17500, 1000.0, 1003),
    # parity-only sizes: several kernel tiles with ragged tails, oracle still fast
    "small": Config("small", 6, 22, 70, 50, 110, 30.0, 1010),
    "medium": Config("medium", 14, 66, 210, 170, 420, 30.0, 1011),
    # wider occupied spaces: the fused exchange kernel's o <= 64 and o <= 128 instantiations
    "occ40": Config("occ40", 40, 56, 200, 130, 300, 30.0, 1012),
    "occ70": Config("occ70", 70, 30, 150, 120, 260, 30.0, 1013),
    # o in (40, 48], (48, 56] and (56, 64]: the exchange kernel's first product stops at 12, 14
    # and 16 k-steps
    "occ46": Config("occ46", 46, 24, 120, 110, 260, 30.0, 1015),
    "occ53": Config("occ53", 53, 20, 110, 100, 240, 30.0, 1016),
    "occ60": Config("occ60", 60, 18, 110, 100, 240, 30.0, 1017),
    # o in (128, 200]: the exchange kernel's 13-row-block instantiation (o = 136 keeps the
    # oracle's o^4 block at 2.7 GB)
    "occ136": Config("occ136", 136, 4, 24, 120, 300, 30.0, 1021),
    # a rank large enough for the benchmark's kernel paths with an oracle that still runs in
    # seconds: 704-padded H ranks (about 43 H-kernel generations, so the backward grid-point walk
    # of odd generations), 128 x 128 tiles for the split symmetric Alg. 1 product
    "wide": Config("wide", 8, 100, 100, 700, 780, 30.0, 1020),
    # degenerate sizes: one occupied orbital; a pair basis and ERI grid as large as the o v
    # pairs (complete: THC-CCSD is then CD-CCSD)
    "one_occ": Config("one_occ", 1, 9, 12, 7, 9, 30.0, 1014),
    "complete": Config("complete", 3, 2, 10, 6, 6, 30.0, 1039),
}


def learned_config(s: int) -> Config:
    """System s (0..255) of the learned-guess set: o in [30, 80], v = 9o, nL = 30o,
    nP = 20o, nQ = 50o; seed 2000 + s."""
    o = 30 + int(bits(7, 0, np.array([s]))[0] % np.uint64(51))
    return Config(f"learn{s}", o, 9 * o, 30 * o, 20 * o, 50 * o, 30.0, 2000 + s)


def orbital_energies(cfg: Config) -> np.ndarray:
    eo = -1.5 + 1.2 * uniform(cfg.seed, STREAM_EPS_O, np.arange(cfg.o))
    ev = 0.1 + 4.9 * uniform(cfg.seed, STREAM_EPS_V, np.arange(cfg.v))
    return np.concatenate([np.sort(eo), np.sort(ev)])


def cholesky_unscaled(cfg: Config, dtype=np.float64) -> np.ndarray:
    """L^K_pq / gamma as an (nL, n, n) array, symmetric in (p, q)."""
    n = cfg.n
    iu, ju = np.triu_indices(n)
    flat = (iu * n + ju).astype(np.uint64)
    out = np.empty((cfg.nL, n, n), dtype=dtype)
    for K in range(cfg.nL):
        vals = normal(cfg.seed, STREAM_L, np.uint64(K * n * n) + flat) * decay_factor(K, cfg.decay)
        m = out[K]
        m[iu, ju] = vals
        m[ju, iu] = vals
    return out


def _lambda_max_ov(Lov: np.ndarray, iters: int = 200) -> float:
    """Largest eigenvalue of the (ov x ov) Gram sum_K L^K (L^K)^T through the small
    (nL x nL) Gram, by power iteration from a fixed start (deterministic)."""
    M = Lov.reshape(Lov.shape[0], -1)
    G = M @ M.T
    x = np.ones(G.shape[0]) / np.sqrt(G.shape[0])
    lam = 0.0
    for _ in range(iters):
        y = G @ x
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam


def make_system(cfg: Config) -> dict:
    """All inputs of one system as FP64 numpy arrays:
    eps (n), L (nL, n, n), Xo (o, nP), Xv (v, nP), xo (o, nQ), xv (v, nQ), gamma."""
    o, v = cfg.o, cfg.v
    eps = orbital_energies(cfg)
    L = cholesky_unscaled(cfg)
    if cfg.gamma is None:
        dmin = 2.0 * (eps[o] - eps[o - 1])
        lam = _lambda_max_ov(L[:, :o, o:])
        gamma = float(np.sqrt(cfg.coupling * dmin / lam))
    else:
        gamma = float(cfg.gamma)
    L *= gamma
    Xo = normal(cfg.seed, STREAM_XO_AMP, np.arange(o * cfg.nP)).reshape(o, cfg.nP) / np.sqrt(cfg.nP)
    Xv = normal(cfg.seed, STREAM_XV_AMP, np.arange(v * cfg.nP)).reshape(v, cfg.nP) / np.sqrt(cfg.nP)
    xo = normal(cfg.seed, STREAM_XO_ERI, np.arange(o * cfg.nQ)).reshape(o, cfg.nQ) / np.sqrt(cfg.nQ)
    xv = normal(cfg.seed, STREAM_XV_ERI, np.arange(v * cfg.nQ)).reshape(v, cfg.nQ) / np.sqrt(cfg.nQ)
    return dict(eps=eps, L=L, Xo=Xo, Xv=Xv, xo=xo, xv=xv, gamma=gamma, cfg=cfg)


def complete_basis(o: int, v: int):
    """Indicator collocation spanning the whole ov pair space: X_o[i, (i'a')] = delta_ii',
    X_v[a, (i'a')] = delta_aa' (column index i'*v + a').  With it the Khatri-Rao product of
    the factors is the identity on ov, so every projection is exact."""
    Xo = np.zeros((o, o * v))
    Xv = np.zeros((v, o * v))
    for i in range(o):
        for a in range(v):
            Xo[i, i * v + a] = 1.0
            Xv[a, i * v + a] = 1.0
    return Xo, Xv
