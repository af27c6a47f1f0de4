"""Mixed-precision path (precision = 1): FP32-MFMA contractions and FP32 H-kernel operands with
FP64 accumulation of H, FP64 energy, denominators, fit and DIIS; precision = 2 with the
contractions as compensated split-BF16 products (each FP32-rounded operand split exactly into
three bf16 pieces, the six largest cross products on BF16 MFMA, FP32 accumulation).

Bounds.  Rounding the operands of a product to FP32 (unit roundoff 2^-24 = 6e-8) and accumulating
in FP32 over K terms gives a relative error of order sqrt(K) 2^-24 for each term group; with
K <= 1e4 here that is ~6e-6.  The split products add only the dropped cross terms, O(2^-24) of
each product.  Each term group must match the FP64 oracle to 5e-5 of its largest element in both
modes.  A mixed solve finishes with FP64 iterations, so its converged energy must match the FP64
solve to 1e-8 Eh."""
import numpy as np
import pytest

import oracle
from oracle import ccsd
from paper_2111_11473_amd import synth

pytestmark = pytest.mark.gpu
RTOL_MIXED = {1: 5e-5, 2: 5e-5}


def _say(*a):
    print("[gpu-mixed]", *a, flush=True)


@pytest.fixture(scope="module")
def thc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc as mod
    mod.load()
    return mod


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _make(thc, cfg, **kw):
    s = synth.make_system(cfg)
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, **kw)
    Z0 = ctx.build_factors(_dev(s["L"]), _dev(s["eps"]), _dev(s["Xo"]), _dev(s["Xv"]), _dev(s["xo"]), _dev(s["xv"]))
    return s, ctx, _host(Z0)


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("name", ["tiny", "medium", "occ40", "occ53", "occ70", "occ136"])
def test_mixed_residual_terms_within_bound(thc, name, precision):
    cfg = synth.CONFIGS[name]
    _say("terms", name, "precision", precision)
    s, ctx, Z0 = _make(thc, cfg, precision=precision)
    rng = np.random.default_rng(3)
    P = Z0.shape[0]
    R = rng.standard_normal((P, P))
    Z = Z0 + 0.3 * np.abs(Z0).max() * (R + R.T)
    t1 = 0.02 * rng.standard_normal((cfg.o, cfg.v))
    z, _ = oracle.eri_fit(s["L"], cfg.o, s["xo"], s["xv"])
    V = oracle.eri_thc_dense(s["xo"], s["xv"], z)
    ref, refs = oracle.thc_residual(s["eps"], s["L"], s["Xo"], s["Xv"], Z, t1, V, terms=True)
    ref["eq32+33"] = ref.pop("eq32") + ref.pop("eq33")
    worst = 0.0
    for key, mask in thc.TERMS.items():
        sig, sig1 = ctx.residual(_dev(Z), _dev(t1), mask=mask)
        got, want = (_host(sig1), refs[key]) if key in ("eq38", "eq42") else (_host(sig), ref[key])
        err = np.abs(got - want).max() / np.abs(want).max()
        worst = max(worst, err)
        _say(f"  {key}: relative error {err:.2e}")
        assert err < RTOL_MIXED[precision], (key, err)
    _say("worst term error", worst)


@pytest.mark.parametrize("i_chunk", [0, 200])
def test_mixed_wide_rank_h_path(thc, i_chunk):
    """Eq. 32 + 33 in mixed precision at a rank (nP = 700) where the FP32 H-kernel runs many
    generations of resident tiles (odd ones walking the grid points backwards) and, with 200-point
    chunks, adds each chunk's FP32 sums into the FP64 H of the previous ones."""
    cfg = synth.CONFIGS["wide"]
    _say("wide mixed i_chunk", i_chunk)
    s, ctx, Z0 = _make(thc, cfg, precision=1, i_chunk=i_chunk, flags=thc.FLAG_QUARTIC)
    plan = ctx.plan()
    assert plan["quintic"] == 0 and plan["i_chunks"] == (1 if i_chunk == 0 else 4)
    rng = np.random.default_rng(4)
    P = Z0.shape[0]
    R = rng.standard_normal((P, P))
    Z = Z0 + 0.3 * np.abs(Z0).max() * (R + R.T)
    t1 = 0.02 * rng.standard_normal((cfg.o, cfg.v))
    z, _ = oracle.eri_fit(s["L"], cfg.o, s["xo"], s["xv"])
    V = oracle.eri_thc_dense(s["xo"], s["xv"], z)
    ref, _ = oracle.thc_residual(s["eps"], s["L"], s["Xo"], s["Xv"], Z, t1, V, terms=True)
    want = ref["eq32"] + ref["eq33"]
    sig, _ = ctx.residual(_dev(Z), _dev(t1), mask=thc.TERM_EQ32)
    err = np.abs(_host(sig) - want).max() / np.abs(want).max()
    _say("  eq32+33 relative error %.2e" % err)
    assert err < RTOL_MIXED[1]


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_solve_reaches_fp64_energy(thc, precision):
    cfg = synth.CONFIGS["medium"]
    _say("solve medium, precision", precision)
    _, c64, _ = _make(thc, cfg, tol_energy=1e-10)
    it64, _, ok64 = c64.iterate(tol=1e-8, maxit=60)
    e64 = c64.energy()
    _, cmx, _ = _make(thc, cfg, tol_energy=1e-10, precision=precision)
    itmx, _, okmx = cmx.iterate(tol=1e-8, maxit=60)
    emx = cmx.energy()
    flags = cmx.history_precision()
    _say("fp64 iterations", it64, "mixed iterations", itmx, "precision flags", flags, "dE", abs(emx - e64))
    assert ok64 and okmx
    assert abs(emx - e64) < 1e-8
    assert flags[0] == 1 and flags[-1] == 0 and sum(flags) >= 1
    assert all(a >= b for a, b in zip(flags, flags[1:]))  # mixed first, then FP64 only
