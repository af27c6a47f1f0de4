"""The benchmark workload itself (fp64: o=50 v=450 nL=1500 nP=1000 nQ=2500), built and run in
the launch configuration bench.py times, against what the oracle computes at that size.

The dense oracle cannot hold this system (the v^4 integral block), so the checks are the
quantities it computes through the factors, each pinned against the dense oracle on small
systems (tests/test_oracle.py):
  - the residual at zero amplitudes is the projected driver M^T M (every other term vanishes);
  - the energy of the MP2 guess from the factors (Coulomb and exchange per Cholesky vector);
and properties that hold at any size: the residual of a symmetric core is symmetric, it does not
depend on the blocking of the Cholesky pass, the grid-point chunk or the X block, and both
mixed-precision modes stay within their error bound of the FP64 residual."""
import numpy as np
import pytest

import oracle
from paper_2111_11473_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-full]", *a, flush=True)


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc
    thc.load()
    cfg = synth.CONFIGS["fp64"]
    _say("generating", cfg)
    s = synth.make_system(cfg)
    dev = {k: torch.from_numpy(np.ascontiguousarray(s[k])).to("cuda") for k in ("L", "eps", "Xo", "Xv", "xo", "xv")}
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ)
    Z0 = ctx.build_factors(dev["L"], dev["eps"], dev["Xo"], dev["Xv"], dev["xo"], dev["xv"])
    yield thc, cfg, s, dev, ctx, Z0.cpu().numpy()
    ctx.close()


def test_zero_amplitude_residual_is_the_projected_driver(full):
    import torch
    thc, cfg, s, dev, ctx, Z0 = full
    _say("zero-amplitude residual")
    z = torch.zeros((cfg.nP, cfg.nP), dtype=torch.float64, device="cuda")
    t1 = torch.zeros((cfg.o, cfg.v), dtype=torch.float64, device="cuda")
    sig, sig1 = ctx.residual(z, t1)
    ref = oracle.driver_projection(s["L"], s["Xo"], s["Xv"])
    err = np.abs(sig.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say("relative error", err)
    assert err < 1e-11
    assert np.abs(sig1.cpu().numpy()).max() < 1e-12 * np.abs(ref).max()


def test_energy_of_the_mp2_guess_from_factors(full):
    thc, cfg, s, dev, ctx, Z0 = full
    _say("energy of the MP2 guess")
    e_gpu = ctx.energy()
    e_ref = oracle.energy_from_factors(s["L"], s["Xo"], s["Xv"], Z0)
    _say("gpu", e_gpu, "oracle", e_ref)
    assert abs(e_gpu - e_ref) < 1e-10 * max(1.0, abs(e_ref)) and abs(e_gpu - e_ref) < 1e-12


def test_residual_symmetric_and_blocking_invariant(full):
    import torch
    thc, cfg, s, dev, ctx, Z0 = full
    rng = np.random.default_rng(11)
    R = rng.standard_normal(Z0.shape)
    Z = Z0 + 0.2 * np.abs(Z0).max() * (R + R.T)
    t1 = 0.01 * rng.standard_normal((cfg.o, cfg.v))
    Zd, t1d = torch.from_numpy(Z).to("cuda"), torch.from_numpy(t1).to("cuda")
    _say("residual (default blocking)")
    a, a1 = ctx.residual(Zd, t1d)
    a, a1 = a.cpu().numpy(), a1.cpu().numpy()
    scale = np.abs(a).max()
    asym = np.abs(a - a.T).max() / scale
    _say("asymmetry", asym)
    assert asym < 1e-12
    _say("residual (Cholesky block 40, grid chunk 300, X block 320)")
    c2 = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, a_block=40, i_chunk=300, x_block=320)
    c2.build_factors(dev["L"], dev["eps"], dev["Xo"], dev["Xv"], dev["xo"], dev["xv"])
    b, b1 = c2.residual(Zd, t1d)
    b, b1 = b.cpu().numpy(), b1.cpu().numpy()
    c2.close()
    d = np.abs(a - b).max() / scale
    d1 = np.abs(a1 - b1).max() / np.abs(a1).max()
    _say("blocking difference", d, d1)
    assert d < 1e-11 and d1 < 1e-11


def test_mixed_residual_at_full_size_within_bound(full):
    """Both mixed-precision modes at the benchmark workload, in the launch configuration the bench
    times (the FP32 H-kernel over 63 generations of 16 x 16 block pairs per grid-point chunk, four
    chunks): the projected and singles residuals stay within the mixed bound (5e-5 of the largest
    element) of the FP64 residual, itself checked above."""
    import torch
    thc, cfg, s, dev, ctx, Z0 = full
    rng = np.random.default_rng(12)
    R = rng.standard_normal(Z0.shape)
    Z = Z0 + 0.2 * np.abs(Z0).max() * (R + R.T)
    t1 = 0.01 * rng.standard_normal((cfg.o, cfg.v))
    Zd, t1d = torch.from_numpy(Z).to("cuda"), torch.from_numpy(t1).to("cuda")
    a, a1 = ctx.residual(Zd, t1d)
    a, a1 = a.cpu().numpy(), a1.cpu().numpy()
    for prec in (1, 2):
        _say("mixed residual, precision", prec)
        c = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, precision=prec)
        c.build_factors(dev["L"], dev["eps"], dev["Xo"], dev["Xv"], dev["xo"], dev["xv"])
        assert c.plan()["i_chunks"] == ctx.plan()["i_chunks"]
        b, b1 = c.residual(Zd, t1d)
        b, b1 = b.cpu().numpy(), b1.cpu().numpy()
        c.close()
        d = np.abs(a - b).max() / np.abs(a).max()
        d1 = np.abs(a1 - b1).max() / np.abs(a1).max()
        _say("  relative difference", d, d1)
        assert d < 5e-5 and d1 < 5e-5
