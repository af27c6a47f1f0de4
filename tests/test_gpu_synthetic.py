"""The library's on-device generator of the synthetic inputs against the Python generator that
feeds the oracle (bit for bit), and residual parity of a context whose inputs were generated on
the device (thc_set_synthetic), with the vv Cholesky block held or regenerated per block."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2111_11473_amd import synth
from test_gpu_parity import _check_terms, _host

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def thc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc as mod
    mod.load()
    return mod


def _same_bits(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint64), np.ascontiguousarray(b).view(np.uint64))


@pytest.mark.parametrize("stream", range(7))
def test_device_normals_bitwise(thc, stream):
    n = 10 ** 6
    for seed, first, div in ((1002, 0, 1.0), (2077, 123456789012, np.sqrt(4000.0))):
        _say("normals", stream, seed, first)
        got = _host(thc.synth_normals(seed, stream, first, n, div))
        want = synth.normal(seed, stream, np.arange(n, dtype=np.uint64) + np.uint64(first)) / div
        assert _same_bits(got, want), (seed, stream, int(np.sum(got != want)))


def test_device_cholesky_and_energies_bitwise(thc):
    cfg = synth.CONFIGS["small"]
    s = synth.make_system(cfg)
    _say("cholesky small")
    L = _host(thc.synth_cholesky(cfg.seed, cfg.n, 0, cfg.nL, cfg.decay, s["gamma"]))
    assert _same_bits(L, s["L"])
    part = _host(thc.synth_cholesky(cfg.seed, cfg.n, 17, 5, cfg.decay, 1.0))
    assert _same_bits(part, synth.cholesky_unscaled(cfg)[17:22])
    assert _same_bits(np.array(thc.synth_energies(cfg.seed, cfg.o, cfg.v)), s["eps"])


def _synthetic_ctx(thc, cfg, **kw):
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=True, **kw)
    ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling)
    Z0 = ctx.build_synthetic()
    return ctx, _host(Z0)


@pytest.mark.parametrize("name,flags,a_block", [("small", 0, 0), ("tiny", "stream", 16), ("medium", "stream", 0)])
def test_generated_inputs_residual_matches_oracle(thc, name, flags, a_block):
    """Inputs made on the device: the scale gamma from the device's power iteration agrees with
    the Python rule; with the oracle fed the same gamma the inputs are identical, and every term
    group of the residual matches the oracle -- also with the vv Cholesky block regenerated for
    each block of the fused pass instead of held."""
    cfg = synth.CONFIGS[name]
    fl = thc.FLAG_STREAM_LVV if flags == "stream" else 0
    _say("synthetic ctx", name, flags, a_block)
    ctx, Z0 = _synthetic_ctx(thc, cfg, flags=fl, a_block=a_block)
    plan = ctx.plan()
    assert plan["lvv_resident"] == (0 if fl else 1)
    g = ctx.synth_gamma()
    s_rule = synth.make_system(cfg)
    assert abs(g - s_rule["gamma"]) < 1e-12 * s_rule["gamma"]
    s = synth.make_system(dataclasses.replace(cfg, gamma=g))
    Zref = oracle.mp2_guess(s["eps"], s["L"], s["Xo"], s["Xv"])
    assert np.abs(Z0 - Zref).max() < 1e-9 * np.abs(Zref).max()
    _check_terms(thc, cfg, s, ctx, Z0)
    ctx.close()
