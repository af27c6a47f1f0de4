"""Two context options of the C ABI, through the library:

* split_mask -- which contraction chains of a mixed-precision residual run as compensated
  split-BF16 products instead of FP32 MFMA.  Every chain set is bit-for-bit precision 2, none is
  bit-for-bit precision 1, a chain that does not run in this configuration (Alg. 4-5 under Alg. 6)
  changes nothing, and one that does (Alg. 6) changes the result but stays within the mixed
  bound of the FP64 residual.
* guess = 1 -- the library starts the first iterate() from the attached network's prediction.
  With a network whose output is a constant (zero weights, the output mean set by hand) the run is
  bit-for-bit the one made by hand from thc_guess_features / thc_mlp_infer / thc_guess_apply; a
  prediction far off diverges and the solve restarts from the MP2 guess and ends at the plain
  energy; without a network iterate() refuses; after set_state() no learned start is applied."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2111_11473_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-options]", *a, flush=True)


@pytest.fixture(scope="module")
def thc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc as mod
    mod.load()
    return mod


def _ctx(thc, cfg, **kw):
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=True, tol_energy=1e-10, **kw)
    ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling)
    return ctx


def _residual(thc, cfg, Z, t1, **kw):
    ctx = _ctx(thc, cfg, **kw)
    ctx.build_synthetic()
    sig, sig1 = ctx.residual(Z, t1)
    torch.cuda.synchronize()
    out = torch.cat([sig.flatten(), sig1.flatten()]).cpu().numpy()
    ctx.close()
    return out


def test_split_mask_routes_chains(thc):
    cfg = synth.CONFIGS["medium"]
    ctx = _ctx(thc, cfg)
    Z0 = ctx.build_synthetic()
    ctx.close()
    g = torch.Generator().manual_seed(5)
    Z = (Z0 + 0.1 * Z0.abs().max() * torch.randn(Z0.shape, generator=g, dtype=torch.float64).to("cuda"))
    Z = (0.5 * (Z + Z.T)).contiguous()
    t1 = (1e-2 * torch.randn((cfg.o, cfg.v), generator=g, dtype=torch.float64)).to("cuda")
    _say("config", cfg)
    ref64 = _residual(thc, cfg, Z, t1)
    p1 = _residual(thc, cfg, Z, t1, precision=1)
    p2 = _residual(thc, cfg, Z, t1, precision=2)
    every = _residual(thc, cfg, Z, t1, precision=1, split_mask=thc.CHAIN_ALL)
    none = _residual(thc, cfg, Z, t1, precision=1, split_mask=0)
    assert np.array_equal(every, p2)
    assert np.array_equal(none, p1)
    assert not np.array_equal(p1, p2)
    scale = np.abs(ref64).max()
    alg45 = _residual(thc, cfg, Z, t1, precision=1, split_mask=thc.CHAIN_ALG45)
    assert np.array_equal(alg45, p1)  # Alg. 6 runs here, so the Alg. 4-5 chain has no products
    for name in ("CHAIN_FUSED", "CHAIN_ASSEMBLY", "CHAIN_ALG6", "CHAIN_ALG7", "CHAIN_SINGLES"):
        r = _residual(thc, cfg, Z, t1, precision=1, split_mask=getattr(thc, name))
        err = np.abs(r - ref64).max() / scale
        _say(name, "differs from FP32:", not np.array_equal(r, p1), "error vs FP64 %.2e" % err)
        assert err < 5e-5, (name, err)
        if name == "CHAIN_ALG6":
            assert not np.array_equal(r, p1)
    with pytest.raises(thc.ThcError):
        thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, precision=1, split_mask=1 << 6)


def _constant_net(thc, c, d):
    net = thc.MLP(10, 256, 2, seed=3)
    net.set_params(torch.zeros(net.n_params, dtype=torch.float32, device="cuda"))
    net.set_norm([0.0] * 10, [1.0] * 10, [c, d], [1.0, 1.0])
    return net


def test_learned_start_in_the_library_equals_the_manual_one(thc):
    cfg = synth.CONFIGS["tiny"]
    net = _constant_net(thc, 0.05, 0.01)
    # by hand
    a = _ctx(thc, cfg)
    a.build_synthetic()
    a.guess_apply(net.infer(a.guess_features()))
    it_a, _, ok_a = a.iterate(tol=1e-9, maxit=60)
    e_a, r_a, _ = a.history()
    # in the library
    b = _ctx(thc, cfg, guess=1)
    b.set_guess_network(net)
    b.build_synthetic()
    it_b, _, ok_b = b.iterate(tol=1e-9, maxit=60)
    e_b, r_b, _ = b.history()
    flags = b.history_flags()
    _say("manual", it_a, e_a[-1], "library", it_b, e_b[-1], flags)
    assert ok_a and ok_b and it_a == it_b
    assert e_a == e_b and r_a == r_b
    assert all(f & thc.ITER_LEARNED for f in flags)
    # a second iterate() continues from the converged state: no second learned start
    b.iterate(tol=1e-9, maxit=5)
    assert not any(f & thc.ITER_LEARNED for f in b.history_flags())
    a.close()
    b.close()


def test_learned_start_falls_back_when_it_diverges(thc):
    cfg = synth.CONFIGS["tiny"]
    plain = _ctx(thc, cfg)
    plain.build_synthetic()
    plain.iterate(tol=1e-9, maxit=60)
    e_plain = plain.energy()
    plain.close()
    far = _constant_net(thc, 99.0, 99.0)  # start 100^2 times the guess, steps 100 times too short
    ctx = _ctx(thc, cfg, guess=1)
    ctx.set_guess_network(far)
    ctx.build_synthetic()
    it, _, ok = ctx.iterate(tol=1e-9, maxit=80)
    flags = ctx.history_flags()
    _say("far prediction", it, flags, ctx.energy(), e_plain)
    assert ok
    assert flags[0] & thc.ITER_LEARNED
    restart = [k for k, f in enumerate(flags) if f & thc.ITER_RESTARTED]
    assert len(restart) == 1 and not any(f & thc.ITER_LEARNED for f in flags[restart[0]:])
    assert abs(ctx.energy() - e_plain) < 1e-9
    ctx.close()


def test_learned_start_needs_a_network_and_a_fresh_guess(thc):
    cfg = synth.CONFIGS["tiny"]
    ctx = _ctx(thc, cfg, guess=1)
    Z0 = ctx.build_synthetic()
    with pytest.raises(thc.ThcError) as e:
        ctx.iterate(tol=1e-9, maxit=5)
    assert e.value.rc == thc.THC_ESTATE
    ctx.close()
    net = _constant_net(thc, 0.05, 0.0)
    ctx = _ctx(thc, cfg, guess=1)
    ctx.set_guess_network(net)
    Z0 = ctx.build_synthetic()
    ctx.set_state(Z0)  # an explicit state replaces the pending learned start
    ctx.iterate(tol=1e-9, maxit=60)
    assert not any(f & thc.ITER_LEARNED for f in ctx.history_flags())
    ctx.close()
    with pytest.raises(thc.ThcError):
        bad = thc.MLP(10, 128, 2, seed=1)
        c2 = _ctx(thc, cfg, guess=1)
        try:
            c2.set_guess_network(bad)
        finally:
            c2.close()
