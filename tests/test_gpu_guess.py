"""Learned-guess pieces on the GPU against the FP64 reference (oracle/guess.py, oracle.solve):
the network's FP32 forward, loss and gradient, the Adam update, BF16 inference, the features,
the training targets, and a solve started from a scaled guess with shifted denominators."""
import numpy as np
import pytest

import oracle
from oracle import guess
from paper_2111_11473_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-guess]", *a, flush=True)


@pytest.fixture(scope="module")
def thc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc as mod
    mod.load()
    return mod


def _t(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda")


def _h(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _net(thc, rows=300, seed=5):
    rng = np.random.default_rng(seed)
    net = thc.MLP(guess.N_FEAT, 256, guess.N_OUT, seed=seed)
    norm = (rng.standard_normal(guess.N_FEAT), rng.uniform(0.5, 2.0, guess.N_FEAT), rng.standard_normal(guess.N_OUT),
            rng.uniform(0.5, 2.0, guess.N_OUT))
    norm = tuple(np.asarray(x, dtype=np.float32).astype(np.float64) for x in norm)
    net.set_norm(*norm)
    X = rng.standard_normal((rows, guess.N_FEAT)).astype(np.float32)
    T = rng.standard_normal((rows, guess.N_OUT)).astype(np.float32)
    return net, norm, X, T


def test_network_forward_loss_and_gradient_match_oracle(thc):
    """FP32 kernels against the FP64 reference on the same parameters (rows not a multiple of 64)."""
    _say("mlp forward/grad")
    net, norm, X, T = _net(thc)
    dims = (guess.N_FEAT, 256, guess.N_OUT)
    p = _h(net.get_params())
    assert p.size == guess.n_params(*dims)
    y_ref, _, _ = guess.forward(p, dims, X.astype(np.float64), norm)
    y = _h(net.forward(_t(X, np.float32)))
    assert np.abs(y - y_ref).max() < 2e-5 * np.abs(y_ref).max()
    loss, g = net.loss_grad(_t(X, np.float32), _t(T, np.float32))
    loss_ref, g_ref = guess.loss_and_grad(p, dims, X.astype(np.float64), T.astype(np.float64), norm)
    assert abs(loss - loss_ref) < 1e-5 * loss_ref
    g = _h(g)
    # per parameter block: W1, b1, W2, b2, W3, b3
    sizes = [dims[0] * 256, 256, 256 * 256, 256, 256 * dims[2], dims[2]]
    k = 0
    for n in sizes:
        a, b = g[k:k + n], g_ref[k:k + n]
        assert np.abs(a - b).max() < 1e-4 * np.abs(b).max(), (k, np.abs(a - b).max(), np.abs(b).max())
        k += n


def test_adam_steps_match_the_update_rule(thc):
    """Two training steps: the parameters move exactly as Adam prescribes for the gradients the
    kernels computed at each point."""
    _say("mlp adam")
    net, norm, X, T = _net(thc, rows=130, seed=6)
    Xd, Td = _t(X, np.float32), _t(T, np.float32)
    lr = 1e-3
    p0 = _h(net.get_params())
    _, g0 = net.loss_grad(Xd, Td)
    g0 = _h(g0)
    net.train_step(Xd, Td, lr)
    p1 = _h(net.get_params())
    want1, m, v = guess.adam(p0, g0, np.zeros_like(p0), np.zeros_like(p0), 1, lr)
    assert np.abs(p1 - want1).max() < 2e-6 * max(1.0, np.abs(p0).max())
    _, g1 = net.loss_grad(Xd, Td)
    g1 = _h(g1)
    net.train_step(Xd, Td, lr)
    p2 = _h(net.get_params())
    want2, _, _ = guess.adam(p1, g1, m, v, 2, lr)
    assert np.abs(p2 - want2).max() < 2e-6 * max(1.0, np.abs(p0).max())


def test_bf16_inference_tracks_fp32(thc):
    """BF16 MFMA inference (FP32 accumulation) against the FP32 forward: the error bound is the
    BF16 unit roundoff 2^-8 amplified by the three layers; stated in standardized output units."""
    _say("mlp bf16")
    net, norm, X, T = _net(thc, rows=1000, seed=7)
    Xd = _t(X, np.float32)
    y32 = _h(net.forward(Xd))
    y16 = _h(net.infer(Xd))
    err = np.abs((y16 - y32) / norm[3]).max()
    _say("bf16 max error (standardized):", err)
    assert err < 0.05


def _system(thc, name, singles=True):
    import torch
    cfg = synth.CONFIGS[name]
    s = synth.make_system(cfg)
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=singles, tol_energy=1e-11)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    Z0 = ctx.build_factors(d(s["L"]), d(s["eps"]), d(s["Xo"]), d(s["Xv"]), d(s["xo"]), d(s["xv"]))
    return cfg, s, ctx, _h(Z0)


def test_features_and_targets_match_oracle(thc):
    _say("features/targets tiny")
    cfg, s, ctx, Z0 = _system(thc, "tiny")
    e, W = oracle.pseudo_canonical(s["Xo"], s["Xv"], s["eps"])
    S = oracle.metric(s["Xo"], s["Xv"])
    Th0_ref = W.T @ S @ Z0 @ S @ W          # eigenvector signs may differ; the features do not
    phi = _h(ctx.guess_features())
    phi_ref = guess.features(Th0_ref, e, s["eps"], cfg.o)
    assert np.abs(phi - phi_ref).max() < 1e-5 * np.abs(phi_ref).max(axis=0).clip(1e-30).max()
    for k in range(guess.N_FEAT):
        assert np.abs(phi[:, k] - phi_ref[:, k]).max() <= 1e-5 * max(1e-12, np.abs(phi_ref[:, k]).max()), k
    Th0, sig0 = ctx.working(residual=True)
    it, rn, ok = ctx.iterate(tol=1e-10, maxit=60)
    assert ok
    Ts, _ = ctx.working()
    c, d = ctx.guess_targets(Th0, Ts, sig0)
    c_ref = guess.fit_scaling(_h(Th0), _h(Ts))
    d_ref = guess.fit_shift(e, _h(Th0), _h(Ts), _h(sig0))
    assert np.abs(_h(c) - c_ref).max() < 1e-8 * max(1.0, np.abs(c_ref).max())
    assert np.abs(_h(d) - d_ref).max() < 1e-7 * max(1.0, np.abs(d_ref).max())


@pytest.mark.parametrize("singles", [True, False])
def test_scaled_guess_and_shift_match_oracle_solve(thc, singles):
    """A state scaled by (1 + c) and denominators shifted by delta: the GPU solve follows the
    oracle's iteration for iteration and converges to the same energy as the plain solve."""
    import torch
    _say("guess apply tiny singles", singles)
    cfg, s, ctx, Z0 = _system(thc, "tiny", singles=singles)
    rng = np.random.default_rng(21)
    c = (0.2 * rng.standard_normal(cfg.nP)).astype(np.float32)
    dl = (0.3 * rng.standard_normal(cfg.nP)).astype(np.float32)
    pred = torch.from_numpy(np.stack([c, dl], axis=1)).to("cuda")
    ctx.guess_apply(pred)
    it, rn, ok = ctx.iterate(tol=1e-10, maxit=80)
    assert ok
    r = oracle.solve(s["eps"], s["L"], s["Xo"], s["Xv"], s["xo"], s["xv"], Z0=Z0, singles=singles, tol=1e-10,
                     tol_e=1e-11, maxit=80, scale=c.astype(np.float64), shift=dl.astype(np.float64))
    assert r.converged
    assert abs(ctx.energy() - r.energy) < 1e-9
    assert abs(it - r.iterations) <= 2
    plain = oracle.solve(s["eps"], s["L"], s["Xo"], s["Xv"], s["xo"], s["xv"], Z0=Z0, singles=singles, tol=1e-10,
                         tol_e=1e-11, maxit=80)
    assert abs(r.energy - plain.energy) < 1e-9   # the fixed point does not depend on the start
    ctx.set_shift(None)
