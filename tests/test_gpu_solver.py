"""Failure handling of the solver (thc_iterate), each condition forced from the host: a NaN
state, a start a hundred times the MP2 guess, an iteration limit of one, and inputs on which the
plain iteration itself diverges (the unscaled synthetic Cholesky vectors); and checkpoint/resume
of an interrupted solve in a fresh context."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2111_11473_amd import synth

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


def _ctx(thc, cfg, gamma=0.0):
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=True, tol_energy=1e-10)
    ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling, gamma)
    Z0 = ctx.build_synthetic()
    return ctx, Z0


@pytest.fixture(scope="module")
def plain(thc):
    cfg = synth.CONFIGS["tiny"]
    ctx, Z0 = _ctx(thc, cfg)
    it, rn, ok = ctx.iterate(tol=1e-9, maxit=60)
    assert ok and not any(f & thc.ITER_RESTARTED for f in ctx.history_flags())
    e = ctx.energy()
    ctx.close()
    _say("plain solve", it, e)
    return cfg, it, e


def test_nan_state_restarts_from_the_mp2_guess(thc, plain):
    cfg, it_plain, e_plain = plain
    ctx, Z0 = _ctx(thc, cfg)
    Z = Z0.clone()
    Z[3, 5] = float("nan")
    ctx.set_state(Z)
    it, rn, ok = ctx.iterate(tol=1e-9, maxit=60)
    flags = ctx.history_flags()
    _say("nan", it, flags)
    assert ok
    assert [k for k, f in enumerate(flags) if f & thc.ITER_RESTARTED] == [1]
    assert abs(ctx.energy() - e_plain) < 1e-9
    # after the restart the iteration is the plain one from the guess
    assert abs((it - 1) - it_plain) <= 1
    ctx.close()


@pytest.mark.parametrize("factor", [100.0, 1.0e4])
def test_far_start_reaches_the_plain_solution(thc, plain, factor):
    """Starts 100 and 10^4 times the MP2 guess end at the plain solution: by DIIS (whose oldest
    vectors are dropped when the subspace becomes ill-conditioned) or after one restart."""
    cfg, it_plain, e_plain = plain
    ctx, Z0 = _ctx(thc, cfg)
    ctx.set_state(Z0 * factor)
    it, rn, ok = ctx.iterate(tol=1e-9, maxit=60)
    flags = ctx.history_flags()
    _say("times", factor, it, flags)
    assert ok and sum(1 for f in flags if f & thc.ITER_RESTARTED) <= 1
    assert abs(ctx.energy() - e_plain) < 1e-9
    ctx.close()


def test_iteration_limit_then_continue(thc, plain):
    cfg, it_plain, e_plain = plain
    ctx, _ = _ctx(thc, cfg)
    it, rn, ok = ctx.iterate(tol=1e-9, maxit=1, raise_on_notconv=False)
    assert (it, ok) == (1, False)
    with pytest.raises(thc.ThcError, match="THC_ENOTCONV"):
        ctx.iterate(tol=1e-9, maxit=1)
    it, rn, ok = ctx.iterate(tol=1e-9, maxit=60)
    assert ok and abs(ctx.energy() - e_plain) < 1e-9
    ctx.close()


def test_divergence_after_restart_is_reported(thc):
    """With the unscaled Cholesky vectors (gamma = 1: amplitudes of order ten, far past the
    convergence radius) the plain iteration diverges from the MP2 guess, restarts once, diverges
    again, and the call ends with THC_EDIVERGED."""
    cfg = synth.CONFIGS["tiny"]
    ctx, _ = _ctx(thc, cfg, gamma=1.0)
    with pytest.raises(thc.ThcError, match="THC_EDIVERGED"):
        ctx.iterate(tol=1e-9, maxit=60)
    flags = ctx.history_flags()
    _say("unscaled", len(flags), flags)
    assert sum(1 for f in flags if f & thc.ITER_RESTARTED) == 1
    ctx.close()


def test_checkpoint_resumes_the_iteration_exactly(thc, plain):
    """Two iterations, a checkpoint saved to host memory, a fresh context built on the same inputs
    loading it and iterating on: every energy and residual norm equals the uninterrupted solve's,
    bit for bit, and so does the iteration count; a checkpoint from another size is refused."""
    import numpy as np
    cfg, it_plain, e_plain = plain
    a, _ = _ctx(thc, cfg)
    it_a, _, ok = a.iterate(tol=1e-9, maxit=60)
    e_a, r_a, _ = a.history()
    a.close()
    b, _ = _ctx(thc, cfg)
    it_b, _, ok_b = b.iterate(tol=1e-9, maxit=2, raise_on_notconv=False)
    assert (it_b, ok_b) == (2, False)
    e_b, r_b, _ = b.history()
    ck = b.save_checkpoint()
    b.close()
    c, _ = _ctx(thc, cfg)
    c.load_checkpoint(ck)
    it_c, _, ok_c = c.iterate(tol=1e-9, maxit=60)
    e_c, r_c, _ = c.history()
    _say("checkpoint", len(ck), "bytes;", it_a, "=", it_b, "+", it_c)
    assert ok and ok_c and it_a == it_b + it_c
    assert e_b + e_c == e_a and r_b + r_c == r_a
    assert abs(c.energy() - e_plain) < 1e-9
    c.close()
    other = synth.CONFIGS["small"]
    d, _ = _ctx(thc, other)
    with pytest.raises(thc.ThcError, match="THC_EINVAL"):
        d.load_checkpoint(ck)
    with pytest.raises(thc.ThcError, match="THC_EINVAL"):
        d.load_checkpoint(np.zeros(16, dtype=np.uint8))
    d.close()


def test_step_checking_mode_and_iteration_log(thc, plain):
    """THC_FLAG_CHECK (a wait after every device step) changes no result: the solve's history is
    bit for bit the plain one's; the per-iteration log carries the history."""
    import json
    cfg, it_plain, e_plain = plain
    a, _ = _ctx(thc, cfg)
    a.iterate(tol=1e-9, maxit=60)
    ref = a.history()
    a.close()
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=True, tol_energy=1e-10, flags=thc.FLAG_CHECK)
    ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling, 0.0)
    ctx.build_synthetic()
    it, _, ok = ctx.iterate(tol=1e-9, maxit=60)
    got = ctx.history()
    assert ok and got[0] == ref[0] and got[1] == ref[1]
    log = ctx.iteration_log()
    assert [r["iteration"] for r in log] == list(range(1, it + 1))
    assert [r["energy"] for r in log] == got[0] and log[0]["dE"] is None
    assert not any(r["mixed"] or r["restarted"] or r["learned"] for r in log)
    json.dumps(log)
    ctx.close()
