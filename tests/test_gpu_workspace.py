"""A context whose device working memory is the caller's workspace (thc_create_with_workspace):
the library allocates no device memory, and the blocking its planner picks for a tight budget
(several H blocks, several grid-point chunks, Alg. 7 row chunks) gives the oracle's residual."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2111_11473_amd import synth
from test_gpu_parity import _check_terms, _dev, _host, _state

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


def _tight_plan(thc, cfg):
    """The smallest budget (in 2% steps down from a generous one) whose plan still fits, and
    that plan: it has to split H, the grid and Alg. 7."""
    big = thc.plan_query(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, 1e12)
    budget, plan = big["device_bytes"], big
    while True:
        try:
            p = thc.plan_query(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, int(budget * 0.98))
        except thc.ThcError:
            return plan
        budget, plan = budget * 0.98, p


def _device_taken():
    """Device bytes in use by anyone but torch's caching allocator (that is, by the library)."""
    free, total = torch.cuda.mem_get_info()
    return total - free - torch.cuda.memory_reserved()


def test_workspace_context_allocates_nothing_and_matches_oracle(thc):
    cfg = synth.CONFIGS["medium"]
    plan = _tight_plan(thc, cfg)
    _say("tight plan", plan)
    assert plan["x_blocks"] >= 2 and plan["i_chunks"] >= 2 and plan["x7_chunks"] >= 2
    s = synth.make_system(cfg)
    inputs = [_dev(s[k]) for k in ("L", "eps", "Xo", "Xv", "xo", "xv")]
    ws = torch.empty(plan["device_bytes"], dtype=torch.uint8, device="cuda")
    # one ordinary context first: the runtime loads the library's code object on its first launch
    warm = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ)
    warm.residual(warm.build_factors(*inputs))
    warm.close()
    torch.cuda.synchronize()
    taken0 = _device_taken()
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, workspace=ws)
    Z0 = ctx.build_factors(*inputs)
    torch.cuda.synchronize()
    assert ctx.plan()["device_bytes"] <= plan["device_bytes"]
    assert {k: ctx.plan()[k] for k in ("x_block", "i_chunk", "x7_chunk")} == \
        {k: plan[k] for k in ("x_block", "i_chunk", "x7_chunk")}
    Z, t1 = _state(s, _host(Z0), 4)
    Zd, t1d = _dev(Z), _dev(t1)
    ctx.residual(Zd, t1d)
    torch.cuda.synchronize()
    # neither the build nor the residual took device memory outside the workspace
    assert _device_taken() == taken0, (_device_taken(), taken0)
    _check_terms(thc, cfg, s, ctx, _host(Z0))
    ctx.close()


def test_workspace_too_small_is_refused(thc):
    cfg = synth.CONFIGS["small"]
    s = synth.make_system(cfg)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, workspace=ws)
    with pytest.raises(thc.ThcError, match="THC_ENOMEM"):
        ctx.build_factors(*[_dev(s[k]) for k in ("L", "eps", "Xo", "Xv", "xo", "xv")])
    ctx.close()
