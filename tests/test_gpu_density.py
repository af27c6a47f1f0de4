"""The MP2 one-particle density of THC amplitudes (paper App. II) by the library's O(N^4)
evaluation (Eq. 51-56) against the dense definition (Eq. 47-48) of the oracle, at the MP2 guess
and at a perturbed core, in one and in several blocks of the outer index."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2111_11473_amd import synth
from test_gpu_parity import _dev, _host, _make, _state

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


@pytest.mark.parametrize("name,a_block", [("small", 0), ("tiny", 0), ("medium", 5), ("occ40", 0), ("wide", 0)])
def test_mp2_density_matches_oracle(thc, name, a_block):
    cfg = synth.CONFIGS[name]
    _say("density", name)
    s, ctx, Z0 = _make(thc, cfg, a_block=a_block)
    for Z in (Z0, _state(s, Z0, 5)[0]):
        Doo, Dvv = ctx.mp2_density(_dev(Z))
        Ro, Rv = oracle.mp2_density(s["Xo"], s["Xv"], Z)
        eo = np.abs(_host(Doo) - Ro).max() / np.abs(Ro).max()
        ev = np.abs(_host(Dvv) - Rv).max() / np.abs(Rv).max()
        _say("  relative errors", eo, ev)
        assert eo < 1e-10 and ev < 1e-10
    # default argument: the current state (the MP2 guess after the set-up)
    Doo, _ = ctx.mp2_density()
    Ro, _ = oracle.mp2_density(s["Xo"], s["Xv"], Z0)
    assert np.abs(_host(Doo) - Ro).max() < 1e-10 * np.abs(Ro).max()
    ctx.close()
