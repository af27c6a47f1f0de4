"""Host-side pieces of the learned-guess study (paper_2111_11473_amd/learned.py), on the CPU: the
time-to-target measure and the system recipe."""
import pytest

pytest.importorskip("torch")

from paper_2111_11473_amd import learned, synth


def test_to_target_counts_until_the_energy_stays_within_the_threshold():
    e_ref = -1.0
    secs = [0.1, 0.2, 0.3, 0.4, 0.5]
    # falls into the window at the third iteration and stays
    assert learned._to_target([-0.9, -0.99, -1.0000005, -0.9999999, -1.0], secs, e_ref) == (3, 0.3)
    # enters, leaves, re-enters: counted from the last entry
    assert learned._to_target([-1.0, -0.9, -1.0, -1.0, -1.0], secs, e_ref) == (3, 0.3)
    # within from the first iteration
    assert learned._to_target([-1.0] * 5, secs, e_ref) == (1, 0.1)
    # never settles (the last one is outside)
    assert learned._to_target([-1.0, -1.0, -0.5], secs[:3], e_ref) == (None, None)
    # the threshold is strict and configurable
    assert learned._to_target([-0.9, -1.001], secs[:2], e_ref, thresh=1e-2) == (2, 0.2)


def test_study_systems_are_the_learned_set():
    for s in range(256):
        a, b = learned.system_config(s, 30, 80), synth.learned_config(s)
        assert (a.o, a.v, a.nL, a.nP, a.nQ, a.seed) == (b.o, b.v, b.nL, b.nP, b.nQ, b.seed)
    small = [learned.system_config(s, 10, 24).o for s in range(200)]
    assert min(small) == 10 and max(small) == 24
