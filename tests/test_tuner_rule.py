"""CPU checks of the tuner's decision rule (meld_tune_choose, a pure host function)."""
import os

import pytest


def _meld():
    import paper_2107_05681_amd as meld
    if not os.path.exists(meld.LIB_PATH):
        from paper_2107_05681_amd import build
        build.build()
    return meld


def test_fastest_wins_without_ties():
    meld = _meld()
    # forms: (lo, hi) = (0,0), (1,0), (0,1), (1,1)
    lo, hi = [0, 1, 0, 1], [0, 0, 1, 1]
    assert meld.tune_choose([4.0, 3.0, 5.0, 6.0], lo, hi, 1.0, 0.0) == 1
    assert meld.tune_choose([4.0, 3.0, 5.0, 2.0], lo, hi, 0.0, 0.0) == 3


def test_probe_breaks_ties_towards_melding_mixed_stages():
    meld = _meld()
    lo, hi = [0, 1, 0, 1], [0, 0, 1, 1]
    t = [1.000, 1.010, 1.005, 1.015]  # all within 2 %
    # low stage mixed, high stage uniform: melded low, divergent high
    assert meld.tune_choose(t, lo, hi, 0.9, 0.0) == 1
    # both uniform: divergent everywhere
    assert meld.tune_choose(t, lo, hi, 0.1, 0.0) == 0
    # both mixed: melded everywhere
    assert meld.tune_choose(t, lo, hi, 0.6, 0.7) == 3
    # outside the tie window timing decides
    assert meld.tune_choose([1.0, 1.5, 1.5, 1.5], lo, hi, 0.9, 0.9) == 0


def test_theta_and_degenerate_inputs():
    meld = _meld()
    lo, hi = [0, 1], [0, 1]
    assert meld.tune_choose([1.0, 1.0], lo, hi, 0.5, 0.5, theta=0.5) == 1
    assert meld.tune_choose([1.0, 1.0], lo, hi, 0.49, 0.49, theta=0.5) == 0
    assert meld.tune_choose([], [], [], 0.0, 0.0) == -1
