"""Host logic of the gradient (no GPU): how WaveProp keeps the forward states."""

import numpy as np
import pytest

from paper_1410_1387_amd.autograd import GradientProblem, keeps_all_states


def _problem(**kw):
    base = dict(r=4, h=10.0, dt=1e-3, nsteps=2000, source=(1, 1, 1), receivers=np.zeros((1, 3), dtype=np.int64))
    base.update(kw)
    return GradientProblem(**base)


def test_explicit_modes_are_obeyed():
    # "all" keeps every state and "checkpoint" never does, whatever the memory (the device
    # is not consulted for them, so this runs without a GPU)
    assert keeps_all_states(_problem(states="all"), 1 << 40, None)
    assert not keeps_all_states(_problem(states="checkpoint"), 1, None)


def test_unknown_mode_rejected():
    with pytest.raises(ValueError):
        keeps_all_states(_problem(states="everything"), 1, None)


def test_default_is_auto():
    assert GradientProblem(r=4, h=10.0, dt=1e-3, nsteps=10, source=(0, 0, 0),
                           receivers=np.zeros((1, 3))).states == "auto"
