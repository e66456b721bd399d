"""The device integrator's choice of fixed-tree intervals (host logic of
paper_1609_08621_amd/kdk.py) against the oracle's rule (oracle/kdk.py),
on random rung distributions.  CPU only."""
import types

import numpy as np
import pytest

from oracle import kdk

torch = pytest.importorskip("torch")


def _integrator(rung, R, dual_below):
    from paper_1609_08621_amd.kdk import Integrator
    it = object.__new__(Integrator)  # the schedule only: no device state
    it.torch = torch
    it.R, it.n, it.dual_below, it.dual_mode = R, rung.size, dual_below, "fixed"
    it.store = types.SimpleNamespace(rung=torch.from_numpy(rung.astype(np.int32)))
    return it


@pytest.mark.parametrize("R", [2, 3, 4, 5])
def test_fixed_rung_choice_matches_the_oracle(R):
    rng = np.random.default_rng(R)
    opened = 0
    for trial in range(40):
        # a bulk on shallow rungs and a thin tail, of varying weight
        n = int(rng.integers(50, 400))
        p = rng.dirichlet(np.r_[np.full(R - 1, 5.0), 0.3, 0.1][:R + 1])
        rung = rng.choice(R + 1, size=n, p=p)
        it = _integrator(rung, R, 0.05)
        for k in range(1 << R):
            r = kdk.fixed_rung(rung, k, R, 0.05)
            assert it._fixed_rung(k) == r, (R, trial, k)
            opened += r is not None
    assert opened > 0  # the draws open intervals
    # "rebuild" mode never opens an interval
    it = _integrator(np.array([0] * 99 + [R]), R, 0.05)
    it.dual_mode = "rebuild"
    assert it._fixed_rung(0) is None
