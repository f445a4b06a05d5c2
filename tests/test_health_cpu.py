"""Pins of the cases behind status bits 4 and 8 (CPU, oracle): with the
planned step count the final state is resolved (neighbouring points a few
1e-3 apart); with half the steps, dt is above the stability radius and the
oracle's final state is grid-scale noise (neighbours more than 0.5 apart)
while every |m| stays 1 and every value finite, which a non-finite check alone
cannot see."""
import numpy as np
import pytest

from health_cases import case
from oracle import micro

ROUGH_MAX = 0.5   # the library's threshold for bit 4


def _final(dim, forced):
    b, coef, init = case(dim, forced)
    r = micro.solve_box(b, coef, init_fn=init, want_state=True)
    mf = r["mfinal"].reshape((3,) + (b["n"],) * dim)
    d = np.sqrt(((mf[..., 1:] - mf[..., :-1]) ** 2).sum(0))   # x1 neighbours
    return r["out"], mf, d


@pytest.mark.parametrize("dim", [1, 2])
def test_planned_steps_leave_a_resolved_state(dim):
    H, mf, d = _final(dim, False)
    assert d.max() < 0.01 and np.isfinite(H).all()


@pytest.mark.parametrize("dim", [1, 2])
def test_forced_steps_leave_finite_grid_scale_noise(dim):
    H, mf, d = _final(dim, True)
    print("dim", dim, "largest neighbour distance", d.max())
    assert np.isfinite(H).all() and np.isfinite(mf).all()
    assert np.abs(np.linalg.norm(mf, axis=0) - 1).max() < 1e-12
    assert d.max() > 2 * ROUGH_MAX
