"""Per-stage timing (dpd_profile_steps): each stage is timed by events that
its first kernel records as it starts and its last as it ends, so a stage
that does not run reads zero and the stages of one step add up to less than
the step's wall time between two host synchronisations."""
import time

import numpy as np
import pytest

from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu


def _box(cells, rho, **kw):
    pos, vel = inputs.uniform_state(cells, density=rho, seed=31)
    b = dpd.Box(cells, len(pos), params=dpd.make_params(**kw), seed=31)
    b.set_state(pos, vel)
    return b


def test_stage_times_of_the_fused_step():
    b = _box((16, 16, 16), 3.0)
    b.step(3)
    t0 = time.perf_counter()
    st = b.profile_steps(5)
    wall_ms = (time.perf_counter() - t0) * 1e3 / 5
    assert st["bin"] > 0.0 and st["force"] > 0.0
    assert st["virial"] == 0.0 and st["integrate"] == 0.0     # no virial; kick-drift fused
    assert st["bin"] + st["force"] < wall_ms
    assert b.stats()["step"] == 8
    b.close()


def test_stage_times_with_virial_and_the_separate_integrate():
    # the reference force path runs the integrate kernel on its own
    b = _box((12, 10, 9), 3.0, flags=dpd.FLAG_VIRIAL | dpd.FLAG_REFERENCE_FORCE)
    st = b.profile_steps(4)
    assert st["virial"] > 0.0 and st["integrate"] > 0.0 and st["force"] > 0.0 and st["bin"] > 0.0
    assert np.isfinite(b.stats()["virial"])
    b.close()
