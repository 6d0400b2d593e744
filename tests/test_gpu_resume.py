"""Checkpoint and resume: a run stopped after k steps, read back (positions,
velocities v^{n-1/2}, species, frozen marks) and loaded into a new box with
the step counter set to k continues bit for bit as the uninterrupted run.
The random term is a pure function of (ids, step, seed) and forces are
order-independent fixed-point sums, so the internal order the new box
builds does not matter."""
import numpy as np
import pytest

from paper_1911_04712_amd import dpd, inputs, walls

pytestmark = pytest.mark.gpu


def _snap(b):
    return b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)


@pytest.mark.parametrize("kind", ["plain", "species", "walls"])
def test_resume_continues_bit_for_bit(kind):
    cells = (9, 10, 8) if kind != "walls" else (6, 14, 14)
    if kind == "walls":
        p = dpd.make_params(dt=0.01, wall_kind=dpd.WALL_CYLINDERS, wall_h=5.5, wall_r_in=2.5, omega_out=0.2)
        pos, vel, frozen = walls.carve(cells, 3.0, dpd.make_params(dt=0.01), dpd.WALL_CYLINDERS, 5.5, seed=80,
                                       equil_steps=100, wall_r_in=2.5)
    else:
        p = dpd.make_params(dt=0.01, body_f=0.05, profile_bins=10)
        pos, vel = inputs.uniform_state(cells, density=3.0, seed=80)
        frozen = None
    types = inputs.species_types(len(pos), [0.5, 0.5], seed=80) if kind == "species" else None
    tabs = ([[25.0, 30.0], [30.0, 25.0]], [[4.5, 9.0], [9.0, 4.5]], [[1.0, 0.8], [0.8, 1.0]])

    def fresh(x, v):
        b = dpd.Box(cells, len(pos), params=p, seed=80)
        b.set_state(x, v)
        if types is not None:
            b.set_species(*tabs)
            b.set_types(types)
        if frozen is not None:
            b.set_frozen(frozen)
        return b

    a = fresh(pos, vel)
    a.step(25)
    ref = _snap(a)
    a.close()
    b = fresh(pos, vel)
    b.step(11)
    x, v = b.read(dpd.POS), b.read(dpd.VEL)
    b.close()
    c = fresh(x, v)
    c.set_step(11)
    c.step(14)
    got = _snap(c)
    assert c.stats()["step"] == 25
    c.close()
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(r, g)


def test_set_step_needs_a_state():
    b = dpd.Box((4, 4, 4), 10, params=dpd.make_params(), seed=1)
    with pytest.raises(dpd.DPDError) as e:
        b.set_step(3)
    assert e.value.code == dpd.ESTATE
    b.close()
