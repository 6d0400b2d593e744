"""dpd_run_static (the box in the library's static per-GPU array, no
device allocation by the library) against the workspace path it mirrors:
dpd_create + set_params + set_seed + set_state + set_step + step + read +
get_stats.  Both run the same kernels, so positions, velocities and the
FP64 diagnostics agree bit for bit.  Two calls in a row, the second on a
smaller box, then the first again: the array keeps the last call's
contents, and each call clears what must start at zero."""
import numpy as np
import pytest

from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu

STAT_KEYS = ("momentum", "ke_half", "ke_centred", "kT_centred", "sum_kT_centred", "sum_momentum", "nsamples", "step",
             "nonfinite", "escaped")


def _workspace_run(cells, pos, vel, params, seed, step0, nsteps):
    with dpd.Box(cells, len(pos), params=params, seed=seed) as b:
        b.set_state(pos, vel)
        if step0:
            b.set_step(step0)
        b.step(nsteps)
        return b.read(dpd.POS), b.read(dpd.VEL), b.stats()


def _static_run(cells, pos, vel, params, seed, step0, nsteps):
    po, vo, st = dpd.run_static(cells, pos, vel, params, seed, nsteps, step0=step0)
    return po.cpu().numpy(), vo.cpu().numpy(), st


def _same(a, b):
    pa, va, sa = a
    pb, vb, sb = b
    assert np.array_equal(pa, pb)
    assert np.array_equal(va, vb)
    for k in STAT_KEYS:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k


CASES = [
    # cells, density, seed, step0, steps, params
    ((16, 16, 16), 3.0, 11, 0, 70, dict(a=25.0, gamma=4.5, kT=1.0, dt=0.01)),
    ((8, 9, 10), 8.0, 12, 5, 7, dict(a=10.0, gamma=10.0, kT=1.0, dt=0.005, body_f=0.05, profile_bins=9)),
]


def test_static_run_equals_workspace_run_twice_in_a_row():
    runs = []
    for cells, rho, seed, step0, steps, kw in CASES:
        print(f"run_static case cells={cells} rho={rho} steps={steps}", flush=True)
        pos, vel = inputs.uniform_state(cells, density=rho, seed=seed)
        p = dpd.make_params(**kw)
        got = _static_run(cells, pos, vel, p, seed, step0, steps)
        _same(got, _workspace_run(cells, pos, vel, p, seed, step0, steps))
        assert got[2]["step"] == step0 + steps
        runs.append((cells, pos, vel, p, seed, step0, steps, got))
    # the first case again, after the smaller one has used the array
    cells, pos, vel, p, seed, step0, steps, first = runs[0]
    _same(_static_run(cells, pos, vel, p, seed, step0, steps), first)


def test_static_run_with_walls_equals_workspace_run():
    # a pipe's fluid without its frozen layer: the walls' bounce-back runs in
    # the force kernel's write-out on both paths
    from paper_1911_04712_amd import walls
    cells, R, seed = (6, 11, 12), 4.0, 13
    pos, vel, frozen = walls.carve(cells, 3.0, dpd.make_params(dt=0.01), dpd.WALL_PIPE, R, seed=seed,
                                   equil_steps=50)
    pos, vel = pos[~frozen], vel[~frozen]
    p = dpd.make_params(wall_kind=dpd.WALL_PIPE, wall_h=R, flags=dpd.FLAG_BODY_UNIFORM, body_f=0.2, dt=0.01,
                        profile_bins=6)
    print(f"run_static walls case cells={cells} n={len(pos)}", flush=True)
    got = _static_run(cells, pos, vel, p, seed, 0, 12)
    _same(got, _workspace_run(cells, pos, vel, p, seed, 0, 12))


def test_static_run_of_zero_steps_returns_the_grid_rounded_state():
    cells = (5, 6, 7)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=3)
    p = dpd.make_params()
    got = _static_run(cells, pos, vel, p, 3, 0, 0)
    _same(got, _workspace_run(cells, pos, vel, p, 3, 0, 0))


def test_static_run_rejects_a_box_beyond_the_array():
    cells = (48, 48, 48)
    pos = np.zeros((884736, 3), np.float32)
    with pytest.raises(dpd.DPDError) as e:
        dpd.run_static(cells, pos, pos, dpd.make_params(), 1, 1)
    assert e.value.code == dpd.ENOMEM
