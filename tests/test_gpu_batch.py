"""Batches of independent boxes: every box computes in a batch exactly the
bits it computes alone (same kernels, same per-box work partition; ids,
step counters and seeds are per box), whatever the batch holds."""
import numpy as np
import pytest

from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu


def _make(spec):
    cells, n, seed = spec["cells"], spec["n"], spec["seed"]
    pos, vel = inputs.uniform_state(cells, n=n, seed=seed)
    b = dpd.Box(cells, n, params=dpd.make_params(**spec.get("params", {})), seed=seed)
    b.set_state(pos, vel)
    return b


def _snapshot(b):
    st = b.stats(allow_nonfinite=True)
    out = [b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)]
    if b.params.profile_bins:
        out.extend(b.profile())
    return out, st


def _assert_same(a, b, label):
    (arrs_a, st_a), (arrs_b, st_b) = a, b
    for x, y in zip(arrs_a, arrs_b):
        np.testing.assert_array_equal(x, y, err_msg=label)
    for k in ("ke_half", "ke_centred", "kT_centred", "pressure", "sum_kT_centred", "step", "nsamples"):
        assert st_a[k] == st_b[k], (label, k, st_a[k], st_b[k])
    np.testing.assert_array_equal(st_a["momentum"], st_b["momentum"])


SPECS = [b for b in inputs.batch_boxes(nboxes=10, lo=3, hi=14, density=3.0, rng_seed=40)]


def test_batch_equals_alone_uneven_boxes():
    steps = 23
    alone = []
    for s in SPECS:
        b = _make(s)
        b.step(steps)
        alone.append(_snapshot(b))
        b.close()
    boxes = [_make(s) for s in SPECS]
    batch = dpd.Batch(boxes)
    batch.step(steps)
    for i, (b, ref) in enumerate(zip(boxes, alone)):
        _assert_same(_snapshot(b), ref, f"box {i} {SPECS[i]['cells']}")
    batch.close()
    for b in boxes:
        b.close()


def test_batch_mixed_parameters_and_flags():
    specs = [
        {"cells": (6, 5, 4), "n": 360, "seed": 1, "params": dict(a=25.0, gamma=4.5, dt=0.01)},
        {"cells": (5, 5, 5), "n": 1000, "seed": 2,
         "params": dict(a=10.0, gamma=10.0, dt=0.005, body_f=0.05, profile_bins=5)},
        {"cells": (3, 4, 3), "n": 100, "seed": 3, "params": dict(a=25.0, gamma=4.5, dt=0.01, flags=dpd.FLAG_VIRIAL)},
        {"cells": (7, 3, 5), "n": 315, "seed": 4,
         "params": dict(a=18.75, gamma=4.5, dt=0.005, flags=dpd.FLAG_REFERENCE_FORCE)},
        {"cells": (4, 4, 4), "n": 0, "seed": 5, "params": dict()},
        {"cells": (3, 3, 3), "n": 1, "seed": 6, "params": dict(body_f=0.3)},
    ]
    steps = 40
    alone = []
    for s in specs:
        b = _make(s)
        b.step(steps)
        alone.append(_snapshot(b))
        b.close()
    boxes = [_make(s) for s in specs]
    batch = dpd.Batch(boxes)
    batch.step(17)          # one graph of 17 steps ...
    batch.step(23)          # ... then another shape: captured again
    for i, (b, ref) in enumerate(zip(boxes, alone)):
        _assert_same(_snapshot(b), ref, f"mixed box {i}")
    # boxes keep working alone after the batch
    boxes[0].step(3)
    assert boxes[0].stats()["step"] == steps + 3
    batch.close()
    for b in boxes:
        b.close()


def test_batch_errors():
    b1 = dpd.Box((4, 4, 4), 50, params=dpd.make_params(), seed=1)
    with pytest.raises(dpd.DPDError) as e:
        dpd.Batch([b1, b1])
    assert e.value.code == dpd.EINVAL
    batch = dpd.Batch([b1])
    with pytest.raises(dpd.DPDError) as e:
        batch.step(1)                       # no state yet
    assert e.value.code == dpd.ESTATE
    pos, vel = inputs.uniform_state((4, 4, 4), n=50, seed=1)
    b1.set_state(pos, vel)
    b2 = dpd.Box((5, 4, 4), 60, params=dpd.make_params(), seed=2)
    b2.set_state(*inputs.uniform_state((5, 4, 4), n=60, seed=2))
    pair = dpd.Batch([b1, b2])
    b1.build_cells()
    with pytest.raises(dpd.DPDError) as e:
        pair.step(1)                        # one box holds a bare cell list, the other not
    assert e.value.code == dpd.ESTATE
    batch.step(1)                           # every box of this batch does: it starts from the lists
    b1.step(1)
    batch.step(2)
    assert b1.stats()["step"] == 4
    pair.close()
    batch.close()
    b1.close()
    b2.close()


def test_batch_tuner_changes_no_bits():
    cells = [(9, 8, 8), (16, 12, 10), (6, 6, 6), (24, 9, 11)]
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    states = [inputs.uniform_state(c, density=3.0, seed=60 + k) for k, c in enumerate(cells)]
    alone = []
    for k, (c, (p, v)) in enumerate(zip(cells, states)):
        b = dpd.Box(c, len(p), params=params, seed=60 + k)
        b.set_state(p, v)
        b.step(9)
        alone.append((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)))
        b.close()
    boxes = []
    for k, (c, (p, v)) in enumerate(zip(cells, states)):
        b = dpd.Box(c, len(p), params=params, seed=60 + k)
        b.set_state(p, v)
        boxes.append(b)
    batch = dpd.Batch(boxes)
    batch.step(4)
    tile, ms = batch.tune(reps=2)
    assert ms > 0
    if tile is not None:
        assert all(b.get_tile() == tuple(min(t, c) for t, c in zip(tile, b_cells))
                   for b, b_cells in zip(boxes, cells))
    batch.step(5)
    for b, ref in zip(boxes, alone):
        assert b.stats()["step"] == 9
        np.testing.assert_array_equal(b.read(dpd.POS), ref[0])
        np.testing.assert_array_equal(b.read(dpd.VEL), ref[1])
        np.testing.assert_array_equal(b.read(dpd.FORCE), ref[2])
    batch.close()
    for b in boxes:
        b.close()


def test_autotuner_picks_a_tile_and_changes_no_bits():
    cells = (20, 16, 12)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=41)
    ref = dpd.Box(cells, len(pos), params=dpd.make_params(), seed=41)
    ref.set_state(pos, vel)
    ref.step(12)
    tuned = dpd.Box(cells, len(pos), params=dpd.make_params(), seed=41)
    tuned.set_state(pos, vel)
    tuned.step(5)
    tile, ms = tuned.tune_tile(reps=3)
    assert all(1 <= t <= 16 for t in tile) and ms > 0
    assert tuned.get_tile() == tile
    tuned.step(7)
    for what in (dpd.POS, dpd.VEL, dpd.FORCE):
        np.testing.assert_array_equal(tuned.read(what), ref.read(what))
    ref.close()
    tuned.close()


def test_batch_of_boxes_with_other_workgroup_sizes_equals_alone():
    # a batch launches with its first box's workgroup size; boxes tuned for
    # another size are laid out for it in the batch's copy of their descriptors
    cells = [(9, 8, 8), (12, 10, 7), (7, 6, 9)]
    threads = [256, 1024, 512]
    states = [inputs.uniform_state(c, density=3.0, seed=70 + k) for k, c in enumerate(cells)]
    alone = []
    for k, (c, (p, v)) in enumerate(zip(cells, states)):
        b = dpd.Box(c, len(p), params=dpd.make_params(), seed=70 + k)
        b.set_state(p, v)
        b.step(6)
        alone.append((b.read(dpd.POS), b.read(dpd.VEL)))
        b.close()
    boxes = []
    for k, (c, (p, v)) in enumerate(zip(cells, states)):
        b = dpd.Box(c, len(p), params=dpd.make_params(), seed=70 + k)
        b.set_force_threads(threads[k])
        b.set_state(p, v)
        boxes.append(b)
    batch = dpd.Batch(boxes)
    batch.step(6)
    for b, ref in zip(boxes, alone):
        np.testing.assert_array_equal(b.read(dpd.POS), ref[0])
        np.testing.assert_array_equal(b.read(dpd.VEL), ref[1])
    assert [b.get_force_threads() for b in boxes] == threads      # the boxes keep their own setting
    batch.close()
    for b in boxes:
        b.close()
