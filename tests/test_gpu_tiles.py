"""The LDS tile force kernel against the one-thread-per-particle gather
kernel: same bits for every tile shape, for overfull tiles (gather fallback
inside the tile kernel) and for boxes smaller than a tile.  Forces are sums
of exactly antisymmetric pair forces in 64-bit fixed point, so the result
cannot depend on which kernel, tile or lane evaluates a pair."""
import numpy as np
import pytest

import oracle
from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu


def _run(cells, pos, vel, params, seed, steps, tile=None, reference=False, threads=0):
    p = dpd.make_params(**params, flags=dpd.FLAG_REFERENCE_FORCE if reference else 0)
    b = dpd.Box(cells, len(pos), params=p, seed=seed)
    if tile is not None:
        b.set_tile(tile)
    b.set_force_threads(threads)
    if threads or tile is not None:
        assert b.get_force_threads() == (threads or 512)
    b.set_state(pos, vel)
    b.step(steps)
    out = (b.read(dpd.FORCE), b.read(dpd.POS), b.read(dpd.VEL))
    st = b.stats()
    b.close()
    assert st["nonfinite"] == 0
    return out


P3 = dict(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
P8 = dict(a=10.0, gamma=10.0, kT=1.0, dt=0.005, body_f=0.05)


@pytest.mark.parametrize("cells,rho,params", [((12, 12, 12), 3.0, P3), ((10, 9, 7), 8.0, P8), ((3, 3, 3), 3.0, P3),
                                               ((5, 4, 3), 8.0, P8)])
def test_tiled_equals_reference_one_step(cells, rho, params):
    pos, vel = inputs.uniform_state(cells, density=rho, seed=21)
    ref = _run(cells, pos, vel, params, 21, 1, reference=True)
    til = _run(cells, pos, vel, params, 21, 1)
    np.testing.assert_array_equal(til[0], ref[0])
    # and both match the oracle
    ids = np.arange(len(pos), dtype=np.uint32)
    f, s, _ = oracle.forces(pos, vel, ids, cells, oracle.make_params(**params), 0, 21)
    assert np.all(np.linalg.norm(til[0] - f, axis=1) <= 1e-5 * s)


@pytest.mark.parametrize("tile", [(1, 1, 1), (2, 3, 4), (4, 4, 4), (6, 6, 6), (16, 2, 3), (4, 4, 2), (3, 2, 2),
                                  (5, 3, 2), (8, 3, 3), (1, 4, 4), (7, 1, 3)])
def test_tile_shape_does_not_change_trajectory(tile):
    cells = (12, 10, 9)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=22)
    ref = _run(cells, pos, vel, P3, 22, 20, reference=True)
    til = _run(cells, pos, vel, P3, 22, 20, tile=tile)
    for a, b in zip(til, ref):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("threads", [256, 1024])
@pytest.mark.parametrize("cells,rho,params,tile", [((12, 10, 9), 3.0, P3, (8, 3, 3)), ((12, 10, 9), 3.0, P3, (2, 2, 2)),
                                                    ((9, 7, 6), 8.0, P8, (4, 2, 2)), ((9, 7, 6), 8.0, P8, (6, 4, 4))])
def test_workgroup_size_does_not_change_trajectory(threads, cells, rho, params, tile):
    # 4 or 16 waves share a tile instead of 8: other waves take other home
    # units, the queue region is laid out for the launch's waves
    pos, vel = inputs.uniform_state(cells, density=rho, seed=27)
    ref = _run(cells, pos, vel, params, 27, 8, reference=True)
    til = _run(cells, pos, vel, params, 27, 8, tile=tile, threads=threads)
    for a, b in zip(til, ref):
        np.testing.assert_array_equal(a, b)


def test_workgroup_size_errors():
    b = dpd.Box((6, 6, 6), 648, params=dpd.make_params(), seed=1)
    for bad in (128, 300, 2048, -1):
        with pytest.raises(dpd.DPDError) as e:
            b.set_force_threads(bad)
        assert e.value.code == dpd.EINVAL
    b.close()


@pytest.mark.parametrize("tile", [(4, 2, 2), (3, 3, 3), (5, 2, 3)])
def test_tile_shape_dense_fluid(tile):
    # rho = 8: one-cell home units and candidate lists longer than a wave
    cells = (9, 7, 6)
    pos, vel = inputs.uniform_state(cells, density=8.0, seed=26)
    ref = _run(cells, pos, vel, P8, 26, 5, reference=True)
    til = _run(cells, pos, vel, P8, 26, 5, tile=tile)
    for a, b in zip(til, ref):
        np.testing.assert_array_equal(a, b)


def test_overfull_tiles_fall_back_to_gather():
    cells = (8, 8, 8)
    # a dense clump: cells of 40+ particles overflow the staging buffers
    cp, cv = inputs.clumped_state(cells, 900, centre=(3.5, 3.5, 3.5), radius=1.2, seed=23)
    up, uv = inputs.uniform_state(cells, n=1200, seed=24)
    pos, vel = np.vstack([cp, up]), np.vstack([cv, uv])
    ref = _run(cells, pos, vel, P3, 23, 5, reference=True)
    til = _run(cells, pos, vel, P3, 23, 5)
    for a, b in zip(til, ref):
        np.testing.assert_array_equal(a, b)


def test_large_box_tiled_equals_reference():
    cells = (48, 48, 48)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=25)
    ref = _run(cells, pos, vel, P3, 25, 3, reference=True)
    til = _run(cells, pos, vel, P3, 25, 3)
    for a, b in zip(til, ref):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("cells,n,tile,threads", [
    ((48, 48, 48), 3 * 48 ** 3, (6, 6, 4), 1024),     # large dilute box: the large shape
    ((16, 16, 16), 3 * 16 ** 3, (4, 4, 4), 512),      # small: more, smaller tiles
    ((64, 64, 64), 8 * 64 ** 3, (8, 4, 4), 1024),     # large dense box
    ((12, 10, 9), 8 * 1080, (4, 2, 2), 512),          # small dense box
])
def test_default_tile_follows_density_and_size(cells, n, tile, threads):
    b = dpd.Box(cells, n, params=dpd.make_params(), seed=1)
    assert b.get_tile() == tile and b.get_force_threads() == threads
    b.close()


def test_bad_tile_rejected():
    # (16, 16, 16) would need more LDS than a CU has
    b = dpd.Box((32, 32, 32), 3 * 32 ** 3)
    for t in [(0, 4, 4), (17, 1, 1), (-1, 2, 2), (16, 16, 16)]:
        with pytest.raises(dpd.DPDError) as e:
            b.set_tile(t)
        assert e.value.code == dpd.EINVAL
    b.set_tile((0, 0, 0))
    b.close()
