"""GPU parity of species (per species-pair a and gamma) against the oracle.

Several fluids in one box, each pair of species with its own a and gamma
(Sec. 2.3, Sec. 5.2, Sec. 5.3).  Bars as in the single-species parity tests:
forces within 1e-5 of the oracle's per-particle force scale, the tile kernel
and the reference gather kernel bit-identical, batches bit-identical to
boxes run alone, species read back exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu

TOL_F = 1e-5

A3 = np.array([[25.0, 18.0, 40.0], [18.0, 12.0, 30.0], [40.0, 30.0, 25.0]])
G3 = np.array([[4.5, 0.0, 9.0], [0.0, 22.5, 3.0], [9.0, 3.0, 1.0]])


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _orc_params(p):
    return oracle.make_params(a=p.a, gamma=p.gamma, kT=p.kT, dt=p.dt, mass=p.mass, body_f=p.body_f,
                              flow_axis=p.flow_axis, grad_axis=p.grad_axis, kexp=p.kexp)


def _mixture(cells, rho, seed, fractions, a_tab, g_tab, **kw):
    pos, vel = inputs.uniform_state(cells, density=rho, seed=seed)
    types = inputs.species_types(len(pos), fractions, seed=seed)
    p = dpd.make_params(**kw)
    b = dpd.Box(cells, len(pos), params=p, seed=seed)
    b.set_state(pos, vel)
    b.set_species(a_tab, g_tab)
    b.set_types(types)
    return b, pos, vel, types, p


def _force_check(f_gpu, f_orc, s_orc, label):
    err = np.linalg.norm(f_gpu.astype(np.float64) - f_orc, axis=1)
    worst = np.max(err / np.maximum(s_orc, 1e-300)) if len(err) else 0.0
    _say(f"[{label}] max |df|/S = {worst:.3e}")
    assert np.all(err <= TOL_F * s_orc + 1e-30), (label, worst)


@pytest.mark.parametrize("cells,rho,kexp", [((8, 7, 9), 3.0, 1.0), ((10, 6, 5), 8.0, 1.0), ((7, 7, 7), 4.0, 0.25)])
def test_mixture_forces_match_oracle(cells, rho, kexp):
    b, pos, vel, types, p = _mixture(cells, rho, 41, [0.5, 0.25, 0.25], A3, G3, kexp=kexp, dt=0.005,
                                     flags=dpd.FLAG_VIRIAL)
    b.step(1)
    f = b.read(dpd.FORCE)
    vir = b.stats()["virial"]
    b.close()
    ids = np.arange(len(pos), dtype=np.uint32)
    q = oracle.with_species(_orc_params(p), types, A3, G3)
    fo, so, vo = oracle.forces(pos, vel, ids, cells, q, 0, 41)
    _force_check(f, fo, so, f"mixture {cells} rho={rho} k={kexp}")
    assert vir == pytest.approx(vo, rel=1e-5)
    # the reference gather kernel gives the same bits as the tile kernel
    br, *_ = _mixture(cells, rho, 41, [0.5, 0.25, 0.25], A3, G3, kexp=kexp, dt=0.005,
                      flags=dpd.FLAG_REFERENCE_FORCE)
    br.step(1)
    np.testing.assert_array_equal(br.read(dpd.FORCE), f)
    br.close()


def test_mixture_ten_steps_track_the_oracle():
    cells = (8, 8, 8)
    b, pos, vel, types, p = _mixture(cells, 3.0, 42, [0.5, 0.5], A3[:2, :2], G3[:2, :2], dt=0.01)
    b.step(10)
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    q = oracle.with_species(_orc_params(p), types, A3[:2, :2], G3[:2, :2])
    oracle.step(x, v, np.arange(len(x), dtype=np.uint32), cells, q, 42, 0, 10, want_diag=False)
    dx = np.abs(b.read(dpd.POS) - x)
    dx = np.minimum(dx, 8.0 - dx)
    dv = np.abs(b.read(dpd.VEL) - v)
    _say(f"mixture 10 steps: max |dx| {dx.max():.3e}, max |dv| {dv.max():.3e}")
    assert dx.max() < 1e-3 and dv.max() < 1e-2
    np.testing.assert_array_equal(b.get_types(), types)      # species ride along with the particles
    b.close()


def test_identical_tables_are_the_single_species_bits():
    cells = (9, 8, 7)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=43)
    types = inputs.species_types(len(pos), [0.3, 0.3, 0.4], seed=43)
    p = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    out = []
    for mode in ("params", "one", "three"):
        b = dpd.Box(cells, len(pos), params=p, seed=43)
        b.set_state(pos, vel)
        if mode == "one":
            b.set_species([[25.0]], [[4.5]])
        elif mode == "three":
            b.set_species(np.full((3, 3), 25.0), np.full((3, 3), 4.5))
            b.set_types(types)
        b.step(5)
        out.append((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)))
        b.close()
    for other in out[1:]:
        for x, y in zip(out[0], other):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("tile", [(4, 4, 4), (8, 3, 3), (3, 2, 2), (5, 3, 2)])
def test_species_tiles_change_no_bits(tile):
    cells = (11, 9, 10)
    ref = None
    for t in ((0, 0, 0), tile):
        b, *_ = _mixture(cells, 3.0, 44, [0.4, 0.3, 0.3], A3, G3)
        b.set_tile(t)
        b.step(3)
        got = (b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE))
        b.close()
        if ref is None:
            ref = got
        else:
            for x, y in zip(ref, got):
                np.testing.assert_array_equal(x, y)


def test_batch_of_mixed_boxes_equals_alone():
    specs = [((6, 5, 7), 3.0, 1, True), ((5, 5, 5), 3.0, 2, False), ((7, 4, 6), 8.0, 3, True), ((4, 6, 5), 3.0, 4, False)]

    def make(cells, rho, seed, species):
        pos, vel = inputs.uniform_state(cells, density=rho, seed=seed)
        b = dpd.Box(cells, len(pos), params=dpd.make_params(dt=0.005), seed=seed)
        b.set_state(pos, vel)
        if species:
            b.set_species(A3, G3)
            b.set_types(inputs.species_types(len(pos), [0.3, 0.3, 0.4], seed=seed))
        return b

    alone = []
    for s in specs:
        b = make(*s)
        b.step(7)
        alone.append((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)))
        b.close()
    boxes = [make(*s) for s in specs]
    batch = dpd.Batch(boxes)
    batch.step(7)
    for i, b in enumerate(boxes):
        for x, y in zip((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)), alone[i]):
            np.testing.assert_array_equal(x, y, err_msg=f"box {i}")
    batch.close()
    for b in boxes:
        b.close()


def test_species_equipartition_on_gpu():
    """Each species keeps kT (fluctuation-dissipation per species pair), with
    the plasma / cytoplasm tables: gamma 4.5, 22.5 and 0 across."""
    cells = (16, 16, 16)
    t = inputs.MIXTURE_TABLES
    b, pos, vel, types, p = _mixture(cells, 3.0, 45, t["fractions"], t["a"], t["gamma"], dt=0.005)
    b.step(2000)
    kts = []
    for _ in range(200):
        b.step(10)
        vc = b.read(dpd.VEL_CENTRED).astype(np.float64)
        ke = 0.5 * (vc * vc).sum(axis=1)
        kts.append([2.0 * ke[types == s].sum() / (3.0 * (types == s).sum()) for s in range(2)])
    b.close()
    m = np.mean(kts, axis=0)
    _say(f"species kT {m}")
    # the time-centred estimator keeps a discretisation bias of about 1 % at
    # this dt and gamma (the same for both species; a sigma that ignored the
    # pair's gamma would put them a factor of about 5 apart)
    assert np.all(np.abs(m - 1.0) < 0.02), m
    assert abs(m[0] - m[1]) < 0.005, m


def test_species_errors():
    cells = (5, 5, 5)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=46)
    b = dpd.Box(cells, len(pos), params=dpd.make_params(), seed=46)
    types = inputs.species_types(len(pos), [0.5, 0.5], seed=46)
    with pytest.raises(dpd.DPDError) as e:
        b.set_types(types)                                   # no state
    assert e.value.code == dpd.ESTATE
    b.set_state(pos, vel)
    with pytest.raises(dpd.DPDError) as e:
        b.set_types(types)                                   # no species tables
    assert e.value.code == dpd.ESTATE
    ok = np.full((2, 2), 25.0)
    for a_tab, g_tab in (([[25.0, 20.0], [21.0, 25.0]], [[4.5, 1.0], [1.0, 4.5]]),
                         (ok, [[4.5, -1.0], [-1.0, 4.5]]),
                         (ok, [[4.5, np.inf], [np.inf, 4.5]]),
                         (np.full((9, 9), 25.0), np.full((9, 9), 4.5))):
        with pytest.raises(dpd.DPDError) as e:
            b.set_species(a_tab, g_tab)
        assert e.value.code == dpd.EINVAL
    b.set_species(ok, np.full((2, 2), 4.5))
    assert b.get_species() == 2
    bad = types.copy()
    bad[7] = 2
    with pytest.raises(dpd.DPDError) as e:
        b.set_types(bad)
    assert e.value.code == dpd.EINVAL
    b.set_types(types)
    np.testing.assert_array_equal(b.get_types(), types)
    with pytest.raises(dpd.DPDError) as e:
        b.set_species([[25.0]], [[4.5]])                     # species 1 exists
    assert e.value.code == dpd.EINVAL
    b.set_species()                                          # back to one species from params
    assert b.get_species() == 0
    b.step(2)
    assert b.stats()["nonfinite"] == 0
    b.set_state(pos, vel)                                    # a new state: every particle species 0
    b.set_species([[25.0]], [[4.5]])
    np.testing.assert_array_equal(b.get_types(), np.zeros(len(pos), dtype=np.int32))
    b.close()


RC3 = np.array([[1.0, 0.8, 0.9], [0.8, 0.6, 0.7], [0.9, 0.7, 1.0]])


@pytest.mark.parametrize("cells,rho,kexp", [((8, 7, 9), 3.0, 1.0), ((9, 6, 5), 8.0, 1.0), ((7, 7, 7), 4.0, 0.25)])
def test_pair_cutoffs_match_oracle(cells, rho, kexp):
    # a cutoff per species pair (Sec. 3.1 keeps several): w = 1 - r / r_c
    pos, vel = inputs.uniform_state(cells, density=rho, seed=47)
    types = inputs.species_types(len(pos), [0.4, 0.3, 0.3], seed=47)
    p = dpd.make_params(kexp=kexp, dt=0.005, flags=dpd.FLAG_VIRIAL)
    out = []
    for flags in (dpd.FLAG_VIRIAL, dpd.FLAG_REFERENCE_FORCE):
        p.flags = flags
        b = dpd.Box(cells, len(pos), params=p, seed=47)
        b.set_state(pos, vel)
        b.set_species(A3, G3, RC3)
        b.set_types(types)
        b.step(1)
        out.append((b.read(dpd.FORCE), b.stats()["virial"]))
        b.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])           # tile kernel = gather kernel
    ids = np.arange(len(pos), dtype=np.uint32)
    q = oracle.with_species(_orc_params(p), types, A3, G3, RC3)
    fo, so, vo = oracle.forces(pos, vel, ids, cells, q, 0, 47)
    _force_check(out[0][0], fo, so, f"cutoffs {cells} rho={rho} k={kexp}")
    assert out[0][1] == pytest.approx(vo, rel=1e-5)


def test_unit_cutoffs_are_the_same_bits():
    cells = (9, 8, 7)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=48)
    types = inputs.species_types(len(pos), [0.4, 0.3, 0.3], seed=48)
    out = []
    for rc in (None, np.ones((3, 3))):
        b = dpd.Box(cells, len(pos), params=dpd.make_params(), seed=48)
        b.set_state(pos, vel)
        b.set_species(A3, G3, rc)
        b.set_types(types)
        b.step(4)
        out.append((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)))
        b.close()
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)


def test_one_species_with_its_own_cutoff():
    cells = (8, 8, 8)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=49)
    p = dpd.make_params(a=25.0, gamma=4.5)
    b = dpd.Box(cells, len(pos), params=p, seed=49)
    b.set_state(pos, vel)
    b.set_species([[25.0]], [[4.5]], [[0.75]])
    b.step(1)
    f = b.read(dpd.FORCE)
    b.close()
    ids = np.arange(len(pos), dtype=np.uint32)
    q = _orc_params(p)
    q.rc = 0.75                     # the oracle's one-species cutoff
    fo, so, _ = oracle.forces(pos, vel, ids, cells, q, 0, 49)
    _force_check(f, fo, so, "one species, r_c = 0.75")


def test_cutoff_errors():
    b = dpd.Box((5, 5, 5), 375, params=dpd.make_params(), seed=50)
    a, g = np.full((2, 2), 25.0), np.full((2, 2), 4.5)
    for rc in ([[1.0, 1.2], [1.2, 1.0]], [[1.0, 0.8], [0.7, 1.0]], [[1.0, 0.01], [0.01, 1.0]]):
        with pytest.raises(dpd.DPDError) as e:
            b.set_species(a, g, rc)
        assert e.value.code == dpd.EINVAL
    b.close()
