"""GPU parity: the HIP path through the C-ABI against the CPU oracle on the
same seeded inputs.

Bars (written at each test):
  - integer work (cell lists, Philox words, ids): bit-exact;
  - forces after one step: |f_gpu - f_orc| <= 1e-5 * S_i per particle, with
    S_i the oracle's sum of the magnitudes of all force terms on i;
  - one-step state: |dv| <= dt * 1e-5 * S_i + 4 ulp(v), |dx| <= 2 q + dt |dv|
    (q the position grid);
  - statistics over long runs within three combined standard errors.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu

TOL_F = 1e-5


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _box(cells, pos, vel, params, seed):
    b = dpd.Box(cells, len(pos), params=params, seed=seed)
    b.set_state(pos, vel)
    return b


def _orc_params(p):
    return oracle.make_params(a=p.a, gamma=p.gamma, kT=p.kT, dt=p.dt, mass=p.mass, body_f=p.body_f,
                              flow_axis=p.flow_axis, grad_axis=p.grad_axis, kexp=p.kexp)


def _force_check(f_gpu, f_orc, s_orc, label):
    err = np.linalg.norm(f_gpu.astype(np.float64) - f_orc, axis=1)
    worst = np.max(err / np.maximum(s_orc, 1e-300)) if len(err) else 0.0
    _say(f"[{label}] max |df|/S = {worst:.3e}")
    assert np.all(err <= TOL_F * s_orc + 1e-30), (label, worst)
    return worst


# ---------------------------------------------------------------------------
# random term
# ---------------------------------------------------------------------------

def test_philox_words_bit_exact():
    rng = np.random.default_rng(100)
    n = 200_000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[:, 3][: n // 2] = 0
    got = dpd.philox(ctr, key)
    ref = np.vstack([oracle.philox4x32_10(ctr[k:k + 1], key[k]) for k in range(0, 2000)])
    np.testing.assert_array_equal(got[:2000], ref)
    # bulk: same key for a batch so the oracle call is vectorised
    key1 = np.tile(key[0], (n, 1))
    np.testing.assert_array_equal(dpd.philox(ctr, key1), oracle.philox4x32_10(ctr, key[0]))


def test_box_muller_exhaustive_24bit_maps():
    """All 2^24 values of each uniform: u1 with u2 = 0 (cos = 1), and u2 with
    u1 = 1/2 (radius sqrt(2 ln 2)).  FP32 GPU vs FP64 oracle."""
    k = np.arange(1 << 24, dtype=np.uint32) << 8
    zeros = np.zeros_like(k)
    half = np.full_like(k, ((1 << 23) - 1) << 8)
    g1 = dpd.box_muller(k, zeros).astype(np.float64)
    r1 = oracle.box_muller_batch(k, zeros)
    g2 = dpd.box_muller(half, k).astype(np.float64)
    r2 = oracle.box_muller_batch(half, k)
    e1, e2 = np.abs(g1 - r1), np.abs(g2 - r2)
    rel1 = e1 / np.maximum(np.abs(r1), 1e-30)
    _say(f"radius map: max abs err {e1.max():.3e}, max rel err {rel1[r1 > 1e-3].max():.3e}; "
         f"cos map: max abs err {e2.max():.3e}")
    assert e1.max() < 4e-6 and e2.max() < 4e-6


# ---------------------------------------------------------------------------
# cell lists: bit-exact against the oracle's stable counting sort
# ---------------------------------------------------------------------------

def _check_cells(cells, pos, label):
    vel = np.zeros_like(pos)
    b = dpd.Box(cells, len(pos), params=dpd.make_params(), seed=0)
    b.set_state(pos, vel)
    b.build_cells()
    p4, v4, cs = b.read_raw()
    order, start = oracle.bin_cells(pos, cells)
    np.testing.assert_array_equal(cs, start, err_msg=label)
    ids = p4[:, 3].view(np.int32)
    np.testing.assert_array_equal(ids, order.astype(np.int32), err_msg=label)
    np.testing.assert_array_equal(p4[:, :3], pos[order], err_msg=label)
    b.close()


@pytest.mark.parametrize("cells,n,seed", [((8, 8, 8), 1536, 0), ((3, 3, 3), 81, 1), ((5, 7, 3), 400, 2),
                                          ((48, 48, 48), 331776, 3), ((3, 3, 3), 1, 4), ((4, 4, 4), 0, 5)])
def test_cell_list_bit_exact_uniform(cells, n, seed):
    pos, _ = inputs.uniform_state(cells, n=n, seed=seed)
    _check_cells(cells, pos, f"uniform {cells} n={n}")


@pytest.mark.parametrize("cells,n,seed", [((6, 5, 4), 700, 6), ((9, 9, 9), 4000, 7)])
def test_cell_list_bit_exact_faces(cells, n, seed):
    pos, _ = inputs.face_state(cells, n, seed=seed)
    _check_cells(cells, pos, f"faces {cells}")


def test_cell_list_bit_exact_clumped():
    pos, _ = inputs.clumped_state((8, 8, 8), 600, centre=(4.0, 4.0, 4.0), radius=0.9, seed=8)
    _check_cells((8, 8, 8), pos, "clumped")


def test_cell_list_stays_stable_while_stepping():
    """Over 30 steps each cell list is valid and keeps, inside every cell, the
    order the particles had after the previous step."""
    cells = (6, 6, 6)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=9)
    b = _box(cells, pos, vel, dpd.make_params(), 9)
    b.step(1)
    prev_ids = b.read_raw()[0][:, 3].view(np.int32).copy()
    for _ in range(30):
        b.step(1)
        p4, _, cs = b.read_raw()
        ids = p4[:, 3].view(np.int32)
        where = np.empty(len(ids), dtype=np.int64)
        where[prev_ids] = np.arange(len(ids))
        c = np.floor(p4[:, :3].astype(np.float64)).astype(np.int64)
        key = c[:, 0] + 6 * (c[:, 1] + 6 * c[:, 2])
        assert np.all(np.diff(key) >= 0)
        assert np.all(np.diff(cs) >= 0) and cs[-1] == len(ids)
        for k in range(216):
            seg = ids[cs[k]:cs[k + 1]]
            assert np.all(key[cs[k]:cs[k + 1]] == k)
            assert np.all(np.diff(where[seg]) > 0)
        prev_ids = ids.copy()


def test_cell_list_dilute_ragged_box_while_stepping():
    """A dilute box whose cell count is not a multiple of the 64-cell
    counters and has more counters than particles: after every step the
    cell list equals the oracle's stable sort of the new positions taken in
    the previous step's order, bit for bit."""
    cells = (37, 29, 23)                     # 24 679 cells, 386 counters, 200 particles
    pos, vel = inputs.uniform_state(cells, n=200, kT=25.0, seed=13)
    b = _box(cells, pos, vel, dpd.make_params(a=0.0, gamma=0.5, kT=25.0, dt=0.05), 13)
    b.build_cells()
    prev_ids = b.read_raw()[0][:, 3].view(np.int32).copy()
    moved = 0
    for step in range(12):
        b.step(1)
        p4, _, cs = b.read_raw()
        ids = p4[:, 3].view(np.int32)
        by_id = np.empty((len(ids), 3), np.float32)
        by_id[ids] = p4[:, :3]
        order, start = oracle.bin_cells(by_id[prev_ids], cells)
        np.testing.assert_array_equal(cs, start, err_msg=f"step {step}")
        np.testing.assert_array_equal(ids, prev_ids[order], err_msg=f"step {step}")
        moved += int(np.any(ids != prev_ids))
        prev_ids = ids.copy()
    assert b.stats()["escaped"] == 0
    assert moved > 0                          # the order did change along the way
    b.close()


# ---------------------------------------------------------------------------
# forces and one step
# ---------------------------------------------------------------------------

CASES = {
    "cube8_rho3": dict(cells=(8, 8, 8), rho=3.0, p=dict(a=25.0, gamma=4.5, kT=1.0, dt=0.01), seed=0),
    "ragged_5x7x3": dict(cells=(5, 7, 3), rho=3.0, p=dict(a=25.0, gamma=4.5, kT=1.0, dt=0.01), seed=11),
    "rho8_poiseuille": dict(cells=(12, 10, 8), rho=8.0,
                            p=dict(a=10.0, gamma=10.0, kT=1.0, dt=0.005, body_f=0.05, profile_bins=10), seed=2),
    "cube3_rho8": dict(cells=(3, 3, 3), rho=8.0, p=dict(a=25.0, gamma=4.5, kT=1.0, dt=0.01), seed=12),
}


@pytest.mark.parametrize("name", list(CASES))
def test_forces_one_step(name):
    c = CASES[name]
    pos, vel = inputs.uniform_state(c["cells"], density=c["rho"], seed=c["seed"])
    params = dpd.make_params(**c["p"])
    b = _box(c["cells"], pos, vel, params, c["seed"])
    b.step(1)
    f_gpu = b.read(dpd.FORCE)
    ids = np.arange(len(pos), dtype=np.uint32)
    f_orc, s_orc, _ = oracle.forces(pos, vel, ids, c["cells"], _orc_params(params), step=0, seed=c["seed"])
    _force_check(f_gpu, f_orc, s_orc, name)


def test_forces_clumped_cells():
    cells = (8, 8, 8)
    pos, vel = inputs.clumped_state(cells, 500, centre=(0.2, 7.9, 4.0), radius=0.8, seed=13)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    b = _box(cells, pos, vel, params, 13)
    b.step(1)
    ids = np.arange(len(pos), dtype=np.uint32)
    f_orc, s_orc, _ = oracle.forces(pos, vel, ids, cells, _orc_params(params), 0, 13)
    _force_check(b.read(dpd.FORCE), f_orc, s_orc, "clumped")


def test_one_step_state_and_stats():
    cells = (8, 8, 8)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=0)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, profile_bins=8, body_f=0.02)
    b = _box(cells, pos, vel, params, 0)
    b.step(1)
    x = pos.astype(np.float64).copy()
    v = vel.astype(np.float64).copy()
    ids = np.arange(len(pos), dtype=np.uint32)
    diag, ps, pc, f_orc = oracle.step(x, v, ids, cells, _orc_params(params), 0, 0, 1, nbins=8)
    _, s_orc, _ = oracle.forces(pos, vel, ids, cells, _orc_params(params), 0, 0)
    vg, xg = b.read(dpd.VEL).astype(np.float64), b.read(dpd.POS).astype(np.float64)
    q = dpd.position_grid(cells)
    dv = np.abs(vg - v)
    tol_v = 0.01 * TOL_F * s_orc[:, None] + 4 * np.spacing(np.abs(v).astype(np.float32)).astype(np.float64)
    assert np.all(dv <= tol_v)
    dx = np.abs(xg - x)
    dx = np.minimum(dx, 8.0 - dx)                      # periodic
    assert np.all(dx <= 2 * q + 0.01 * dv + 1e-12)
    vc_gpu = b.read(dpd.VEL_CENTRED).astype(np.float64)
    vc_orc = vel.astype(np.float64) + 0.5 * 0.01 * f_orc
    assert np.all(np.abs(vc_gpu - vc_orc) <= 0.5 * tol_v + 4 * np.spacing(np.float32(8.0)))
    st = b.stats()
    assert st["step"] == 1 and st["nsamples"] == 1 and st["nonfinite"] == 0
    np.testing.assert_allclose(st["momentum"], diag["momentum"][0], rtol=0, atol=1e-4)
    assert st["ke_half"] == pytest.approx(diag["ke_half"][0], rel=1e-6)
    assert st["ke_centred"] == pytest.approx(diag["ke_centred"][0], rel=1e-6)
    sv, cn = b.profile()
    np.testing.assert_array_equal(cn, pc)
    np.testing.assert_allclose(sv, ps, rtol=0, atol=1e-4)


def test_ten_steps_track_the_oracle():
    """Trajectories are chaotic; over 10 steps FP32 and FP64 still agree to
    far below the particle spacing."""
    cells = (8, 8, 8)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=14)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    b = _box(cells, pos, vel, params, 14)
    b.step(10)
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    oracle.step(x, v, np.arange(len(x), dtype=np.uint32), cells, _orc_params(params), 14, 0, 10, want_diag=False)
    dx = np.abs(b.read(dpd.POS) - x)
    dx = np.minimum(dx, 8.0 - dx)
    dv = np.abs(b.read(dpd.VEL) - v)
    _say(f"10 steps: max |dx| {dx.max():.3e}, max |dv| {dv.max():.3e}")
    assert dx.max() < 1e-3 and dv.max() < 1e-2


# ---------------------------------------------------------------------------
# full-size workloads: sampled particles against the oracle
# ---------------------------------------------------------------------------

def _body_force_sum(pos, w):
    """Sum of the periodic-Poiseuille body force over the particles (flow
    axis x, gradient axis y, -f where y <= L_y / 2)."""
    if w.body_f == 0.0:
        return 0.0
    lower = np.count_nonzero(pos[:, 1].astype(np.float64) <= 0.5 * w.cells[1])
    return w.body_f * (len(pos) - 2 * lower)


def _momentum_check(f_gpu, pos, w, label):
    """Pair forces are exactly antisymmetric fixed-point sums: the forces of
    the whole box add up to the body-force sum up to the final FP32 rounding
    of each particle's force."""
    f = f_gpu.astype(np.float64)
    tot = f.sum(axis=0)
    tot[0] -= _body_force_sum(pos, w)
    bound = np.sum(np.spacing(np.abs(f).astype(np.float32)).astype(np.float64), axis=0)
    _say(f"[{label}] |sum f - body| = {np.abs(tot)}, rounding bound {bound}")
    assert np.all(np.abs(tot) <= bound), (label, tot, bound)


@pytest.mark.parametrize("name", ["cube48_rho3", "pp192x96x96_rho8"])
def test_full_size_forces_sampled(name):
    """Full-size boxes at step 0 on the harness's state and again at a later
    step on the GPU's own state (the tile shape the benchmark tunes), on 4000
    sampled particles; the momentum balance over the whole box both times."""
    w = inputs.WORKLOADS[name]
    _say(f"[{name}] generating {w.n} particles")
    pos, vel = inputs.uniform_state(w.cells, n=w.n, kT=w.kT, seed=w.seed)
    params = dpd.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, body_f=w.body_f, profile_bins=w.profile_bins)
    b = _box(w.cells, pos, vel, params, w.seed)
    b.tune_tile(reps=2)
    b.step(1)
    f_gpu = b.read(dpd.FORCE)
    rng = np.random.default_rng(15)
    sample = np.sort(rng.choice(w.n, size=4000, replace=False))
    ids = np.arange(w.n, dtype=np.uint32)
    f_orc, s_orc, _ = oracle.forces(pos, vel, ids, w.cells, _orc_params(params), 0, w.seed, which=sample)
    _force_check(f_gpu[sample], f_orc, s_orc, name)
    _momentum_check(f_gpu, pos, w, name)
    st = b.stats()
    assert st["nonfinite"] == 0 and st["escaped"] == 0
    # a later step on the GPU's own state
    later = 40
    b.step(later - 1)
    pe, ve = b.read(dpd.POS), b.read(dpd.VEL)
    b.step(1)
    f_gpu = b.read(dpd.FORCE)
    f_orc, s_orc, _ = oracle.forces(pe, ve, ids, w.cells, _orc_params(params), later, w.seed, which=sample)
    _force_check(f_gpu[sample], f_orc, s_orc, f"{name} step {later}")
    _momentum_check(f_gpu, pe, w, f"{name} step {later}")
    st = b.stats()
    assert st["step"] == later + 1 and st["nonfinite"] == 0 and st["escaped"] == 0
    b.close()


def test_full_box_forces_cube48_at_step_100():
    """Every particle of the 48^3 box at step 100, on the GPU's own state,
    against the oracle over the whole box."""
    w = inputs.WORKLOADS["cube48_rho3"]
    pos, vel = inputs.uniform_state(w.cells, n=w.n, kT=w.kT, seed=w.seed)
    params = dpd.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt)
    b = _box(w.cells, pos, vel, params, w.seed)
    b.step(100)
    pe, ve = b.read(dpd.POS), b.read(dpd.VEL)
    b.step(1)
    f_gpu = b.read(dpd.FORCE)
    ids = np.arange(w.n, dtype=np.uint32)
    f_orc, s_orc, _ = oracle.forces(pe, ve, ids, w.cells, _orc_params(params), 100, w.seed)
    _force_check(f_gpu, f_orc, s_orc, "cube48_rho3 full box, step 100")
    err = np.linalg.norm(f_gpu.astype(np.float64) - f_orc, axis=1) / np.maximum(np.linalg.norm(f_orc, axis=1), 1e-300)
    _say(f"[cube48 step 100] relative |df|/|f|: max {err.max():.3e}, p99.99 {np.quantile(err, 0.9999):.3e}")
    _momentum_check(f_gpu, pe, w, "cube48 step 100")
    b.close()


@pytest.mark.parametrize("cells,rho,seed", [((8, 8, 8), 3.0, 21), ((48, 48, 48), 3.0, 22), ((13, 7, 19), 8.0, 23)])
def test_cell_list_matches_oracle_at_steps_1_10_100(cells, rho, seed):
    """The cell list the GPU builds at steps 1, 10 and 100 of its own run
    equals, bit for bit, the oracle's stable counting sort of the positions
    in the order the previous step left them."""
    pos, vel = inputs.uniform_state(cells, density=rho, seed=seed)
    b = _box(cells, pos, vel, dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01), seed)
    done = 0
    for target in (1, 10, 100):
        if target - 1 > done:
            b.step(target - 1 - done)
            done = target - 1
        if done == 0:
            ids_prev = np.arange(len(pos), dtype=np.int32)       # the state's own (id) order
        else:
            ids_prev = b.read_raw()[0][:, 3].view(np.int32).copy()
        by_id = b.read(dpd.POS)
        b.step(1)
        done += 1
        p4, _, cs = b.read_raw()
        order, start = oracle.bin_cells(by_id[ids_prev], cells)
        np.testing.assert_array_equal(cs, start, err_msg=f"step {target}")
        np.testing.assert_array_equal(p4[:, 3].view(np.int32), ids_prev[order], err_msg=f"step {target}")
        np.testing.assert_array_equal(p4[:, :3], by_id[ids_prev][order], err_msg=f"step {target}")
    b.close()


@pytest.mark.parametrize("L", [8, 48, 192])
def test_offgrid_fp32_inputs(L):
    """Positions handed over as arbitrary FP32 numbers (finer than the box's
    position grid q): the library rounds them to q, and its forces are those
    of the rounded state, within 1e-5 S_i of the oracle on that state.
    Against the oracle on the raw positions the difference is that bar plus
    what the rounding (at most q/2 per coordinate) moves the exact forces."""
    if L == 192:
        cells, w = (192, 8, 8), inputs.WORKLOADS["pp192x96x96_rho8"]
    elif L == 48:
        cells, w = (48, 24, 24), inputs.WORKLOADS["cube48_rho3"]
    else:
        cells, w = (8, 8, 8), inputs.WORKLOADS["cube8_rho3"]
    n = int(round(w.density * cells[0] * cells[1] * cells[2]))
    pos, vel = inputs.offgrid_state(cells, n, kT=w.kT, seed=30 + L)
    params = dpd.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, body_f=w.body_f)
    b = _box(cells, pos, vel, params, 31)
    rounded = b.read(dpd.POS)
    q = dpd.position_grid(cells)
    d = np.abs(rounded.astype(np.float64) - pos)
    d = np.minimum(d, np.array(cells, dtype=np.float64) - d)      # a coordinate next to L wraps to 0
    assert np.all(d <= 0.5 * q)
    assert np.count_nonzero(rounded != pos) > n // 4              # the inputs were off the grid
    b.step(1)
    f_gpu = b.read(dpd.FORCE)
    ids = np.arange(n, dtype=np.uint32)
    op = _orc_params(params)
    f_r, s_r, _ = oracle.forces(rounded, vel, ids, cells, op, 0, 31)
    _force_check(f_gpu, f_r, s_r, f"off-grid L={L}, rounded state")
    # against the oracle on the raw positions: the contract is the forces of
    # the grid-rounded state, so the bar is 1e-5 S_i plus what the rounding
    # itself moves the exact (FP64) forces, |f_orc(rounded) - f_orc(raw)|
    f_raw, s_raw, _ = oracle.forces(pos, vel, ids, cells, op, 0, 31)
    moved = np.linalg.norm(f_r - f_raw, axis=1)
    err = np.linalg.norm(f_gpu.astype(np.float64) - f_raw, axis=1)
    _say(f"[off-grid L={L}] raw positions: max |df|/S = {np.max(err / s_raw):.3e}; "
         f"rounding alone moves the exact forces by up to {np.max(moved / s_raw):.3e} S")
    assert np.all(err <= TOL_F * s_raw + moved + 1e-30)
    b.close()


def test_profile_bins_match_oracle_statistics():
    """The time-averaged flow profile of a driven box, GPU against oracle,
    bin by bin within three combined standard errors (eight blocks each)."""
    cells, nb = (8, 8, 8), 8
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=24)
    params = dpd.make_params(a=25.0, gamma=6.75, kT=1.0, dt=0.04, body_f=0.2, profile_bins=nb)
    b = _box(cells, pos, vel, params, 24)
    b.step(600)
    gp = []
    for _ in range(8):
        b.reset_accumulators()
        b.step(400)
        sv, cn = b.profile()
        gp.append(sv / cn)
    b.close()
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    ids = np.arange(len(x), dtype=np.uint32)
    op = _orc_params(params)
    oracle.step(x, v, ids, cells, op, 24, 0, 600, want_diag=False)
    op_ = []
    for k in range(8):
        _, ps, pc, _ = oracle.step(x, v, ids, cells, op, 24, 600 + 400 * k, 400, nbins=nb, want_diag=False)
        op_.append(ps / pc)
    gp, op_ = np.array(gp), np.array(op_)
    gm, ge = gp.mean(axis=0), gp.std(axis=0, ddof=1) / math.sqrt(8)
    om, oe = op_.mean(axis=0), op_.std(axis=0, ddof=1) / math.sqrt(8)
    z = np.abs(gm - om) / np.hypot(ge, oe)
    _say(f"profile GPU {np.round(gm, 4)}\n        orc {np.round(om, 4)}\n        z {np.round(z, 2)}")
    assert np.all(gm[: nb // 2] < 0) and np.all(gm[nb // 2:] > 0)
    assert np.all(z < 3.0), z


# ---------------------------------------------------------------------------
# determinism, statistics, errors
# ---------------------------------------------------------------------------

def test_run_twice_bitwise_identical():
    cells = (10, 9, 8)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=16)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, body_f=0.05, profile_bins=9)
    out = []
    for _ in range(2):
        b = _box(cells, pos, vel, params, 16)
        b.step(57)
        out.append((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE), b.stats(), b.profile()))
        b.close()
    for k in range(3):
        np.testing.assert_array_equal(out[0][k], out[1][k])
    assert out[0][3]["ke_half"] == out[1][3]["ke_half"]
    np.testing.assert_array_equal(out[0][4][0], out[1][4][0])


def test_pair_forces_conserve_momentum_exactly():
    """Fixed-point accumulation of exactly antisymmetric pair forces: the sum
    of all pair forces is zero up to the final FP32 rounding of each force."""
    cells = (16, 16, 16)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=17)
    b = _box(cells, pos, vel, dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01), 17)
    b.step(1)
    f = b.read(dpd.FORCE).astype(np.float64)
    tot = np.abs(f.sum(axis=0))
    bound = np.sum(np.spacing(np.abs(f).astype(np.float32)).astype(np.float64), axis=0)
    assert np.all(tot <= bound), (tot, bound)


def test_equilibrium_statistics_match_oracle():
    cells = (8, 8, 8)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=11)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, flags=dpd.FLAG_VIRIAL)
    b = _box(cells, pos, vel, params, 11)
    b.step(1000)
    kts, prs = [], []
    for blk in range(10):
        b.reset_accumulators()
        b.step(500)
        st = b.stats()
        kts.append(st["sum_kT_centred"] / st["nsamples"])
        prs.append(st["sum_pressure"] / st["nsamples"])
    kt, se_kt = np.mean(kts), np.std(kts, ddof=1) / math.sqrt(len(kts))
    pr, se_pr = np.mean(prs), np.std(prs, ddof=1) / math.sqrt(len(prs))
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    diag, _, _, _ = oracle.step(x, v, np.arange(len(x), dtype=np.uint32), cells,
                                oracle.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01), 11, 0, 6000)
    okt = diag["kT_centred"][1000:].reshape(10, -1).mean(axis=1)
    opr = diag["pressure"][1000:].reshape(10, -1).mean(axis=1)
    _say(f"GPU kT {kt:.4f}+-{se_kt:.4f} p {pr:.3f}+-{se_pr:.3f}; oracle kT {okt.mean():.4f} p {opr.mean():.3f}")
    assert abs(kt - 1.0) < 0.01
    se_o = okt.std(ddof=1) / math.sqrt(10)
    assert abs(kt - okt.mean()) < 3 * math.hypot(se_kt, se_o) + 1e-3
    sp_o = opr.std(ddof=1) / math.sqrt(10)
    assert abs(pr - opr.mean()) < 3 * math.hypot(se_pr, sp_o) + 0.02


def test_poiseuille_profile_on_gpu():
    cells = (8, 8, 8)
    nb = 16
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=13)
    params = dpd.make_params(a=25.0, gamma=6.75, kT=1.0, dt=0.04, body_f=0.1, profile_bins=nb)
    b = _box(cells, pos, vel, params, 13)
    b.step(1500)
    prof = []
    for blk in range(10):
        b.reset_accumulators()
        b.step(300)
        sv, cn = b.profile()
        prof.append(sv / cn)
    prof = np.array(prof)
    mean, err = prof.mean(axis=0), prof.std(axis=0, ddof=1) / math.sqrt(10)
    L = 8.0
    def shape(y0, y1):
        yy = np.linspace(y0, y1, 201)
        s = np.mod(yy, L / 2)
        return np.mean(np.where(yy <= L / 2, -1.0, 1.0) * s * (L / 2 - s))
    g = np.array([shape(i * L / nb, (i + 1) * L / nb) for i in range(nb)])
    w = 1.0 / err ** 2
    c = np.sum(w * g * mean) / np.sum(w * g * g)
    eta = 3.0 * 0.1 / (2.0 * c)
    _say(f"GPU Poiseuille eta = {eta:.3f}")
    assert np.all(mean[: nb // 2] < 0) and np.all(mean[nb // 2:] > 0)
    assert abs(eta - 0.91) < 0.15 * 0.91


def test_error_paths():
    cells = (4, 4, 4)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=18)
    b = dpd.Box(cells, len(pos))
    with pytest.raises(dpd.DPDError) as e:
        b.step(1)
    assert e.value.code == dpd.ESTATE
    b.set_params(dpd.make_params())
    b.set_seed(1)
    bad = pos.copy()
    bad[5, 1] = 4.0                                    # == L: outside [0, L)
    with pytest.raises(dpd.DPDError) as e:
        b.set_state(bad, vel)
    assert e.value.code == dpd.EINVAL
    nanv = vel.copy()
    nanv[3, 0] = np.nan
    with pytest.raises(dpd.DPDError) as e:
        b.set_state(pos, nanv)
    assert e.value.code == dpd.EINVAL
    with pytest.raises(dpd.DPDError) as e:
        b.read(dpd.POS)
    assert e.value.code == dpd.ESTATE
    for kw in [dict(dt=0.0), dict(gamma=-1.0), dict(flow_axis=1, grad_axis=1), dict(profile_bins=5000),
               dict(kT=float("nan"))]:
        with pytest.raises(dpd.DPDError) as e:
            b.set_params(dpd.make_params(**kw))
        assert e.value.code == dpd.EINVAL
    b.set_state(pos, vel)
    with pytest.raises(dpd.DPDError) as e:
        b.read(dpd.FORCE)
    assert e.value.code == dpd.ESTATE
    # an absurd time step makes particles jump more than a cell: reported
    b.set_params(dpd.make_params(dt=5.0))
    b.step(2)
    st = b.stats(allow_nonfinite=True)
    assert st["escaped"] == 1
    b.close()


def test_pair_force_beyond_the_fixed_point_range_is_reported():
    """Pair forces are summed as 64-bit fixed point, 2^31 units per force
    unit, with a range of 2^19 per pair (include/dpd.h, DPD_ENONFINITE).  Two
    particles 0.5 apart closing at relative speed 2V feel a dissipative
    force of 2 gamma w^2 V = 2.25 V: at V = 1e4 it is summed (and matches the
    FP64 oracle), at V = 1e6 it is beyond the range, adds nothing and is
    reported."""
    cells = (4, 4, 4)
    pos = np.array([[1.25, 2.0, 2.0], [1.75, 2.0, 2.0]], np.float32)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=1e-6)
    ids = np.arange(2, dtype=np.uint32)
    for v, reported in [(1e4, False), (1e6, True)]:
        vel = np.array([[v, 0.0, 0.0], [-v, 0.0, 0.0]], np.float32)
        b = _box(cells, pos, vel, params, 5)
        b.step(1)
        st = b.stats(allow_nonfinite=True)
        assert st["nonfinite"] == (1 if reported else 0), v
        if not reported:
            f_gpu = b.read(dpd.FORCE)
            assert f_gpu[0, 0] < -2.0e4 and f_gpu[1, 0] == -f_gpu[0, 0]
            f_orc, s_orc, _ = oracle.forces(pos, vel, ids, cells, _orc_params(params), step=0, seed=5)
            _force_check(f_gpu, f_orc, s_orc, f"closing pair v={v:g}")
        b.close()


def test_empty_and_single_particle_boxes():
    b = dpd.Box((3, 3, 3), 0, params=dpd.make_params(), seed=0)
    b.set_state(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32))
    b.step(5)
    assert b.read(dpd.POS).shape == (0, 3)
    assert b.stats()["step"] == 5
    b.close()
    pos = np.array([[1.5, 1.5, 1.5]], np.float32)
    vel = np.array([[0.5, -0.25, 0.125]], np.float32)
    b = dpd.Box((3, 3, 3), 1, params=dpd.make_params(dt=0.01, body_f=0.2), seed=0)
    b.set_state(pos, vel)
    b.step(3)
    f = b.read(dpd.FORCE)
    np.testing.assert_array_equal(f, [[np.float32(-0.2), 0.0, 0.0]])
    b.close()


def test_periodic_pair_worked_example():
    # the two-particle example across the periodic face of an 8^3 box
    # (Eqs. 3-5 worked by hand; the same numbers pin the oracle), through
    # the C-ABI: the force after one step is the step-0 force
    pos = np.array([[0.125, 4.0, 4.0], [7.75, 4.25, 3.875]], np.float32)
    vel = np.array([[0.5, -0.25, 0.125], [-0.25, 0.5, 0.0]], np.float32)
    fc = np.array([10.669593143432, -7.113062095621, 3.556531047811])
    fd = np.array([-1.058714025971, 0.705809350647, -0.352904675324])
    fr1 = np.array([12.803511772118, -8.535674514745, 4.267837257373])
    for kT, seed in ((0.0, 3), (1.0, 11)):
        b = _box((8, 8, 8), pos, vel, dpd.make_params(a=25.0, gamma=4.5, kT=kT, dt=0.01), seed)
        b.step(1)
        f = b.read(dpd.FORCE).astype(np.float64)
        b.close()
        expect = fc + fd + (oracle.xi(0, 1, 0, seed) * fr1 if kT else 0.0)
        s = np.abs(fc).sum() + np.abs(fd).sum() + (np.abs(fr1).sum() * 4.0 if kT else 0.0)
        _say(f"[example B] kT={kT}: gpu {f[0]}, expect {expect}")
        assert np.all(np.abs(f[0] - expect) <= TOL_F * s), (f[0], expect)
        np.testing.assert_array_equal(f[1], -f[0])          # the pair halves are exact negatives


# ---------------------------------------------------------------------------
# kernel exponent k (w_R = w^k, w_D = w_R^2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k,cells,rho", [(0.25, (10, 9, 8), 4.0), (0.15, (7, 12, 9), 3.0), (0.5, (5, 5, 5), 8.0)])
def test_kernel_exponent_forces(k, cells, rho):
    pos, vel = inputs.uniform_state(cells, density=rho, seed=31)
    p = dpd.make_params(a=18.75, gamma=4.5, kT=1.0, dt=0.005, kexp=k)
    b = _box(cells, pos, vel, p, 31)
    b.step(1)
    f = b.read(dpd.FORCE)
    b.close()
    ids = np.arange(len(pos), dtype=np.uint32)
    fo, so, _ = oracle.forces(pos, vel, ids, cells, _orc_params(p), 0, 31)
    _force_check(f, fo, so, f"k={k}")
    # the reference gather kernel gives the same bits as the tile kernel
    pr = dpd.make_params(a=18.75, gamma=4.5, kT=1.0, dt=0.005, kexp=k, flags=dpd.FLAG_REFERENCE_FORCE)
    br = _box(cells, pos, vel, pr, 31)
    br.step(1)
    np.testing.assert_array_equal(br.read(dpd.FORCE), f)
    br.close()


def test_kernel_exponent_one_and_zero_are_linear():
    cells = (9, 8, 7)
    pos, vel = inputs.uniform_state(cells, density=3.0, seed=32)
    out = []
    for k in (1.0, 0.0):
        b = _box(cells, pos, vel, dpd.make_params(kexp=k), 32)
        b.step(3)
        out.append((b.read(dpd.POS), b.read(dpd.VEL), b.read(dpd.FORCE)))
        b.close()
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)
    b = dpd.Box(cells, len(pos), seed=1)
    for bad in (-0.1, 1.5, float("nan")):
        with pytest.raises(dpd.DPDError) as e:
            b.set_params(dpd.make_params(kexp=bad))
        assert e.value.code == dpd.EINVAL
    b.close()
