"""Serving: admission by HBM footprint, continuous batching, and the same
result for a request alone and in a mix."""
import numpy as np
import pytest

from paper_1911_04712_amd import dpd, inputs

pytestmark = pytest.mark.gpu

P3 = dict(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
P8 = dict(a=10.0, gamma=10.0, kT=1.0, dt=0.01, body_f=0.05)


def _run_until_done(srv, tickets, quantum, arrivals=()):
    """Pump until all tickets are done; `arrivals` are (after_pump_k, submit_fn)
    pairs that submit more requests while others run."""
    out, pumps = {}, 0
    arrivals = list(arrivals)
    while len(out) < len(tickets) or arrivals:
        while arrivals and arrivals[0][0] <= pumps:
            tickets.append(arrivals.pop(0)[1]())
        srv.pump(quantum)
        pumps += 1
        for t in tickets:
            if t not in out:
                r = srv.poll(t, want_state=True)
                if r is not None:
                    out[t] = r
        assert pumps < 10000
    return out


def test_request_alone_equals_request_in_mix():
    cells, n = (9, 7, 6), 1134
    pos, vel = inputs.uniform_state(cells, n=n, seed=50)
    alone = dpd.Server(64 << 20, max_slots=8)
    t = alone.submit(cells, n, P3, seed=50, nsteps=60, pos=pos, vel=vel)
    ref = _run_until_done(alone, [t], quantum=20)[t]
    alone.close()

    mix = dpd.Server(64 << 20, max_slots=8)
    tk = [mix.submit((5, 6, 7), 210 * 8, P8, seed=51, nsteps=90, init_kT=1.0, init_seed=7),
          mix.submit((4, 4, 4), 192, P3, seed=52, nsteps=30, init_kT=1.0, init_seed=8)]
    target = []

    def late():
        target.append(mix.submit(cells, n, P3, seed=50, nsteps=60, pos=pos, vel=vel))
        return target[0]
    arrivals = [(1, late), (2, lambda: mix.submit((8, 3, 5), 360, P3, seed=53, nsteps=45, init_kT=0.5, init_seed=9))]
    got = _run_until_done(mix, tk, quantum=20, arrivals=arrivals)
    res, p, v = got[target[0]]
    assert res["status"] == dpd.OK
    assert res["stats"]["step"] == 60
    np.testing.assert_array_equal(p, ref[1])
    np.testing.assert_array_equal(v, ref[2])
    assert res["stats"]["ke_half"] == ref[0]["stats"]["ke_half"]
    for r in got.values():
        assert r[0]["status"] == dpd.OK
        assert r[0]["t_submit"] <= r[0]["t_admit"] <= r[0]["t_done"]
    mix.close()


def test_admission_waits_for_memory():
    cells, n = (10, 10, 10), 3000
    def a256(x):
        return (x + 255) // 256 * 256
    need = a256(dpd.workspace_bytes(cells, n))
    # room for two requests plus the batch tables, not three
    srv = dpd.Server(a256(dpd.batch_workspace_bytes(16)) + 2 * need + need // 2, max_slots=16)
    tk = [srv.submit(cells, n, P3, seed=60 + k, nsteps=40, init_kT=1.0, init_seed=k) for k in range(3)]
    srv.pump(10)
    q, a, _ = srv.counts()
    assert (q, a) == (1, 2)
    out = _run_until_done(srv, tk, quantum=10)
    t_admit = [out[t][0]["t_admit"] for t in tk]
    t_done = [out[t][0]["t_done"] for t in tk]
    assert t_admit[2] >= min(t_done[0], t_done[1])          # admitted only after memory was freed
    srv.close()


def test_server_rejects_and_edge_requests():
    srv = dpd.Server(8 << 20, max_slots=4)
    with pytest.raises(dpd.DPDError) as e:
        srv.submit((64, 64, 64), 3 * 64 ** 3, P3, seed=1, nsteps=10)   # can never fit
    assert e.value.code == dpd.ENOMEM
    t0 = srv.submit((4, 4, 4), 100, P3, seed=2, nsteps=0, init_kT=1.0)
    t1 = srv.submit((3, 3, 3), 0, P3, seed=3, nsteps=5)
    out = _run_until_done(srv, [t0, t1], quantum=4)
    assert out[t0][0]["status"] == dpd.OK and out[t0][0]["stats"]["step"] == 0
    assert out[t1][0]["status"] == dpd.OK
    with pytest.raises(dpd.DPDError) as e:
        srv.poll(t0)
    assert e.value.code == dpd.ENOTFOUND
    srv.close()


def test_init_random_state():
    cells = (16, 12, 10)
    n = 3 * 16 * 12 * 10
    b = dpd.Box(cells, n, params=dpd.make_params(mass=2.0), seed=1)
    b.init_random(kT=1.5, seed=77)
    p, v = b.read(dpd.POS), b.read(dpd.VEL).astype(np.float64)
    assert np.all(p >= 0) and np.all(p < np.array(cells, dtype=np.float32))
    q = dpd.position_grid(cells)
    assert np.all(np.mod(p.astype(np.float64), q) == 0)
    assert np.all(np.abs(v.mean(axis=0)) < 1e-6)
    # per-component variance kT/m = 0.75 within 5 standard errors
    var = v.var(axis=0)
    assert np.all(np.abs(var - 0.75) < 5 * 0.75 * np.sqrt(2.0 / n))
    # uniform positions: occupancy of the 8 octants within 5 sigma
    octant = (p[:, 0] >= 8).astype(int) + 2 * (p[:, 1] >= 6) + 4 * (p[:, 2] >= 5)
    cnt = np.bincount(octant, minlength=8)
    assert np.all(np.abs(cnt - n / 8) < 5 * np.sqrt(n / 8))
    # same seed, same state; the box steps from it
    b2 = dpd.Box(cells, n, params=dpd.make_params(mass=2.0), seed=1)
    b2.init_random(kT=1.5, seed=77)
    np.testing.assert_array_equal(b2.read(dpd.VEL), b.read(dpd.VEL))
    b.step(5)
    assert b.stats()["step"] == 5
    b.close()
    b2.close()


# ---------------------------------------------------------------------------
# served requests against the CPU oracle (not only against themselves alone)
# ---------------------------------------------------------------------------

TOL_F = 1e-5


def _orc(p):
    import oracle
    return oracle.make_params(a=p["a"], gamma=p["gamma"], kT=p["kT"], dt=p["dt"], body_f=p.get("body_f", 0.0))


def _mix(srv):
    """Three other requests of other sizes and fluids that share the pumps."""
    return [srv.submit((5, 6, 7), 210 * 8, P8, seed=91, nsteps=25, init_kT=1.0, init_seed=3),
            srv.submit((4, 4, 4), 192, P3, seed=92, nsteps=3, init_kT=1.0, init_seed=4),
            srv.submit((11, 3, 6), 594, P3, seed=93, nsteps=14, init_kT=0.5, init_seed=5)]


def test_served_one_step_matches_oracle():
    """A one-step request served in a mix: its final state and diagnostics
    against the FP64 oracle's step from the same state (velocities within
    dt 1e-5 S_i plus 4 ulp, positions within two grid spacings)."""
    import oracle
    cells, n = (9, 7, 6), 1134
    p = dict(P8, profile_bins=0)
    pos, vel = inputs.uniform_state(cells, n=n, seed=94)
    srv = dpd.Server(64 << 20, max_slots=8)
    tk = _mix(srv)
    target = srv.submit(cells, n, dict(a=10.0, gamma=10.0, kT=1.0, dt=0.01, body_f=0.05), seed=94, nsteps=1,
                        pos=pos, vel=vel)
    got = _run_until_done(srv, tk + [target], quantum=4)
    res, pg, vg = got[target]
    assert res["status"] == dpd.OK and res["stats"]["step"] == 1
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    ids = np.arange(n, dtype=np.uint32)
    op = _orc(dict(a=10.0, gamma=10.0, kT=1.0, dt=0.01, body_f=0.05))
    diag, _, _, _ = oracle.step(x, v, ids, cells, op, 94, 0, 1)
    _, s_orc, _ = oracle.forces(pos, vel, ids, cells, op, 0, 94)
    dv = np.abs(vg.astype(np.float64) - v)
    tol_v = 0.01 * TOL_F * s_orc[:, None] + 4 * np.spacing(np.abs(v).astype(np.float32)).astype(np.float64)
    print(f"served one step: max |dv| / tol = {np.max(dv / tol_v):.3e}", flush=True)
    assert np.all(dv <= tol_v)
    dx = np.abs(pg.astype(np.float64) - x)
    L = np.array(cells, dtype=np.float64)
    dx = np.minimum(dx, L - dx)
    assert np.all(dx <= 2 * dpd.position_grid(cells) + 0.01 * dv + 1e-12)
    st = res["stats"]
    np.testing.assert_allclose(st["momentum"], diag["momentum"][0], rtol=0, atol=1e-4)
    assert st["ke_half"] == pytest.approx(diag["ke_half"][0], rel=1e-6)
    assert st["ke_centred"] == pytest.approx(diag["ke_centred"][0], rel=1e-6)
    assert st["kT_centred"] == pytest.approx(diag["kT_centred"][0], rel=1e-6)
    srv.close()


def test_served_request_tracks_oracle_over_ten_steps():
    """A ten-step request that runs over several pumps while other requests
    come and go: its final state stays within the ten-step tracking bound of
    FP32 against the FP64 oracle."""
    import oracle
    cells, n = (8, 8, 8), 1536
    pos, vel = inputs.uniform_state(cells, n=n, seed=95)
    srv = dpd.Server(64 << 20, max_slots=8)
    tk = _mix(srv)
    target = srv.submit(cells, n, P3, seed=95, nsteps=10, pos=pos, vel=vel)
    late = [(1, lambda: srv.submit((6, 6, 6), 648, P3, seed=96, nsteps=5, init_kT=1.0, init_seed=6))]
    got = _run_until_done(srv, tk + [target], quantum=3, arrivals=late)
    res, pg, vg = got[target]
    assert res["status"] == dpd.OK and res["stats"]["step"] == 10
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    oracle.step(x, v, np.arange(n, dtype=np.uint32), cells, _orc(P3), 95, 0, 10, want_diag=False)
    dx = np.abs(pg - x)
    dx = np.minimum(dx, 8.0 - dx)
    dv = np.abs(vg - v)
    print(f"served 10 steps: max |dx| {dx.max():.3e}, max |dv| {dv.max():.3e}", flush=True)
    assert dx.max() < 1e-3 and dv.max() < 1e-2
    srv.close()


def test_nonfinite_request_is_retired_and_others_unaffected():
    """A request whose velocities are absurd (1e30) overflows the force
    range: it is retired with DPD_ENONFINITE, while the requests beside it
    finish with the same bits as alone."""
    cells, n = (6, 6, 6), 648
    pos, vel = inputs.uniform_state(cells, n=n, seed=97)
    bad_vel = vel.copy()
    bad_vel[::50] = 1e30
    ok_cells, ok_n = (7, 5, 6), 630
    ok_pos, ok_vel = inputs.uniform_state(ok_cells, n=ok_n, seed=98)
    alone = dpd.Server(64 << 20, max_slots=4)
    t = alone.submit(ok_cells, ok_n, P3, seed=98, nsteps=12, pos=ok_pos, vel=ok_vel)
    ref = _run_until_done(alone, [t], quantum=5)[t]
    alone.close()
    srv = dpd.Server(64 << 20, max_slots=4)
    tb = srv.submit(cells, n, P3, seed=97, nsteps=12, pos=pos, vel=bad_vel)
    tg = srv.submit(ok_cells, ok_n, P3, seed=98, nsteps=12, pos=ok_pos, vel=ok_vel)
    got = _run_until_done(srv, [tb, tg], quantum=5)
    assert got[tb][0]["status"] == dpd.ENONFINITE
    assert got[tb][0]["stats"]["nonfinite"] == 1
    res, p, v = got[tg]
    assert res["status"] == dpd.OK
    np.testing.assert_array_equal(p, ref[1])
    np.testing.assert_array_equal(v, ref[2])
    srv.close()
