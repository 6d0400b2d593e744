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
