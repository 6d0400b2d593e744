"""Pins of the oracle's walls: SDF surface, frozen particles, bounce-back.

Walls are the zero isosurface of a signed distance function with a layer of
frozen particles (thickness r_c) behind it that interact through the usual
DPD forces and never move (Sec. 2.3); a fluid particle whose drift ends
inside the wall is put at the collision point, the SDF's zero along the
drift, with its velocity reversed (Sec. 3.3).  Pins, none a retyped line of
the oracle:

  - a crossing of a plate lands on the plane where the drift meets it, a
    crossing of a pipe where the drift meets the circle (the root of the
    quadratic |p + t d| = R), velocities reversed; particles that stay in
    the fluid move as without walls;
  - frozen particles never move and are left out of the diagnostics;
  - over a long run no fluid particle is ever found inside a wall;
  - channel (plane Poiseuille) flow between frozen walls has the parabolic
    profile v = rho f (h^2 - y^2) / (2 eta) with the viscosity the periodic
    Poiseuille measurement gives for the same fluid;
  - rotating coaxial cylinders (Taylor-Couette, Sec. 4.3): a crossing of
    either cylinder lands on it with the velocity reversed in the frame of
    that wall (v -> 2 omega x r - v), a turning cylinder's frozen layer turns
    rigidly with it, and the azimuthal profile is A r + B / r.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1911_04712_amd import inputs


def _two_particles(p0, v0, far=(0.5, 0.5, 0.5)):
    x = np.array([p0, far], dtype=np.float64)
    v = np.array([v0, (0.0, 0.0, 0.0)], dtype=np.float64)
    return x, v, np.arange(2, dtype=np.uint32)


def test_plate_crossing_lands_on_the_plane():
    cells = (6, 8, 6)                      # plates normal to y (grad axis 1) at y = 4 -+ 2.5
    p = oracle.with_walls(oracle.make_params(a=0.0, gamma=0.0, kT=0.0, dt=0.01), 1, 2.5)
    y0, vy, vx = 6.49, 2.0, 0.75
    x, v, ids = _two_particles((3.0, y0, 3.0), (vx, vy, 0.0), far=(3.0, 4.0, 3.0))
    oracle.step(x, v, ids, cells, p, 0, 0, 1, want_diag=False)
    t = (6.5 - y0) / (vy * 0.01)           # fraction of the drift that reaches the plane
    assert x[0, 1] == pytest.approx(6.5, abs=1e-12) and oracle.sdf(x[0], cells, p)[0] <= 0.0
    assert x[0, 0] == pytest.approx(3.0 + t * vx * 0.01, abs=1e-12)
    np.testing.assert_array_equal(v[0], [-vx, -vy, 0.0])
    # the lower plate, and a particle that stays in the fluid
    x, v, ids = _two_particles((3.0, 1.505, 3.0), (0.0, -1.0, 0.0), far=(3.0, 4.0, 3.0))
    v[1] = (0.3, 0.4, -0.2)
    oracle.step(x, v, ids, cells, p, 0, 0, 1, want_diag=False)
    assert x[0, 1] == pytest.approx(1.5, abs=1e-12) and oracle.sdf(x[0], cells, p)[0] <= 0.0
    np.testing.assert_array_equal(v[0], [0.0, 1.0, 0.0])
    np.testing.assert_allclose(x[1], [3.003, 4.004, 2.998], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(v[1], [0.3, 0.4, -0.2])


@pytest.mark.parametrize("seed", range(5))
def test_pipe_crossing_lands_on_the_circle(seed):
    cells = (5, 12, 12)                    # pipe along x (flow axis 0) through (y, z) = (6, 6)
    R = 4.0
    p = oracle.with_walls(oracle.make_params(a=0.0, gamma=0.0, kT=0.0, dt=0.01), 2, R)
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0, 2 * math.pi)
    r0 = R - rng.uniform(0.001, 0.01)
    p0 = np.array([2.0, 6.0 + r0 * math.cos(ang), 6.0 + r0 * math.sin(ang)])
    out = np.array([0.0, math.cos(ang), math.sin(ang)])
    vel = 1.5 * out + rng.normal(0, 0.4, 3)
    x, v, ids = _two_particles(p0, vel, far=(2.0, 6.0, 6.0))
    oracle.step(x, v, ids, cells, p, 0, 0, 1, want_diag=False)
    d = vel * 0.01
    # |q + t e|^2 = R^2 in the cross-section, q = p0 - centre, e = drift
    q, e = p0[1:] - 6.0, d[1:]
    A, B, C = e @ e, 2 * q @ e, q @ q - R * R
    t = (-B + math.sqrt(B * B - 4 * A * C)) / (2 * A)
    assert 0 < t < 1
    np.testing.assert_allclose(x[0], p0 + t * d, rtol=0, atol=1e-12)
    assert oracle.sdf(x[0], cells, p)[0] <= 0.0
    np.testing.assert_array_equal(v[0], -vel)


def _channel_state(cells, h, rho, seed, equil_steps=300, params=None):
    """An equilibrated periodic fluid carved into a channel: particles within
    r_c behind each plate are frozen (zero velocity), those further in are
    dropped, as the paper builds its wall layers from the fluid itself."""
    pos, vel = inputs.uniform_state(cells, density=rho, seed=seed)
    x, v = pos.astype(np.float64), vel.astype(np.float64)
    ids = np.arange(len(x), dtype=np.uint32)
    p = params or oracle.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    oracle.step(x, v, ids, cells, p, seed, 0, equil_steps, want_diag=False)
    s = oracle.sdf(x, cells, oracle.with_walls(p, 1, h))
    keep = s <= 1.0
    frozen = (s[keep] > 0.0).astype(np.uint8)
    x, v = x[keep].copy(), v[keep].copy()
    v[frozen == 1] = 0.0
    return x, v, frozen


def test_frozen_particles_stay_and_are_not_counted():
    cells = (6, 8, 6)
    x, v, frozen = _channel_state(cells, 2.5, 3.0, 51, equil_steps=50)
    ids = np.arange(len(x), dtype=np.uint32)
    p = oracle.with_walls(oracle.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, body_f=0.05), 1, 2.5, frozen)
    x0 = x.copy()
    diag, _, _, _ = oracle.step(x, v, ids, cells, p, 51, 0, 20)
    fz = frozen == 1
    np.testing.assert_array_equal(x[fz], x0[fz])
    np.testing.assert_array_equal(v[fz], 0.0)
    np.testing.assert_allclose(diag["momentum"][-1], v[~fz].sum(axis=0), rtol=1e-12, atol=1e-12)
    ke = 0.5 * (v[~fz] ** 2).sum()
    assert diag["ke_half"][-1] == pytest.approx(ke, rel=1e-12)


@pytest.mark.slow
def test_no_fluid_particle_enters_a_wall():
    cells = (6, 8, 6)
    h = 2.5
    x, v, frozen = _channel_state(cells, h, 3.0, 52)
    ids = np.arange(len(x), dtype=np.uint32)
    p = oracle.with_walls(oracle.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, body_f=0.2), 1, h, frozen)
    fluid = frozen == 0
    worst = -1.0
    for k in range(20):
        oracle.step(x, v, ids, cells, p, 52, 50 * k, 50, want_diag=False)
        worst = max(worst, oracle.sdf(x[fluid], cells, p).max())
    assert worst <= 0.0, worst


@pytest.mark.slow
def test_channel_flow_parabola_and_viscosity():
    """Groot-Warren fluid of Table 1 (a = 25, gamma = 6.75, rho = 3, kT = 1,
    dt = 0.04; eta = 0.89-0.91) between frozen walls 2h = 8 apart, uniform
    drive f: the mean profile is a parabola vanishing near the walls, and its
    curvature gives eta."""
    cells, h, rho, f = (6, 12, 6), 4.0, 3.0, 0.01
    base = oracle.make_params(a=25.0, gamma=6.75, kT=1.0, dt=0.04)
    x, v, frozen = _channel_state(cells, h, rho, 53, equil_steps=200, params=base)
    ids = np.arange(len(x), dtype=np.uint32)
    p = oracle.with_walls(oracle.make_params(a=25.0, gamma=6.75, kT=1.0, dt=0.04, body_f=f, flow_axis=0, grad_axis=1),
                          1, h, frozen)
    nb = 24
    oracle.step(x, v, ids, cells, p, 53, 0, 2500, want_diag=False)          # spin-up, ~4.6 relaxation times
    _, ps, pc, _ = oracle.step(x, v, ids, cells, p, 53, 2500, 6000, nbins=nb, want_diag=False)
    yc = (np.arange(nb) + 0.5) * cells[1] / nb - cells[1] / 2
    inside = np.abs(yc) < h - 0.5
    prof = ps[inside] / pc[inside]
    # least squares v = c0 - c2 y^2
    X = np.stack([np.ones(inside.sum()), -yc[inside] ** 2], axis=1)
    c0, c2 = np.linalg.lstsq(X, prof, rcond=None)[0]
    eta = rho * f / (2 * c2)
    y0 = math.sqrt(c0 / c2)                # where the fitted parabola vanishes
    resid = prof - X @ np.array([c0, c2])
    print(f"channel eta {eta:.3f} y0 {y0:.3f} c0 {c0:.4f}")
    assert np.max(np.abs(resid)) < 0.1 * c0, (resid, c0)
    assert 0.75 < eta < 1.05, eta
    assert abs(y0 - h) < 0.5, y0           # no-slip up to a fraction of r_c


# ---------------------------------------------------------------------------
# rotating coaxial cylinders (Taylor-Couette, Sec. 4.3)
# ---------------------------------------------------------------------------

def _couette_params(base, frozen=None, r_in=2.0, r_out=5.0, w_in=0.0, w_out=0.3):
    return oracle.with_walls(base, 3, r_out, frozen, body_uniform=True, r_in=r_in, omega_in=w_in, omega_out=w_out)


@pytest.mark.parametrize("outward", [True, False])
def test_rotating_wall_bounce_closed_form(outward):
    cells = (4, 12, 12)                    # cylinders along x through (y, z) = (6, 6)
    r_in, r_out, w_in, w_out = 2.0, 5.0, -0.2, 0.3
    p = _couette_params(oracle.make_params(a=0.0, gamma=0.0, kT=0.0, dt=0.01), None, r_in, r_out, w_in, w_out)
    ang = 0.7
    radial = np.array([0.0, math.cos(ang), math.sin(ang)])
    r0, R, w = (r_out - 0.004, r_out, w_out) if outward else (r_in + 0.004, r_in, w_in)
    p0 = np.array([2.0, 6.0, 6.0]) + r0 * radial
    vel = (1.0 if outward else -1.0) * 1.2 * radial + np.array([0.3, -0.4, 0.25])
    x, v, ids = _two_particles(p0, vel, far=(2.0, 6.0 + 3.5 * math.cos(ang + 2), 6.0 + 3.5 * math.sin(ang + 2)))
    oracle.step(x, v, ids, cells, p, 0, 0, 1, want_diag=False)
    d = vel * 0.01
    q, e = p0[1:] - 6.0, d[1:]
    A, B, C = e @ e, 2 * q @ e, q @ q - R * R
    roots = np.roots([A, B, C])
    t = min(r for r in roots.real if r > 0)          # the first crossing of that circle
    xc = p0 + t * d
    np.testing.assert_allclose(x[0], xc, rtol=0, atol=1e-12)
    u = np.cross([w, 0.0, 0.0], xc - np.array([xc[0], 6.0, 6.0]))    # omega x r about the axis
    np.testing.assert_allclose(v[0], 2 * u - vel, rtol=0, atol=1e-12)


def test_frozen_layer_turns_with_its_cylinder():
    # a turning cylinder's frozen particles turn rigidly with it, omega dt per
    # step about the axis, and carry omega x r; the resting cylinder's stay
    cells = (4, 12, 12)
    p0 = oracle.make_params(a=0.0, gamma=0.0, kT=0.0, dt=0.05)
    x = np.array([[1.0, 6.0 + 5.5, 6.0], [1.0, 6.0, 6.0 - 1.6], [1.0, 6.0, 6.0 + 3.5], [1.0, 6.0 - 3.5, 6.0]])
    frozen = np.array([1, 1, 0, 0], dtype=np.uint8)
    p = _couette_params(p0, frozen, 2.0, 5.0, 0.0, 0.3)
    v = np.zeros((4, 3))
    v[:2] = oracle.wall_velocity(x[:2], cells, p)
    ids = np.arange(4, dtype=np.uint32)
    oracle.step(x, v, ids, cells, p, 0, 0, 10, want_diag=False)
    ang = 0.3 * 0.05 * 10
    np.testing.assert_allclose(x[0], [1.0, 6.0 + 5.5 * math.cos(ang), 6.0 + 5.5 * math.sin(ang)], rtol=0, atol=1e-12)
    np.testing.assert_allclose(v[0], np.cross([0.3, 0.0, 0.0], x[0] - [1.0, 6.0, 6.0]), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(x[1], [1.0, 6.0, 6.0 - 1.6])          # inner cylinder at rest
    np.testing.assert_array_equal(v[1], 0.0)


def _annulus_state(cells, rho, params, seed, equil_steps=300):
    """Equilibrated fluid cut into an annulus: within r_c behind either
    cylinder frozen, carrying the wall's velocity; farther out dropped."""
    pos, vel = inputs.uniform_state(cells, density=rho, seed=seed)
    x, v = pos.astype(np.float64), vel.astype(np.float64)
    ids = np.arange(len(x), dtype=np.uint32)
    free = oracle.make_params(a=params.a, gamma=params.gamma, kT=params.kT, dt=params.dt)
    oracle.step(x, v, ids, cells, free, seed, 0, equil_steps, want_diag=False)
    s = oracle.sdf(x, cells, params)
    keep = s <= 1.0
    x, v = x[keep].copy(), v[keep].copy()
    frozen = (s[keep] > 0.0).astype(np.uint8)
    v[frozen == 1] = oracle.wall_velocity(x[frozen == 1], cells, params)
    return x, v, frozen


@pytest.mark.slow
def test_taylor_couette_profile():
    """Inner cylinder at rest, outer turning (the paper's Sec. 4.3 setting):
    the azimuthal velocity follows A r + B / r with A, B from the radii and
    angular velocities (the general form of Eq. 12)."""
    cells, rho = (4, 18, 18), 3.0
    r_in, r_out, w_out = 3.0, 7.5, 0.06
    base = oracle.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    geo = _couette_params(base, None, r_in, r_out, 0.0, w_out)
    x, v, frozen = _annulus_state(cells, rho, geo, 54)
    p = _couette_params(base, frozen, r_in, r_out, 0.0, w_out)
    ids = np.arange(len(x), dtype=np.uint32)
    oracle.step(x, v, ids, cells, p, 54, 0, 3000, want_diag=False)          # spin-up, ~5 relaxation times
    edges = np.linspace(r_in, r_out, 10)
    acc, cnt = np.zeros(9), np.zeros(9)
    fl = frozen == 0
    for k in range(80):
        oracle.step(x, v, ids, cells, p, 54, 3000 + 100 * k, 100, want_diag=False)
        c = x[fl][:, 1:] - 9.0
        r = np.hypot(c[:, 0], c[:, 1])
        vt = (c[:, 0] * v[fl][:, 2] - c[:, 1] * v[fl][:, 1]) / r
        b = np.clip(np.searchsorted(edges, r) - 1, 0, 8)
        np.add.at(acc, b, vt)
        np.add.at(cnt, b, 1)
    rm = 0.5 * (edges[1:] + edges[:-1])
    prof = acc / cnt
    A = w_out * r_out ** 2 / (r_out ** 2 - r_in ** 2)
    B = -w_out * r_in ** 2 * r_out ** 2 / (r_out ** 2 - r_in ** 2)
    want = A * rm + B / rm
    print("taylor-couette", np.round(prof, 4), np.round(want, 4))
    inner = (rm > r_in + 0.6) & (rm < r_out - 0.6)
    assert np.max(np.abs(prof[inner] - want[inner])) < 0.08 * w_out * r_out
