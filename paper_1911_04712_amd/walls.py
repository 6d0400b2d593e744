"""Walls: frozen-particle layers cut from an equilibrated fluid, and the pipe
Poiseuille viscosity measurement.

A wall is the zero isosurface of a signed distance function (negative in the
fluid) with a layer of frozen particles of thickness r_c = 1 behind it that
interact through the usual DPD forces and never move (Sec. 2.3); fluid
particles that cross it bounce back (Sec. 3.3).  The frozen layer must have
the fluid's own structure, so it is cut from a periodic fluid equilibrated
with the same parameters: particles with sdf <= 0 stay fluid, those with
0 < sdf <= 1 are frozen (velocity 0) and the rest are dropped.

Table 1's viscosities come from pipe flow (Sec. 4.1): a uniform body force f
along the pipe of radius R drives Poiseuille flow with mean velocity
u_avg = rho f R^2 / (8 eta).

    python -m paper_1911_04712_amd.walls           # Table 1 through pipe flow
    python -m paper_1911_04712_amd.walls couette   # the Taylor-Couette test
"""
import json
import math
import sys

import numpy as np

from . import dpd


def carve(cells, rho, params, wall_kind, wall_h, seed=1, equil_steps=1000, wall_r_in=0.0):
    """Equilibrate a periodic box of the fluid `params` describes (no walls,
    no body force), then cut walls into it.  Returns (pos, vel, frozen) in id
    order, ready for a box whose params carry the same wall (dpd_set_frozen
    then gives the frozen particles their wall's velocity)."""
    n = int(round(rho * cells[0] * cells[1] * cells[2]))
    p0 = dpd.make_params(a=params.a, gamma=params.gamma, kT=params.kT, dt=params.dt, mass=params.mass,
                         kexp=params.kexp, flow_axis=params.flow_axis, grad_axis=params.grad_axis)
    with dpd.Box(cells, n, params=p0, seed=seed) as b:
        b.init_random(params.kT, seed)
        b.step(equil_steps)
        pos, vel = b.read(dpd.POS), b.read(dpd.VEL)
        pw = dpd.make_params(a=params.a, gamma=params.gamma, kT=params.kT, dt=params.dt, mass=params.mass,
                             kexp=params.kexp, flow_axis=params.flow_axis, grad_axis=params.grad_axis,
                             wall_kind=wall_kind, wall_h=wall_h, wall_r_in=wall_r_in)
        b.set_params(pw)
        sdf = b.wall_sdf()
    keep = sdf <= 1.0
    frozen = sdf[keep] > 0.0
    vel = vel[keep].copy()
    vel[frozen] = 0.0
    return np.ascontiguousarray(pos[keep]), np.ascontiguousarray(vel), frozen


def pipe_viscosity(a, gamma, rho, k, kT, dt, eta_guess, R=8.0, length=16, seed=1, warm_tau=6.0, avg_tau=6.0,
                   f=None, rc=1.0):
    """Pipe Poiseuille viscosity on the GPU (Sec. 4.1): a pipe of radius R
    (cells of edge r_c) along x, uniform drive f, eta = rho f R^2 / (8 u_avg)
    with u_avg the mean flow velocity of the fluid particles over avg_tau
    momentum relaxation times rho R^2 / (5.78 eta) after warm_tau of them.
    eta_guess sets only f (a peak flow of 0.2 sqrt(kT)) and the run length.
    A cutoff rc != 1 runs in units of rc (the same exact change of units as
    the periodic measurement)."""
    if rc != 1.0:
        from .viscosity import unit_cutoff
        a1, g1, rho1, kT1, _ = unit_cutoff(a, gamma, rho, kT, 0.0, rc)
        r = pipe_viscosity(a1, g1, rho1, k, kT1, dt, eta_guess * rc, R, length, seed, warm_tau, avg_tau,
                           None if f is None else f / rc)
        r.update(eta=r["eta"] / rc, f=r["f"] * rc, u_avg=r["u_avg"] * rc)
        return r
    side = int(math.ceil(2 * (R + 1.0))) + 2
    cells = (int(length), side, side)
    if f is None:
        f = 0.2 * math.sqrt(kT) * 4.0 * eta_guess / (rho * R * R)       # peak 2 u_avg = rho f R^2 / (4 eta)
    tau = rho * R * R / (5.783 * eta_guess)                             # slowest mode, j_0,1^2 = 5.783
    base = dpd.make_params(a=a, gamma=gamma, kT=kT, dt=dt, kexp=k)
    pos, vel, frozen = carve(cells, rho, base, dpd.WALL_PIPE, R, seed=seed,
                             equil_steps=max(200, int(round(2.0 / dt))))
    p = dpd.make_params(a=a, gamma=gamma, kT=kT, dt=dt, kexp=k, body_f=f, flags=dpd.FLAG_BODY_UNIFORM,
                        wall_kind=dpd.WALL_PIPE, wall_h=R)
    nfluid = int((~frozen).sum())
    with dpd.Box(cells, len(pos), params=p, seed=seed + 1000) as b:
        b.set_state(pos, vel)
        b.set_frozen(frozen)
        b.step(int(round(warm_tau * tau / dt)))
        b.reset_accumulators()
        nsteps = int(round(avg_tau * tau / dt))
        b.step(nsteps)
        st = b.stats()
    u_avg = st["sum_momentum"][0] / st["nsamples"] / (nfluid * p.mass)
    rho_fluid = nfluid / (math.pi * R * R * length)
    eta = rho_fluid * f * R * R / (8.0 * u_avg)
    return {"eta": eta, "u_avg": u_avg, "f": f, "R": R, "length": length, "cells": list(cells),
            "fluid": nfluid, "frozen": int(frozen.sum()), "rho_fluid": rho_fluid, "steps": nsteps,
            "kT_centred": st["sum_kT_centred"] / st["nsamples"]}


def couette_profile(r, r_in, r_out, omega_in, omega_out):
    """Azimuthal velocity between coaxial cylinders (Sec. 4.3, Eq. 12 in
    its general form): A r + B / r with A = (omega_out R_out^2 - omega_in
    R_in^2) / (R_out^2 - R_in^2), B = (omega_in - omega_out) R_in^2 R_out^2 /
    (R_out^2 - R_in^2)."""
    d = r_out ** 2 - r_in ** 2
    A = (omega_out * r_out ** 2 - omega_in * r_in ** 2) / d
    B = (omega_in - omega_out) * r_in ** 2 * r_out ** 2 / d
    return A * np.asarray(r) + B / np.asarray(r)


def taylor_couette(r_in=10.0, r_out=32.0, omega_in=0.0, omega_out=0.01, rho=10.0, a=10.0, gamma=10.0, kT=0.5,
                   k=0.125, dt=0.001, length=6, eta_guess=49.0, warm_tau=5.0, avg_tau=5.0, samples=100, nbins=22,
                   seed=1):
    """Taylor-Couette flow on the GPU (Sec. 4.3; the defaults are the
    paper's setting): fluid between coaxial cylinders along x, frozen layers
    cut from the equilibrated fluid, the cylinders turning at omega_in and
    omega_out.  After warm_tau momentum-diffusion times rho (R_out - R_in)^2
    / (pi^2 eta) the azimuthal velocity of the fluid particles is averaged
    over avg_tau more in radial bins and returned with the analytic profile."""
    side = int(math.ceil(2 * (r_out + 1.0))) + 2
    cells = (int(length), side, side)
    base = dpd.make_params(a=a, gamma=gamma, kT=kT, dt=dt, kexp=k)
    pos, vel, frozen = carve(cells, rho, base, dpd.WALL_CYLINDERS, r_out, seed=seed,
                             equil_steps=max(200, int(round(2.0 / dt))), wall_r_in=r_in)
    p = dpd.make_params(a=a, gamma=gamma, kT=kT, dt=dt, kexp=k, wall_kind=dpd.WALL_CYLINDERS, wall_h=r_out,
                        wall_r_in=r_in, omega_in=omega_in, omega_out=omega_out)
    tau = rho * (r_out - r_in) ** 2 / (math.pi ** 2 * eta_guess)
    edges = np.linspace(r_in, r_out, nbins + 1)
    acc, cnt = np.zeros(nbins), np.zeros(nbins)
    fluid = ~frozen
    centre = np.array([cells[1], cells[2]], dtype=np.float64) / 2
    with dpd.Box(cells, len(pos), params=p, seed=seed + 1000) as b:
        b.set_state(pos, vel)
        b.set_frozen(frozen)
        b.step(int(round(warm_tau * tau / dt)))
        every = max(1, int(round(avg_tau * tau / dt / samples)))
        for _ in range(samples):
            b.step(every)
            x = b.read(dpd.POS)[fluid].astype(np.float64)
            v = b.read(dpd.VEL_CENTRED)[fluid].astype(np.float64)
            c = x[:, 1:] - centre
            r = np.hypot(c[:, 0], c[:, 1])
            vt = (c[:, 0] * v[:, 2] - c[:, 1] * v[:, 1]) / r
            bi = np.clip(np.searchsorted(edges, r) - 1, 0, nbins - 1)
            np.add.at(acc, bi, vt)
            np.add.at(cnt, bi, 1)
        st = b.stats()
    rm = 0.5 * (edges[1:] + edges[:-1])
    return {"r": rm, "v": acc / np.maximum(cnt, 1), "v_analytic": couette_profile(rm, r_in, r_out, omega_in, omega_out),
            "fluid": int(fluid.sum()), "frozen": int(frozen.sum()), "cells": list(cells),
            "kT_centred": st["kT_centred"], "steps": int(round(warm_tau * tau / dt)) + samples * every}


def main(argv=None):
    """Table 1 through pipe flow, R = 20 (the paper's radius) unless given,
    in the units of the table (R / r_c cells for the r_c = 1.5 rows);
    `couette` instead runs the paper's Taylor-Couette setting."""
    if argv and argv[0] == "couette":
        r = taylor_couette()
        dev = np.abs(r["v"] - r["v_analytic"])
        print(json.dumps({"r": np.round(r["r"], 3).tolist(), "v": np.round(r["v"], 5).tolist(),
                          "v_analytic": np.round(r["v_analytic"], 5).tolist(), "max_abs_dev": float(dev.max()),
                          "max_dev_over_wall_speed": float(dev.max() / (0.01 * 32.0)), "fluid": r["fluid"],
                          "frozen": r["frozen"], "cells": r["cells"], "steps": r["steps"],
                          "kT_centred": r["kT_centred"]}), flush=True)
        return 0
    from .viscosity import TABLE1
    R = float(argv[0]) if argv else 20.0
    rows = [int(x) for x in argv[1].split(",")] if argv and len(argv) > 1 else range(len(TABLE1))
    for i in rows:
        row = TABLE1[i]
        par = {k: row[k] for k in ("a", "gamma", "rho", "k", "kT", "dt")}
        rc = row.get("rc", 1.0)
        runs = []
        for s in (1, 2, 3):
            runs.append(pipe_viscosity(**par, eta_guess=sum(row["eta_paper"]) / 2, R=R / rc, seed=s, rc=rc))
            print(json.dumps({"row": i, "seed": s, "eta": runs[-1]["eta"], "steps": runs[-1]["steps"]}), flush=True)
        etas = np.array([r["eta"] for r in runs])
        print(json.dumps({"row": i, "params": dict(par, rc=rc), "R": R, "eta": float(etas.mean()),
                          "eta_err": float(etas.std(ddof=1) / math.sqrt(len(etas))),
                          "eta_runs": [round(float(e), 4) for e in etas], "eta_paper": row["eta_paper"],
                          "eta_ref": row["eta_ref"], "fluid": runs[0]["fluid"], "frozen": runs[0]["frozen"],
                          "rho_fluid": runs[0]["rho_fluid"], "kT_centred": runs[0]["kT_centred"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
