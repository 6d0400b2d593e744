"""Viscosity of the DPD fluid from periodic (reverse) Poiseuille flow.

The paper measures the viscosity of its fluids with Poiseuille flow
(Sec. 4.1, Table 1: eta = rho f R^2 / (8 u_avg) in a pipe) and introduces the
wall-free periodic form (Sec. 4.2, Eq. 11): a body force -f along the flow
axis where the gradient coordinate is <= L/2 and +f above drives two
counter-flowing parabolas.  For a Newtonian fluid of mass density rho the
flow-axis velocity is, with s = y mod L/2,

    v(y) = -/+ rho f s (L/2 - s) / (2 eta)   (lower / upper half),

so eta follows from a least-squares fit of the measured profile to that
shape.  The profile is accumulated on the GPU (fixed point, per slab of the
gradient axis, time-centred velocities) in blocks whose scatter gives the
statistical error.

    python -m paper_1911_04712_amd.viscosity      # the r_c = 1 rows of Table 1
"""
import json
import math
import sys

import numpy as np

from . import dpd

# Table 1: DPD parameters, the paper's measured range and the literature
# value it compares with.  TABLE1_RC1 holds the r_c = 1 rows; the two
# r_c = 1.5 rows follow in TABLE1.
TABLE1_RC1 = [
    dict(a=0.9375, gamma=115.6, rho=4, k=1.0, kT=0.05, dt=0.01, eta_paper=(4.4, 4.6), eta_ref=4.7),
    dict(a=6.0, gamma=20.0, rho=3, k=0.15, kT=0.1, dt=0.002, eta_paper=(8.0, 8.3), eta_ref=8.1),
    dict(a=25.0, gamma=6.75, rho=3, k=1.0, kT=1.0, dt=0.04, eta_paper=(0.89, 0.9), eta_ref=0.91),
    dict(a=18.75, gamma=4.5, rho=4, k=1.0, kT=1.0, dt=0.005, eta_paper=(1.07, 1.08), eta_ref=1.08),
    dict(a=18.75, gamma=4.5, rho=4, k=0.25, kT=1.0, dt=0.005, eta_paper=(2.44, 2.45), eta_ref=2.59),
    dict(a=0.0, gamma=20.25, rho=6, k=1.0, kT=0.5, dt=0.01, eta_paper=(2.08, 2.1), eta_ref=2.09),
]
TABLE1 = TABLE1_RC1 + [
    dict(a=4.0, gamma=8.0, rho=3, k=0.15, kT=0.1, dt=0.001, rc=1.5, eta_paper=(24.7, 26.3), eta_ref=26.3),
    dict(a=4.0, gamma=40.0, rho=3, k=0.15, kT=0.1, dt=0.0002, rc=1.5, eta_paper=(122.5, 129.5), eta_ref=126.0),
]
# Boxes of the periodic measurement: 16^3 cells, 24^3 for the r_c = 1.5 rows,
# whose dissipation-dominated viscosity still moved by 5 % from 16^3 to 24^3
# (116.7 -> 122.6 for the last row) while the others stay within the noise.
CELLS = {6: (24, 24, 24), 7: (24, 24, 24)}


def unit_cutoff(a, gamma, rho, kT, f, rc):
    """The same fluid with r_c as the length unit (an exact change of units;
    time and mass are kept): lengths and velocities scale by 1/r_c, forces
    by 1/r_c, so a' = a / r_c, gamma' = gamma, sigma' = sigma / r_c
    (kT' = kT / r_c^2), number density rho' = rho r_c^3, body force
    f' = f / r_c; a viscosity measured in these units is eta' = eta r_c."""
    return a / rc, gamma, rho * rc ** 3, kT / rc ** 2, f / rc


def _shape(nb, L):
    """Bin average of sign(y) s (L/2 - s), s = y mod L/2, over nb slabs."""
    g = np.empty(nb)
    for i in range(nb):
        yy = np.linspace(i * L / nb, (i + 1) * L / nb, 201)
        s = np.mod(yy, L / 2)
        g[i] = np.mean(np.where(yy <= L / 2, -1.0, 1.0) * s * (L / 2 - s))
    return g


def fit_eta(profiles, rho, f, L, skip=1.0):
    """profiles: blocks x slabs of mean flow velocity.  Returns (eta, its
    standard error, reduced chi^2 of the fit).

    The DPD stress reaches one cutoff (here 1 length unit), so within that
    distance of a plane where the body force flips the profile bends away
    from the two parabolas and, further out, each half is still the exact
    parabola (a symmetric stress kernel maps a linear shear rate to eta
    times itself) shifted by a constant.  The fit therefore leaves out slabs
    whose centre is within `skip` of y = 0, L/2, L and gives each half its
    own offset: v = A_half + c sign(y) s (L/2 - s) with c = rho f / (2 eta)."""
    prof = np.asarray(profiles)
    mean = prof.mean(axis=0)
    nb = len(mean)
    err = prof.std(axis=0, ddof=1) / math.sqrt(len(prof))
    g = _shape(nb, L)
    yc = (np.arange(nb) + 0.5) * L / nb
    dist = np.minimum.reduce([yc, np.abs(yc - L / 2), L - yc])
    use = dist > skip
    upper = yc > L / 2
    X = np.stack([g, ~upper, upper], axis=1).astype(np.float64)[use]
    w = 1.0 / np.maximum(err[use], 1e-12) ** 2
    Xw = X * w[:, None]
    cov = np.linalg.inv(X.T @ Xw)
    beta = cov @ (Xw.T @ mean[use])
    c, dc = beta[0], math.sqrt(cov[0, 0])
    chi2 = float(np.sum(w * (mean[use] - X @ beta) ** 2) / max(int(use.sum()) - 3, 1))
    eta = rho * f / (2.0 * c)
    return eta, eta * dc / abs(c), chi2


def measure(a, gamma, rho, k, kT, dt, eta_guess, f=None, cells=(16, 16, 16), warm_tau=10.0, blocks=10,
            block_tau=3.0, seed=1, rc=1.0):
    """Periodic-Poiseuille viscosity on the GPU.  Flow along x, gradient along
    y (cells[1] slabs of one cell).  The expected viscosity eta_guess sets
    only the drive and the run length: f gives a peak flow of about
    0.2 sqrt(kT), and the warm-up and each of the averaging blocks last
    warm_tau and block_tau momentum relaxation times rho (L/2)^2 / (pi^2 eta).
    eta_err is the block-scatter error of one run; slow flow fluctuations
    make runs with other seeds scatter about three times more, so main()
    reports the scatter over seeds.  A cutoff rc != 1 is run in units of
    rc (unit_cutoff): cells are then cells of edge rc, and eta, eta_err and
    f are returned in the original units."""
    if rc != 1.0:
        a1, g1, rho1, kT1, _ = unit_cutoff(a, gamma, rho, kT, 0.0, rc)
        r = measure(a1, g1, rho1, k, kT1, dt, eta_guess * rc, None if f is None else f / rc, cells, warm_tau,
                    blocks, block_tau, seed)
        r.update(eta=r["eta"] / rc, eta_err=r["eta_err"] / rc, f=r["f"] * rc, kT_centred=r["kT_centred"] * rc * rc)
        return r
    L = float(cells[1])
    n = int(round(rho * cells[0] * cells[1] * cells[2]))
    tau = rho * (L / 2) ** 2 / (math.pi ** 2 * eta_guess)
    if f is None:
        f = 0.2 * math.sqrt(kT) * 32.0 * eta_guess / (rho * L * L)
    warm_steps = int(round(warm_tau * tau / dt))
    block_steps = max(100, int(round(block_tau * tau / dt)))
    nb = cells[1]
    p = dpd.make_params(a=a, gamma=gamma, kT=kT, dt=dt, body_f=f, flow_axis=0, grad_axis=1, profile_bins=nb,
                        kexp=k)
    box = dpd.Box(cells, n, params=p, seed=seed)
    try:
        box.init_random(kT, seed)
        box.step(warm_steps)
        profiles = []
        for _ in range(blocks):
            box.reset_accumulators()
            box.step(block_steps)
            sv, cn = box.profile()
            profiles.append(sv / np.maximum(cn, 1.0))
        st = box.stats()
    finally:
        box.close()
    eta, deta, chi2 = fit_eta(profiles, rho, f, L)
    return {"eta": eta, "eta_err": deta, "chi2": chi2, "f": f, "particles": n, "cells": list(cells),
            "steps": warm_steps + blocks * block_steps,
            "kT_centred": st["sum_kT_centred"] / max(st["nsamples"], 1)}      # mean over the last block


def main(argv=None):
    seeds = range(1, 5)
    rows = [int(x) for x in argv[0].split(",")] if argv else range(len(TABLE1))
    for i in rows:
        row = TABLE1[i]
        par = {k: row[k] for k in ("a", "gamma", "rho", "k", "kT", "dt")}
        par["rc"] = row.get("rc", 1.0)
        runs = [measure(**par, eta_guess=sum(row["eta_paper"]) / 2, seed=s, cells=CELLS.get(i, (16, 16, 16)))
                for s in seeds]
        etas = np.array([r["eta"] for r in runs])
        print(json.dumps({"row": i, "params": par, "eta": float(etas.mean()),
                          "eta_err": float(etas.std(ddof=1) / math.sqrt(len(etas))),
                          "eta_runs": [round(float(e), 4) for e in etas], "eta_paper": row["eta_paper"],
                          "eta_ref": row["eta_ref"], "cells": runs[0]["cells"], "particles": runs[0]["particles"],
                          "steps_per_run": runs[0]["steps"], "f": runs[0]["f"],
                          "kT_centred": float(np.mean([r["kT_centred"] for r in runs]))}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
