"""Viscosity of the DPD fluid on the GPU from periodic Poiseuille flow
(Sec. 4.2, Eq. 11) against the paper's Table 1 (r_c = 1 rows, kernel
exponents k = 1, 1/4 and 0.15).  The paper measures in a pipe; the
periodic form needs no walls and measures the same Newtonian viscosity, so
the bar is 10 % of the paper's value (its own range and the literature value
it compares with differ by up to 6 %; one run of this length scatters by
about 3 % from seed to seed)."""
import sys

import pytest

from paper_1911_04712_amd import viscosity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("row", [2, 4, 1], ids=["groot_k1", "fan_k0.25", "fedosov_k0.15"])
def test_viscosity_matches_table1(row):
    r = viscosity.TABLE1_RC1[row]
    eta_p = sum(r["eta_paper"]) / 2
    par = {k: r[k] for k in ("a", "gamma", "rho", "k", "kT", "dt")}
    print(f"[viscosity] row {row}: {par}", file=sys.stderr, flush=True)
    m = viscosity.measure(**par, eta_guess=eta_p, seed=70 + row)
    print(f"[viscosity] eta = {m['eta']:.3f} +- {m['eta_err']:.3f} (paper {r['eta_paper']}), chi2 {m['chi2']:.2f}",
          file=sys.stderr, flush=True)
    # the time-centred kT estimate carries an O(dt) error (a few % at dt = 0.04)
    assert abs(m["kT_centred"] - r["kT"]) < 0.05 * r["kT"]
    assert m["chi2"] < 6.0                      # the two-half parabola fits
    assert abs(m["eta"] - eta_p) < 0.10 * eta_p
