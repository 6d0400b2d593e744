"""Host-side profile fits of the viscosity measurements (no GPU, no oracle).

The periodic-Poiseuille fit leaves out the slabs within one cutoff of the
planes where the drive flips and gives each half its own offset; a profile
that is the exact two-half parabola away from those planes, with the planes'
neighbourhood bent and each half shifted, must give back the viscosity it
was made with.
"""
import numpy as np
import pytest

from paper_1911_04712_amd.viscosity import _shape, fit_eta, unit_cutoff


@pytest.mark.parametrize("eta,L", [(0.9, 16.0), (8.2, 16.0), (120.0, 24.0)])
def test_fit_recovers_eta_despite_kinks_and_offsets(eta, L):
    nb = int(L)
    rho, f = 3.0, 0.01
    g = _shape(nb, L)
    v = rho * f / (2 * eta) * g
    yc = (np.arange(nb) + 0.5) * L / nb
    bent = v.copy()
    bent[yc < L / 2] += 0.02 * v.max()
    bent[yc > L / 2] -= 0.02 * v.max()
    for k in (0, nb // 2 - 1, nb // 2, nb - 1):          # slabs touching a plane
        bent[k] *= 0.6
    rng = np.random.default_rng(1)
    prof = bent[None, :] + rng.normal(0, 1e-3 * v.max(), size=(12, nb))
    e, de, chi2 = fit_eta(prof, rho, f, L)
    assert e == pytest.approx(eta, rel=5 * de / e + 1e-3)
    assert chi2 < 3.0


def test_unit_cutoff_is_a_change_of_units():
    # r_c as the unit of length: a/r_c, gamma, rho r_c^3, kT/r_c^2, f/r_c
    a, g, rho, kT, f = unit_cutoff(4.0, 8.0, 3.0, 0.1, 0.3, 1.5)
    assert (a, g, rho, kT, f) == pytest.approx((4.0 / 1.5, 8.0, 3.0 * 3.375, 0.1 / 2.25, 0.2))
