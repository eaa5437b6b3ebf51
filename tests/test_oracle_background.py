"""Pins of the coupled-quintessence background oracle (Sec. 4.3, background
cosmology solver) against things other than itself: the radiation density of
a 2.7255 K black body, the LCDM limit in closed form, the identity
dE/dN = 2D that ties the Friedmann and Raychaudhuri forms to the field
equation, insensitivity to the initial field, and H(a=1) = H0 after the
shooting."""
import math

import numpy as np
import pytest

from oracle import cq_background as bg

OM, H = 0.3089, 0.6774


def test_photon_density_of_cmb():
    # Omega_gamma h^2 = 2.47e-5 for T_CMB = 2.7255 K (standard value)
    og_h2 = bg.omega_r(H, n_eff=0.0) * H * H
    assert abs(og_h2 / 2.4728e-5 - 1.0) < 2e-3
    # massless neutrinos: 3.046 * 7/8 (4/11)^(4/3) = 0.6918 of the photons
    assert abs(bg.omega_r(H) / bg.omega_r(H, n_eff=0.0) - 1.69179) < 1e-4


def test_lcdm_limit_closed_form():
    """alpha = beta = 0: constant potential, no coupling, the field stays put;
    lambda^2 = 3 Omega_Lambda and H(a) is the LCDM expansion rate."""
    lam, orr, tab = bg.table(OM, H, 0.0, 0.0, n_table=200)
    ol = 1.0 - OM - orr
    assert abs(lam * lam / 3.0 / ol - 1.0) < 1e-10
    a = tab[:, 0]
    e = orr * a ** -4 + OM * a ** -3 + ol
    assert np.allclose(tab[:, 1], np.sqrt(e), rtol=1e-10, atol=0)
    hdot = 0.5 * (-4 * orr * a ** -4 - 3 * OM * a ** -3)
    assert np.allclose(tab[:, 2], hdot, rtol=1e-9, atol=0)
    assert np.all(tab[:, 3] == 1e-6) and np.all(tab[:, 4] == 0.0)


@pytest.mark.parametrize("alpha,beta", [(0.1, -0.1), (0.1, -0.2), (0.5, -0.2)])
def test_friedmann_raychaudhuri_and_field_equation_agree(alpha, beta):
    """Along the solution, the derivative of E = (aH/H0)^2 from the Friedmann
    form equals 2D = 2 a^2 (H^2 + dH/dt)/H0^2 from the Raychaudhuri form; the
    identity holds only when the potential terms of both and the potential
    force of the field equation carry consistent coefficients."""
    nt = 40001
    lam, orr, tab = bg.table(OM, H, alpha, beta, n_table=nt)
    a = tab[:, 0]
    N = np.log(a)
    E = (a * tab[:, 1]) ** 2
    D = a * a * (tab[:, 1] ** 2 + tab[:, 2])
    dE = (E[2:] - E[:-2]) / (N[2:] - N[:-2])
    # relative to E: D passes through zero where the expansion starts to accelerate
    rel = np.abs(dE - 2 * D[1:-1]) / E[1:-1]
    assert rel.max() < 1e-6
    # the same check with the potential coefficient lambda^2 instead of
    # lambda^2/3 in E and D fails: the pin can see that reading
    P, Q = tab[:, 3], tab[:, 4] * a
    pot = lam * lam * np.exp(2 * N) * P ** (-alpha)
    mat = OM * np.exp(-N) * np.exp(beta * P)
    rad = orr * np.exp(-2 * N)
    E2 = (rad + mat + pot) / (1 - Q * Q / 6)
    D2 = -Q * Q * E2 / 3 + pot - rad - 0.5 * mat
    dE2 = (E2[2:] - E2[:-2]) / (N[2:] - N[:-2])
    assert (np.abs(dE2 - 2 * D2[1:-1]) / E2[1:-1]).max() > 1e-3


def test_h0_today_and_initial_field_insensitivity():
    alpha, beta = 0.1, -0.2
    lam1, orr, t1 = bg.table(OM, H, alpha, beta, n_table=64, phi_init=1e-6)
    assert abs(t1[-1, 0] - 1.0) < 1e-15 and abs(t1[-1, 1] - 1.0) < 1e-11
    lam2, _, t2 = bg.table(OM, H, alpha, beta, n_table=64, phi_init=1e-8)
    lam3, _, t3 = bg.table(OM, H, alpha, beta, n_table=64, phi_init=1e-5, dphi_init=1e-6)
    for lam, t in ((lam2, t2), (lam3, t3)):
        assert abs(lam / lam1 - 1.0) < 1e-6
        assert abs(t[-1, 3] / t1[-1, 3] - 1.0) < 1e-5
    # the coupling (beta < 0) and the runaway potential push phi-bar up
    assert np.all(np.diff(t1[:, 3]) > 0) and 0.05 < t1[-1, 3] < 5.0


def test_interp_is_linear_in_a():
    lam, orr, tab = bg.table(OM, H, 0.1, -0.1, n_table=300)
    r = 200
    am = 0.5 * (tab[r, 0] + tab[r + 1, 0])
    assert np.allclose(bg.interp(tab, am), 0.5 * (tab[r] + tab[r + 1]), rtol=1e-14, atol=0)
