"""FP64 oracle for the coupled-quintessence background (Sec. 4.3, "background
cosmology solver"): the homogeneous field phi-bar(a), H(a), and the lambda of
eq:csf_param_lambda that makes H(a=1) = H0.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: it shares nothing with
the HIP library.  The integrator is scipy's DOP853 (a library primitive used
as one step); the shooting on lambda is scipy's brentq.

Equations (time variable N = ln a, E = (conformal H / H0)^2,
D = conformal-time derivative of conformal H over H0^2, P = phi-bar,
Q = dP/dN), as printed in the code-unit forms that follow
eq:csf_background_Raychaudhuri, with the printed potential coefficient read as
lambda^2/3 (see ``POTENTIAL_COEF``):

    E = [Om_r e^-2N + Om_m e^-N e^{beta P} + (lambda^2/3) e^2N P^-alpha] / (1 - Q^2/6)
    D = -(1/3) Q^2 E + (lambda^2/3) e^2N P^-alpha - Om_r e^-2N - (1/2) Om_m e^-N e^{beta P}
    E dQ/dN + (2E + D) Q - alpha lambda^2 e^2N P^-(1+alpha) + 3 beta Om_m e^-N e^{beta P} = 0

(eq:csf_background_eom_codeunit with the same reading: its potential force
3 alpha (lambda^2/3) equals the alpha lambda^2 of eq:csf_eom_code.)
"""
import math

import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

# CODATA 2018 / IAU values
K_B = 1.380649e-23  # J/K
HBAR = 1.054571817e-34  # J s
C_LIGHT = 299792458.0  # m/s
G_NEWTON = 6.67430e-11  # m^3 kg^-1 s^-2
MPC = 3.0856775814913673e22  # m


def potential_coef(lam):
    """Coefficient of e^2N P^-alpha in E and D.  The paper prints "lambda"
    there; with V = M_Pl^2 H0^2 lambda^2 phi^-alpha (eq:csf_potential,
    eq:csf_param_lambda) the Friedmann equation carries V / (3 M_Pl^2), so the
    coefficient is lambda^2 / 3 (the LCDM limit alpha = beta = 0 then gives
    lambda^2 = 3 Omega_Lambda)."""
    return lam * lam / 3.0


def omega_r(h, t_cmb=2.7255, n_eff=3.046):
    """Present radiation density parameter: CMB photons at t_cmb plus n_eff
    massless neutrino species, each 7/8 (4/11)^(4/3) of the photons."""
    rho_gamma = (math.pi ** 2 / 15.0) * (K_B * t_cmb) ** 4 / (HBAR * C_LIGHT) ** 3 / C_LIGHT ** 2
    h0 = 100.0 * h * 1e3 / MPC  # 1/s
    rho_crit = 3.0 * h0 * h0 / (8.0 * math.pi * G_NEWTON)
    og = rho_gamma / rho_crit
    return og * (1.0 + n_eff * 7.0 / 8.0 * (4.0 / 11.0) ** (4.0 / 3.0))


def _e_d(N, P, Q, lam, om, orr, alpha, beta):
    pot = potential_coef(lam) * math.exp(2 * N) * P ** (-alpha)
    mat = om * math.exp(-N) * math.exp(beta * P)
    rad = orr * math.exp(-2 * N)
    E = (rad + mat + pot) / (1.0 - Q * Q / 6.0)
    D = -Q * Q * E / 3.0 + pot - rad - 0.5 * mat
    return E, D


def _rhs(lam, om, orr, alpha, beta):
    def f(N, y):
        P, Q = y
        E, D = _e_d(N, P, Q, lam, om, orr, alpha, beta)
        force = alpha * lam * lam * math.exp(2 * N) * P ** (-(1 + alpha)) \
            - 3 * beta * om * math.exp(-N) * math.exp(beta * P)
        return [Q, (force - (2 * E + D) * Q) / E]
    return f


def evolve(lam, om, orr, alpha, beta, z_init=1e5, phi_init=1e-6, dphi_init=0.0, n_eval=None):
    """Integrate from a = 1/(1+z_init) to a = 1; returns the scipy solution."""
    n0 = -math.log1p(z_init)
    t_eval = None if n_eval is None else np.asarray(n_eval, dtype=float)
    return solve_ivp(_rhs(lam, om, orr, alpha, beta), (n0, 0.0), [phi_init, dphi_init],
                     method="DOP853", rtol=1e-12, atol=1e-15, t_eval=t_eval)


def h_today(lam, om, orr, alpha, beta, **kw):
    s = evolve(lam, om, orr, alpha, beta, **kw)
    P, Q = s.y[0, -1], s.y[1, -1]
    return math.sqrt(_e_d(0.0, P, Q, lam, om, orr, alpha, beta)[0])


def shoot_lambda(om, orr, alpha, beta, **kw):
    """lambda such that H(a=1) = H0 (the paper adjusts lambda until the two
    agree); brentq on H(1)/H0 - 1 over a bracket grown from lambda = 1."""
    g = lambda lam: h_today(lam, om, orr, alpha, beta, **kw) - 1.0
    lo, hi = 0.0, 1.0
    while g(hi) < 0.0:
        lo, hi = hi, 2.0 * hi
    return brentq(g, lo, hi, xtol=1e-14, rtol=1e-14)


def table(om, h, alpha, beta, n_table=1024, z_init=1e5, phi_init=1e-6, dphi_init=0.0,
          t_cmb=2.7255, n_eff=3.046):
    """The stored background: rows uniform in ln a from a_init to 1, columns
    (a, H/H0, (dH/dt)/H0^2, phi-bar, d phi-bar/da, (d phi-bar/dt)/H0).
    Returns (lambda, Omega_r, table)."""
    orr = omega_r(h, t_cmb, n_eff)
    kw = dict(z_init=z_init, phi_init=phi_init, dphi_init=dphi_init)
    lam = shoot_lambda(om, orr, alpha, beta, **kw)
    Ns = np.linspace(-math.log1p(z_init), 0.0, n_table)
    s = evolve(lam, om, orr, alpha, beta, n_eval=Ns, **kw)
    out = np.empty((n_table, 6))
    for r, N in enumerate(Ns):
        P, Q = s.y[0, r], s.y[1, r]
        E, D = _e_d(N, P, Q, lam, om, orr, alpha, beta)
        a = math.exp(N)
        hh = math.sqrt(E) / a  # conformal H = a H
        out[r] = (a, hh, (D - E) / (a * a), P, Q / a, hh * Q)
    return lam, orr, out


def interp(tab, a):
    """Linear interpolation of every column in a (the paper's lookup)."""
    col = tab[:, 0]
    return np.array([np.interp(a, col, tab[:, c]) for c in range(tab.shape[1])])
