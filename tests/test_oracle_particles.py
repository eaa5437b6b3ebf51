"""Oracle pins for the particle side after the fifth force: CIC
interpolation to particles, the Newtonian FFT Poisson potential and its
gradient, the symmetron friction term.

Pins: interpolation is the exact transpose of the (separately pinned) CIC
assignment; it reproduces cell values at cell centres, constants, and linear
fields exactly.  The Poisson potential satisfies the 7-point discrete
equation (checked by finite differences, not by the FFT), has zero mean, and
matches the closed form for a single Fourier mode.  The friction term's
coefficient is derived here a second way, numerically: the last term of
eq:csf_particle_geodesic_qsa in code units is -(dA/dphi)(d phi-bar/da) p~,
with A of eq:sym_coupling_function, phi_* of eq:varphi_ast and phi-bar(a) of
eq:varphi_min_symm, differentiated by mpmath at a != 1 (which exposes the
a^-4 factor); its interpolation part is pinned through interp.
"""
import numpy as np
import pytest

import oracle

OM = 0.3


def test_interp_is_transpose_of_cic_assignment():
    n, npart = 12, 3000
    rng = np.random.default_rng(1)
    pos = rng.uniform(0, n, (npart, 3))
    F = rng.standard_normal((n, n, n))
    count = (oracle.cic(n, pos) + 1.0) * npart / n ** 3  # sum of CIC weights per cell
    lhs = oracle.interp(n, pos, F).sum()
    rhs = np.sum(F * count)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(F * count))


def test_interp_cell_centres_constants_and_linear_fields():
    n = 10
    rng = np.random.default_rng(2)
    F = rng.standard_normal((3, n, n, n))
    cells = rng.integers(0, n, (50, 3))
    pos = cells + 0.5
    got = oracle.interp(n, pos, F)
    ref = F[:, cells[:, 2], cells[:, 1], cells[:, 0]].T
    assert np.array_equal(got, ref)
    const = np.full((n, n, n), 2.5)
    assert np.allclose(oracle.interp(n, rng.uniform(0, n, (100, 3)), const), 2.5, rtol=0, atol=1e-14)
    # a field linear in x is reproduced exactly away from the periodic seam
    i = np.arange(n, dtype=float)
    lin = np.broadcast_to(0.3 * (i + 0.5), (n, n, n)).copy()
    p = rng.uniform(1.0, n - 1.0, (200, 3))
    assert np.allclose(oracle.interp(n, p, lin), 0.3 * p[:, 0], rtol=0, atol=1e-13)


def _lap(phi):
    return sum(np.roll(phi, s, a) for a in range(3) for s in (1, -1)) - 6.0 * phi


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_poisson_satisfies_discrete_equation_with_zero_mean(a):
    n = 16
    P = oracle.params(oracle.FR, n, float(n), a=a, omega_m=OM)
    d = np.random.default_rng(3).standard_normal((n, n, n))
    d -= d.mean()
    phi = oracle.poisson_newton(P, d)
    src = 1.5 * OM / a * d
    assert np.abs(_lap(phi) - src).max() <= 1e-12 * np.abs(src).max()
    assert abs(phi.mean()) < 1e-14


def test_poisson_single_mode_closed_form():
    n, m = 24, 3
    P = oracle.params(oracle.FR, n, float(n), omega_m=OM)
    x = np.arange(n)
    d = np.broadcast_to(np.sin(2 * np.pi * m * x / n)[None, :, None], (n, n, n)).copy()  # y mode
    phi = oracle.poisson_newton(P, d)
    ref = -1.5 * OM * d / (4.0 * np.sin(np.pi * m / n) ** 2)
    assert np.abs(phi - ref).max() <= 1e-13


def test_gradient_of_sine_is_exact_central_difference():
    n, m = 20, 2
    x = np.arange(n)
    s = np.sin(2 * np.pi * m * x / n)
    phi = np.broadcast_to(s[:, None, None], (n, n, n)).copy()  # varies along z
    g = oracle.gradient(phi)
    ref = -np.sin(2 * np.pi * m / n) * np.cos(2 * np.pi * m * x / n)
    assert np.abs(g[2] - ref[:, None, None]).max() < 1e-14
    assert np.abs(g[0]).max() == 0.0 and np.abs(g[1]).max() == 0.0


def _friction_coef_from_geodesic(a, a_star, xi, beta_star, om, u):
    """-(dA/dphi)(d phi-bar/da) at phi = phi_* u, in units M_Pl = 1, by
    numerical differentiation (50 digits).  The paper's parameters: phi_* =
    6 Omega_m beta_* xi^2 a_*^-3 (eq:varphi_ast); beta_* = M_Pl phi_* / M^2
    fixes M^2; A = 1 + phi^2 / (2 M^2) (eq:sym_coupling_function); phi-bar
    = phi_* sqrt(1 - (a_*/a)^3) (eq:varphi_min_symm).  The field's time
    derivative is the background's (quasi-static approximation), and
    dp~/da = (dp~/dt)/a-dot turns phi-dot into d phi-bar / da."""
    import mpmath as mp
    mp.mp.dps = 50
    a, a_star, xi, beta_star, om, u = (mp.mpf(x) for x in (a, a_star, xi, beta_star, om, u))
    phi_star = 6 * om * beta_star * xi ** 2 / a_star ** 3
    M2 = phi_star / beta_star

    def A(phi):
        return 1 + phi ** 2 / (2 * M2)

    def phibar(aa):
        return phi_star * mp.sqrt(1 - (a_star / aa) ** 3)

    return float(-mp.diff(A, phi_star * u) * mp.diff(phibar, a))


@pytest.mark.parametrize("a", [1.0, 0.8, 0.6])
def test_friction_coefficient_from_the_geodesic_equation(a):
    """The oracle's friction per unit momentum equals the coefficient
    derived numerically from the geodesic equation, at a = 1, 0.8, 0.6
    (a_* = 0.5), for fields u of either side of the background."""
    n, ast, xi, bst = 8, 0.5, 2e-3, 1.3
    P = oracle.params(oracle.SYM, n, float(n), a=a, a_star=ast, xi=xi, beta_star=bst, omega_m=OM)
    rng = np.random.default_rng(4)
    pos = (np.arange(n)[rng.integers(0, n, (6, 3))] + 0.5).astype(np.float64)  # cell centres
    for uval in (0.3, 0.9, 1.4):
        u = np.full((n, n, n), uval)
        mom = rng.standard_normal((6, 3))
        f = oracle.sym_friction(P, u, pos, mom)
        coef = _friction_coef_from_geodesic(a, ast, xi, bst, OM, uval)
        assert np.allclose(f, coef * mom, rtol=1e-12, atol=0), (a, uval)
    # eq:F_x_codeunit as printed carries u-bar = sqrt(1 - (a_*/a)^3) where the
    # derivation gives 1 / u-bar: the printed value is u-bar^2 times this one
    ubar2 = 1 - (ast / a) ** 3
    printed = -9 * OM * bst ** 2 * xi ** 2 * np.sqrt(ubar2) / a ** 4 * 0.9
    derived = _friction_coef_from_geodesic(a, ast, xi, bst, OM, 0.9)
    assert abs(printed / derived - ubar2) < 1e-12


def test_friction_is_interpolated_field_times_momentum():
    n, a, ast, xi, bst = 8, 0.8, 0.5, 2e-3, 1.3
    P = oracle.params(oracle.SYM, n, float(n), a=a, a_star=ast, xi=xi, beta_star=bst)
    rng = np.random.default_rng(4)
    u = rng.uniform(0.5, 1.0, (n, n, n))
    pos = rng.uniform(0, n, (40, 3))
    mom = rng.standard_normal((40, 3))
    f = oracle.sym_friction(P, u, pos, mom)
    coef = _friction_coef_from_geodesic(a, ast, xi, bst, OM, 1.0)  # linear in u
    assert np.allclose(f, coef * oracle.interp(n, pos, u)[:, None] * mom, rtol=1e-12, atol=0)


@pytest.mark.parametrize("model", ["fr", "cq"])
def test_total_force_single_modes_closed_form(model):
    """Phi_N varies along x, the scalar field along y: the x component is the
    Newtonian force (scaled by exp(beta phibar) for CQ), the y component the
    fifth force (-1/2 c~^2 f_R for f(R), beta phi~ for CQ), z vanishes."""
    n, m1, m2 = 16, 1, 3
    x = np.arange(n)
    sx = np.sin(2 * np.pi * m1 * x / n)
    sy = np.sin(2 * np.pi * m2 * x / n)
    phin = np.broadcast_to(sx[None, None, :], (n, n, n)).copy()
    if model == "fr":
        P = oracle.params(oracle.FR, n, 64.0, omega_m=OM)
        # the oracle's f(R) variable is w = -f_R > 0, and Phi5 = c~^2 w / 2
        v = 1e-6 * (1.5 + np.broadcast_to(sy[None, :, None], (n, n, n)))
        sn, amp = 1.0, 0.5 * oracle.ctilde(n, 64.0) ** 2 * 1e-6
    else:
        P = oracle.params(oracle.CQ, n, 64.0, omega_m=OM, beta=-0.2, phibar=0.5)
        v = 3.0 * np.broadcast_to(sy[None, :, None], (n, n, n)).copy()
        sn, amp = np.exp(-0.2 * 0.5), -0.2 * 3.0
    g = oracle.total_force(P, phin, v)
    gx = -sn * np.sin(2 * np.pi * m1 / n) * np.cos(2 * np.pi * m1 * x / n)
    gy = -amp * np.sin(2 * np.pi * m2 / n) * np.cos(2 * np.pi * m2 * x / n)
    scale = max(abs(sn), abs(amp))
    assert np.abs(g[0] - gx[None, None, :]).max() <= 1e-13 * scale
    assert np.abs(g[1] - gy[None, :, None]).max() <= 1e-13 * scale
    assert np.abs(g[2]).max() <= 1e-13 * scale
