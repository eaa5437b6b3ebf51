"""Pins for the oracle's discrete operators and FAS multigrid against what the
paper and the mathematics fix (Ruan et al., arXiv:2110.00328):

* uniform density -> background field (eq:field_uniform_dens_test), and the
  closed-form uniform solutions for a uniform non-zero contrast;
* manufactured single Fourier modes (eq:sine_field_fR, eq:sine_field_sym,
  eq:sine_field_cs), using the discrete Laplacian symbol so that the sine is an
  exact solution of the discrete system;
* the linear limit against an exact FFT Yukawa/Helmholtz solve whose mass is
  the paper's m_eff (point-mass test, Sec. 4.2.3);
* brute-force dense Newton on 8^3;
* independence of the converged result from cycle type and sweep counts.
"""
import numpy as np
import pytest

import oracle

CH = oracle.C_OVER_H0


def sine_phase(n, axis):
    th = 2.0 * np.pi * (np.arange(n) + 0.5) / n
    shape = [1, 1, 1]
    shape[2 - axis] = n  # arrays are [k][j][i]; axis 0 = x = i
    return np.broadcast_to(th.reshape(shape), (n, n, n))


def disc_k2(n, h=1.0):
    """Eigenvalue of -Laplacian_h on sin(2 pi x / N): (4/h^2) sin^2(pi/N)."""
    return 4.0 / h ** 2 * np.sin(np.pi / n) ** 2


# ---------------------------------------------------------------------------
# Homogeneous and uniform-contrast densities
# ---------------------------------------------------------------------------

def test_homogeneous_fr_random_guess():
    """delta = 0 -> f_R = f_R-bar from random initial f_R/f_R-bar in [0,2]
    (n=1, f_R0 = -1e-5; Sec. 4.2.1)."""
    n = 16
    P = oracle.params(oracle.FR, n, 32.0, fr0=1e-5)
    wbar = oracle.background(P)
    rng = np.random.default_rng(0)
    v0 = wbar * rng.uniform(1e-3, 2.0, (n, n, n))
    v, cyc, rel, _ = oracle.solve(P, np.zeros((n, n, n)), v0, tol=1e-13, max_cycles=60)
    assert np.max(np.abs(v / wbar - 1.0)) < 1e-12


@pytest.mark.parametrize("a", [1.0, 0.8])
def test_homogeneous_sym_random_guess(a):
    """delta = 0 -> u = sqrt(1-(a*/a)^3) (eq:varphi_min_symm) from random u in
    (0,1]; a*=0.5, xi=1e-3, beta*=0.1 (Sec. 4.2.1), at a = 1 and a = 0.8."""
    n = 16
    P = oracle.params(oracle.SYM, n, 256.0, a=a, a_star=0.5, xi=1e-3, beta_star=0.1)
    ubar = oracle.background(P)
    assert abs(ubar - np.sqrt(1 - (0.5 / a) ** 3)) < 1e-15
    rng = np.random.default_rng(1)
    v0 = rng.uniform(0.05, 1.0, (n, n, n))
    v, cyc, rel, _ = oracle.solve(P, np.zeros((n, n, n)), v0, tol=1e-13, max_cycles=60)
    assert np.max(np.abs(v - ubar)) < 1e-12


def test_homogeneous_cq_random_guess():
    """delta = 0 -> phi~ = 0 from random delta-phi in [-0.5,0.5] (times c~^2);
    alpha = 0.1, beta = -0.2 (Sec. 4.2.1)."""
    n = 8
    P = oracle.params(oracle.CQ, n, 16.0, alpha=0.1, beta=-0.2, phibar=0.5)
    ct2 = oracle.ctilde(n, 16.0) ** 2
    rng = np.random.default_rng(2)
    v0 = ct2 * rng.uniform(-0.5, 0.5, (n, n, n)) * 1e-3
    v, cyc, rel, _ = oracle.solve(P, np.zeros((n, n, n)), v0, tol=1e-14, max_cycles=200)
    assert np.max(np.abs(v)) < 1e-12 * ct2


@pytest.mark.parametrize("fr_n", [0, 1, 2])
def test_uniform_contrast_fr_closed_form(fr_n):
    """Uniform delta0: Laplacian vanishes, eq:fR_eom_codeunit2 gives
    w = wbar (K / (K + Om delta0 / a))^{n+1}, K = R-bar a^2 / 3 (eq:R_bar)."""
    n, a, om, fr0, d0 = 8, 0.6, 0.3, 3e-6, 4.0
    P = oracle.params(oracle.FR, n, 8.0, a=a, omega_m=om, fr_n=fr_n, fr0=fr0)
    oml = 1 - om
    K = (om / a ** 3 + 4 * oml) * a ** 2
    wbar = fr0 * ((om + 4 * oml) / (om / a ** 3 + 4 * oml)) ** (fr_n + 1)
    assert abs(oracle.background(P) / wbar - 1) < 1e-14
    w_exact = wbar * (K / (K + om * d0 / a)) ** (fr_n + 1)
    v, _, _, _ = oracle.solve(P, np.full((n, n, n), d0), tol=1e-14, max_cycles=100)
    assert np.max(np.abs(v / w_exact - 1)) < 1e-12


@pytest.mark.parametrize("a", [1.0, 0.8])
def test_uniform_contrast_sym_closed_form(a):
    """Uniform delta0 in eq:sym_eom_code_unit: u^2 = 1 - (1+delta0) a*^3/a^3."""
    n, ast, d0 = 8, 0.5, 2.0 if a == 1.0 else 1.5
    P = oracle.params(oracle.SYM, n, 8.0, a=a, a_star=ast, xi=2e-3)
    u_exact = np.sqrt(1 - (1 + d0) * (ast / a) ** 3)
    v, _, _, _ = oracle.solve(P, np.full((n, n, n), d0), tol=1e-14, max_cycles=100)
    assert np.max(np.abs(v - u_exact)) < 1e-12


def test_uniform_contrast_cq_scalar_root():
    """Uniform delta0 in eq:csf_eom_code: the uniform phi0 solves a scalar
    equation, solved here by 60-digit bisection."""
    import mpmath as mp
    mp.mp.dps = 60
    n, box, a, om, al, be, pb, d0 = 8, 4.0, 0.8, 0.3, 0.1, -0.2, 0.5, 0.3
    P = oracle.params(oracle.CQ, n, box, a=a, omega_m=om, alpha=al, beta=be, phibar=pb)
    lam2 = (1 - om) * pb ** al
    ct2 = mp.mpf(n * CH / box) ** 2

    def rhs(ph):
        return (3 * be * om / a * mp.e ** (be * pb) * (mp.e ** (be * ph / ct2) * (1 + d0) - 1)
                - al * lam2 * a * a * ((pb + ph / ct2) ** (-(1 + al)) - mp.mpf(pb) ** (-(1 + al))))

    lo, hi = -0.4 * ct2, 0.4 * ct2
    assert rhs(lo) * rhs(hi) < 0
    for _ in range(300):
        mid = (lo + hi) / 2
        if rhs(lo) * rhs(mid) <= 0:
            hi = mid
        else:
            lo = mid
    phi0 = float((lo + hi) / 2)
    v, _, _, _ = oracle.solve(P, np.full((n, n, n), d0), tol=1e-14, max_cycles=200)
    # phi0 ~ 1e7 while the uniform mode's restoring term is ~1e-8 per cell:
    # FP64 rounding of the Laplacian limits the uniform mode to ~1e-8 relative
    assert np.max(np.abs(v - phi0)) < 1e-7 * abs(phi0)


# ---------------------------------------------------------------------------
# Single Fourier modes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fr_n", [0, 1, 2])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sine_mode_fr(fr_n, axis):
    """f_R/f_R-bar = 1 + A sin(2 pi x/N), A = 0.5, f_R0 = -1e-5 (eq:sine_field_fR)
    with the density from the printed formula, (2 pi/N)^2 -> discrete symbol."""
    n, box, a, om, A = 32, 64.0, 1.0, 0.3, 0.5
    P = oracle.params(oracle.FR, n, box, a=a, omega_m=om, fr_n=fr_n, fr0=1e-5)
    ct2 = (n * CH / box) ** 2
    fbar = -oracle.background(P)
    Rbar_a2_3 = (om / a ** 3 + 4 * (1 - om)) * a * a  # (1/3) R-bar a^2
    s = np.sin(sine_phase(n, axis))
    delta = a / om * (ct2 * fbar * disc_k2(n) * A * s + Rbar_a2_3 * (1 + A * s) ** (-1.0 / (fr_n + 1))
                      - Rbar_a2_3)
    exact = -fbar * (1 + A * s)
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-13, max_cycles=100)
    assert rel < 1e-12
    assert np.max(np.abs(v - exact)) / np.max(np.abs(exact + fbar)) < 1e-10


@pytest.mark.parametrize("a", [1.0, 0.8])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sine_mode_sym(axis, a):
    """u = 1/2 + A sin(2 pi x/N) (eq:sine_field_sym) with A = 0.25 (A = 0.5 would
    drive u through zero); a*=0.5, xi=1e-3, beta*=0.1, density from the printed
    formula with the discrete symbol, at a = 1 and a = 0.8 (where the printed
    density's a^3/a*^3 and 2/a^2 factors differ from 8 and 2)."""
    n, box, ast, xi, A = 32, 256.0, 0.5, 1e-3, 0.25
    P = oracle.params(oracle.SYM, n, box, a=a, a_star=ast, xi=xi, beta_star=0.1)
    ct2 = (n * CH / box) ** 2
    s = np.sin(sine_phase(n, axis))
    u = 0.5 + A * s
    delta = a ** 3 / ast ** 3 * (1 - u * u - 2 / a ** 2 * xi ** 2 * ct2 * A * disc_k2(n) * s / u) - 1
    assert delta.min() > -1
    v, cyc, rel, _ = oracle.solve(P, delta, v0=np.full_like(u, 0.5), tol=1e-13, max_cycles=100)
    assert np.max(np.abs(v - u)) / A < 1e-10


@pytest.mark.parametrize("A", [0.5, 1.0])
def test_sine_mode_cq(A):
    """phi~ = A sin(2 pi x/N) (eq:sine_field_cs).  The printed density is
    inconsistent with eq:csf_eom_code (sign of beta phibar, exponent of the
    potential term), so delta is derived from eq:csf_eom_code itself."""
    n, box, a, om, al, be, pb = 16, 32.0, 1.0, 0.3, 0.1, -0.2, 0.5
    P = oracle.params(oracle.CQ, n, box, a=a, omega_m=om, alpha=al, beta=be, phibar=pb)
    lam2 = (1 - om) * pb ** al
    ct2 = (n * CH / box) ** 2
    phi = A * np.sin(sine_phase(n, 1))
    lap = -disc_k2(n) * phi
    src = 3 * be * om / a * np.exp(be * pb)
    pot = al * lam2 * a * a * ((pb + phi / ct2) ** (-(1 + al)) - pb ** (-(1 + al)))
    one_plus = ((lap + pot) / src + 1.0) / np.exp(be * phi / ct2)
    delta = one_plus - 1
    assert delta.min() > -1
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-14, max_cycles=200)
    assert np.max(np.abs(v - phi)) / A < 1e-9


# ---------------------------------------------------------------------------
# Linear limit against an exact FFT Helmholtz solve
# ---------------------------------------------------------------------------

def fft_helmholtz(rhs, m2, h=1.0):
    """Solve (Lap_h - m2) x = rhs exactly on the periodic grid."""
    n = rhs.shape[0]
    k = 4.0 / h ** 2 * np.sin(np.pi * np.fft.fftfreq(n)) ** 2
    sym = -(k[:, None, None] + k[None, :, None] + k[None, None, :]) - m2
    return np.real(np.fft.ifftn(np.fft.fftn(rhs) / sym))


def small_field(n, seed, amp):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n, n))
    g -= g.mean()
    return amp * g / g.std()


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_linear_limit_fr_matches_paper_meff(a):
    """delta ~ 1e-6: w - wbar solves (Lap - m^2) x = (Om/(a c~^2)) delta with the
    paper's m_eff (point-mass test) times a^2 for comoving code units."""
    n, box, om, fr_n, fr0 = 32, 32.0, 0.3, 1, 1e-5
    P = oracle.params(oracle.FR, n, box, a=a, omega_m=om, fr_n=fr_n, fr0=fr0)
    ct2 = (n * CH / box) ** 2
    oml = 1 - om
    meff2 = om / (ct2 * (fr_n + 1) * fr0) * (a ** -3 + 4 * oml / om) ** (fr_n + 2) / (
        1 + 4 * oml / om) ** (fr_n + 1)
    m2 = meff2 * a * a
    delta = small_field(n, 3, 1e-6)
    x = fft_helmholtz(om / (a * ct2) * delta, m2)
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-13, max_cycles=100)
    wbar = oracle.background(P)
    err = np.linalg.norm(v - wbar - x) / np.linalg.norm(x)
    assert err < 1e-5, err


@pytest.mark.parametrize("a", [1.0, 0.8])
def test_linear_limit_sym(a):
    """delta ~ 1e-6: u - ubar solves (Lap - m^2) x = s delta with
    m^2 = a^2 (1 - a*^3/a^3) / (xi c~)^2 and s = a*^3 ubar / (2 xi^2 c~^2 a),
    the linearisation of eq:sym_eom_code_unit about eq:varphi_min_symm."""
    n, box, ast, xi = 32, 32.0, 0.5, 1.0 / CH
    P = oracle.params(oracle.SYM, n, box, a=a, a_star=ast, xi=xi)
    ct2 = (n * CH / box) ** 2
    ubar = np.sqrt(1 - (ast / a) ** 3)
    m2 = a * a * (1 - ast ** 3 / a ** 3) / (xi * xi * ct2)
    s = ast ** 3 * ubar / (2 * xi * xi * ct2 * a)
    delta = small_field(n, 4, 1e-6)
    x = fft_helmholtz(s * delta, m2)
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-13, max_cycles=100)
    err = np.linalg.norm(v - ubar - x) / np.linalg.norm(x)
    assert err < 1e-5, err


@pytest.mark.parametrize("keep_exp", [1, 0])
def test_linear_limit_cq(keep_exp):
    n, box, a, om, al, be, pb = 16, 16.0, 1.0, 0.3, 0.1, -0.2, 0.5
    P = oracle.params(oracle.CQ, n, box, a=a, omega_m=om, alpha=al, beta=be, phibar=pb,
                      cq_keep_exp=keep_exp)
    lam2 = (1 - om) * pb ** al
    ct2 = (n * CH / box) ** 2
    src = 3 * be * om / a * np.exp(be * pb)
    m2 = (keep_exp * 3 * be * be * om / a * np.exp(be * pb) +
          al * (1 + al) * lam2 * a * a * pb ** (-(2 + al))) / ct2
    delta = small_field(n, 5, 1e-6)
    x = fft_helmholtz(src * delta, m2)
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-14, max_cycles=300)
    err = np.linalg.norm(v - x) / np.linalg.norm(x)
    assert err < 1e-5, err


def test_point_mass_far_field_decays_as_yukawa():
    """delta_{000} = 1e-4 (N^3 - 1), -1e-4 elsewhere (eqn:deltaijk_point_mass):
    far from the mass, r delta-f_R(r) ~ exp(-m_eff r) (eq:fR_point_mass_soln).
    At this amplitude the field is linear, so the exact periodic lattice
    Green's function must match to O(amplitude)."""
    n, box, om, fr0 = 64, 64.0, 0.3, 1e-5
    P = oracle.params(oracle.FR, n, box, fr0=fr0)
    ct2 = (n * CH / box) ** 2
    delta = np.full((n, n, n), -1e-4)
    delta[0, 0, 0] = 1e-4 * (n ** 3 - 1)
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-12, max_cycles=100)
    wbar = oracle.background(P)
    dfr = -(v - wbar)
    meff = np.sqrt((om + 4 * (1 - om)) / (ct2 * 2 * fr0))
    x = fft_helmholtz(om / ct2 * delta, meff ** 2)
    assert np.linalg.norm(dfr + x) / np.linalg.norm(x) < 2e-3
    # along +x away from the lattice scale and the periodic images, after
    # removing the uniform response to the -1e-4 background contrast
    offset = om / ct2 * (-1e-4) / meff ** 2
    r = np.arange(6, 16, dtype=float)
    prof = dfr[0, 0, 6:16] - offset
    slope = np.polyfit(r, np.log(np.abs(r * prof)), 1)[0]
    assert abs(-slope / meff - 1) < 0.1, (slope, meff)


# ---------------------------------------------------------------------------
# Brute force: dense Newton on 8^3
# ---------------------------------------------------------------------------

def _lap_np(v):
    return sum(np.roll(v, s, ax) for ax in range(3) for s in (1, -1)) - 6 * v


def _F_np(model, P, delta, v):
    ct2 = (P.n * CH / P.box) ** 2
    a, om = P.a, P.omega_m
    if model == oracle.FR:
        K = (om / a ** 3 + 4 * (1 - om)) * a * a
        wb = oracle.background(P)
        m = 1.0 / (P.fr_n + 1)
        F = -ct2 * _lap_np(v) + om / a * delta + K - K * wb ** m * v ** (-m)
        dF = 6 * ct2 + K * wb ** m * m * v ** (-m - 1)
        off = -ct2
    elif model == oracle.SYM:
        sa = a * a / (2 * P.xi ** 2)
        sr = (P.a_star / a) ** 3
        F = ct2 * _lap_np(v) - sa * (((1 + delta) * sr - 1) * v + v ** 3)
        dF = -6 * ct2 - sa * (((1 + delta) * sr - 1) + 3 * v * v)
        off = ct2
    else:
        src = 3 * P.beta * om / a * np.exp(P.beta * P.phibar)
        pot = P.alpha * P.lam ** 2 * a * a
        E = np.exp(P.beta * v / ct2)
        Y = P.phibar + v / ct2
        # accurate forms of e^x (1+d) - 1 and Y^-(1+al) - pb^-(1+al) (phi/c^2 ~ 1e-14)
        F = (_lap_np(v) - src * (np.expm1(P.beta * v / ct2) * (1 + delta) + delta) +
             pot * P.phibar ** (-(1 + P.alpha)) *
             np.expm1(-(1 + P.alpha) * np.log1p(v / (ct2 * P.phibar))))
        dF = -6 - src * P.beta / ct2 * E * (1 + delta) - pot * (1 + P.alpha) / ct2 * Y ** (-(2 + P.alpha))
        off = 1.0
    return F, dF, off


def dense_newton_np(model, P, delta, v0):
    n = delta.shape[0]
    m = n ** 3
    idx = np.arange(m).reshape(n, n, n)
    nbrs = [np.roll(idx, s, ax).ravel() for ax in range(3) for s in (1, -1)]
    v = v0.copy()
    for _ in range(100):
        F, dF, off = _F_np(model, P, delta, v)
        if np.max(np.abs(F)) < 1e-14 * (1 + np.max(np.abs(dF * v))):
            break
        J = np.zeros((m, m))
        J[np.arange(m), np.arange(m)] = dF.ravel()
        for nb in nbrs:
            np.add.at(J, (np.arange(m), nb), off)
        step = np.linalg.solve(J, -F.ravel()).reshape(n, n, n)
        t = 1.0
        f0 = np.linalg.norm(F)
        while True:  # damped so that w stays positive and |F| decreases
            vn = v + t * step
            if model != oracle.FR or vn.min() > 0:
                Fn = _F_np(model, P, delta, vn)[0]
                if np.linalg.norm(Fn) < f0 or t < 1e-6:
                    break
            t *= 0.5
        v = vn
    return v


@pytest.mark.parametrize("model", [oracle.FR, oracle.SYM, oracle.CQ])
def test_dense_newton_8cube(model):
    n = 8
    rng = np.random.default_rng(7)
    g = rng.standard_normal((n, n, n))
    delta = np.exp(0.8 * g - 0.32) - 1
    delta -= delta.mean()
    if model == oracle.FR:
        # |f_R0| = 1e-6 on 1 Mpc/h cells: screened, strongly nonlinear (at 1e-5
        # the 8^3 problem is nearly linear and both solvers sit on the FP64
        # residual floor, ~1e-10 in the field)
        P = oracle.params(model, n, 8.0, fr0=1e-6)
        v0 = np.full((n, n, n), oracle.background(P))
    elif model == oracle.SYM:
        P = oracle.params(model, n, 8.0, a_star=0.5, xi=1.0 / CH)
        v0 = np.full((n, n, n), oracle.background(P))
    else:
        P = oracle.params(model, n, 8.0)
        v0 = np.zeros((n, n, n))
    ref = dense_newton_np(model, P, delta, v0)
    v, cyc, rel, _ = oracle.solve(P, delta, tol=1e-14, max_cycles=300)
    bg = 0.0 if model == oracle.CQ else oracle.background(P)
    if model == oracle.CQ:
        # the uniform mode is restored only by the tiny CQ mass (m^2 ~ 4e-8 per
        # cell^2): at the FP64 residual floor it is fixed to ~1e-9 relative
        assert abs(v.mean() - ref.mean()) < 1e-7 * np.max(np.abs(ref))
        v = v - v.mean()
        ref = ref - ref.mean()
    err = np.linalg.norm(v - ref) / np.linalg.norm(ref - bg)
    assert err < 1e-11, err


# ---------------------------------------------------------------------------
# Multigrid reaches the definition's unique result
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("model", [oracle.FR, oracle.CQ])
def test_cycle_type_and_sweeps_do_not_change_result(model):
    n = 32
    rng = np.random.default_rng(8)
    g = rng.standard_normal((n, n, n))
    delta = np.exp(g - 0.5) - 1
    delta -= delta.mean()  # a CIC contrast has zero mean
    P = oracle.params(model, n, 32.0, fr0=1e-5)
    bg = oracle.background(P)
    ref, _, rel, _ = oracle.solve(P, delta, tol=1e-12, cycle="V", nu1=1, nu2=1)
    assert rel < 1e-12
    for cyc, nu1, nu2 in (("F", 1, 1), ("W", 2, 1), ("V", 2, 2), ("V", 0, 1)):
        v, c, rel, _ = oracle.solve(P, delta, tol=1e-12, cycle=cyc, nu1=nu1, nu2=nu2, max_cycles=300)
        assert rel < 1e-12
        dv = v - ref
        if model == oracle.CQ:  # uniform mode: condition ~ 1/m^2, see the 8^3 test
            assert abs(dv.mean()) < 1e-6 * np.max(np.abs(ref))
            dv = dv - dv.mean()
        assert np.linalg.norm(dv) / np.linalg.norm(ref - bg) < 1e-10


def test_multigrid_equals_plain_gauss_seidel():
    """A massive f(R) field on 8^3: red-black Gauss-Seidel alone converges;
    the multigrid result is the same solution."""
    n = 8
    P = oracle.params(oracle.FR, n, 16.0, fr0=1e-6)
    rng = np.random.default_rng(9)
    delta = np.exp(rng.standard_normal((n, n, n)) * 0.7 - 0.245) - 1
    v = np.full((n, n, n), oracle.background(P))
    for _ in range(3000):
        v = oracle.relax_colour(P, delta, v, 0)
        v = oracle.relax_colour(P, delta, v, 1)
    ref, _, rel, _ = oracle.solve(P, delta, tol=1e-14, max_cycles=100)
    assert np.linalg.norm(v - ref) / np.linalg.norm(ref - oracle.background(P)) < 1e-11


def test_half_sweep_zeroes_residual_of_its_colour():
    """After a nonlinear Gauss-Seidel half-sweep each updated cell satisfies its
    own discrete equation exactly (Sec. 3.2.4-3.2.5)."""
    n = 16
    rng = np.random.default_rng(10)
    delta = np.exp(rng.standard_normal((n, n, n)) - 0.5) - 1
    for model, kw in ((oracle.FR, dict(fr0=1e-5)), (oracle.SYM, dict(a_star=0.5, xi=2.0 / CH))):
        P = oracle.params(model, n, 16.0, **kw)
        v = oracle.background(P) * rng.uniform(0.5, 1.5, (n, n, n))
        v = oracle.relax_colour(P, delta, v, 0)
        d, _ = oracle.residual(P, delta, v)
        i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        even = ((i + j + k) % 2) == 0
        scale = np.max(np.abs(d[~even]))
        assert np.max(np.abs(d[even])) < 1e-9 * scale


# ---------------------------------------------------------------------------
# Transfer operators
# ---------------------------------------------------------------------------

def test_prolongation_stencil_weights():
    """A unit coarse spike spreads with 27/64, 9/64, 3/64 and 1/64 to the fine
    cells it is parent, face-, edge- and corner-neighbour of (Sec. 3.2.1)."""
    nc = 4
    c = np.zeros((nc, nc, nc))
    c[1, 1, 1] = 1.0
    f = oracle.prolong_add(c, np.zeros((8, 8, 8)))
    w1 = np.array([0, 1, 3, 3, 1, 0, 0, 0]) / 4.0  # fine cells 1..4 around coarse 1
    expected = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    assert np.max(np.abs(f - expected)) < 1e-16
    vals = sorted(set(np.round(f[f > 0] * 64).astype(int)))
    assert vals == [1, 3, 9, 27]


def test_restriction_and_prolongation_on_polynomials():
    n = 16
    rng = np.random.default_rng(12)
    c0 = rng.standard_normal()
    assert np.allclose(oracle.restrict(np.full((n, n, n), c0)), c0, atol=0, rtol=1e-15)
    assert np.allclose(oracle.prolong_add(np.full((8, 8, 8), c0), np.zeros((n, n, n))), c0,
                       atol=0, rtol=1e-15)
    # linear in x (cell centres i + 1/2): R exact everywhere, P exact away from the wrap
    x = (np.arange(n) + 0.5)[None, None, :] * np.ones((n, n, n))
    Rx = oracle.restrict(x)
    X = 2 * (np.arange(8) + 0.5)[None, None, :]
    assert np.max(np.abs(Rx - X)) < 1e-13
    Px = oracle.prolong_add(Rx, np.zeros((n, n, n)))
    assert np.max(np.abs(Px[:, :, 1:-1] - x[:, :, 1:-1])) < 1e-13


def test_prolongation_second_order_on_sines():
    errs = []
    for n in (16, 32, 64):
        th = 2 * np.pi * (np.arange(n) + 0.5) / n
        f = np.sin(th)[None, None, :] * np.ones((n, n, n))
        c = np.sin(2 * np.pi * (2 * np.arange(n // 2) + 1.0) / n)[None, None, :] * np.ones((n // 2,) * 3)
        errs.append(np.max(np.abs(oracle.prolong_add(c, np.zeros((n, n, n))) - f)))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.8 < errs[1] / errs[2] < 4.2


# ---------------------------------------------------------------------------
# Force
# ---------------------------------------------------------------------------

def test_force_of_sine_fields_is_exact_central_difference():
    """g5 = -grad Phi5 with 3-point differences (Sec. 3.1): for Phi5 ~ sin the
    difference is sin(2 pi/N) cos(.) exactly.  Prefactors from eq:F5_fR_codeunit
    (f(R)), eq:F_5_codeunit (symmetron, without H0/a-dot) and
    eq:csf_particle_geodesic_code2 (CQ)."""
    n, box = 16, 32.0
    ct2 = (n * CH / box) ** 2
    th = 2 * np.pi * (np.arange(n) + 0.5) / n
    for axis in range(3):
        shape = [1, 1, 1]
        shape[2 - axis] = n
        s = np.broadcast_to(np.sin(th).reshape(shape), (n, n, n))
        c = np.broadcast_to(np.cos(th).reshape(shape), (n, n, n))
        d = np.sin(2 * np.pi / n) * c  # (s_{i+1} - s_{i-1}) / 2
        # f(R): F5 = 1/2 c~^2 grad f_R, with f_R = -w
        P = oracle.params(oracle.FR, n, box)
        w = 1e-5 * (1 + 0.3 * s)
        g = oracle.force(P, w)
        assert np.max(np.abs(g[axis] - 0.5 * ct2 * (-1e-5 * 0.3 * d))) < 1e-12 * ct2 * 1e-5
        assert np.max(np.abs(np.delete(g, axis, 0))) == 0.0
        # CQ: F5 = -beta grad phi~
        P = oracle.params(oracle.CQ, n, box, beta=-0.2)
        g = oracle.force(P, 2.0 * s)
        assert np.max(np.abs(g[axis] - 0.2 * 2.0 * d)) < 1e-14
        # symmetron: F5 = -3 xi^2 Om beta*^2 c~^2 a*^-3 grad(u^2)
        xi, bs, ast, om = 1e-3, 0.7, 0.5, 0.3
        P = oracle.params(oracle.SYM, n, box, a_star=ast, xi=xi, beta_star=bs, omega_m=om)
        u = 0.5 + 0.2 * s
        u2 = u * u
        du2 = (np.roll(u2, -1, 2 - axis) - np.roll(u2, 1, 2 - axis)) / 2
        pref = 3 * xi * xi * om * bs * bs * ct2 / ast ** 3
        g = oracle.force(P, u)
        assert np.max(np.abs(g[axis] + pref * du2)) < 1e-13 * pref


def test_force_gr_limits():
    """Zero coupling: CQ beta = 0 gives phi~ = 0 and no force; symmetron
    beta* = 0 leaves the field equation unchanged (eq:sym_eom_code_unit has no
    beta*) but zeroes the force; f(R) with |f_R0| -> 0 screens everything."""
    n = 16
    rng = np.random.default_rng(13)
    delta = np.exp(rng.standard_normal((n, n, n)) - 0.5) - 1
    delta -= delta.mean()
    P = oracle.params(oracle.CQ, n, 16.0, beta=0.0)
    v, _, _, _ = oracle.solve(P, delta, tol=1e-12)
    assert np.max(np.abs(v)) < 1e-9
    assert np.max(np.abs(oracle.force(P, v))) < 1e-9
    P = oracle.params(oracle.SYM, n, 16.0, a_star=0.5, xi=1.0 / CH, beta_star=0.0)
    v, _, _, _ = oracle.solve(P, delta, tol=1e-12)
    assert np.max(np.abs(oracle.force(P, v))) == 0.0
    g = []
    for fr0 in (1e-5, 1e-7, 1e-9, 1e-11, 1e-13):
        P = oracle.params(oracle.FR, n, 16.0, fr0=fr0)
        v, _, _, _ = oracle.solve(P, delta, tol=1e-12)
        g.append(np.max(np.abs(oracle.force(P, v))))
    # once m^2 = K/(2 c~^2 |f_R0|) dominates every lattice k^2 the force falls
    # in proportion to |f_R0|
    assert g[0] > g[1] > g[2]
    for a, b in zip(g[2:], g[3:]):
        assert 80 < a / b < 120


# ---------------------------------------------------------------------------
# CIC
# ---------------------------------------------------------------------------

def test_cic_invariants():
    n = 16
    rng = np.random.default_rng(14)
    pos = rng.uniform(0, n, (5000, 3))
    d = oracle.cic(n, pos)
    assert abs((1 + d).sum() - n ** 3) < 1e-9  # mass conservation
    # unperturbed lattice at cell centres -> delta = 0
    q = (np.arange(n) + 0.5)
    lat = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3)
    assert np.max(np.abs(oracle.cic(n, lat))) < 1e-14
    # one particle at a cell centre -> one cell
    one = oracle.cic(n, np.array([[3.5, 7.5, 11.5]]))
    mean = 1.0 / n ** 3
    assert abs((one[11, 7, 3] + 1) * mean - 1) < 1e-15
    assert np.count_nonzero(one + 1) == 1
    # shift by whole cells = periodic roll
    shifted = oracle.cic(n, np.mod(pos + np.array([1.0, 2.0, 3.0]), n))
    assert np.max(np.abs(shifted - np.roll(d, (3, 2, 1), (0, 1, 2)))) < 1e-12


def test_cic_golden_weights():
    """Hand-computed CIC weights (tests/golden/cic_small.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "cic_small.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    n = int(rows[0][1])
    pos = np.array([[float(x) for x in r[1:4]] for r in rows if r[0] == "p"])
    d = oracle.cic(n, pos)
    mass = (1 + d) * pos.shape[0] / n ** 3
    for r in rows:
        if r[0] == "c":
            i, j, k = int(r[1]), int(r[2]), int(r[3])
            num, den = (int(x) for x in r[4].split("/"))
            assert abs(mass[k, j, i] - num / den) < 1e-14, r
    total = sum(int(r[4].split("/")[0]) / int(r[4].split("/")[1]) for r in rows if r[0] == "c")
    assert abs(total - pos.shape[0]) < 1e-14
