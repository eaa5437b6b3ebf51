"""Pins for the oracle's adjoint: d(Loss)/d(delta) through the converged field.

The forward map is defined by F(v(delta), delta) = 0, so
dL/d(delta) = -(dF/d(delta)) J^{-1} dL/dv with the symmetric Jacobian
J = dF/dv ("Laplacian plus diagonal").  Pins: symmetry of J, an exact FFT
inverse at a uniform field, agreement of multigrid and conjugate gradients,
and central finite differences (h = 1e-4) of the full nonlinear solve.
"""
import numpy as np
import pytest

import oracle

CH = oracle.C_OVER_H0


def _delta(n, seed, sig=0.8):
    g = np.random.default_rng(seed).standard_normal((n, n, n))
    d = np.exp(sig * g - 0.5 * sig * sig) - 1
    return d - d.mean()


# the symmetron also at a = 0.8 (a_* = 0.5), where the a^2/(2 xi^2) and
# (a_*/a)^3 factors of eq:sym_eom_code_unit differ from their a = 1 values
SYM08 = "sym08"
MODELS = [oracle.FR, oracle.SYM, SYM08, oracle.CQ]


def _model(model, n, box):
    if model == oracle.FR:
        return oracle.params(model, n, box, fr0=1e-5)
    if model in (oracle.SYM, SYM08):
        return oracle.params(oracle.SYM, n, box, a=0.8 if model == SYM08 else 1.0, a_star=0.5,
                             xi=2.0 / CH, beta_star=1.0)
    return oracle.params(model, n, box)


@pytest.mark.parametrize("model", MODELS)
def test_jacobian_is_symmetric(model):
    n = 8
    P = _model(model, n, 8.0)
    delta = _delta(n, 1)
    v, _, _, _ = oracle.solve(P, delta, tol=1e-13)
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((2, n, n, n))
    a = np.vdot(oracle.apply_jacobian(P, delta, v, x), y)
    b = np.vdot(x, oracle.apply_jacobian(P, delta, v, y))
    assert abs(a - b) < 1e-12 * abs(a)


def test_jacobian_matches_finite_difference_of_operator():
    """J x = d/de F(v + e x) at e = 0 (central difference of the residual)."""
    n = 8
    for model in MODELS:
        P = _model(model, n, 8.0)
        delta = _delta(n, 3)
        v, _, _, _ = oracle.solve(P, delta, tol=1e-13)
        x = np.random.default_rng(4).standard_normal((n, n, n))
        scale = max(np.max(np.abs(v)), 1.0 if model == oracle.CQ else 0.0)
        e = 1e-6 * scale
        fp, _ = oracle.residual(P, delta, v + e * x)
        fm, _ = oracle.residual(P, delta, v - e * x)
        jx = oracle.apply_jacobian(P, delta, v, x)
        fd = (fp - fm) / (2 * e)
        assert np.linalg.norm(fd - jx) / np.linalg.norm(jx) < 1e-6


def test_adjoint_at_background_matches_fft():
    """At the uniform background field (delta = 0) J is constant-coefficient,
    J = -c~^2 Lap + K/((n+1) wbar), and inverts exactly by FFT."""
    n = 16
    P = oracle.params(oracle.FR, n, 16.0, fr0=1e-5)
    wbar = oracle.background(P)
    ct2 = (n * CH / 16.0) ** 2
    K = 0.3 + 4 * 0.7
    delta = np.zeros((n, n, n))
    v = np.full((n, n, n), wbar)
    g = np.random.default_rng(5).standard_normal((n, n, n))
    got, it, rel = oracle.adjoint(P, delta, v, g, tol=1e-14)
    k = 4.0 * np.sin(np.pi * np.fft.fftfreq(n)) ** 2
    sym = ct2 * (k[:, None, None] + k[None, :, None] + k[None, None, :]) + K / (2 * wbar)
    lam = np.real(np.fft.ifftn(np.fft.fftn(g) / sym))
    ref = -0.3 * lam  # dL/ddelta = -(Om/a) lambda
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("model", MODELS)
def test_multigrid_adjoint_equals_cg(model):
    n = 16
    P = _model(model, n, 16.0)
    delta = _delta(n, 6)
    v, _, _, _ = oracle.solve(P, delta, tol=1e-13)
    g = np.random.default_rng(7).standard_normal((n, n, n))
    if model == oracle.CQ:
        # a force-adjoint gradient is a divergence (zero mean); a non-zero mean
        # would excite the nearly singular uniform mode (m^2 ~ 4e-8)
        g -= g.mean()
    a, it1, r1 = oracle.adjoint(P, delta, v, g, tol=1e-13, solver="mg")
    b, it2, r2 = oracle.adjoint(P, delta, v, g, tol=1e-13, solver="cg")
    assert r1 < 1e-13 and r2 < 1e-13
    d = a - b
    if model == oracle.CQ:  # the uniform mode has condition ~ 1/m^2
        assert abs(d.mean()) < 1e-8 * np.max(np.abs(b))
        d = d - d.mean()
    assert np.linalg.norm(d) / np.linalg.norm(b) < 1e-10


def test_force_adjoint_is_transpose():
    """<G v, g> = <v, G^T g> for the linear force maps; for the symmetron,
    whose force is quadratic in u, G^T g is the derivative of <g5(u), g>."""
    n = 8
    rng = np.random.default_rng(8)
    for model in (oracle.FR, oracle.CQ, oracle.SYM, SYM08):
        P = _model(model, n, 8.0)
        v = 0.5 + 0.1 * rng.standard_normal((n, n, n))
        gf = rng.standard_normal((3, n, n, n))
        gv = oracle.force_adjoint(P, v, gf)
        if model not in (oracle.SYM, SYM08):
            assert abs(np.vdot(oracle.force(P, v), gf) - np.vdot(v, gv)) < 1e-10 * abs(np.vdot(v, gv))
        else:
            x = rng.standard_normal((n, n, n))
            e = 1e-6
            fd = (np.vdot(oracle.force(P, v + e * x), gf) - np.vdot(oracle.force(P, v - e * x), gf)) / (2 * e)
            assert abs(fd - np.vdot(x, gv)) < 1e-7 * abs(fd)


def _loss_and_grad_force(P, v, cells):
    g = oracle.force(P, v)
    flat = g.reshape(3, -1)
    L = float(np.sum(flat[:, cells] ** 2))
    gf = np.zeros_like(flat)
    gf[:, cells] = 2.0 * flat[:, cells]
    return L, gf.reshape(g.shape)


@pytest.mark.parametrize("model", MODELS)
def test_adjoint_matches_central_finite_differences(model):
    """Loss = sum of |g5|^2 over a seeded cell set; dL/d(delta) at probe cells
    against central differences with h = 1e-4 and forward solves to 1e-13."""
    n = 16
    P = _model(model, n, 16.0)
    delta = _delta(n, 9)
    rng = np.random.default_rng(10)
    cells = rng.choice(n ** 3, 200, replace=False)
    # forward solves are driven to the FP64 floor (fixed 40 cycles): the FD
    # quotient divides the solves' stopping noise by 2h
    v, _, _, _ = oracle.solve(P, delta, tol=1e-16, max_cycles=40)
    L0, gf = _loss_and_grad_force(P, v, cells)
    gv = oracle.force_adjoint(P, v, gf)
    gd, it, rel = oracle.adjoint(P, delta, v, gv, tol=1e-14)
    probes = list(cells[:4]) + list(rng.choice(n ** 3, 4, replace=False))
    h = 1e-4
    for c in probes:
        dp = delta.copy().reshape(-1)
        dm = delta.copy().reshape(-1)
        dp[c] += h
        dm[c] -= h
        vp, _, _, _ = oracle.solve(P, dp.reshape(delta.shape), v0=v, tol=1e-16, max_cycles=40)
        vm, _, _, _ = oracle.solve(P, dm.reshape(delta.shape), v0=v, tol=1e-16, max_cycles=40)
        fd = (_loss_and_grad_force(P, vp, cells)[0] - _loss_and_grad_force(P, vm, cells)[0]) / (2 * h)
        got = gd.reshape(-1)[c]
        assert abs(got - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(gd))), (c, got, fd)
