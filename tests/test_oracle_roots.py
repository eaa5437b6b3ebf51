"""Pins for the oracle's per-cell roots (eq:fR_cubic_solns, eq:sym_cubic_solns,
eq:fR_quartic_solns, eq:fR_quadratic_solns) against 50-digit mpmath bisection."""
import mpmath as mp
import numpy as np
import pytest

import oracle

mp.mp.dps = 50


def _bisect_pos(f, hi):
    """Unique positive root of an increasing-through-zero f on (0, hi]."""
    lo = mp.mpf(0)
    hi = mp.mpf(hi)
    while f(hi) < 0:
        hi *= 2
    for _ in range(220):
        mid = (lo + hi) / 2
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


def _samples(rng, m):
    # |p| from 1e-8 to 1e3 (both signs), q from -1e-14 to -1e2: covers deep
    # screening (p^{3/2} >> |q|) where the printed Cardano form fails
    p = rng.choice([-1, 1], m) * 10.0 ** rng.uniform(-8, 3, m)
    q = -(10.0 ** rng.uniform(-14, 2, m))
    return p, q


def test_cubic_unique_positive_root_matches_bisection():
    rng = np.random.default_rng(11)
    p, q = _samples(rng, 400)
    got = oracle.cubic_root(p, q)
    worst = 0.0
    for pi, qi, gi in zip(p, q, got):
        P, Q = mp.mpf(pi), mp.mpf(qi)
        ref = _bisect_pos(lambda t: t ** 3 + P * t + Q, 1 + abs(P) + abs(Q))
        worst = max(worst, float(abs((mp.mpf(gi) - ref) / ref)))
    assert worst < 4e-15, worst


def test_cubic_branch_is_largest_real_root_when_q_positive():
    """For q >= 0 (coarse-level symmetron sources) the paper's branches give the
    single real root (Delta > 0) or the largest root (Delta < 0)."""
    rng = np.random.default_rng(12)
    for _ in range(300):
        p = rng.choice([-1, 1]) * 10.0 ** rng.uniform(-3, 2)
        q = 10.0 ** rng.uniform(-4, 2)
        roots = mp.polyroots([1, 0, p, q], maxsteps=200, extraprec=200)
        real = [mp.re(r) for r in roots if abs(mp.im(r)) < mp.mpf(10) ** -30 * (1 + abs(r))]
        ref = max(real)
        got = oracle.cubic_root(p, q)[0]
        assert abs(got - float(ref)) <= 1e-13 * max(1.0, abs(float(ref))), (p, q, got, ref)


def test_cubic_matches_paper_closed_form_where_well_conditioned():
    """Where Cardano does not cancel (Delta != 0, moderate |p|^{3/2}/|q|), the
    paper's printed branches, evaluated at 50 digits, give our root."""
    rng = np.random.default_rng(13)
    for _ in range(200):
        p = rng.choice([-1, 1]) * 10.0 ** rng.uniform(-1, 1)
        q = -(10.0 ** rng.uniform(-1, 1))
        P, Q = mp.mpf(p), mp.mpf(q)
        d0, d1 = -3 * P, 27 * Q
        disc = d1 ** 2 - 4 * d0 ** 3
        if disc > 0:
            x = (d1 + mp.sqrt(disc)) / 2
            C = mp.sign(x) * mp.cbrt(abs(x))  # real cube root
            ref = -(C + d0 / C) / 3
        else:
            th = mp.acos(d1 / (2 * mp.sqrt(d0 ** 3)))
            ref = -mp.mpf(2) / 3 * mp.sqrt(d0) * mp.cos(th / 3 + 2 * mp.pi / 3)
        got = oracle.cubic_root(p, q)[0]
        assert abs(got - float(ref)) <= 1e-14 * abs(float(ref)), (p, q)


def test_printed_delta_zero_branch_is_not_a_root():
    """Reading: for q < 0 the Delta = 0 case means a double root at -sqrt(-p/3)
    and a simple root 3q/p; cbrt(-q) is not a root unless p = 0."""
    q = -2.0
    p = -3.0 * (q * q / 4.0) ** (1.0 / 3.0)  # 4p^3 + 27q^2 = 0
    u = oracle.cubic_root(p, q)[0]
    assert abs(u - 3 * q / p) < 1e-12
    c = (-q) ** (1.0 / 3.0)
    assert abs(c ** 3 + p * c + q) > 0.1


@pytest.mark.parametrize("n", [0, 2])
def test_fr_root_n0_n2_matches_bisection(n):
    rng = np.random.default_rng(20 + n)
    p, q = _samples(rng, 300)
    got = oracle.fr_root(n, p, q)
    for pi, qi, gi in zip(p, q, got):
        P, Q = mp.mpf(pi), mp.mpf(qi)
        ref = _bisect_pos(lambda u: u ** (n + 2) + P * u + Q, 1 + abs(P) + abs(Q))
        assert abs((mp.mpf(gi) - ref) / ref) < 4e-15, (n, pi, qi, gi, ref)
