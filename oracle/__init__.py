"""FP64 CPU oracle for the MG-GLAM scalar-field hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check and the bench's
``cpu_baseline`` leg may import this package.  It wraps ``mg_oracle.c`` (plain
C, FP64, natural ``[k][j][i]`` layout) through ctypes and shares nothing with
the HIP library.  Citations refer to Ruan et al., arXiv:2110.00328.

Conventions: the solved variable is ``w = -f_R`` for f(R), ``u = phi/phi_*``
for the symmetron and ``phi~ = c~^2 delta-phi`` for coupled quintessence.
"""
import ctypes
import os

import numpy as np

from . import build as _build

FR, SYM, CQ = 0, 1, 2
C_OVER_H0 = 2997.92458  # Mpc/h

_lib = None


class Params(ctypes.Structure):
    """Mirror of ``ora_params`` in mg_oracle.c."""

    _fields_ = [
        ("model", ctypes.c_int),
        ("n", ctypes.c_int),
        ("box", ctypes.c_double),
        ("a", ctypes.c_double),
        ("omega_m", ctypes.c_double),
        ("fr_n", ctypes.c_int),
        ("fr0", ctypes.c_double),
        ("a_star", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("beta_star", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("phibar", ctypes.c_double),
        ("lam", ctypes.c_double),
        ("cq_keep_exp", ctypes.c_int),
    ]


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(Params)
        L.ora_ctilde.restype = ctypes.c_double
        L.ora_ctilde.argtypes = [ctypes.c_int, ctypes.c_double]
        L.ora_background.restype = ctypes.c_double
        L.ora_background.argtypes = [P]
        L.ora_cubic_root.restype = ctypes.c_double
        L.ora_cubic_root.argtypes = [ctypes.c_double, ctypes.c_double]
        L.ora_fr_root.restype = ctypes.c_double
        L.ora_fr_root.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.ora_cubic_root_vec.argtypes = [ctypes.c_int64, dp, dp, dp]
        L.ora_fr_root_vec.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp]
        L.ora_residual.restype = ctypes.c_double
        L.ora_residual.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp, dp, dp]
        L.ora_relax_colour.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp, dp, ctypes.c_int]
        L.ora_relax.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.ora_restrict.argtypes = [ctypes.c_int, dp, dp]
        L.ora_prolong_add.argtypes = [ctypes.c_int, dp, dp]
        L.ora_num_levels.restype = ctypes.c_int
        L.ora_num_levels.argtypes = [ctypes.c_int]
        L.ora_background_resid_rms.restype = ctypes.c_double
        L.ora_background_resid_rms.argtypes = [P, dp]
        L.ora_solve.restype = ctypes.c_int
        L.ora_solve.argtypes = [P, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, dp, dp]
        L.ora_force.argtypes = [P, dp, dp]
        L.ora_cic.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp]
        L.ora_dense_solve.restype = ctypes.c_int
        L.ora_dense_solve.argtypes = [ctypes.c_int, dp, dp]
        L.ora_cg.restype = ctypes.c_int
        L.ora_cg.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, ctypes.c_double,
                             ctypes.c_int, dp]
        L.ora_lin_mg.restype = ctypes.c_int
        L.ora_lin_mg.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, ctypes.c_double,
                                 ctypes.c_int, dp]
        L.ora_adjoint.restype = ctypes.c_int
        L.ora_adjoint.argtypes = [P, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        L.ora_apply_jacobian.argtypes = [P, dp, dp, dp, dp]
        L.ora_force_adjoint.argtypes = [P, dp, dp, dp]
        L.ora_interp.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, ctypes.c_int, dp]
        L.ora_sym_friction.argtypes = [P, dp, dp, dp, ctypes.c_int64, dp]
        L.ora_gradient.argtypes = [ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    assert x.dtype == np.float64 and x.flags["C_CONTIGUOUS"]
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def params(model, n, box, a=1.0, omega_m=0.3, fr_n=1, fr0=1e-5, a_star=0.5,
           xi=1.0 / C_OVER_H0, beta_star=1.0, alpha=0.1, beta=-0.2, phibar=0.5,
           lam=None, cq_keep_exp=1):
    """Model parameters in the paper's notation (Sec. 2).  ``lam`` defaults
    to the stand-in ``lambda^2 = Omega_L phibar^alpha`` (no CQ background
    solve is part of this path)."""
    if lam is None:
        lam = float(np.sqrt((1.0 - omega_m) * phibar ** alpha))
    return Params(model, n, box, a, omega_m, fr_n, fr0, a_star, xi, beta_star, alpha,
                  beta, phibar, lam, cq_keep_exp)


def ctilde(n, box):
    """c~ = N (c/H0) / L (Sec. 3.1.1)."""
    return lib().ora_ctilde(n, box)


def background(P):
    """Background value of the solved variable (eq:field_uniform_dens_test)."""
    return lib().ora_background(ctypes.byref(P))


def cubic_root(p, q):
    p = _f64(np.atleast_1d(p))
    q = _f64(np.atleast_1d(q))
    out = np.empty_like(p)
    lib().ora_cubic_root_vec(p.size, _ptr(p), _ptr(q), _ptr(out))
    return out


def fr_root(n, p, q):
    p = _f64(np.atleast_1d(p))
    q = _f64(np.atleast_1d(q))
    out = np.empty_like(p)
    lib().ora_fr_root_vec(n, p.size, _ptr(p), _ptr(q), _ptr(out))
    return out


def residual(P, delta, v, S=None, h=1.0):
    """d = L^h(v) - S (eq:residual_d).  Returns (d, sum of d^2)."""
    delta = _f64(delta)
    v = _f64(v)
    S = None if S is None else _f64(S)
    d = np.empty_like(v)
    n = v.shape[0]
    ss = lib().ora_residual(ctypes.byref(P), n, h, _ptr(delta), _ptr(S), _ptr(v), _ptr(d))
    return d, ss


def relax_colour(P, delta, v, colour, S=None, h=1.0):
    """One half-sweep on cells with (i+j+k)%2 == colour; returns a new array."""
    delta = _f64(delta)
    out = _f64(v).copy()
    S = None if S is None else _f64(S)
    lib().ora_relax_colour(ctypes.byref(P), out.shape[0], h, _ptr(delta), _ptr(S), _ptr(out),
                           colour)
    return out


def restrict(f):
    f = _f64(f)
    n = f.shape[0]
    c = np.empty((n // 2,) * 3)
    lib().ora_restrict(n, _ptr(f), _ptr(c))
    return c


def prolong_add(c, f):
    """Returns f + P(c) (eq:solution_correction)."""
    c = _f64(c)
    out = _f64(f).copy()
    lib().ora_prolong_add(c.shape[0], _ptr(c), _ptr(out))
    return out


def num_levels(n):
    return lib().ora_num_levels(n)


def background_resid_rms(P, delta):
    return lib().ora_background_resid_rms(ctypes.byref(P), _ptr(_f64(delta)))


_CYCLES = {"V": 0, "F": 1, "W": 2}


def solve(P, delta, v0=None, tol=1e-12, max_cycles=200, nu1=1, nu2=1, cycle="V"):
    """FAS multigrid solve of L(v) = 0 (Sec. 3.2.1).  Returns
    (v, cycles, final relative residual, history)."""
    delta = _f64(delta)
    n = delta.shape[0]
    if v0 is None:
        v = np.full((n, n, n), background(P))
    else:
        v = _f64(v0).copy()
    rel = ctypes.c_double(0.0)
    hist = np.zeros(max(max_cycles, 1))
    cyc = lib().ora_solve(ctypes.byref(P), _ptr(delta), _ptr(v), tol, max_cycles, nu1, nu2,
                          _CYCLES[cycle], ctypes.byref(rel), _ptr(hist))
    return v, cyc, rel.value, hist[:cyc].copy()


def force(P, v):
    """g5 = -grad Phi5 by central differences; shape (3, N, N, N)."""
    v = _f64(v)
    out = np.empty((3,) + v.shape)
    lib().ora_force(ctypes.byref(P), _ptr(v), _ptr(out))
    return out


def cic(n, pos):
    """CIC density contrast from positions (np, 3) in code units [0, n)."""
    pos = _f64(pos).reshape(-1, 3)
    out = np.empty((n, n, n))
    lib().ora_cic(n, pos.shape[0], _ptr(pos), _ptr(out))
    return out


def dense_solve(A, b):
    A = _f64(A).copy()
    b = _f64(b).copy()
    rc = lib().ora_dense_solve(b.size, _ptr(A), _ptr(b))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return b


def cg(kap, dg, b, tol=1e-12, maxit=100000):
    dg = _f64(dg)
    b = _f64(b)
    x = np.zeros_like(b)
    rel = ctypes.c_double(0.0)
    it = lib().ora_cg(b.shape[0], kap, _ptr(dg), _ptr(b), _ptr(x), tol, maxit, ctypes.byref(rel))
    return x, it, rel.value


def lin_mg(kap, dg, b, tol=1e-12, maxit=500):
    dg = _f64(dg)
    b = _f64(b)
    x = np.zeros_like(b)
    rel = ctypes.c_double(0.0)
    it = lib().ora_lin_mg(b.shape[0], kap, _ptr(dg), _ptr(b), _ptr(x), tol, maxit,
                          ctypes.byref(rel))
    return x, it, rel.value


def adjoint(P, delta, v, grad_v, tol=1e-12, solver="mg"):
    """dL/d(delta) from dL/dv at the converged field v."""
    delta = _f64(delta)
    v = _f64(v)
    grad_v = _f64(grad_v)
    out = np.empty_like(v)
    rel = ctypes.c_double(0.0)
    it = lib().ora_adjoint(ctypes.byref(P), _ptr(delta), _ptr(v), _ptr(grad_v), _ptr(out), tol,
                           1 if solver == "cg" else 0, ctypes.byref(rel))
    return out, it, rel.value


def apply_jacobian(P, delta, v, x):
    delta, v, x = _f64(delta), _f64(v), _f64(x)
    y = np.empty_like(x)
    lib().ora_apply_jacobian(ctypes.byref(P), _ptr(delta), _ptr(v), _ptr(x), _ptr(y))
    return y


def force_adjoint(P, v, gforce):
    v = _f64(v)
    gforce = _f64(gforce)
    out = np.empty_like(v)
    lib().ora_force_adjoint(ctypes.byref(P), _ptr(v), _ptr(gforce), _ptr(out))
    return out


# --- the particle side after the fifth force --------------------------------
def interp(n, pos, grid):
    """CIC interpolation of a mesh field (ncomp, N, N, N) or (N, N, N) to
    particles (np, 3); returns (np, ncomp) or (np,)."""
    g = _f64(grid)
    scalar = g.ndim == 3
    g = g.reshape(1 if scalar else g.shape[0], -1)
    pos = _f64(pos).reshape(-1, 3)
    out = np.empty((pos.shape[0], g.shape[0]))
    lib().ora_interp(n, pos.shape[0], _ptr(pos), _ptr(np.ascontiguousarray(g)), g.shape[0],
                     _ptr(out))
    return out[:, 0] if scalar else out


def sym_friction(P, u, pos, mom):
    """Symmetron friction force per particle (eq:F_x_codeunit)."""
    pos = _f64(pos).reshape(-1, 3)
    mom = _f64(mom).reshape(-1, 3)
    out = np.empty_like(pos)
    lib().ora_sym_friction(ctypes.byref(P), _ptr(_f64(u)), _ptr(pos), _ptr(mom), pos.shape[0],
                           _ptr(out))
    return out


def gradient(phi):
    """-grad phi by central differences, shape (3, N, N, N)."""
    phi = _f64(phi)
    out = np.empty((3,) + phi.shape)
    lib().ora_gradient(phi.shape[0], _ptr(phi), _ptr(out))
    return out


def total_force(P, phi_n, v):
    """Newtonian plus fifth force, -grad(s_N Phi_N + Phi5): the two potentials
    are summed on the grid and then differenced (the paper's treatment of
    coupled quintessence after eq:csf_particle_geodesic_code2).  For CQ the
    standard Poisson potential is scaled by exp(beta phibar), the background
    factor of eq:csf_poisson_code, which the paper applies to the Newtonian
    force instead of the source.  gradient() and force() are both linear in
    the potential, so their sum is the difference of the summed potential."""
    sn = np.exp(P.beta * P.phibar) if P.model == CQ else 1.0
    return gradient(sn * _f64(phi_n)) + force(P, v)


def poisson_newton(P, delta):
    """Newtonian potential of eq:GR_poisson_codeunit on the grid: the
    zero-mean solution of (7-point Laplacian) Phi = (3/2) Omega_m a^-1 delta,
    by FFT (numpy) with the discrete symbol -4 sum sin^2(pi m_i / N)."""
    d = _f64(delta)
    n = d.shape[0]
    s = np.sin(np.pi * np.fft.fftfreq(n)) ** 2  # sin^2(pi m / N)
    sr = np.sin(np.pi * np.fft.rfftfreq(n)) ** 2
    k2 = 4.0 * (s[:, None, None] + s[None, :, None] + sr[None, None, :])
    k2[0, 0, 0] = 1.0
    src = 1.5 * P.omega_m / P.a * np.fft.rfftn(d)
    phik = -src / k2
    phik[0, 0, 0] = 0.0
    return np.fft.irfftn(phik, s=d.shape, axes=(0, 1, 2))
