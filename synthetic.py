"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module holds no part of the method's arithmetic: it only produces
particle positions and density-contrast fields that both the HIP path and the
CPU oracle consume.  The cosmological linear power spectrum the paper uses
(from CAMB) is not available, so a power law stands in for it.

Recipes (all arrays ``[k][j][i]``, i fastest; frequencies in cell units):

* Gaussian field: white noise filtered by ``k^-0.75`` (P(k) ~ k^-1.5), mean
  removed, normalised to unit variance.
* Zel'dovich positions: ``delta_L = sigma_lin g``; displacement
  ``psi = IFFT(i k / k^2 FFT(delta_L))`` (so ``div psi = -delta_L``);
  particle ``q`` on the ``np^3`` lattice sits at ``(q + 1/2) s + psi(q) s``
  modulo N, with ``s = N/np`` the lattice spacing in cells.
* Lognormal field: ``delta = exp(sigma_g g - sigma_g^2/2) - 1`` with
  ``sigma_g^2 = ln(1 + sigma_delta^2)``.
* NFW-like clumps: centres uniform in the box, ``r_s ~ U[1, 4]`` cells, peak
  log-uniform in ``[1e2, 1e4]``, profile ``peak min(1, rho(r)/rho(1/2))`` with
  ``rho = 1/((r/r_s)(1 + r/r_s)^2)``, truncated at ``10 r_s``, minimum-image
  distances; added to ``1 + delta`` which is then renormalised to mean 1.
"""
import numpy as np
import scipy.fft as sfft

C_OVER_H0 = 2997.92458  # Mpc/h


def _kgrid(n):
    k1 = 2.0 * np.pi * np.fft.fftfreq(n)
    kr = 2.0 * np.pi * np.fft.rfftfreq(n)
    return k1[:, None, None], k1[None, :, None], kr[None, None, :]


def gaussian_field(n, rng, slope=-0.75):
    """Unit-variance Gaussian random field with |g_k| ~ k^slope, g(k=0)=0."""
    white = rng.standard_normal((n, n, n))
    kz, ky, kx = _kgrid(n)
    k = np.sqrt(kz * kz + ky * ky + kx * kx)
    k[0, 0, 0] = 1.0
    gk = sfft.rfftn(white, workers=-1) * k ** slope
    gk[0, 0, 0] = 0.0
    g = sfft.irfftn(gk, s=(n, n, n), workers=-1)
    g /= g.std()
    return g


def zeldovich_positions(n_grid, n_part, seed, sigma_lin=1.0, dtype=np.float64):
    """Particle positions (n_part^3, 3) in code units [0, n_grid), columns x,y,z."""
    rng = np.random.default_rng(seed)
    g = gaussian_field(n_part, rng)
    dk = sfft.rfftn(sigma_lin * g, workers=-1)
    kz, ky, kx = _kgrid(n_part)
    k2 = kz * kz + ky * ky + kx * kx
    k2[0, 0, 0] = 1.0
    s = n_grid / n_part
    q = (np.arange(n_part) + 0.5) * s
    out = np.empty((n_part, n_part, n_part, 3), dtype=dtype)
    for axis, kk, grid_shape in ((0, kx, (1, 1, n_part)), (1, ky, (1, n_part, 1)),
                                 (2, kz, (n_part, 1, 1))):
        psi = sfft.irfftn(1j * kk / k2 * dk, s=(n_part,) * 3, workers=-1) * s
        pos = psi + q.reshape(grid_shape)
        out[..., axis] = np.mod(pos, n_grid)
        del psi, pos
    out = out.reshape(-1, 3)
    # a float32 value can round up to exactly n_grid; keep [0, n_grid)
    if dtype == np.float32:
        out[out >= n_grid] = 0.0
    return out


def lognormal_delta(n, seed, sigma_delta=2.0):
    rng = np.random.default_rng(seed)
    g = gaussian_field(n, rng)
    sg2 = np.log1p(sigma_delta ** 2)
    return np.expm1(np.sqrt(sg2) * g - 0.5 * sg2)


def add_nfw_clumps(delta, seed, n_clumps=20, peak_range=(1e2, 1e4), rs_range=(1.0, 4.0)):
    n = delta.shape[0]
    rng = np.random.default_rng(seed)
    rho = 1.0 + delta
    idx = np.arange(n, dtype=np.float64) + 0.5
    for _ in range(n_clumps):
        c = rng.uniform(0.0, n, size=3)
        rs = rng.uniform(*rs_range)
        peak = 10.0 ** rng.uniform(np.log10(peak_range[0]), np.log10(peak_range[1]))
        rmax = 10.0 * rs
        lo = np.floor(c - rmax).astype(int)
        hi = np.ceil(c + rmax).astype(int)
        ii = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        dxs = []
        for a in range(3):
            d = (ii[a] % n) + 0.5 - c[a]
            d = d - n * np.round(d / n)  # minimum image
            dxs.append(d)
        r = np.sqrt(dxs[2][:, None, None] ** 2 + dxs[1][None, :, None] ** 2 +
                    dxs[0][None, None, :] ** 2)
        x = np.maximum(r, 1e-12) / rs
        prof = 1.0 / (x * (1.0 + x) ** 2)
        x0 = 0.5 / rs
        ref = 1.0 / (x0 * (1.0 + x0) ** 2)
        val = peak * np.minimum(1.0, prof / ref)
        val[r > rmax] = 0.0
        kk = (ii[2] % n)[:, None, None]
        jj = (ii[1] % n)[None, :, None]
        iw = (ii[0] % n)[None, None, :]
        np.add.at(rho, (kk, jj, iw), val)
    del idx
    rho /= rho.mean()
    return rho - 1.0


# ---------------------------------------------------------------------------
# The five workloads (sizes, seeds and model parameters)
# ---------------------------------------------------------------------------

def c1_inputs():
    """32^3 grid, 64 Mpc/h box, 32^3 Zel'dovich particles (FP64), seed 1."""
    return dict(n=32, box=64.0, pos=zeldovich_positions(32, 32, seed=1))


def c2_delta(n=256, seed=2):
    """Lognormal sigma_delta = 2 plus 20 NFW-like clumps (peak <= 1e4)."""
    d = lognormal_delta(n, seed)
    return add_nfw_clumps(d, seed + 10000, n_clumps=20)


def c3_positions(n=512, seed=3):
    """n^3 FP32 Zel'dovich particles on an n^3 grid, sigma_lin = 1."""
    return zeldovich_positions(n, n, seed=seed, dtype=np.float32)


def c4_boxes(n_box=64):
    """Per-box (N, box, model, params, delta) for the batched sweep."""
    boxes = []
    for b in range(n_box):
        n = (64, 96, 128)[b % 3]
        rng = np.random.default_rng(4000 + b)
        if b % 2 == 0:
            model = "fr"
            par = dict(fr_n=1, fr0=float(10.0 ** rng.uniform(-7.0, -4.0)))
        else:
            model = "sym"
            par = dict(beta_star=float(rng.uniform(0.5, 2.0)), a_star=0.5, xi=1.0 / C_OVER_H0)
        delta = lognormal_delta(n, 4000 + b)
        boxes.append(dict(n=n, box=float(n), model=model, params=par, delta=delta))
    return boxes


def c5_delta(n=256, seed=5):
    return lognormal_delta(n, seed)


def c5_loss_cells(n=256, count=4096, seed=5005):
    return np.sort(np.random.default_rng(seed).choice(n ** 3, count, replace=False))
