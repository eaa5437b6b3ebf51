"""GPU parity of the particle side after the fifth force: CIC interpolation
of mesh fields to particles, the Newtonian FFT Poisson potential, its
gradient, the symmetron friction term; against the oracle on the same
seeded inputs."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from paper_2110_00328_amd import api

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n,npart", [(24, 20001), (64, 64 ** 3)])
def test_interp_to_particles_matches_oracle(n, npart):
    say("interp", n, npart)
    rng = np.random.default_rng(n)
    pos = rng.uniform(0, n, (npart, 3)).astype(np.float32)
    pos[:50] = rng.integers(0, n, (50, 3)) + 0.0  # on cell corners, incl. the seam
    pos[50:100] = np.float32(n) - np.float32(1e-4)
    grid = rng.standard_normal((3, n, n, n)).astype(np.float32)
    mg = api.Context(n, device=DEV)
    got = mg.interp_to_particles(torch.from_numpy(grid).to(DEV), torch.from_numpy(pos).to(DEV))
    ref = oracle.interp(n, pos.astype(np.float64), grid.astype(np.float64))
    err = np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max()
    say(f"  max rel {err:.1e}")
    assert err < 1e-6
    tpos = torch.from_numpy(pos).to(DEV)
    for nc in (1, 2):  # fewer components, and a plain (n, n, n) grid
        sub = mg.interp_to_particles(torch.from_numpy(np.ascontiguousarray(grid[:nc])).to(DEV), tpos)
        assert sub.shape == (npart, nc)
        assert np.abs(sub.cpu().numpy() - ref[:, :nc]).max() <= 1e-6 * np.abs(ref).max()
    one = mg.interp_to_particles(torch.from_numpy(np.ascontiguousarray(grid[2])).to(DEV), tpos)
    assert one.shape == (npart,)
    assert np.abs(one.cpu().numpy() - ref[:, 2]).max() <= 1e-6 * np.abs(ref).max()
    f64 = rng.standard_normal((n, n, n))
    g1 = mg.interp_field_to_particles(torch.from_numpy(f64).to(DEV), torch.from_numpy(pos).to(DEV))
    r1 = oracle.interp(n, pos.astype(np.float64), f64)
    assert np.abs(g1.cpu().numpy() - r1).max() <= 1e-13 * np.abs(r1).max()
    mg.close()


@pytest.mark.parametrize("n", [18, 32, 48, 128])
def test_poisson_newton_and_gradient_match_oracle(n):
    say("poisson", n)
    P = oracle.params(oracle.FR, n, float(n), a=0.8)
    prm = api.model_params(float(n), a=0.8)
    d = synthetic.lognormal_delta(n, 300 + n, sigma_delta=2.0).astype(np.float32)
    mg = api.Context(n, device=DEV)
    phi = mg.poisson_newton(prm, torch.from_numpy(d).to(DEV))
    ref = oracle.poisson_newton(P, d.astype(np.float64))
    err = np.linalg.norm(phi.cpu().numpy() - ref) / np.linalg.norm(ref)
    g = mg.gradient(phi).cpu().numpy().astype(np.float64)
    gref = oracle.gradient(ref)
    gerr = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"  phi {err:.1e} grad {gerr:.1e}")
    assert err < 1e-12 and gerr < 1e-6
    mg.close()


@pytest.mark.parametrize("a", [1.0, 0.8])
def test_symmetron_friction_matches_oracle(a):
    n, npart = 32, 5000
    say("symmetron friction, a =", a)
    kw = dict(a=a, a_star=0.5, xi=1.0 / oracle.C_OVER_H0, beta_star=1.2)
    P = oracle.params(oracle.SYM, n, float(n), **kw)
    prm = api.model_params(float(n), **kw)
    rng = np.random.default_rng(9)
    u = rng.uniform(0.3, 1.0, (n, n, n))
    pos = rng.uniform(0, n, (npart, 3)).astype(np.float32)
    pos[:20, 0] = np.float32(n - 0.25)  # lower cell n - 1: the x pair wraps the seam
    pos[20:40, 0] = np.float32(0.25)    # lower cell -1 -> n - 1
    mom = rng.standard_normal((npart, 3)).astype(np.float32)
    mg = api.Context(n, device=DEV)
    got = mg.symmetron_friction(prm, torch.from_numpy(u).to(DEV), torch.from_numpy(pos).to(DEV),
                                torch.from_numpy(mom).to(DEV)).cpu().numpy()
    ref = oracle.sym_friction(P, u, pos.astype(np.float64), mom.astype(np.float64))
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
    with pytest.raises(api.MGError):
        mg.symmetron_friction(api.model_params(float(n), a=0.4, a_star=0.5),
                              torch.from_numpy(u).to(DEV), torch.from_numpy(pos).to(DEV),
                              torch.from_numpy(mom).to(DEV))
    mg.close()


@pytest.mark.parametrize("model,n", [("fr", 32), ("sym", 18), ("cq", 40), ("cq", 18)])
def test_total_force_matches_oracle(model, n):
    """Newtonian and fifth-force potentials summed, then differenced; both
    force kernels (z-marching for n % 4 == 0, per cell otherwise)."""
    say("total force", model, n)
    rng = np.random.default_rng(70 + n)
    mid = {"fr": oracle.FR, "sym": oracle.SYM, "cq": oracle.CQ}[model]
    P = oracle.params(mid, n, 2.0 * n, a=0.9)
    prm = api.model_params(2.0 * n, a=0.9)
    phin = 1e-3 * rng.standard_normal((n, n, n))
    if model == "fr":
        w = 1e-6 * rng.uniform(0.5, 2.0, (n, n, n))
        field, vora = -w, w  # the library's f(R) field is f_R = -w
    elif model == "sym":
        field = rng.uniform(0.0, 1.0, (n, n, n))
        vora = field
    else:
        field = rng.standard_normal((n, n, n))
        vora = field
    mg = api.Context(n, device=DEV)
    g = mg.total_force(model, prm, torch.from_numpy(phin).to(DEV),
                       torch.from_numpy(np.ascontiguousarray(field)).to(DEV)).cpu().numpy()
    ref = oracle.total_force(P, phin, vora)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    say(f"  max rel {err:.1e}")
    assert err < 1e-6
    mg.close()


def test_empty_particle_sets_are_no_ops():
    n = 16
    mg = api.Context(n, device=DEV)
    pos = torch.empty((0, 3), dtype=torch.float32, device=DEV)
    g = torch.zeros((3, n, n, n), dtype=torch.float32, device=DEV)
    assert mg.interp_to_particles(g, pos).shape == (0, 3)
    f = torch.zeros((n, n, n), dtype=torch.float64, device=DEV)
    assert mg.interp_field_to_particles(f, pos).shape == (0,)
    prm = api.model_params(float(n), a=1.0, a_star=0.5)
    assert mg.symmetron_friction(prm, f + 0.5, pos, pos.clone()).shape == (0, 3)
    mg.close()


def test_particle_side_error_paths():
    """Bad arguments are rejected with MG_EINVAL and leave the context usable."""
    n = 16
    mg = api.Context(n, device=DEV)
    L = mg.lib
    prm = api.model_params(float(n))
    g = torch.zeros((4, n, n, n), dtype=torch.float32, device=DEV)
    pos = torch.full((10, 3), 1.5, dtype=torch.float32, device=DEV)
    out = torch.empty((10, 4), dtype=torch.float32, device=DEV)
    import ctypes
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.mg_interp_to_particles(mg.ptr, vp(g), 4, vp(pos), 10, vp(out)) == api.L.MG_EINVAL
    assert L.mg_interp_to_particles(mg.ptr, vp(g), 0, vp(pos), 10, vp(out)) == api.L.MG_EINVAL
    assert L.mg_interp_to_particles(mg.ptr, vp(g), 3, vp(pos), -1, vp(out)) == api.L.MG_EINVAL
    assert L.mg_interp_to_particles(mg.ptr, None, 3, vp(pos), 10, vp(out)) == api.L.MG_EINVAL
    phi = torch.zeros((n, n, n), dtype=torch.float64, device=DEV)
    f = torch.empty((3, n, n, n), dtype=torch.float32, device=DEV)
    assert L.mg_gradient(mg.ptr, None, vp(f)) == api.L.MG_EINVAL
    assert L.mg_total_force(mg.ptr, api.L.MG_FR, ctypes.byref(prm), None, vp(phi), vp(f)) == \
        api.L.MG_EINVAL
    assert L.mg_total_force(mg.ptr, 7, ctypes.byref(prm), vp(phi), vp(phi), vp(f)) == api.L.MG_EINVAL
    bad = api.model_params(float(n), a=-1.0)
    assert L.mg_poisson_newton(mg.ptr, ctypes.byref(bad), vp(g), vp(phi)) == api.L.MG_EINVAL
    with pytest.raises(api.MGError):
        mg.symmetron_friction(api.model_params(float(n), a=0.5, a_star=0.5), phi + 0.5, pos, pos)
    assert mg.lib.mg_last_error(mg.ptr)  # a message is kept
    # the context still works after the rejected calls
    d = torch.zeros((n, n, n), dtype=torch.float32, device=DEV)
    out_phi = mg.poisson_newton(prm, d)
    assert torch.count_nonzero(out_phi).item() == 0
    mg.close()


@pytest.mark.parametrize("n", [64, 128, 48])
@pytest.mark.parametrize("model", ["fr", "sym", "cq"])
def test_force_kernels_bit_identical(model, n):
    """The tiled z-marching force kernel (n % 64 == 0), the row-chunk one
    (n % 4 == 0) and the per-cell one (taken for an output that is not
    16-byte aligned) do the same arithmetic: fifth force, total force and
    the force adjoint agree bit for bit."""
    say("force kernels", model, n)
    rng = np.random.default_rng(90 + n)
    prm = api.model_params(2.0 * n, a=0.9)
    if model == "fr":
        field = -1e-6 * rng.uniform(0.5, 2.0, (n, n, n))
    elif model == "sym":
        field = rng.uniform(0.0, 1.0, (n, n, n))
    else:
        field = rng.standard_normal((n, n, n))
    f = torch.from_numpy(field).to(DEV)
    phin = torch.from_numpy(1e-3 * rng.standard_normal((n, n, n))).to(DEV)
    mg = api.Context(n, device=DEV)
    for total in (False, True):
        fast = mg.total_force(model, prm, phin, f) if total else mg.force(model, prm, f)
        big = torch.empty(3 * n ** 3 + 1, dtype=torch.float32, device=DEV)
        slow = big[1:].view(3, n, n, n)
        if total:
            mg.total_force(model, prm, phin, f, out=slow)
        else:
            mg.force(model, prm, f, out=slow)
        a, b = fast.cpu().numpy(), slow.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (total, np.abs(a - b).max())
    # the force adjoint: tiled (n % 64 == 0) or per cell, the same bits
    gfo = torch.from_numpy(rng.standard_normal((3, n, n, n)).astype(np.float32)).to(DEV)
    fast = mg.force_adjoint(model, prm, f, gfo)
    big = torch.empty(n ** 3 + 1, dtype=torch.float64, device=DEV)
    slow = big[1:].view(n, n, n)
    mg.force_adjoint(model, prm, f, gfo, out=slow)
    a, b = fast.cpu().numpy(), slow.cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), np.abs(a - b).max()
    mg.close()
