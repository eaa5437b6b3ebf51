"""Full-size parity: the workloads the benchmark and the parity cases name,
at their real sizes, against the FP64 CPU oracle.

- 512^3 f(R) (|f_R0| = 1e-5 and 1e-6), the bench's pipeline and launch
  configuration (CIC of 512^3 FP32 Zel'dovich particles, FP32-refined
  V(1,1) to relative residual 1e-6): CIC against the oracle's CIC; field and
  force against the oracle's solve of the oracle's own density to 1e-10; the
  oracle's residual of the GPU field; the plain FP64 GPU solve beside it;
  the fused prolongation/half-sweep kernels against the separate ones, bit
  for bit, through the forward solve and the adjoint.
- 512^3 coupled quintessence, with and without exp(beta phi~/c~^2) before
  (1+delta): field and force against the oracle's solve of the same density,
  the oracle's residual of the GPU field, FP32-refined against FP64.
- 256^3 f(R) and symmetron on a lognormal field with 20 NFW-like clumps
  (peak delta up to 1e4): field and force against the oracle.
- 256^3 f(R) adjoint of Loss = sum over 4096 cells of |F5|^2: against the
  oracle's FP64 adjoint and against central finite differences of FP64 GPU
  solves (h = 1e-4 on delta at 16 probe cells).
- The autograd path (solve_force + backward) against the explicit adjoint
  chain.
- 512^3 particle side in the bench's configuration (512^3 particles): the FFT
  potential through the discrete Poisson equation at sampled cells (a
  property at any size), the total force and the CIC interpolation to
  sampled particles and the symmetron friction against the oracle.

Error metrics as in the other parity tests: field_err =
||x - x_ora|| / ||x_ora - x_bg||, force_err = ||g - g_ora|| / ||g_ora||, and
the same ratios in the max norm.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import synthetic
from paper_2110_00328_amd import api

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
CH = oracle.C_OVER_H0


def say(*a):
    print(*a, flush=True)


def rel_err(x, ref, bg=0.0):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref - bg))


def max_err(x, ref, bg=0.0):
    """max |x - ref| / max |ref - bg|: an error confined to a few cells (a
    clump) shows here long before it moves the L2 ratio."""
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref - bg)))


@pytest.fixture(scope="module")
def c3():
    n = 512
    t0 = time.perf_counter()
    pos32 = synthetic.c3_positions(n)
    say(f"c3 positions {time.perf_counter() - t0:.1f} s")
    pos = torch.from_numpy(pos32).to(DEV)
    mg = api.Context(n, device=DEV)
    delta = mg.cic(pos)
    t0 = time.perf_counter()
    d_ora = oracle.cic(n, pos32.astype(np.float64))
    say(f"oracle CIC {time.perf_counter() - t0:.1f} s")
    d_gpu = delta.cpu().numpy()
    err = np.max(np.abs(d_gpu - d_ora)) / np.max(np.abs(d_ora))
    say(f"512^3 CIC max|diff|/max|delta| = {err:.2e}, sigma_delta = {d_ora.std():.3f}")
    del pos
    yield dict(n=n, mg=mg, delta=delta, d_ora=d_ora, cic_err=err, pos32=pos32)
    mg.close()


def test_c3_cic_matches_oracle(c3):
    assert c3["cic_err"] < 1e-6


@pytest.mark.parametrize("fr0", [1e-5, 1e-6])
def test_c3_fr_solve_and_force_match_oracle(c3, fr0):
    n, mg, delta = c3["n"], c3["mg"], c3["delta"]
    P = oracle.params(oracle.FR, n, float(n), fr0=fr0)
    prm = api.model_params(float(n), fr0=fr0)
    t0 = time.perf_counter()
    ref, cyc, rel_o, _ = oracle.solve(P, c3["d_ora"], tol=1e-10, max_cycles=100)
    say(f"fr0={fr0:g}: oracle solve {time.perf_counter() - t0:.1f} s, {cyc} cycles, rel {rel_o:.1e}")
    g_ref = oracle.force(P, ref)
    bg = -oracle.background(P)
    ref = -ref  # f_R
    out = {}
    for prec in ("fp32", "fp64"):
        field, st = mg.solve("fr", prm, delta, tol=1e-6, opts=api.solver_opts(precision=prec))
        g = mg.force("fr", prm, field).cpu().numpy().astype(np.float64)
        x = field.cpu().numpy()
        ferr, gerr = rel_err(x, ref, bg), rel_err(g, g_ref)
        fmax, gmax = max_err(x, ref, bg), max_err(g, g_ref)
        # the oracle's own relative residual of the GPU field (on the GPU's density)
        r, _ = oracle.residual(P, delta.cpu().numpy().astype(np.float64), -x)
        rel_by_oracle = np.sqrt(np.mean(r * r)) / oracle.background_resid_rms(
            P, delta.cpu().numpy().astype(np.float64))
        say(f"  {prec}: V-cycles={st.vcycles} rel={st.rel_resid:.2e} oracle-rel={rel_by_oracle:.2e} "
            f"field_err={ferr:.2e} (max {fmax:.2e}) force_err={gerr:.2e} (max {gmax:.2e})")
        out[prec] = (ferr, gerr, fmax, gmax, rel_by_oracle, st.rel_resid)
    for prec, (ferr, gerr, fmax, gmax, rel_o2, rel_g) in out.items():
        assert rel_o2 <= 1e-6 and abs(rel_o2 - rel_g) <= 1e-3 * rel_g + 1e-12
        assert ferr < 1e-5 and gerr < 1e-5 and fmax < 1e-5 and gmax < 1e-5


def test_c3_fused_prolongation_is_bit_identical(c3, monkeypatch):
    """The bench's pipeline and launch configuration (512^3, 16-bit level-0
    storage): the prolongation fused into the first post-smoothing
    half-sweep of the finest level, forward and adjoint, gives the same
    field and density gradient, bit for bit, as the separate kernels."""
    n, delta = c3["n"], c3["delta"]
    prm = api.model_params(float(n), fr0=1e-5)
    cells = torch.from_numpy(np.random.default_rng(7).choice(n ** 3, 4096, replace=False)).to(DEV)
    opts = api.solver_opts(precision="fp32")
    outs = []
    for pk in (None, "0"):
        if pk is None:
            monkeypatch.delenv("MGGPU_PROLONG_SMOOTH_KT", raising=False)
        else:
            monkeypatch.setenv("MGGPU_PROLONG_SMOOTH_KT", pk)
        mg = api.Context(n, device=DEV)
        field, st = mg.solve("fr", prm, delta, tol=1e-6, opts=opts)
        _, gforce = mg.loss_force_sq(mg.force("fr", prm, field), cells)
        gfield = mg.force_adjoint("fr", prm, field, gforce)
        gd, st2 = mg.solve_adjoint("fr", prm, delta, field, gfield, tol=1e-6, opts=opts)
        outs.append((field.cpu().numpy(), gd.cpu().numpy(), st.vcycles, st2.vcycles))
        say(f"  fused={pk is None}: V-cycles {st.vcycles} / {st2.vcycles}")
        mg.close()
    assert outs[0][2:] == outs[1][2:]
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("keep_exp", [1, 0])
def test_c3_cq_solve_and_force_match_oracle(c3, keep_exp):
    """512^3 coupled quintessence, eq:csf_eom_code as printed (keep_exp = 1)
    and with exp(beta phi~/c~^2) dropped as the paper's runs do (keep_exp =
    0): field (uniform mode removed: it is fixed only to ~tol/m^2 and the
    force does not see it) and force against the oracle's solve of the same
    density to 1e-9; the oracle's residual of the GPU field; FP32-refined
    against FP64 on the GPU."""
    n, mg, delta = c3["n"], c3["mg"], c3["delta"]
    P = oracle.params(oracle.CQ, n, float(n), cq_keep_exp=keep_exp)
    prm = api.model_params(float(n), cq_keep_exp=keep_exp)
    d64 = delta.cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    ref, cyc, rel_ref, _ = oracle.solve(P, d64, tol=1e-9, max_cycles=200)
    say(f"cq keep_exp={keep_exp}: oracle solve {time.perf_counter() - t0:.1f} s, {cyc} cycles, "
        f"rel {rel_ref:.1e}")
    g_ref = oracle.force(P, ref)
    ref0 = ref - ref.mean()
    eps_bg = oracle.background_resid_rms(P, d64)
    fields = {}
    for prec in ("fp32", "fp64"):
        field, st = mg.solve("cq", prm, delta, tol=1e-6, opts=api.solver_opts(precision=prec))
        x = field.cpu().numpy()
        r, _ = oracle.residual(P, d64, x)
        rel_o = np.sqrt(np.mean(r * r)) / eps_bg
        g = mg.force("cq", prm, field).cpu().numpy().astype(np.float64)
        x0 = x - x.mean()
        ferr, fmax = rel_err(x0, ref0), max_err(x0, ref0)
        gerr, gmax = rel_err(g, g_ref), max_err(g, g_ref)
        say(f"  cq {prec}: V-cycles={st.vcycles} rel={st.rel_resid:.2e} oracle-rel={rel_o:.2e} "
            f"field_err={ferr:.2e} (max {fmax:.2e}) force_err={gerr:.2e} (max {gmax:.2e})")
        assert rel_o <= 1e-6 and abs(rel_o - st.rel_resid) <= 1e-3 * st.rel_resid + 1e-12
        assert ferr < 1e-5 and gerr < 1e-5 and fmax < 1e-5 and gmax < 1e-5
        fields[prec] = x
    a, b = fields["fp32"], fields["fp64"]
    err = rel_err(a - a.mean(), b - b.mean())
    say(f"  cq fp32 vs fp64 (uniform mode removed): {err:.2e}")
    assert err < 1e-5


@pytest.fixture(scope="module")
def c2():
    n = 256
    d = synthetic.c2_delta(n).astype(np.float32)
    say(f"c2 delta: sigma={d.std():.2f} max={d.max():.3g}")
    mg = api.Context(n, device=DEV)
    yield dict(n=n, d32=d, delta=torch.from_numpy(d).to(DEV), mg=mg)
    mg.close()


@pytest.mark.parametrize("model", ["fr", "sym"])
def test_c2_fp32_solve_and_force_match_oracle(c2, model):
    n, mg = c2["n"], c2["mg"]
    if model == "fr":
        P = oracle.params(oracle.FR, n, float(n), fr0=1e-5)
        prm = api.model_params(float(n), fr0=1e-5)
    else:
        kw = dict(a_star=0.5, xi=1.0 / CH, beta_star=1.0)
        P = oracle.params(oracle.SYM, n, float(n), **kw)
        prm = api.model_params(float(n), **kw)
    d64 = c2["d32"].astype(np.float64)
    t0 = time.perf_counter()
    ref, cyc, rel_o, _ = oracle.solve(P, d64, tol=1e-10, max_cycles=200)
    say(f"{model}: oracle {time.perf_counter() - t0:.1f} s, {cyc} cycles, rel {rel_o:.1e}")
    g_ref = oracle.force(P, ref)
    sgn = -1.0 if model == "fr" else 1.0
    bg = sgn * oracle.background(P)
    for tol in (1e-6, 1e-8):
        field, st = mg.solve(model, prm, c2["delta"], tol=tol, opts=api.solver_opts(precision="fp32"))
        g = mg.force(model, prm, field).cpu().numpy().astype(np.float64)
        x = field.cpu().numpy()
        ferr, fmax = rel_err(x, sgn * ref, bg), max_err(x, sgn * ref, bg)
        gerr, gmax = rel_err(g, g_ref), max_err(g, g_ref)
        say(f"  tol {tol:g}: V-cycles={st.vcycles} rel={st.rel_resid:.2e} field_err={ferr:.2e} "
            f"(max {fmax:.2e}) force_err={gerr:.2e} (max {gmax:.2e})")
        # the stated 1e-5 at the configured tolerance; 1e-6 when driven to 1e-8
        lim = 1e-5 if tol == 1e-6 else 1e-6
        assert ferr < lim and gerr < lim
        assert fmax < 1e-5 and gmax < 1e-5


@pytest.fixture(scope="module")
def c5():
    n = 256
    d = synthetic.c5_delta(n).astype(np.float32)
    cells = synthetic.c5_loss_cells(n)
    mg = api.Context(n, device=DEV)
    P = oracle.params(oracle.FR, n, float(n), fr0=1e-5)
    prm = api.model_params(float(n), fr0=1e-5)
    yield dict(n=n, d32=d, delta=torch.from_numpy(d).to(DEV), cells=cells,
               cells_t=torch.from_numpy(cells).to(DEV), mg=mg, P=P, prm=prm)
    mg.close()


def _loss64(mg, prm, field, cells_t):
    """Loss in FP64 from an FP64 field (central differences of Phi5 = -c~^2 f_R / 2)."""
    n = field.shape[0]
    ct = n * CH / float(n)  # c~ for 1 Mpc/h cells
    phi = -0.5 * ct * ct * field
    g = []
    for ax in (2, 1, 0):  # x, y, z
        g.append(-0.5 * (torch.roll(phi, -1, dims=ax) - torch.roll(phi, 1, dims=ax)))
    g = torch.stack(g).reshape(3, -1)[:, cells_t]
    return float((g * g).sum()), g


def test_c5_adjoint_matches_oracle_and_finite_differences(c5):
    n, mg, P, prm = c5["n"], c5["mg"], c5["P"], c5["prm"]
    cells_t = c5["cells_t"]
    # forward (FP32-refined, as the bench) and the adjoint chain on the GPU
    field, _ = mg.solve("fr", prm, c5["delta"], tol=1e-10, opts=api.solver_opts(precision="fp32"))
    force = mg.force("fr", prm, field)
    loss, gforce = mg.loss_force_sq(force, cells_t)
    gfield = mg.force_adjoint("fr", prm, field, gforce)
    gd32, st32 = mg.solve_adjoint("fr", prm, c5["delta"], field, gfield, tol=1e-8,
                                  opts=api.solver_opts(precision="fp32"))
    gd64, st64 = mg.solve_adjoint("fr", prm, c5["delta"], field, gfield, tol=1e-11,
                                  opts=api.solver_opts(precision="fp64"))
    gd32, gd64 = gd32.cpu().numpy(), gd64.cpu().numpy()
    # oracle: its own solve and adjoint of the same loss
    d64 = c5["d32"].astype(np.float64)
    t0 = time.perf_counter()
    ref, _, _, _ = oracle.solve(P, d64, tol=1e-12, max_cycles=200)
    g_ora = oracle.force(P, ref).reshape(3, -1)
    gf = np.zeros_like(g_ora)
    gf[:, c5["cells"]] = 2.0 * g_ora[:, c5["cells"]]
    gv = oracle.force_adjoint(P, ref, gf.reshape(3, n, n, n))
    gd_ora, _, _ = oracle.adjoint(P, d64, ref, gv, tol=1e-12)
    say(f"oracle solve + adjoint {time.perf_counter() - t0:.1f} s")
    e32, e64 = rel_err(gd32, gd_ora), rel_err(gd64, gd_ora)
    m32, m64 = max_err(gd32, gd_ora), max_err(gd64, gd_ora)
    say(f"adjoint vs oracle: fp32 {e32:.2e} (max {m32:.2e}, {st32.vcycles} cycles), "
        f"fp64 {e64:.2e} (max {m64:.2e})")
    assert e32 < 1e-5 and e64 < 1e-6 and m32 < 1e-5 and m64 < 1e-6
    # central differences of FP64 GPU solves on delta at 16 probe cells
    rng = np.random.default_rng(5006)
    near = []
    for c in c5["cells"][rng.choice(len(c5["cells"]), 8, replace=False)]:
        k, j, i = np.unravel_index(c, (n, n, n))
        near.append(np.ravel_multi_index((k, j, (i + 1) % n), (n, n, n)))
    probes = np.array(near + list(rng.choice(n ** 3, 8, replace=False)))
    o64 = api.solver_opts(precision="fp64")
    base, _ = mg.solve("fr", prm, c5["delta"], tol=1e-13, opts=o64, allow_noconv=True)
    # the FP64 adjoint of the FP64 loss
    l0, g0 = _loss64(mg, prm, base, cells_t)
    # the FP64 loss differentiates the library's own force
    g_lib = mg.force("fr", prm, base).reshape(3, -1)[:, cells_t].double()
    assert float((g_lib - g0).norm() / g0.norm()) < 1e-6
    gfull = torch.zeros((3, n ** 3), dtype=torch.float64, device=DEV)
    gfull[:, cells_t] = 2.0 * g0
    gfa = mg.force_adjoint("fr", prm, base, gfull.reshape(3, n, n, n).float())
    gda, _ = mg.solve_adjoint("fr", prm, c5["delta"], base, gfa, tol=1e-12, opts=o64,
                              allow_noconv=True)
    gda = gda.cpu().numpy().ravel()
    h = 1e-4
    # Central differences of FP64 solves at their rounding floor scatter by
    # ~1e-9 here (against gradients up to ~3e-3); the bound is 1e-5 relative
    # plus 1e-8 absolute (4e-6 of the largest probe gradient).
    floor = 1e-8
    say(f"loss {l0:.6e}")
    worst = 0.0
    d = c5["d32"].ravel().copy()
    for c in probes:
        dp, dm = d.copy(), d.copy()
        dp[c] = np.float32(d[c] + h)
        dm[c] = np.float32(d[c] - h)
        step = float(dp[c]) - float(dm[c])
        lp = _loss64(mg, prm, mg.solve("fr", prm, torch.from_numpy(dp.reshape(n, n, n)).to(DEV),
                                       field_in=base, tol=1e-13, opts=o64,
                                       allow_noconv=True)[0], cells_t)[0]
        lm = _loss64(mg, prm, mg.solve("fr", prm, torch.from_numpy(dm.reshape(n, n, n)).to(DEV),
                                       field_in=base, tol=1e-13, opts=o64,
                                       allow_noconv=True)[0], cells_t)[0]
        fd = (lp - lm) / step
        e = abs(fd - gda[c]) / (1e-5 * abs(fd) + floor)
        worst = max(worst, e)
        say(f"  probe {c}: fd={fd:.6e} adjoint={gda[c]:.6e} |diff|/(1e-5|fd| + 1e-8)={e:.3f}")
    assert worst < 1.0


def test_autograd_backward_matches_adjoint_chain():
    n = 48
    d = synthetic.lognormal_delta(n, 77, sigma_delta=1.5).astype(np.float32)
    mg = api.Context(n, device=DEV)
    prm = api.model_params(float(n), fr0=1e-5)
    cells = torch.from_numpy(np.sort(np.random.default_rng(78).choice(n ** 3, 500,
                                                                      replace=False))).to(DEV)
    delta = torch.from_numpy(d).to(DEV).requires_grad_(True)
    opts = api.solver_opts(precision="fp32")
    field, force = api.solve_force(mg, "fr", prm, delta, tol=1e-10, opts=opts, adj_tol=1e-10)
    loss = (force.reshape(3, -1)[:, cells] ** 2).sum()
    loss.backward()
    g_auto = delta.grad.double().cpu().numpy()
    # explicit chain through the C ABI
    f2, _ = mg.solve("fr", prm, delta.detach(), tol=1e-10, opts=opts)
    F2 = mg.force("fr", prm, f2)
    _, gF = mg.loss_force_sq(F2, cells)
    gfield = mg.force_adjoint("fr", prm, f2, gF)
    gd, _ = mg.solve_adjoint("fr", prm, delta.detach(), f2, gfield, tol=1e-10, opts=opts)
    e = rel_err(g_auto, gd.cpu().numpy())
    # and the oracle's adjoint of the same loss
    P = oracle.params(oracle.FR, n, float(n), fr0=1e-5)
    ref, _, _, _ = oracle.solve(P, d.astype(np.float64), tol=1e-12)
    g_ora = oracle.force(P, ref).reshape(3, -1)
    gf = np.zeros_like(g_ora)
    cc = cells.cpu().numpy()
    gf[:, cc] = 2.0 * g_ora[:, cc]
    gv = oracle.force_adjoint(P, ref, gf.reshape(3, n, n, n))
    gd_ora, _, _ = oracle.adjoint(P, d.astype(np.float64), ref, gv, tol=1e-12)
    e_ora = rel_err(g_auto, gd_ora)
    say(f"autograd vs explicit chain {e:.2e}, vs oracle {e_ora:.2e}")
    assert e < 1e-6 and e_ora < 1e-5
    mg.close()


def test_c5_1024_fp32_refined_adjoint_matches_fp64():
    """The differentiable solve repeated at 1024^3 (lognormal, seed 5): the
    FP32-refined forward + adjoint against the plain FP64 GPU path (no oracle
    at this size).  Only the forward solution is kept for the backward pass;
    the adjoint rebuilds its own level pyramid from it (the multigrid levels
    are recomputed, not stored)."""
    n = 1024
    t0 = time.perf_counter()
    d = synthetic.c5_delta(n).astype(np.float32)
    cells = torch.from_numpy(synthetic.c5_loss_cells(n)).to(DEV)
    say(f"1024^3 inputs {time.perf_counter() - t0:.1f} s")
    delta = torch.from_numpy(d).to(DEV)
    del d
    mg = api.Context(n, device=DEV)
    prm = api.model_params(float(n), fr0=1e-5)
    out = {}
    for prec in ("fp32", "fp64"):
        o = api.solver_opts(precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        field, st = mg.solve("fr", prm, delta, tol=1e-6, opts=o)
        force = mg.force("fr", prm, field)
        loss, gforce = mg.loss_force_sq(force, cells)
        del force
        gfield = mg.force_adjoint("fr", prm, field, gforce)
        del gforce
        gd, sa = mg.solve_adjoint("fr", prm, delta, field, gfield, tol=1e-6, opts=o)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        say(f"  {prec}: forward {st.vcycles} cycles (rel {st.rel_resid:.1e}), adjoint "
            f"{sa.vcycles} cycles (rel {sa.rel_resid:.1e}), {ms:.0f} ms, "
            f"HBM in use {torch.cuda.memory_allocated() / 2**30:.0f} GiB (tensors)")
        out[prec] = (field.cpu().numpy(), gd.cpu().numpy(), float(loss))
        del field, gfield, gd
    f32, g32, l32 = out["fp32"]
    f64, g64, l64 = out["fp64"]
    ferr = rel_err(f32, f64, f64.mean())
    gerr = rel_err(g32, g64)
    say(f"  fp32 vs fp64: field {ferr:.2e}, dL/d(delta) {gerr:.2e}, loss {abs(l32 - l64) / l64:.1e}")
    assert ferr < 1e-5 and gerr < 1e-5
    mg.close()


def test_c3_particle_side_sampled(c3):
    n, mg, delta = c3["n"], c3["mg"], c3["delta"]
    say("c3 particle side")
    prm = api.model_params(float(n), fr0=1e-5)
    P = oracle.params(oracle.FR, n, float(n), fr0=1e-5)
    field, st = mg.solve("fr", prm, delta, tol=1e-6, opts=api.solver_opts(precision="fp32"))
    phin = mg.poisson_newton(prm, delta)
    ph = phin.cpu().numpy()
    d = delta.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(512)
    cells = rng.choice(n ** 3, 4096, replace=False)
    k, j, i = np.unravel_index(cells, (n, n, n))
    wrap = lambda a: a % n
    lap = (ph[wrap(k + 1), j, i] + ph[wrap(k - 1), j, i] + ph[k, wrap(j + 1), i] +
           ph[k, wrap(j - 1), i] + ph[k, j, wrap(i + 1)] + ph[k, j, wrap(i - 1)] - 6 * ph[k, j, i])
    src = 1.5 * 0.3 * (d[k, j, i] - d.mean())
    perr = np.abs(lap - src).max() / np.abs(src).max()
    # total force at the sampled cells: -(Phi(c+e) - Phi(c-e))/2, Phi = Phi_N + Phi5
    g = mg.total_force("fr", prm, phin, field).cpu().numpy()
    f = field.cpu().numpy()
    pot = lambda kk, jj, ii: ph[kk, jj, ii] - 0.5 * P_ct2(P) * f[kk, jj, ii]
    gx = -0.5 * (pot(k, j, wrap(i + 1)) - pot(k, j, wrap(i - 1)))
    gy = -0.5 * (pot(k, wrap(j + 1), i) - pot(k, wrap(j - 1), i))
    gz = -0.5 * (pot(wrap(k + 1), j, i) - pot(wrap(k - 1), j, i))
    gref = np.stack([gx, gy, gz])
    gerr = np.abs(g[:, k, j, i] - gref).max() / np.abs(gref).max()
    # CIC interpolation of the three components to every particle, checked
    # on 100k sampled particles against the oracle's interpolation of the
    # same mesh values
    pos = torch.from_numpy(c3["pos32"]).to(DEV)
    acc = mg.interp_to_particles(torch.from_numpy(g).to(DEV), pos)
    sel = rng.choice(pos.shape[0], 100000, replace=False)
    ps = c3["pos32"][sel].astype(np.float64)
    aref = oracle.interp(n, ps, g.astype(np.float64))
    ierr = np.abs(acc.cpu().numpy()[sel] - aref).max() / np.abs(aref).max()
    # symmetron friction on the same particles (u in [0.3, 1], unit momenta)
    u = torch.rand((n, n, n), dtype=torch.float64, device=DEV,
                   generator=torch.Generator(device=DEV).manual_seed(3)) * 0.7 + 0.3
    mom = torch.ones_like(pos)
    prms = api.model_params(float(n), a=0.8, a_star=0.5)
    Ps = oracle.params(oracle.SYM, n, float(n), a=0.8, a_star=0.5)
    fr = mg.symmetron_friction(prms, u, pos, mom).cpu().numpy()[sel]
    fref = oracle.sym_friction(Ps, u.cpu().numpy(), ps, np.ones_like(ps))
    ferr = np.abs(fr - fref).max() / np.abs(fref).max()
    say(f"  poisson {perr:.1e} total force {gerr:.1e} interp {ierr:.1e} friction {ferr:.1e}")
    assert perr < 1e-8 and gerr < 1e-6 and ierr < 1e-6 and ferr < 1e-6
    del pos, acc


def P_ct2(P):
    return oracle.ctilde(P.n, P.box) ** 2
