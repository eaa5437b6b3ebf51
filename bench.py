#!/usr/bin/env python
"""Benchmark of the hot path on one MI355X.

One step = the whole hot path over one 512^3 box (1 Mpc/h cells, seeded
Zel'dovich particles standing in for a simulation snapshot):
  CIC of 512^3 FP32 particles -> f(R) n=1 |f_R0|=1e-5 solve, FP32 multigrid
  refined in FP64, to relative residual 1e-6 -> fifth force -> loss over
  4096 seeded cells and its force gradient -> force adjoint -> adjoint solve
  (FP32 refined, 1e-6).
Inputs are resident in HBM before the timed region; every step solves from
the background field.  value = grid cells per second through the step.

Also reported: the plain FP64 GPU step at the same tolerances, the
roofline of the dominant kernel (FP32 finest-level smoother half-sweep,
timed with HIP events on the solve's stream over the timed steps; its
algorithmic bytes are 12 per updated cell),
and the FP64 CPU oracle on the same 512^3 pipeline on all of this machine's
host threads, plus a 192^3 box on one thread.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Algorithmic bytes of the FP32 smoother: 12 B per cell per full sweep, i.e.
# per updated cell of a half-sweep: read the other colour's field and the
# cell's coefficient, write the cell (4 + 4 + 4).
FP32_SMOOTH_BYTES_PER_CELL = 12.0
# This library's correction-form smoother moves exactly that: the
# linearisation point X and the right-hand side rho in 16-bit floats, the
# other colour's FP32 correction, the written correction (2 + 2 + 4 + 4).
# HBM bytes per finest-level launch of that kernel at 512^3, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (scaled by a plain copy of known size).  Set to
# None whenever the kernel changes, until the counters are taken again.
# k_smooth_corr_kv<FR, h16, h16>: 546.8 MB fetched + 268.4 MB written.
FP32_SMOOTH_TRAFFIC_512 = 815.2e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--fr0", type=float, default=1e-5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=512,
                    help="oracle sample box at all host threads (the metric's own 512^3)")
    ap.add_argument("--cpu-n1", type=int, default=192,
                    help="oracle sample box on one host thread")
    ap.add_argument("--cpu-leg", type=int, nargs=2, metavar=("N", "THREADS"),
                    help=argparse.SUPPRESS)  # internal: one oracle run, JSON to stdout
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the |f_R0|=1e-6, coupled-quintessence and batched legs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB FP32 device copy (counter calibration)")
    return ap.parse_args()


def cpu_baseline(n, fr0, tol):
    """The FP64 oracle's pipeline on an n^3 sample box (same 1 Mpc/h cells)."""
    import numpy as np

    import oracle
    import synthetic

    pos = synthetic.zeldovich_positions(n, n, seed=3, dtype=np.float32).astype(np.float64)
    cells = np.sort(np.random.default_rng(5005).choice(n ** 3, 4096 * n ** 3 // 512 ** 3 or 64,
                                                       replace=False))
    P = oracle.params(oracle.FR, n, float(n), fr0=fr0)
    ph = {}
    t0 = t = time.perf_counter()

    def lap(name):
        nonlocal t
        now = time.perf_counter()
        ph[name] = now - t
        t = now

    d = oracle.cic(n, pos)
    lap("cic")
    v, cyc, rel, _ = oracle.solve(P, d, tol=tol, max_cycles=100)
    lap("solve")
    g = oracle.force(P, v).reshape(3, -1)
    gf = np.zeros_like(g)
    gf[:, cells] = 2.0 * g[:, cells]
    lap("force_and_loss")
    gv = oracle.force_adjoint(P, v, gf.reshape(3, n, n, n))
    gd, it, arel = oracle.adjoint(P, d, v, gv, tol=tol)
    lap("adjoint")
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return dict(value=n ** 3 / dt, unit="cells/s", cores=threads, kind="oracle",
                sample=f"{n}^3 box, {n} Mpc/h, same pipeline (CIC, FP64 FAS V(1,1) to {tol:g}, "
                       f"force, loss grad, force adjoint, linear-MG adjoint to {tol:g}); "
                       f"{dt:.1f} s wall, {cyc} cycles",
                seconds=dt, phases_s={k: round(x, 3) for k, x in ph.items()})


def cpu_model():
    """The host CPU as /proc/cpuinfo names it (model name, family/model/stepping)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if not ln.strip():
                    break
                k, _, v = ln.partition(":")
                info[k.strip()] = v.strip()
    except OSError:
        return "unknown"
    return (f"{info.get('model name', '?')} (vendor {info.get('vendor_id', '?')}, family "
            f"{info.get('cpu family', '?')}, model {info.get('model', '?')}, stepping "
            f"{info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz)")


def cpu_leg(n, threads, fr0, tol):
    """One oracle run in a child process with OMP_NUM_THREADS = threads (the
    OpenMP runtime reads it when the oracle library loads)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", str(n),
                        str(threads), "--fr0", repr(fr0)], env=env, capture_output=True,
                       text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baselines(a, tol):
    """The oracle on the metric's pipeline: the full 512^3 box on all host
    threads (the reported value), and a smaller box on one thread."""
    nproc = len(os.sched_getaffinity(0))
    full = cpu_leg(a.cpu_n, nproc, a.fr0, tol)
    one = cpu_leg(a.cpu_n1, 1, a.fr0, tol)
    full.update(cpu_model=cpu_model(), host_threads_available=os.cpu_count(),
                single_thread=dict(value=one["value"], unit="cells/s", cores=1,
                                   sample=one["sample"], seconds=one["seconds"],
                                   phases_s=one["phases_s"]),
                threads_speedup_per_cell=full["value"] / one["value"])
    return full


def m_cells(n):
    return float(n) ** 3


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def cycle_costs(mg, delta, field, n, fr0, tol):
    """V, F and W cycles on the same 512^3 f(R) problem (the comparison of
    the paper's convergence tests): two cycles from the background with no
    convergence test (FP64 FAS; refined: one outer step of two FP32 cycles),
    their time and the residual reduction, then the solve to tol."""
    import math

    from paper_2110_00328_amd import api

    prm = api.model_params(float(n), fr0=fr0)
    rows = []
    for prec in ("fp64", "fp32"):
        for cyc in ("V", "F", "W"):
            k = 2
            o = api.solver_opts(cycle=cyc, precision=prec, fixed_cycles=k)
            st = {}

            def fixed():
                _, s = mg.solve("fr", prm, delta, out=field, tol=tol, opts=o)
                st["rel"] = s.rel_resid

            ms = _timed(fixed, 3)
            ot = api.solver_opts(cycle=cyc, precision=prec)
            tt = {}

            def to_tol():
                _, s = mg.solve("fr", prm, delta, out=field, tol=tol, opts=ot)
                tt.update(cycles=s.vcycles, rel=s.rel_resid)

            ms_tol = _timed(to_tol, 2)
            digits = -math.log10(st["rel"]) if st["rel"] > 0 else float("inf")
            rows.append(dict(cycle=cyc, precision=prec, fixed_cycles=k, ms=ms,
                             rel_after=st["rel"], contraction_per_cycle=st["rel"] ** (1.0 / k),
                             digits_per_ms=digits / ms, ms_to_tol=ms_tol,
                             cycles_to_tol=tt["cycles"], rel_at_tol=tt["rel"]))
    return dict(problem=f"f(R) |f_R0|={fr0:g}, {n}^3 CIC density, from the background",
                tol=tol, rows=rows)


def batched_leg(dev, tol):
    """The 64-box sweep (64^3 / 96^3 / 128^3, f(R) with log-uniform |f_R0|
    and symmetron) through mg_solve_batched after tuning, against the same
    boxes solved one after another, with each box's error against its own
    single-box FP64 solve."""
    import tempfile

    import numpy as np
    import torch

    import synthetic
    from paper_2110_00328_amd import api

    # 64 boxes of 64^3 / 96^3 / 128^3, f(R) with log-uniform |f_R0| and symmetron
    spec = synthetic.c4_boxes()
    boxes = []
    for b in spec:
        nb = b["n"]
        prm = api.model_params(b["box"], **b["params"])
        boxes.append(dict(n=nb, model=b["model"], params=prm,
                          delta=torch.from_numpy(b["delta"].astype(np.float32)).to(dev),
                          field=torch.empty((nb, nb, nb), dtype=torch.float64, device=dev),
                          force=torch.empty((3, nb, nb, nb), dtype=torch.float32, device=dev)))
    cells_total = sum(b["n"] ** 3 for b in boxes)
    o = api.solver_opts(precision="fp32")
    bctx = api.Context(boxes[0]["n"], device=dev)
    os.environ.setdefault("MGGPU_TUNE_CACHE", os.path.join(tempfile.mkdtemp(), "tune.json"))
    t0 = time.perf_counter()
    bctx.batched_tune(boxes, opts=o)
    tune_ms = (time.perf_counter() - t0) * 1e3
    stats = []
    b_ms = _timed(lambda: stats.__setitem__(slice(None), bctx.solve_batched(boxes, tol=tol, opts=o)),
                  3)
    blk, vec, teams = bctx.batched_config()
    bctx.close()
    # each box's batched field and force against its own plain FP64 single-box
    # solve to the same tolerance (max over boxes of the L2 and max-norm ratios)
    singles = {nb: api.Context(nb, device=dev) for nb in (64, 96, 128)}
    worst_field = worst_force = 0.0
    o64 = api.solver_opts(precision="fp64")
    for b in boxes:
        c = singles[b["n"]]
        f64, _ = c.solve(b["model"], b["params"], b["delta"], tol=tol, opts=o64)
        g64 = c.force(b["model"], b["params"], f64).double()
        bg = f64.mean()
        x, g = b["field"], b["force"].double()
        worst_field = max(worst_field, float((x - f64).norm() / (f64 - bg).norm()),
                          float((x - f64).abs().max() / (f64 - bg).abs().max()))
        worst_force = max(worst_force, float((g - g64).norm() / g64.norm()),
                          float((g - g64).abs().max() / g64.abs().max()))
        del f64, g64

    def one_by_one():
        for b in boxes:
            c = singles[b["n"]]
            c.solve(b["model"], b["params"], b["delta"], out=b["field"], tol=tol, opts=o)
            c.force(b["model"], b["params"], b["field"], out=b["force"])

    s_ms = _timed(one_by_one, 2)
    for c in singles.values():
        c.close()
    return dict(
        boxes=len(boxes), cells=cells_total, ms=b_ms, boxes_per_s=len(boxes) / (b_ms * 1e-3),
        cells_per_s=cells_total / (b_ms * 1e-3), block=blk, cells_per_thread=4 if vec else 1,
        teams={0: "persistent launch, single-workgroup teams",
               1: "persistent launch, one sized team per box",
               2: "grouped level launches per (n, model) class"}[teams],
        tune_ms=tune_ms, max_rel_resid=max(s.rel_resid for s in stats),
        max_err_vs_fp64_single_box=dict(field=worst_field, force=worst_force),
        outer_steps=[int(min(s.cycles for s in stats)), int(max(s.cycles for s in stats))],
        one_by_one_ms=s_ms, batched_speedup=s_ms / b_ms)


def warm_start_v2(mg, pos, delta, field, n, fr0, tol):
    """The paper's production mode (Sec. 4.3): two V-cycles per time step,
    warm-started from the previous step's field.  The next step's density
    comes from the same Zel'dovich particles moved on by 1% of their
    displacement (x = q + 1.01 psi, q the Lagrangian grid point); from the
    converged field of the present density, two V(1,1) cycles with no
    convergence test, against the converged field of the next density."""
    import torch

    from paper_2110_00328_amd import api

    prm = api.model_params(float(n), fr0=fr0)
    npart = round(pos.shape[0] ** (1.0 / 3.0))
    s = n / npart
    g = (torch.arange(npart, device=pos.device, dtype=torch.float32) + 0.5) * s
    q = torch.stack(torch.meshgrid(g, g, g, indexing="ij"), dim=-1).reshape(-1, 3)
    q = q.flip(-1)  # particle index is [k][j][i] with i fastest, columns x, y, z
    psi = torch.remainder(pos - q + n / 2, n) - n / 2
    pos2 = torch.remainder(q + 1.01 * psi, n)
    pos2[pos2 >= n] = 0.0
    delta2 = torch.empty_like(delta)
    mg.cic(pos2.contiguous(), out=delta2)
    del q, psi, pos2
    f0, _ = mg.solve("fr", prm, delta, tol=tol)
    ref, _ = mg.solve("fr", prm, delta2, tol=1e-9, opts=api.solver_opts(precision="fp64"))
    bg = ref.mean()
    rows = []
    for prec in ("fp32", "fp64"):
        o = api.solver_opts(precision=prec, fixed_cycles=2)
        st = {}

        def step():
            _, t = mg.solve("fr", prm, delta2, field_in=f0, out=field, tol=tol, opts=o)
            st["rel"] = t.rel_resid

        ms = _timed(step, 3)
        err = float((field - ref).norm() / (ref - bg).norm())
        rows.append(dict(precision=prec, ms=ms, rel_after=st["rel"], field_err_vs_converged=err))
    rel0 = float((f0 - ref).norm() / (ref - bg).norm())
    del f0, ref, delta2
    return dict(problem=f"f(R) |f_R0|={fr0:g}, {n}^3, next density from x = q + 1.01 psi",
                start_field_err=rel0, rows=rows)


def extra_legs(a, mg, pos, delta, field, force, cells, n, tol):
    """The other workloads the metric names, timed outside the main loop:
    |f_R0| = 1e-6 forward+adjoint, coupled quintessence forward (FP32-refined
    and FP64), the particle side after the fifth force, and the 64-box
    batched sweep in one persistent launch against the same boxes solved one
    after another."""
    import tempfile

    import numpy as np
    import torch

    import synthetic
    from paper_2110_00328_amd import api

    dev = pos.device
    out = {}
    gforce = torch.empty_like(force)
    gfield = torch.empty_like(field)
    gdelta = torch.empty_like(field)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    mg.cic(pos, out=delta)
    # f(R) |f_R0| = 1e-6: deeper screening, same pipeline
    prm6 = api.model_params(float(n), fr0=1e-6)
    leg = {}
    for prec in ("fp32", "fp64"):
        o = api.solver_opts(precision=prec)
        st = {}

        def fwd_adj():
            _, s1 = mg.solve("fr", prm6, delta, out=field, tol=tol, opts=o)
            mg.force("fr", prm6, field, out=force)
            mg.loss_force_sq(force, cells, grad_out=gforce, loss_out=loss)
            mg.force_adjoint("fr", prm6, field, gforce, out=gfield)
            _, s2 = mg.solve_adjoint("fr", prm6, delta, field, gfield, out=gdelta, tol=tol, opts=o)
            st.update(fwd_vcycles=s1.vcycles, adj_vcycles=s2.vcycles)

        leg[prec + "_ms"] = _timed(fwd_adj, 2)
        leg[prec + "_cycles"] = dict(st)
    leg["fp64_over_fp32"] = leg["fp64_ms"] / leg["fp32_ms"]
    out["fr0_1e-6_solve_adjoint"] = leg
    # coupled quintessence (alpha=0.1, beta=-0.2) with phibar(a=1) and lambda
    # from the background solve (H(a=1) = H0)
    back = api.cq_background(0.1, -0.2, omega_m=0.3)
    prmq = api.cq_model_params(float(n), 1.0, 0.1, -0.2, omega_m=0.3, background=back)
    leg = dict(phibar=prmq.cq_phibar, lam=prmq.cq_lambda)
    for prec in ("fp32", "fp64"):
        o = api.solver_opts(precision=prec)
        st = {}

        def fwd():
            _, s1 = mg.solve("cq", prmq, delta, out=field, tol=tol, opts=o)
            mg.force("cq", prmq, field, out=force)
            st.update(vcycles=s1.vcycles, rel=s1.rel_resid)

        leg[prec + "_ms"] = _timed(fwd, 2)
        leg[prec + "_cycles"] = dict(st)
    leg["fp64_over_fp32"] = leg["fp64_ms"] / leg["fp32_ms"]
    out["cq_solve_force"] = leg
    out["cycle_costs"] = cycle_costs(mg, delta, field, n, a.fr0, tol)
    out["warm_start_v2"] = warm_start_v2(mg, pos, delta, field, n, a.fr0, tol)
    # the particle side after the fifth force, at the same size: Newtonian
    # potential by FFT, total force (potentials summed, then differenced), CIC
    # interpolation of the three components to every particle, friction term
    prm = api.model_params(float(n), fr0=a.fr0)
    mg.solve("fr", prm, delta, out=field, tol=tol)
    phin = torch.empty_like(field)
    npart = pos.shape[0]
    ppart = torch.empty((npart, 3), dtype=torch.float32, device=dev)
    pfric = torch.empty_like(ppart)
    u = torch.full_like(field, 0.8)
    prms = api.model_params(float(n), a=1.0, a_star=0.5)
    leg = dict(particles=npart)
    leg["poisson_fft_ms"] = _timed(lambda: mg.poisson_newton(prm, delta, out=phin), 3)
    leg["total_force_ms"] = _timed(lambda: mg.total_force("fr", prm, phin, field, out=force), 3)
    leg["interp_ms"] = _timed(lambda: mg.interp_to_particles(force, pos, out=ppart), 3)
    leg["sym_friction_ms"] = _timed(
        lambda: mg.symmetron_friction(prms, u, pos, ppart, out=pfric), 3)
    # algorithmic bytes: positions 12 + result 12 per particle, each grid
    # cell's three components read once (12 per cell)
    leg["interp_GBps"] = (24.0 * npart + 12.0 * m_cells(n)) / (leg["interp_ms"] * 1e6)
    leg["total_force_GBps"] = 28.0 * m_cells(n) / (leg["total_force_ms"] * 1e6)
    out["particle_side"] = leg
    del phin, ppart, pfric, u
    out["batched_c4"] = batched_leg(dev, tol)
    return out


def main():
    a = parse()
    if a.cpu_leg:
        print(json.dumps(cpu_baseline(a.cpu_leg[0], a.fr0, 1e-6)), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synthetic
    from paper_2110_00328_amd import _lib as L
    from paper_2110_00328_amd import api

    dev = torch.device("cuda:0")
    n = a.n
    tol = 1e-6
    pos = torch.from_numpy(synthetic.c3_positions(n)).to(dev)
    cells = torch.from_numpy(np.sort(np.random.default_rng(5005).choice(n ** 3, 4096,
                                                                        replace=False))).to(dev)
    mg = api.Context(n, device=dev)
    prm = api.model_params(float(n), fr0=a.fr0)
    m = n ** 3
    delta = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    field = torch.empty((n, n, n), dtype=torch.float64, device=dev)
    force = torch.empty((3, n, n, n), dtype=torch.float32, device=dev)
    gforce = torch.empty_like(force)
    gfield = torch.empty_like(field)
    gdelta = torch.empty_like(field)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    info = {}

    def step(prec):
        o = api.solver_opts(precision=prec)
        mg.cic(pos, out=delta)
        _, st = mg.solve("fr", prm, delta, out=field, tol=tol, opts=o)
        mg.force("fr", prm, field, out=force)
        mg.loss_force_sq(force, cells, grad_out=gforce, loss_out=loss)
        mg.force_adjoint("fr", prm, field, gforce, out=gfield)
        _, sa = mg.solve_adjoint("fr", prm, delta, field, gfield, out=gdelta, tol=tol, opts=o)
        info[prec] = dict(fwd_checks=st.cycles, fwd_vcycles=st.vcycles, fwd_rel=st.rel_resid,
                          fwd_ms=st.ms_total, adj_checks=sa.cycles, adj_vcycles=sa.vcycles,
                          adj_rel=sa.rel_resid, adj_ms=sa.ms_total)

    for _ in range(a.warmup):
        step("fp32")
    torch.cuda.synchronize()
    mg.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step("fp32")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.steps
    sm_ms, sm_n = mg.prof_read(L.MG_PROF_SMOOTH32)
    mg.prof_enable(False)

    if a.calib_copy:
        # a plain copy of known size: 2^28 floats read + written once
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fp64_ms = None
    if not a.no_fp64:
        step("fp64")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step("fp64")
        torch.cuda.synchronize()
        fp64_ms = (time.perf_counter() - t1) * 1e3

    extra = {} if a.no_extra else extra_legs(a, mg, pos, delta, field, force, cells, n, tol)

    mg.close()
    avg = sm_ms / max(sm_n, 1)
    bytes_per_launch = FP32_SMOOTH_BYTES_PER_CELL * (m / 2)
    achieved = bytes_per_launch / (avg * 1e-3) / 1e9 if sm_n else None
    out = {
        "metric": "512^3 f(R) MG solve to 1e-6 resid: FP32+adjoint vs FP64 time; % HBM peak",
        "value": m / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 grid, {n} Mpc/h box, {n}^3 Zel'dovich FP32 particles "
                               f"(seed 3); f(R) n=1 |f_R0|={a.fr0:g}, Omega_m=0.3, a=1; CIC, "
                               f"FP32-refined V(1,1) solve and adjoint to {tol:g}, force, "
                               f"4096-cell |F5|^2 loss",
                   "grid": n, "tol": tol, "precision": "fp32-refined"},
        "fp64_ms_per_step": fp64_ms,
        "fp64_over_fp32": (fp64_ms / ms) if fp64_ms else None,
        "phases": info,
        **extra,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": FP32_SMOOTH_TRAFFIC_512 if n == 512 else None,
                     "traffic_unit": "bytes per launch (HBM, counted)",
                     "kernel": "k_smooth_corr_kv<FR, h16, h16> (finest-level FP32 half-sweep)",
                     "avg_launch_ms": avg, "launches": sm_n,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "algorithmic_bytes_per_cell": FP32_SMOOTH_BYTES_PER_CELL},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baselines(a, tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
