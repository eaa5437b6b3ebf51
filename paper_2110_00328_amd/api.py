"""Torch-facing wrappers of the C ABI (include/mggpu.h).

PyTorch provides device memory and the stream; every computation is a call
into libmggpu.so.  Tensors must be contiguous CUDA (HIP) tensors of the
documented dtype and shape; nothing falls back to the CPU.
"""
import ctypes

import torch

from . import _lib as L

C_OVER_H0 = 2997.92458  # Mpc/h

MODELS = {"fr": L.MG_FR, "sym": L.MG_SYMMETRON, "cq": L.MG_CQ}
PRECISIONS = {"fp64": L.MG_FP64, "fp32": L.MG_FP32_REFINED}
CYCLES = {"V": L.MG_CYCLE_V, "F": L.MG_CYCLE_F, "W": L.MG_CYCLE_W}


class MGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mggpu error {code}: {msg}")
        self.code = code


def model_id(model):
    return MODELS[model] if isinstance(model, str) else int(model)


def model_params(box, a=1.0, omega_m=0.3, fr_n=1, fr0=1e-5, a_star=0.5, xi=1.0 / C_OVER_H0,
                 beta_star=1.0, alpha=0.1, beta=-0.2, phibar=0.5, lam=None, cq_keep_exp=1):
    """mg_model_params in the paper's notation.  ``lam`` defaults to the
    stand-in lambda^2 = Omega_L phibar^alpha."""
    if lam is None:
        lam = ((1.0 - omega_m) * phibar ** alpha) ** 0.5
    return L.ModelParams(a, omega_m, box, fr_n, fr0, a_star, xi, beta_star, alpha, beta, phibar,
                         lam, cq_keep_exp)


def cq_background(alpha, beta, omega_m=0.3089, h=0.6774, n_table=4096, z_init=1e5,
                  phi_init=1e-6, dphi_init=0.0, t_cmb=2.7255, n_eff=3.046, tol=1e-12):
    """The coupled-quintessence background (mg_cq_background): returns
    (info, table) with table an (n_table, 6) float64 array of rows
    (a, H/H0, (dH/dt)/H0^2, phibar, d phibar/da, (d phibar/dt)/H0) uniform
    in ln a.  Defaults are the paper's Planck 2015 cosmology and start."""
    import numpy as np

    p = L.CqBackgroundParams(omega_m, h, t_cmb, n_eff, alpha, beta, z_init, phi_init, dphi_init,
                             tol)
    tab = np.empty((n_table, 6), dtype=np.float64)
    info = L.CqBackgroundInfo()
    rc = L.load().mg_cq_background(ctypes.byref(p), n_table,
                                  tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(info))
    if rc != L.MG_OK:
        raise MGError(rc, "mg_cq_background failed")
    return info, tab


def cq_background_at(table, a):
    """Row of the background table linearly interpolated at scale factor a."""
    import numpy as np

    tab = np.ascontiguousarray(table, dtype=np.float64)
    row = np.empty(6, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = L.load().mg_cq_background_at(tab.ctypes.data_as(dp), tab.shape[0], float(a),
                                     row.ctypes.data_as(dp))
    if rc != L.MG_OK:
        raise MGError(rc, f"mg_cq_background_at(a={a}) outside the table")
    return row


def cq_model_params(box, a, alpha, beta, omega_m=0.3089, background=None, **kw):
    """mg_model_params for coupled quintessence with phibar(a) and lambda from
    the background solve instead of stand-ins."""
    info, tab = background if background is not None else cq_background(alpha, beta, omega_m)
    row = cq_background_at(tab, a)
    return model_params(box, a=a, omega_m=omega_m, alpha=alpha, beta=beta, phibar=row[3],
                        lam=info.lam, **kw)


def solver_opts(cycle="V", nu_pre=1, nu_post=1, inner_cycles=0, max_cycles=64, precision="fp32",
                coarse_sweeps=0, fixed_cycles=0):
    """mg_solver_opts; inner_cycles = 0 plans the cycles between FP64
    residual checks from the measured contraction; fixed_cycles = k runs
    exactly k cycles with no convergence test (the paper's V2 per step)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cyc = CYCLES[cycle] if isinstance(cycle, str) else int(cycle)
    return L.SolverOpts(cyc, nu_pre, nu_post, inner_cycles, max_cycles, prec, coarse_sweeps,
                        fixed_cycles)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """One mg_ctx: the level pyramid for n^3 grids on one stream."""

    def __init__(self, n, device="cuda", stream=None):
        self.lib = L.load()
        self.n = int(n)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ptr = ctypes.c_void_p()
        rc = self.lib.mg_ctx_create(ctypes.byref(ptr), self.n,
                                    ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise MGError(rc, f"mg_ctx_create(n={n}) failed")
        self.ptr = ptr
        self.levels = self.lib.mg_ctx_levels(self.ptr)

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.mg_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            msg = self.lib.mg_last_error(self.ptr)
            raise MGError(rc, msg.decode() if msg else "")
        return rc

    def _grid(self):
        return (self.n, self.n, self.n)

    # -- the hot path -----------------------------------------------------
    def cic(self, pos, out=None):
        """CIC density contrast from (n_part, 3) float32 positions in [0, n)."""
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("pos must be (n_part, 3)")
        _need(pos, torch.float32, pos.shape, "pos")
        if out is None:
            out = torch.empty(self._grid(), dtype=torch.float32, device=pos.device)
        _need(out, torch.float32, self._grid(), "delta_out")
        self._check(self.lib.cic_assign(self.ptr, _p(pos), pos.shape[0], _p(out)))
        return out

    def solve(self, model, params, delta, field_in=None, out=None, tol=1e-6, opts=None,
              allow_noconv=False):
        """Returns (field, stats).  field is f_R (f(R)), u (symmetron) or phi~ (CQ)."""
        _need(delta, torch.float32, self._grid(), "delta")
        if field_in is not None:
            _need(field_in, torch.float64, self._grid(), "field_in")
        if out is None:
            out = torch.empty(self._grid(), dtype=torch.float64, device=delta.device)
        _need(out, torch.float64, self._grid(), "field_out")
        opts = opts if opts is not None else solver_opts()
        st = L.Stats()
        rc = self.lib.mg_solve(self.ptr, model_id(model), ctypes.byref(params), ctypes.byref(opts),
                               _p(delta), _p(field_in) if field_in is not None else None, _p(out),
                               tol, ctypes.byref(st))
        self._check(rc, allow=(L.MG_ENOCONV,) if allow_noconv else ())
        return out, st

    def solve_noalloc(self, model, params, delta, out, field_in=None, tol=1e-6, opts=None,
                      allow_noconv=False):
        """mg_solve_noalloc: the same solve with its workspace in the library's
        static device array (n <= 64); out (float64, n^3) is caller-provided."""
        _need(delta, torch.float32, self._grid(), "delta")
        if field_in is not None:
            _need(field_in, torch.float64, self._grid(), "field_in")
        _need(out, torch.float64, self._grid(), "field_out")
        opts = opts if opts is not None else solver_opts()
        st = L.Stats()
        rc = self.lib.mg_solve_noalloc(self.ptr, model_id(model), ctypes.byref(params),
                                       ctypes.byref(opts), _p(delta),
                                       _p(field_in) if field_in is not None else None, _p(out),
                                       tol, ctypes.byref(st))
        self._check(rc, allow=(L.MG_ENOCONV,) if allow_noconv else ())
        return out, st

    def residual(self, model, params, delta, field, d_out=None):
        _need(delta, torch.float32, self._grid(), "delta")
        _need(field, torch.float64, self._grid(), "field")
        if d_out is not None:
            _need(d_out, torch.float64, self._grid(), "d_out")
        rel = ctypes.c_double(0.0)
        self._check(self.lib.mg_residual(self.ptr, model_id(model), ctypes.byref(params), _p(delta),
                                         _p(field), _p(d_out) if d_out is not None else None,
                                         ctypes.byref(rel)))
        return rel.value

    def force(self, model, params, field, out=None):
        _need(field, torch.float64, self._grid(), "field")
        if out is None:
            out = torch.empty((3,) + self._grid(), dtype=torch.float32, device=field.device)
        _need(out, torch.float32, (3,) + self._grid(), "force_out")
        self._check(self.lib.mg_force(self.ptr, model_id(model), ctypes.byref(params), _p(field),
                                      _p(out)))
        return out

    def force_adjoint(self, model, params, field, grad_force, out=None):
        _need(field, torch.float64, self._grid(), "field")
        _need(grad_force, torch.float32, (3,) + self._grid(), "grad_force")
        if out is None:
            out = torch.empty(self._grid(), dtype=torch.float64, device=field.device)
        _need(out, torch.float64, self._grid(), "grad_field_out")
        self._check(self.lib.mg_force_adjoint(self.ptr, model_id(model), ctypes.byref(params),
                                              _p(field), _p(grad_force), _p(out)))
        return out

    def solve_adjoint(self, model, params, delta, field, grad_field, out=None, tol=1e-6,
                      opts=None, allow_noconv=False):
        _need(delta, torch.float32, self._grid(), "delta")
        _need(field, torch.float64, self._grid(), "field")
        _need(grad_field, torch.float64, self._grid(), "grad_field")
        if out is None:
            out = torch.empty(self._grid(), dtype=torch.float64, device=field.device)
        _need(out, torch.float64, self._grid(), "grad_delta_out")
        opts = opts if opts is not None else solver_opts()
        st = L.Stats()
        rc = self.lib.mg_solve_adjoint(self.ptr, model_id(model), ctypes.byref(params),
                                       ctypes.byref(opts), _p(delta), _p(field), _p(grad_field),
                                       _p(out), tol, ctypes.byref(st))
        self._check(rc, allow=(L.MG_ENOCONV,) if allow_noconv else ())
        return out, st

    def loss_force_sq(self, force, cells, grad_out=None, loss_out=None):
        """Loss = sum over cells of |g5|^2 and dLoss/dforce."""
        _need(force, torch.float32, (3,) + self._grid(), "force")
        if cells.dtype != torch.int64 or cells.device.type != "cuda" or not cells.is_contiguous():
            raise TypeError("cells must be a contiguous int64 GPU tensor")
        if grad_out is None:
            grad_out = torch.empty_like(force)
        if loss_out is None:
            loss_out = torch.empty(1, dtype=torch.float64, device=force.device)
        _need(grad_out, torch.float32, (3,) + self._grid(), "grad_out")
        _need(loss_out, torch.float64, (1,), "loss_out")
        self._check(self.lib.mg_loss_force_sq(self.ptr, _p(force), _p(cells), cells.numel(),
                                              _p(grad_out), _p(loss_out)))
        return loss_out, grad_out

    # -- the particle side after the fifth force -----------------------------
    def interp_to_particles(self, grid, pos, out=None):
        """CIC interpolation of a float32 mesh field (ncomp, n, n, n) or
        (n, n, n) to particles (n_part, 3)."""
        scalar = grid.dim() == 3
        ncomp = 1 if scalar else grid.shape[0]
        shape = self._grid() if scalar else (ncomp,) + self._grid()
        _need(grid, torch.float32, shape, "grid")
        _need(pos, torch.float32, (pos.shape[0], 3), "pos")
        if out is None:
            out = torch.empty((pos.shape[0], ncomp), dtype=torch.float32, device=pos.device)
        _need(out, torch.float32, (pos.shape[0], ncomp), "out")
        self._check(self.lib.mg_interp_to_particles(self.ptr, _p(grid), ncomp, _p(pos),
                                                    pos.shape[0], _p(out)))
        return out[:, 0] if scalar else out

    def interp_field_to_particles(self, field, pos, out=None):
        _need(field, torch.float64, self._grid(), "field")
        _need(pos, torch.float32, (pos.shape[0], 3), "pos")
        if out is None:
            out = torch.empty(pos.shape[0], dtype=torch.float64, device=pos.device)
        _need(out, torch.float64, (pos.shape[0],), "out")
        self._check(self.lib.mg_interp_field_to_particles(self.ptr, _p(field), _p(pos),
                                                          pos.shape[0], _p(out)))
        return out

    def poisson_newton(self, params, delta, out=None):
        """Newtonian potential (zero mean) of the density contrast."""
        _need(delta, torch.float32, self._grid(), "delta")
        if out is None:
            out = torch.empty(self._grid(), dtype=torch.float64, device=delta.device)
        _need(out, torch.float64, self._grid(), "phi_out")
        self._check(self.lib.mg_poisson_newton(self.ptr, ctypes.byref(params), _p(delta), _p(out)))
        return out

    def gradient(self, phi, out=None):
        """-grad phi by central differences, (3, n, n, n) float32."""
        _need(phi, torch.float64, self._grid(), "phi")
        if out is None:
            out = torch.empty((3,) + self._grid(), dtype=torch.float32, device=phi.device)
        _need(out, torch.float32, (3,) + self._grid(), "force_out")
        self._check(self.lib.mg_gradient(self.ptr, _p(phi), _p(out)))
        return out

    def total_force(self, model, params, phi_n, field, out=None):
        """-grad(s_N phi_n + Phi5(field)), s_N = exp(beta phibar) for CQ, else 1."""
        _need(phi_n, torch.float64, self._grid(), "phi_n")
        _need(field, torch.float64, self._grid(), "field")
        if out is None:
            out = torch.empty((3,) + self._grid(), dtype=torch.float32, device=field.device)
        _need(out, torch.float32, (3,) + self._grid(), "force_out")
        self._check(self.lib.mg_total_force(self.ptr, model_id(model), ctypes.byref(params), _p(phi_n),
                                            _p(field), _p(out)))
        return out

    def symmetron_friction(self, params, u_field, pos, mom, out=None):
        _need(u_field, torch.float64, self._grid(), "u_field")
        _need(pos, torch.float32, (pos.shape[0], 3), "pos")
        _need(mom, torch.float32, pos.shape, "mom")
        if out is None:
            out = torch.empty_like(mom)
        _need(out, torch.float32, (pos.shape[0], 3), "out")
        self._check(self.lib.mg_symmetron_friction(self.ptr, ctypes.byref(params), _p(u_field),
                                                   _p(pos), _p(mom), pos.shape[0], _p(out)))
        return out

    # -- batched boxes ------------------------------------------------------
    def _box_array(self, boxes):
        arr = (L.BoxDesc * len(boxes))()
        for q, b in enumerate(boxes):
            n = int(b["n"])
            _need(b["delta"], torch.float32, (n, n, n), f"boxes[{q}].delta")
            _need(b["field"], torch.float64, (n, n, n), f"boxes[{q}].field")
            force = b.get("force")
            if force is not None:
                _need(force, torch.float32, (3, n, n, n), f"boxes[{q}].force")
            arr[q].n = n
            arr[q].model = model_id(b["model"])
            arr[q].params = b["params"]
            arr[q].delta = b["delta"].data_ptr()
            arr[q].field = b["field"].data_ptr()
            arr[q].force = force.data_ptr() if force is not None else None
            arr[q].field_in = 1 if b.get("field_in") else 0
        return arr

    def solve_batched(self, boxes, tol=1e-6, opts=None, allow_noconv=False):
        """boxes: list of dicts (n, model, params, delta, field[, force, field_in]).
        Returns the per-box stats."""
        arr = self._box_array(boxes)
        opts = opts if opts is not None else solver_opts()
        st = (L.Stats * len(boxes))()
        rc = self.lib.mg_solve_batched(self.ptr, len(boxes), arr, ctypes.byref(opts), tol, st)
        self._check(rc, allow=(L.MG_ENOCONV,) if allow_noconv else ())
        return list(st)

    def batched_tune(self, boxes, opts=None):
        arr = self._box_array(boxes)
        opts = opts if opts is not None else solver_opts()
        blk, vec = ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.mg_batched_tune(self.ptr, len(boxes), arr, ctypes.byref(opts),
                                             ctypes.byref(blk), ctypes.byref(vec)))
        return blk.value, vec.value

    def batched_config(self):
        """(workgroup size, 4 cells per thread?, one sized team per box?)"""
        blk, vec, team = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.mg_batched_config(self.ptr, ctypes.byref(blk), ctypes.byref(vec),
                                               ctypes.byref(team)))
        return blk.value, vec.value, team.value

    def batched_set_config(self, block=0, vec=1, teams=1):
        """Pin the batched tile shape (block=0 unpins)."""
        self._check(self.lib.mg_batched_set_config(self.ptr, block, vec, teams))

    # -- kernel timing ------------------------------------------------------
    def prof_enable(self, on=True):
        self._check(self.lib.mg_prof_enable(self.ptr, 1 if on else 0))

    def prof_read(self, cls):
        """(total ms, launches) of one timed kernel class since prof_enable."""
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        self._check(self.lib.mg_prof_read(self.ptr, cls, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    # -- single operations (parity checks) ---------------------------------
    def relax_halfsweep(self, model, params, delta, field, colour):
        _need(delta, torch.float32, self._grid(), "delta")
        _need(field, torch.float64, self._grid(), "field")
        self._check(self.lib.mg_relax_halfsweep(self.ptr, model_id(model), ctypes.byref(params),
                                                _p(delta), _p(field), colour))
        return field

    def restrict(self, fine, out=None):
        _need(fine, torch.float64, self._grid(), "fine")
        nc = self.n // 2
        if out is None:
            out = torch.empty((nc, nc, nc), dtype=torch.float64, device=fine.device)
        self._check(self.lib.mg_restrict(self.ptr, _p(fine), _p(out)))
        return out

    def prolong_add(self, coarse, fine):
        nc = self.n // 2
        _need(coarse, torch.float64, (nc, nc, nc), "coarse")
        _need(fine, torch.float64, self._grid(), "fine")
        self._check(self.lib.mg_prolong_add(self.ptr, _p(coarse), _p(fine)))
        return fine


class MGSolve(torch.autograd.Function):
    """field = solve(delta); backward by the hand-written adjoint."""

    @staticmethod
    def forward(fctx, delta, mg, model, params, tol, opts, adj_tol):
        delta = delta.contiguous()
        field, _ = mg.solve(model, params, delta, tol=tol, opts=opts)
        fctx.save_for_backward(delta, field)
        fctx.mg, fctx.model, fctx.params, fctx.opts, fctx.adj_tol = mg, model, params, opts, adj_tol
        return field

    @staticmethod
    def backward(fctx, grad_field):
        delta, field = fctx.saved_tensors
        gd, _ = fctx.mg.solve_adjoint(fctx.model, fctx.params, delta, field,
                                      grad_field.contiguous().to(torch.float64), tol=fctx.adj_tol,
                                      opts=fctx.opts)
        return gd.to(delta.dtype), None, None, None, None, None, None


class MGForce(torch.autograd.Function):
    """force = -grad Phi5(field); backward by the transposed difference."""

    @staticmethod
    def forward(fctx, field, mg, model, params):
        force = mg.force(model, params, field.contiguous())
        fctx.save_for_backward(field)
        fctx.mg, fctx.model, fctx.params = mg, model, params
        return force

    @staticmethod
    def backward(fctx, grad_force):
        (field,) = fctx.saved_tensors
        g = fctx.mg.force_adjoint(fctx.model, fctx.params, field,
                                  grad_force.contiguous().to(torch.float32))
        return g, None, None, None


def solve_force(mg, model, params, delta, tol=1e-6, opts=None, adj_tol=None):
    """Differentiable delta -> (field, force)."""
    opts = opts if opts is not None else solver_opts()
    field = MGSolve.apply(delta, mg, model, params, tol, opts, adj_tol or tol)
    force = MGForce.apply(field, mg, model, params)
    return field, force
