"""ctypes binding of libmggpu.so (declarations mirror include/mggpu.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Loading fails loudly if the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmggpu.so")

MG_OK, MG_EINVAL, MG_ENOCONV, MG_ENAN, MG_EHIP = 0, -1, -2, -3, -4
MG_FR, MG_SYMMETRON, MG_CQ = 0, 1, 2
MG_FP64, MG_FP32_REFINED = 0, 1
MG_CYCLE_V, MG_CYCLE_F, MG_CYCLE_W = 0, 1, 2

# every symbol include/mggpu.h declares
EXPORTS = (
    "mg_ctx_create", "mg_ctx_destroy", "mg_last_error", "mg_ctx_levels", "cic_assign",
    "mg_solve", "mg_residual", "mg_force", "mg_force_adjoint", "mg_solve_adjoint",
    "mg_loss_force_sq", "mg_relax_halfsweep", "mg_restrict", "mg_prolong_add",
    "mg_solve_batched", "mg_prof_enable", "mg_prof_read", "mg_batched_tune",
    "mg_batched_config", "mg_batched_set_config", "mg_interp_to_particles",
    "mg_interp_field_to_particles", "mg_poisson_newton", "mg_gradient", "mg_total_force",
    "mg_symmetron_friction", "mg_cq_background", "mg_cq_background_at", "mg_solve_noalloc",
)
MG_PROF_SMOOTH32, MG_PROF_SMOOTH64, MG_PROF_LIN32, MG_PROF_LIN64 = 0, 1, 2, 3


class ModelParams(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double),
        ("omega_m", ctypes.c_double),
        ("box_mpch", ctypes.c_double),
        ("fr_n", ctypes.c_int),
        ("fr_fr0_abs", ctypes.c_double),
        ("sym_a_star", ctypes.c_double),
        ("sym_xi", ctypes.c_double),
        ("sym_beta_star", ctypes.c_double),
        ("cq_alpha", ctypes.c_double),
        ("cq_beta", ctypes.c_double),
        ("cq_phibar", ctypes.c_double),
        ("cq_lambda", ctypes.c_double),
        ("cq_keep_exp", ctypes.c_int),
    ]


class CqBackgroundParams(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in (
        "omega_m", "h", "t_cmb", "n_eff", "alpha", "beta", "z_init", "phi_init", "dphi_init",
        "tol")]


class CqBackgroundInfo(ctypes.Structure):
    _fields_ = [
        ("lam", ctypes.c_double),
        ("omega_r", ctypes.c_double),
        ("h_today", ctypes.c_double),
        ("shots", ctypes.c_int),
        ("steps", ctypes.c_long),
    ]


class SolverOpts(ctypes.Structure):
    _fields_ = [
        ("cycle", ctypes.c_int),
        ("nu_pre", ctypes.c_int),
        ("nu_post", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("max_cycles", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("coarse_sweeps", ctypes.c_int),
        ("fixed_cycles", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int),
        ("status", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("resid_hist", ctypes.c_double * 64),
        ("ms_total", ctypes.c_double),
        ("vcycles", ctypes.c_int),
        ("fallback", ctypes.c_int),
    ]


class BoxDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("model", ctypes.c_int),
        ("params", ModelParams),
        ("delta", ctypes.c_void_p),
        ("field", ctypes.c_void_p),
        ("force", ctypes.c_void_p),
        ("field_in", ctypes.c_int),
    ]


_lib = None


def load():
    """Load libmggpu.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "mg_ctx_create": (ci, [P(vp), ci, vp]),
        "mg_ctx_destroy": (None, [vp]),
        "mg_last_error": (ctypes.c_char_p, [vp]),
        "mg_ctx_levels": (ci, [vp]),
        "cic_assign": (ci, [vp, vp, i64, vp]),
        "mg_solve": (ci, [vp, ci, P(ModelParams), P(SolverOpts), vp, vp, vp, dbl, P(Stats)]),
        "mg_solve_noalloc": (ci, [vp, ci, P(ModelParams), P(SolverOpts), vp, vp, vp, dbl,
                                  P(Stats)]),
        "mg_residual": (ci, [vp, ci, P(ModelParams), vp, vp, vp, P(dbl)]),
        "mg_force": (ci, [vp, ci, P(ModelParams), vp, vp]),
        "mg_force_adjoint": (ci, [vp, ci, P(ModelParams), vp, vp, vp]),
        "mg_solve_adjoint": (ci, [vp, ci, P(ModelParams), P(SolverOpts), vp, vp, vp, vp, dbl,
                                  P(Stats)]),
        "mg_loss_force_sq": (ci, [vp, vp, vp, i64, vp, vp]),
        "mg_relax_halfsweep": (ci, [vp, ci, P(ModelParams), vp, vp, ci]),
        "mg_restrict": (ci, [vp, vp, vp]),
        "mg_prolong_add": (ci, [vp, vp, vp]),
        "mg_solve_batched": (ci, [vp, ci, P(BoxDesc), P(SolverOpts), dbl, P(Stats)]),
        "mg_prof_enable": (ci, [vp, ci]),
        "mg_prof_read": (ci, [vp, ci, P(dbl), P(i64)]),
        "mg_batched_tune": (ci, [vp, ci, P(BoxDesc), P(SolverOpts), P(ci), P(ci)]),
        "mg_batched_config": (ci, [vp, P(ci), P(ci), P(ci)]),
        "mg_batched_set_config": (ci, [vp, ci, ci, ci]),
        "mg_interp_to_particles": (ci, [vp, vp, ci, vp, i64, vp]),
        "mg_interp_field_to_particles": (ci, [vp, vp, vp, i64, vp]),
        "mg_poisson_newton": (ci, [vp, P(ModelParams), vp, vp]),
        "mg_gradient": (ci, [vp, vp, vp]),
        "mg_total_force": (ci, [vp, ci, P(ModelParams), vp, vp, vp]),
        "mg_symmetron_friction": (ci, [vp, P(ModelParams), vp, vp, vp, i64, vp]),
        "mg_cq_background": (ci, [P(CqBackgroundParams), ci, P(dbl), P(CqBackgroundInfo)]),
        "mg_cq_background_at": (ci, [P(dbl), ci, dbl, P(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return _lib
