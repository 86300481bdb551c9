"""Python binding of libhom.so (ctypes): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and law dictionaries into the C structures of ``include/hom.h`` and back.
There is no fallback: if the library is missing or cannot be loaded, every
entry point raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhom.so")

HOM_OK = 0
HOM_E_ARG = -1
HOM_E_OOM = -2
HOM_E_NOT_CONVERGED = -3
HOM_E_NAN = -4
HOM_E_DEVICE = -5
HOM_E_UNSUPPORTED = -6

SCHEME_BASIC = 0
SCHEME_NEWTON_CG = 1
FP64 = 0
FP32 = 1
DISC_COLLOCATION = 0
DISC_ROTATED = 1

FIELD_STRAIN = 0
FIELD_STRESS = 1
FIELD_GRADIENT = 2
FIELD_STATE = 3

OP_PROJECTOR = 0
OP_GAMMA0 = 1
OP_GRAD_PROJECTOR = 2
OP_GAMMA_CONDUCTION = 3
OP_PROJECTOR_ROTATED = 4
OP_GRAD_PROJECTOR_ROTATED = 5

MAX_MAXWELL = 16


class HomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hom error {code}: {msg}")
        self.code = code


class Grid(ct.Structure):
    _fields_ = [("n", ct.c_int32 * 3), ("len", ct.c_double * 3)]


class Law(ct.Structure):
    _fields_ = [
        ("kind", ct.c_int32),
        ("E", ct.c_double), ("nu", ct.c_double), ("alpha0", ct.c_double), ("kappa0", ct.c_double),
        ("c0", ct.c_double), ("theta0", ct.c_double),
        ("n_maxwell", ct.c_int32),
        ("E_i", ct.c_double * MAX_MAXWELL), ("log10_tau_i", ct.c_double * MAX_MAXWELL),
        ("C1", ct.c_double), ("C2", ct.c_double), ("theta_ref", ct.c_double), ("sigma_y0", ct.c_double),
        ("k_h", ct.c_double), ("n_h", ct.c_double), ("eta0", ct.c_double), ("m", ct.c_double),
        ("beta1", ct.c_double), ("beta2", ct.c_double),
    ]


class Options(ct.Structure):
    _fields_ = [
        ("scheme", ct.c_int32), ("precision", ct.c_int32), ("tol", ct.c_double), ("thermal_tol", ct.c_double),
        ("max_iter", ct.c_int32), ("max_krylov", ct.c_int32), ("chunk", ct.c_int32), ("use_graph", ct.c_int32),
        ("profile", ct.c_int32), ("autotune", ct.c_int32), ("stream", ct.c_void_p), ("tangent", ct.c_int32),
        ("discretization", ct.c_int32), ("predictor", ct.c_int32),
    ]


class MacroTemp(ct.Structure):
    _fields_ = [("theta", ct.c_double), ("grad", ct.c_double * 3)]


class Result(ct.Structure):
    _fields_ = [
        ("stress", ct.c_double * 6), ("heat_flux", ct.c_double * 3), ("dissipation", ct.c_double),
        ("coupling", ct.c_double), ("heat_capacity", ct.c_double), ("residual", ct.c_double),
        ("newton_iters", ct.c_int32), ("krylov_iters", ct.c_int32), ("thermal_iters", ct.c_int32),
        ("status", ct.c_int32), ("pipelines", ct.c_double), ("thermal_pipelines", ct.c_double),
        ("strain", ct.c_double * 6), ("theta", ct.c_double), ("stagger_iters", ct.c_int32),
        ("reserved", ct.c_int32),
    ]

    def as_dict(self):
        return dict(stress=np.array(self.stress[:]), heat_flux=np.array(self.heat_flux[:]),
                    dissipation=self.dissipation, coupling=self.coupling, heat_capacity=self.heat_capacity,
                    residual=self.residual, newton_iters=self.newton_iters, krylov_iters=self.krylov_iters,
                    thermal_iters=self.thermal_iters, status=self.status, pipelines=self.pipelines,
                    thermal_pipelines=self.thermal_pipelines, strain=np.array(self.strain[:]), theta=self.theta,
                    stagger_iters=self.stagger_iters)


class Load(ct.Structure):
    _fields_ = [
        ("strain", ct.c_double * 6), ("stress", ct.c_double * 6), ("stress_mask", ct.c_uint32),
        ("adiabatic", ct.c_int32), ("temp", MacroTemp), ("dt", ct.c_double), ("trial", ct.c_int32),
        ("reserved", ct.c_int32),
    ]


def make_load(strain, theta, grad, dt, stress=None, stress_mask=0, adiabatic=False, trial=False) -> Load:
    """hom_load; stress_mask: int bit mask or 6 booleans (True: stress-controlled)."""
    L = Load()
    for c in range(6):
        L.strain[c] = float(strain[c])
        L.stress[c] = 0.0 if stress is None else float(stress[c])
    if not isinstance(stress_mask, (int, np.integer)):
        stress_mask = sum(1 << c for c in range(6) if stress_mask[c])
    L.stress_mask = int(stress_mask)
    L.adiabatic = int(bool(adiabatic))
    L.trial = int(bool(trial))
    L.temp.theta = float(theta)
    for c in range(3):
        L.temp.grad[c] = float(grad[c])
    L.dt = float(dt)
    return L


class Tangent(ct.Structure):
    _fields_ = [
        ("dsde", ct.c_double * 36), ("dsdt", ct.c_double * 6), ("dDde", ct.c_double * 6), ("dDdt", ct.c_double),
        ("solves", ct.c_int32), ("krylov_iters", ct.c_int32), ("pipelines", ct.c_double), ("status", ct.c_int32),
    ]

    def as_dict(self):
        return dict(dsde=np.array(self.dsde[:]).reshape(6, 6), dsdt=np.array(self.dsdt[:]),
                    dDde=np.array(self.dDde[:]), dDdt=self.dDdt, solves=self.solves,
                    krylov_iters=self.krylov_iters, pipelines=self.pipelines, status=self.status)


class DmnTrainOpts(ct.Structure):
    _fields_ = [("lr_max", ct.c_double), ("lr_min", ct.c_double), ("half_period", ct.c_int32),
                ("decay", ct.c_double), ("q", ct.c_double), ("penalty", ct.c_double)]


class DmnResult(ct.Structure):
    _fields_ = [
        ("stress", ct.c_double * 6), ("coupling", ct.c_double), ("dissipation", ct.c_double),
        ("dsde", ct.c_double * 36), ("dsdt", ct.c_double * 6), ("dDde", ct.c_double * 6), ("dDdt", ct.c_double),
        ("residual", ct.c_double), ("newton_iters", ct.c_int32), ("status", ct.c_int32),
    ]

    def as_dict(self):
        return dict(stress=np.array(self.stress[:]), coupling=self.coupling, dissipation=self.dissipation,
                    dsde=np.array(self.dsde[:]).reshape(6, 6), dsdt=np.array(self.dsdt[:]),
                    dDde=np.array(self.dDde[:]), dDdt=self.dDdt, residual=self.residual,
                    newton_iters=self.newton_iters, status=self.status)


# hom_dmn_result as a numpy record (same layout): DmnOnline.step fills an array
# of these in place, so results[i]["stress"], results["dsde"] etc. need no copy
DMN_RESULT_DTYPE = np.dtype([
    ("stress", "<f8", (6,)), ("coupling", "<f8"), ("dissipation", "<f8"), ("dsde", "<f8", (6, 6)),
    ("dsdt", "<f8", (6,)), ("dDde", "<f8", (6,)), ("dDdt", "<f8"), ("residual", "<f8"),
    ("newton_iters", "<i4"), ("status", "<i4"),
])
assert DMN_RESULT_DTYPE.itemsize == ct.sizeof(DmnResult)


# hom_result as a numpy record (same layout), for bulk result arrays
RESULT_DTYPE = np.dtype([
    ("stress", "<f8", (6,)), ("heat_flux", "<f8", (3,)), ("dissipation", "<f8"), ("coupling", "<f8"),
    ("heat_capacity", "<f8"), ("residual", "<f8"), ("newton_iters", "<i4"), ("krylov_iters", "<i4"),
    ("thermal_iters", "<i4"), ("status", "<i4"), ("pipelines", "<f8"), ("thermal_pipelines", "<f8"),
    ("strain", "<f8", (6,)), ("theta", "<f8"), ("stagger_iters", "<i4"), ("reserved", "<i4"),
], align=True)
assert RESULT_DTYPE.itemsize == ct.sizeof(Result)


class SurrogateConfig(ct.Structure):
    _fields_ = [("n_nets", ct.c_int32), ("epochs", ct.c_int32), ("batch", ct.c_int32), ("lr", ct.c_double),
                ("seed", ct.c_uint64), ("target", ct.c_double), ("quantile", ct.c_double),
                ("holdout", ct.c_double), ("floor_scale", ct.c_double), ("theta_init", ct.c_double),
                ("chunk", ct.c_int32), ("max_resident", ct.c_int32)]


class SurrogateReport(ct.Structure):
    _fields_ = [("train_rows", ct.c_int64), ("holdout_rows", ct.c_int64), ("threshold", ct.c_double),
                ("holdout_accepted", ct.c_double), ("holdout_accepted_max_error", ct.c_double),
                ("holdout_accepted_p99_error", ct.c_double), ("holdout_median_error", ct.c_double),
                ("holdout_median_error_forced", ct.c_double), ("skip_median_error", ct.c_double),
                ("fit_seconds", ct.c_double), ("final_loss", ct.c_double * 16)]

    def as_dict(self, nets=16):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "final_loss"}
        d["final_loss"] = list(self.final_loss[:nets])
        return d


class SurrogateStepInfo(ct.Structure):
    _fields_ = [("network_points", ct.c_int32), ("rejected_points", ct.c_int32), ("resident_points", ct.c_int32),
                ("replayed_increments", ct.c_int32), ("network_ms", ct.c_double), ("fallback_ms", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = (
    "hom_default_options", "hom_setup", "hom_solve_increment", "hom_state_size", "hom_get_state",
    "hom_set_state", "hom_get_field", "hom_kernel_stats", "hom_set_profiling", "hom_device_bytes",
    "hom_algorithmic_tangent", "hom_batch_algorithmic_tangent", "hom_solve_load", "hom_batch_solve_load",
    "hom_set_laws", "hom_batch_set_laws",
    "hom_last_error", "hom_destroy",
    "hom_batch_setup", "hom_batch_solve_increment", "hom_batch_kernel_stats", "hom_batch_last_error",
    "hom_batch_destroy", "hom_batch_schedules", "hom_schedules", "hom_apply_operator", "hom_apply_operator_schedule",
    "hom_eval_law",
    "hom_dmn_default_train_opts", "hom_dmn_create", "hom_dmn_get_params", "hom_dmn_set_params",
    "hom_dmn_homogenize", "hom_dmn_loss_grad", "hom_dmn_train", "hom_dmn_last_error", "hom_dmn_destroy",
    "hom_dmn_online_create", "hom_dmn_online_step", "hom_dmn_online_set_predictor", "hom_dmn_online_last_error",
    "hom_dmn_online_destroy",
    "hom_mlp_create", "hom_mlp_param_count", "hom_mlp_set_scaling", "hom_mlp_set_skip", "hom_mlp_fit_skip",
    "hom_mlp_get_params",
    "hom_mlp_set_params",
    "hom_mlp_train", "hom_mlp_forward", "hom_mlp_loss_grad", "hom_mlp_ensemble_infer",
    "hom_mlp_ensemble_infer_static",
    "hom_mlp_last_error",
    "hom_mlp_destroy",
    "hom_surrogate_default_config", "hom_surrogate_create", "hom_surrogate_solve_histories",
    "hom_surrogate_features", "hom_surrogate_train", "hom_surrogate_calibrate", "hom_surrogate_set_threshold",
    "hom_surrogate_threshold", "hom_surrogate_infer", "hom_surrogate_points_create", "hom_surrogate_points_step",
    "hom_surrogate_points_last_error", "hom_surrogate_points_destroy", "hom_surrogate_last_error",
    "hom_surrogate_destroy",
)

_lib = None


def library(path: str | None = None):
    """Load libhom.so (once). Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise HomError(HOM_E_DEVICE, f"{p} is not built; run __graft_entry__.build()")
    # PyTorch (used for device buffers and streams) ships its own HIP runtime;
    # it has to be loaded before this library's, or it finds no GPU later.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(p)
    dp = ct.POINTER(ct.c_double)
    lib.hom_default_options.argtypes = [ct.POINTER(Options)]
    lib.hom_setup.argtypes = [ct.POINTER(Grid), ct.c_void_p, ct.POINTER(Law), ct.c_int32, ct.POINTER(Options),
                              ct.POINTER(ct.c_void_p)]
    lib.hom_solve_increment.argtypes = [ct.c_void_p, dp, ct.POINTER(MacroTemp), ct.c_double, ct.POINTER(Result)]
    lib.hom_state_size.argtypes = [ct.c_void_p]
    lib.hom_state_size.restype = ct.c_size_t
    lib.hom_get_state.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t]
    lib.hom_set_state.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t]
    lib.hom_get_field.argtypes = [ct.c_void_p, ct.c_int32, dp, ct.c_size_t]
    lib.hom_kernel_stats.argtypes = [ct.c_void_p, ct.POINTER(ct.c_char_p), ct.POINTER(ct.c_int64), dp, ct.c_int32]
    lib.hom_set_profiling.argtypes = [ct.c_void_p, ct.c_int32]
    lib.hom_algorithmic_tangent.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(Tangent)]
    lib.hom_solve_load.argtypes = [ct.c_void_p, ct.POINTER(Load), ct.POINTER(Result)]
    lib.hom_set_laws.argtypes = [ct.c_void_p, ct.POINTER(Law), ct.c_int32]
    lib.hom_batch_set_laws.argtypes = [ct.c_void_p, ct.POINTER(Law), ct.c_int32]
    lib.hom_batch_solve_load.argtypes = [ct.c_void_p, ct.POINTER(Load), ct.POINTER(Result)]
    lib.hom_batch_algorithmic_tangent.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(Tangent)]
    lib.hom_device_bytes.argtypes = [ct.c_void_p]
    lib.hom_device_bytes.restype = ct.c_size_t
    lib.hom_last_error.argtypes = [ct.c_void_p]
    lib.hom_last_error.restype = ct.c_char_p
    lib.hom_destroy.argtypes = [ct.c_void_p]
    lib.hom_destroy.restype = None
    lib.hom_batch_setup.argtypes = [ct.c_int32, ct.POINTER(Grid), ct.POINTER(ct.c_void_p), ct.POINTER(Law),
                                    ct.c_int32, ct.POINTER(Options), ct.POINTER(ct.c_void_p)]
    lib.hom_batch_solve_increment.argtypes = [ct.c_void_p, dp, ct.POINTER(MacroTemp), dp, ct.POINTER(Result)]
    lib.hom_batch_kernel_stats.argtypes = [ct.c_void_p, ct.POINTER(ct.c_char_p), ct.POINTER(ct.c_int64), dp,
                                           ct.c_int32]
    lib.hom_batch_last_error.argtypes = [ct.c_void_p]
    lib.hom_batch_last_error.restype = ct.c_char_p
    lib.hom_batch_destroy.argtypes = [ct.c_void_p]
    lib.hom_batch_destroy.restype = None
    lib.hom_apply_operator.argtypes = [ct.POINTER(Grid), ct.c_int32, ct.c_int32, ct.c_double, ct.c_double,
                                       ct.c_int32, dp, dp]
    lib.hom_schedules.argtypes = [ct.c_void_p, ct.POINTER(ct.c_int32), ct.c_int32]
    lib.hom_batch_schedules.argtypes = [ct.c_void_p, ct.POINTER(ct.c_int32), ct.c_int32]
    lib.hom_apply_operator_schedule.argtypes = [ct.POINTER(Grid), ct.c_int32, ct.c_int32, ct.c_double, ct.c_double,
                                                ct.c_int32, ct.c_int32, dp, dp]
    lib.hom_eval_law.argtypes = [ct.POINTER(Law), ct.c_int64, dp, dp, dp, ct.c_double, ct.c_double, ct.c_int32,
                                 dp, dp, dp, dp, dp, dp]
    lib.hom_dmn_default_train_opts.argtypes = [ct.POINTER(DmnTrainOpts)]
    lib.hom_dmn_default_train_opts.restype = None
    lib.hom_dmn_create.argtypes = [ct.c_int32, ct.c_uint64, ct.POINTER(ct.c_void_p)]
    lib.hom_dmn_get_params.argtypes = [ct.c_void_p, dp, dp]
    lib.hom_dmn_set_params.argtypes = [ct.c_void_p, dp, dp]
    lib.hom_dmn_homogenize.argtypes = [ct.c_void_p, ct.c_int64, dp, dp, dp]
    lib.hom_dmn_loss_grad.argtypes = [ct.c_void_p, ct.c_int64, dp, dp, dp, ct.POINTER(DmnTrainOpts), dp, dp, dp]
    lib.hom_dmn_train.argtypes = [ct.c_void_p, ct.c_int64, dp, dp, dp, ct.c_int32, ct.c_int32, ct.c_uint64,
                                  ct.POINTER(DmnTrainOpts), dp]
    lib.hom_dmn_last_error.argtypes = [ct.c_void_p]
    lib.hom_dmn_last_error.restype = ct.c_char_p
    lib.hom_dmn_destroy.argtypes = [ct.c_void_p]
    lib.hom_dmn_destroy.restype = None
    lib.hom_dmn_online_create.argtypes = [ct.c_void_p, ct.POINTER(Law), ct.c_int32, ct.c_double, ct.c_int32,
                                          ct.POINTER(ct.c_void_p)]
    lib.hom_dmn_online_step.argtypes = [ct.c_void_p, dp, dp, dp, ct.c_int32, ct.c_int32, ct.POINTER(DmnResult)]
    lib.hom_dmn_online_set_predictor.argtypes = [ct.c_void_p, ct.c_int32]
    lib.hom_dmn_online_last_error.argtypes = [ct.c_void_p]
    lib.hom_dmn_online_last_error.restype = ct.c_char_p
    lib.hom_dmn_online_destroy.argtypes = [ct.c_void_p]
    lib.hom_dmn_online_destroy.restype = None
    fp = ct.POINTER(ct.c_float)
    lib.hom_mlp_create.argtypes = [ct.c_int32, ct.c_int32, ct.c_uint64, ct.POINTER(ct.c_void_p)]
    lib.hom_mlp_param_count.argtypes = [ct.c_void_p]
    lib.hom_mlp_param_count.restype = ct.c_size_t
    lib.hom_mlp_set_scaling.argtypes = [ct.c_void_p, fp, fp, fp, fp, fp]
    lib.hom_mlp_set_skip.argtypes = [ct.c_void_p, ct.POINTER(ct.c_int32), fp, fp]
    lib.hom_mlp_fit_skip.argtypes = [ct.c_void_p, fp, fp, ct.c_int64, ct.POINTER(ct.c_int32), fp, fp]
    lib.hom_mlp_get_params.argtypes = [ct.c_void_p, fp, ct.c_size_t]
    lib.hom_mlp_set_params.argtypes = [ct.c_void_p, fp, ct.c_size_t]
    lib.hom_mlp_train.argtypes = [ct.c_void_p, fp, fp, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_double, ct.c_uint64,
                                  fp, fp]
    lib.hom_mlp_forward.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p]
    lib.hom_mlp_loss_grad.argtypes = [ct.c_void_p, fp, fp, ct.c_int64, ct.c_int32, ct.POINTER(ct.c_double), fp]
    lib.hom_mlp_ensemble_infer.argtypes = [ct.POINTER(ct.c_void_p), ct.c_int32, ct.c_void_p, ct.c_void_p,
                                           ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_double, ct.c_double,
                                           ct.c_void_p]
    lib.hom_mlp_ensemble_infer_static.argtypes = lib.hom_mlp_ensemble_infer.argtypes
    fp64 = dp
    hist = [ct.c_int32, ct.c_int32, fp64, fp64, fp64, fp64]
    lib.hom_surrogate_default_config.argtypes = [ct.POINTER(SurrogateConfig)]
    lib.hom_surrogate_default_config.restype = None
    lib.hom_surrogate_create.argtypes = [ct.POINTER(Grid), ct.c_void_p, ct.POINTER(Law), ct.c_int32,
                                         ct.POINTER(Options), ct.POINTER(SurrogateConfig), ct.POINTER(ct.c_void_p)]
    lib.hom_surrogate_solve_histories.argtypes = [ct.c_void_p] + hist + [ct.c_void_p, fp64]
    lib.hom_surrogate_features.argtypes = hist + [ct.c_void_p, ct.c_double, fp, fp, fp64]
    lib.hom_surrogate_train.argtypes = [ct.c_void_p] + hist + [ct.c_void_p, ct.POINTER(SurrogateReport)]
    lib.hom_surrogate_calibrate.argtypes = [ct.c_void_p] + hist + [ct.c_void_p, ct.c_double, ct.c_double,
                                                                   ct.POINTER(SurrogateReport)]
    lib.hom_surrogate_set_threshold.argtypes = [ct.c_void_p, ct.c_double]
    lib.hom_surrogate_threshold.argtypes = [ct.c_void_p]
    lib.hom_surrogate_threshold.restype = ct.c_double
    lib.hom_surrogate_infer.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64,
                                        ct.c_void_p]
    lib.hom_surrogate_points_create.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_void_p)]
    lib.hom_surrogate_points_step.argtypes = [ct.c_void_p, fp64, fp64, fp64, fp64, ct.c_void_p, ct.c_void_p,
                                              ct.POINTER(SurrogateStepInfo)]
    lib.hom_surrogate_points_last_error.argtypes = [ct.c_void_p]
    lib.hom_surrogate_points_last_error.restype = ct.c_char_p
    lib.hom_surrogate_points_destroy.argtypes = [ct.c_void_p]
    lib.hom_surrogate_points_destroy.restype = None
    lib.hom_surrogate_last_error.argtypes = [ct.c_void_p]
    lib.hom_surrogate_last_error.restype = ct.c_char_p
    lib.hom_surrogate_destroy.argtypes = [ct.c_void_p]
    lib.hom_surrogate_destroy.restype = None
    lib.hom_mlp_last_error.argtypes = [ct.c_void_p]
    lib.hom_mlp_last_error.restype = ct.c_char_p
    lib.hom_mlp_destroy.argtypes = [ct.c_void_p]
    lib.hom_mlp_destroy.restype = None
    _lib = lib
    return lib


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_law(p: dict) -> Law:
    """hom_law from a parameter dictionary (see workloads.py)."""
    L = Law()
    kind = p["kind"]
    L.kind = 1 if kind == "thermoelastic" else 2
    for k in ("E", "nu", "alpha0", "kappa0", "c0", "theta0"):
        setattr(L, k, float(p[k]))
    if L.kind == 2:
        Ei = list(p["E_i"])
        ti = list(p["log10_tau_i"])
        if len(Ei) > MAX_MAXWELL:
            raise HomError(HOM_E_ARG, "too many Maxwell branches")
        L.n_maxwell = len(Ei)
        for i, (e, t) in enumerate(zip(Ei, ti)):
            L.E_i[i] = e
            L.log10_tau_i[i] = t
        for k in ("C1", "C2", "theta_ref", "sigma_y0", "k_h", "n_h", "eta0", "m", "beta1", "beta2"):
            setattr(L, k, float(p[k]))
    return L


def make_options(scheme=SCHEME_NEWTON_CG, precision=FP32, tol=1e-6, thermal_tol=0.0, max_iter=0, max_krylov=0,
                 chunk=0, use_graph=1, profile=0, autotune=0, stream=None, tangent=0,
                 discretization=0, predictor=0) -> Options:
    o = Options()
    library().hom_default_options(ct.byref(o))
    o.scheme = scheme
    o.precision = precision
    o.tol = tol
    o.thermal_tol = thermal_tol
    o.max_iter = max_iter
    o.max_krylov = max_krylov
    o.chunk = chunk
    o.use_graph = use_graph
    o.profile = profile
    o.autotune = autotune
    o.stream = stream
    o.tangent = tangent
    o.discretization = discretization
    o.predictor = predictor
    return o


def make_grid(shape_zyx, lengths=(1.0, 1.0, 1.0)) -> Grid:
    g = Grid()
    nz, ny, nx = shape_zyx
    g.n[0], g.n[1], g.n[2] = nx, ny, nz
    for i in range(3):
        g.len[i] = lengths[i]
    return g


def _check(code, msg_fn):
    if code != HOM_OK:
        raise HomError(code, msg_fn())


class _Handle:
    """Scope use of an owning handle: `with Context(...) as ctx:` closes it on
    exit, also when the block raises."""

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


class Context(_Handle):
    """One microstructure (hom_setup / hom_solve_increment / ...)."""

    def __init__(self, phases, laws, options: Options | None = None, lengths=(1.0, 1.0, 1.0), **opt_kw):
        lib = library()
        self._lib = lib
        ph = np.ascontiguousarray(phases, dtype=np.uint8)
        self.shape = ph.shape
        self.grid = make_grid(ph.shape, lengths)
        n = len(laws)
        self._laws = (Law * n)(*[make_law(p) for p in laws])
        self.options = options if options is not None else make_options(**opt_kw)
        h = ct.c_void_p()
        rc = lib.hom_setup(ct.byref(self.grid), ph.ctypes.data_as(ct.c_void_p), self._laws, n,
                           ct.byref(self.options), ct.byref(h))
        _check(rc, lambda: lib.hom_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return self._lib.hom_last_error(self._h).decode()

    def solve_increment(self, strain, theta, grad, dt, check=True):
        s = _f64(strain)
        t = MacroTemp()
        t.theta = theta
        for i in range(3):
            t.grad[i] = float(grad[i])
        r = Result()
        rc = self._lib.hom_solve_increment(self._h, _dptr(s), ct.byref(t), float(dt), ct.byref(r))
        if check:
            _check(rc, self.error)
        out = r.as_dict()
        out["rc"] = rc
        return out

    def set_laws(self, laws):
        """hom_set_laws: new parameters for the phase laws (same kinds)."""
        arr = (Law * len(laws))(*[make_law(p) for p in laws])
        _check(self._lib.hom_set_laws(self._h, arr, len(laws)), self.error)
        self._laws = arr

    def solve_load(self, strain, theta, grad, dt, stress=None, stress_mask=0, adiabatic=False, trial=False,
                   check=True):
        """hom_solve_load: mixed boundary conditions and / or the adiabatic heat
        balance (theta is theta^n when adiabatic); trial: commit nothing."""
        L = make_load(strain, theta, grad, dt, stress, stress_mask, adiabatic, trial)
        r = Result()
        rc = self._lib.hom_solve_load(self._h, ct.byref(L), ct.byref(r))
        if check:
            _check(rc, self.error)
        out = r.as_dict()
        out["rc"] = rc
        return out

    def field(self, which):
        nv = int(np.prod(self.shape))
        nc = {FIELD_STRAIN: 6, FIELD_STRESS: 6, FIELD_GRADIENT: 3}.get(which)
        if nc is None:
            nc = self.nstate
        out = np.empty(nc * nv)
        rc = self._lib.hom_get_field(self._h, which, _dptr(out), out.size)
        _check(rc, self.error)
        return out.reshape((nc,) + tuple(self.shape))

    @property
    def nstate(self):
        for L in self._laws:
            if L.kind == 2:
                return 7 + 6 * sum(1 for i in range(L.n_maxwell) if L.E_i[i] > 0)
        return 0

    def get_state(self, as_array=False):
        """Checkpoint (committed fields, internal variables, macro state) as
        bytes, or as a uint8 array without the extra host copy."""
        n = self._lib.hom_state_size(self._h)
        buf = np.empty(n, dtype=np.uint8)
        _check(self._lib.hom_get_state(self._h, buf.ctypes.data_as(ct.c_void_p), n), self.error)
        return buf if as_array else buf.tobytes()

    def set_state(self, data):
        buf = np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(self._lib.hom_set_state(self._h, buf.ctypes.data_as(ct.c_void_p), buf.size), self.error)

    def algorithmic_tangent(self, what=1):
        """Effective algorithmic tangents of the last converged increment
        (hom_algorithmic_tangent): dsde (6, 6), dsdt (6,), dDde (6,), dDdt."""
        t = Tangent()
        _check(self._lib.hom_algorithmic_tangent(self._h, int(what), ct.byref(t)), self.error)
        return t.as_dict()

    def kernel_stats(self):
        return _stats(self._lib.hom_kernel_stats, self._h)

    def schedules(self):
        """The y / z pass schedules (tile width, FFT plan) the autotuner chose."""
        return _schedules(self._lib.hom_schedules, self._h)

    def set_profiling(self, on: bool):
        _check(self._lib.hom_set_profiling(self._h, int(on)), self.error)

    def device_bytes(self):
        return int(self._lib.hom_device_bytes(self._h))


def _schedules(fn, h):
    cap = 16
    buf = (ct.c_int32 * (7 * cap))()
    n = fn(h, buf, cap)
    if n < 0:
        raise HomError(n, "schedule query failed")
    keys = ("grid", "y_mech", "z_mech", "y_thermal", "z_thermal")
    out = []
    for g in range(min(n, cap)):
        r = list(buf[7 * g: 7 * g + 7])
        sched = {k: {"tile": v & 15, "plan": v >> 4} for k, v in zip(keys[1:], r[3:])}
        out.append({"grid": r[:3], **sched})
    return out


def _stats(fn, h):
    cap = 32
    names = (ct.c_char_p * cap)()
    launches = (ct.c_int64 * cap)()
    ms = (ct.c_double * cap)()
    n = fn(h, names, launches, ms, cap)
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(n)}


class Batch(_Handle):
    """Independent microproblems solved together (hom_batch_*)."""

    def __init__(self, phase_list, laws, options: Options | None = None, lengths=(1.0, 1.0, 1.0), **opt_kw):
        lib = library()
        self._lib = lib
        self._phases = [np.ascontiguousarray(p, dtype=np.uint8) for p in phase_list]
        n = len(self._phases)
        self.n = n
        self._grids = (Grid * n)(*[make_grid(p.shape, lengths) for p in self._phases])
        ptrs = (ct.c_void_p * n)(*[p.ctypes.data_as(ct.c_void_p).value for p in self._phases])
        nl = len(laws)
        self._laws = (Law * nl)(*[make_law(p) for p in laws])
        self.options = options if options is not None else make_options(**opt_kw)
        h = ct.c_void_p()
        rc = lib.hom_batch_setup(n, self._grids, ptrs, self._laws, nl, ct.byref(self.options), ct.byref(h))
        _check(rc, lambda: lib.hom_batch_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_increment(self, strains, thetas, grads, dts):
        s = _f64(strains).reshape(self.n, 6)
        temps = (MacroTemp * self.n)()
        for i in range(self.n):
            temps[i].theta = float(thetas[i])
            for c in range(3):
                temps[i].grad[c] = float(grads[i][c])
        d = _f64(dts).reshape(self.n)
        res = (Result * self.n)()
        rc = self._lib.hom_batch_solve_increment(self._h, _dptr(s), temps, _dptr(d), res)
        _check(rc, lambda: self._lib.hom_batch_last_error(self._h).decode())
        return [r.as_dict() for r in res]

    def set_laws(self, laws):
        arr = (Law * len(laws))(*[make_law(p) for p in laws])
        _check(self._lib.hom_batch_set_laws(self._h, arr, len(laws)),
               lambda: self._lib.hom_batch_last_error(self._h).decode())
        self._laws = arr

    def solve_load(self, loads):
        """loads: one dict per problem with the keyword arguments of make_load."""
        arr = (Load * self.n)(*[make_load(**d) for d in loads])
        res = (Result * self.n)()
        rc = self._lib.hom_batch_solve_load(self._h, arr, res)
        _check(rc, lambda: self._lib.hom_batch_last_error(self._h).decode())
        return [r.as_dict() for r in res]

    def algorithmic_tangent(self, what=1):
        out = (Tangent * self.n)()
        _check(self._lib.hom_batch_algorithmic_tangent(self._h, int(what), out),
               lambda: self._lib.hom_batch_last_error(self._h).decode())
        return [t.as_dict() for t in out]

    def kernel_stats(self):
        return _stats(self._lib.hom_batch_kernel_stats, self._h)

    def schedules(self):
        """The y / z pass schedules (tile width, FFT plan) per grid group."""
        return _schedules(self._lib.hom_batch_schedules, self._h)


# schedules of the y and z passes: tile width + 16 x FFT plan variant
SCHEDULES = (2, 4, 8, 18, 20, 24)


def apply_operator(field, op, p0=0.0, p1=0.0, precision=FP64, lengths=(1.0, 1.0, 1.0), schedule=None):
    """IFFT(Op FFT(field)) on the GPU; field (C, nz, ny, nx) float64;
    schedule: one of SCHEDULES, or None for the default."""
    lib = library()
    f = _f64(field)
    C = f.shape[0]
    g = make_grid(f.shape[1:], lengths)
    out = np.empty_like(f)
    if schedule is None:
        rc = lib.hom_apply_operator(ct.byref(g), C, op, p0, p1, precision, _dptr(f), _dptr(out))
    else:
        rc = lib.hom_apply_operator_schedule(ct.byref(g), C, op, p0, p1, precision, int(schedule), _dptr(f),
                                             _dptr(out))
    _check(rc, lambda: lib.hom_last_error(None).decode())
    return out


def eval_law(law: dict, eps, eps_n=None, state=None, theta=293.15, dt=1.0, commit=False):
    """Evaluate one law on the GPU at points eps (6, M) (Mandel)."""
    lib = library()
    L = make_law(law)
    e = _f64(eps)
    m = e.shape[1]
    en = _f64(eps_n) if eps_n is not None else np.zeros_like(e)
    st = _f64(state) if state is not None else None
    sig = np.empty((6, m))
    ab = np.empty((2, m))
    nd = np.zeros((6, m))
    nst = 0 if L.kind == 1 else 7 + 6 * sum(1 for i in range(L.n_maxwell) if L.E_i[i] > 0)
    st_out = np.empty((nst, m)) if (commit and nst) else None
    diss = np.empty(m) if commit else None
    coup = np.empty(m) if commit else None
    rc = lib.hom_eval_law(ct.byref(L), m, _dptr(e), _dptr(en), _dptr(st), float(theta), float(dt), int(commit),
                          _dptr(sig), _dptr(ab), _dptr(nd), _dptr(st_out), _dptr(diss), _dptr(coup))
    _check(rc, lambda: lib.hom_last_error(None).decode())
    return dict(sigma=sig, ab=ab, nd=nd, state=st_out, dissipation=diss, coupling=coup)


def _fptr(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_float))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class MLP(_Handle):
    """The surrogate network (hom_mlp_*). Device arrays are torch tensors."""

    def __init__(self, n_in, n_out, seed=0):
        lib = library()
        self._lib = lib
        h = ct.c_void_p()
        _check(lib.hom_mlp_create(n_in, n_out, seed, ct.byref(h)), lambda: lib.hom_mlp_last_error(None).decode())
        self._h = h
        self.n_in, self.n_out = n_in, n_out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return self._lib.hom_mlp_last_error(self._h).decode()

    @property
    def param_count(self):
        return int(self._lib.hom_mlp_param_count(self._h))

    def set_scaling(self, x_mean, x_std, y_mean, y_std, loss_weight=None):
        lw = _f32(loss_weight) if loss_weight is not None else _f32(np.ones(self.n_out))
        arrs = [_f32(a) for a in (x_mean, x_std, y_mean, y_std)]
        _check(self._lib.hom_mlp_set_scaling(self._h, *[_fptr(a) for a in arrs], _fptr(lw)), self.error)

    N_GATES = 10

    def set_skip(self, gates, G, c):
        """Gated polynomial skip: G [n_out, 10, n_in], c [n_out], gates: 3 input indices."""
        g = (ct.c_int32 * 3)(*[int(v) for v in gates])
        G = _f32(G).reshape(self.n_out, self.N_GATES, self.n_in)
        c = _f32(c).reshape(self.n_out)
        _check(self._lib.hom_mlp_set_skip(self._h, g, _fptr(G), _fptr(c)), self.error)

    def fit_skip(self, x, y, gates, loss_weight=None, row_weight=None):
        x, y = _f32(x), _f32(y)
        g = (ct.c_int32 * 3)(*[int(v) for v in gates])
        lw = _f32(loss_weight) if loss_weight is not None else None
        rw = _f32(row_weight) if row_weight is not None else None
        _check(self._lib.hom_mlp_fit_skip(self._h, _fptr(x), _fptr(y), x.shape[0], g,
                                          _fptr(lw) if lw is not None else None,
                                          _fptr(rw) if rw is not None else None), self.error)

    def get_params(self):
        out = np.empty(self.param_count, dtype=np.float32)
        _check(self._lib.hom_mlp_get_params(self._h, _fptr(out), out.size), self.error)
        return out

    def set_params(self, p):
        p = _f32(p)
        _check(self._lib.hom_mlp_set_params(self._h, _fptr(p), p.size), self.error)

    def layers(self, flat=None):
        """Split a flat parameter vector into [(W [out, in], b [out])]."""
        flat = self.get_params() if flat is None else flat
        sizes = [self.n_in, 256, 256, 256, 256, self.n_out]
        out, o = [], 0
        for i, j in zip(sizes[:-1], sizes[1:]):
            W = flat[o:o + i * j].reshape(j, i)
            o += i * j
            b = flat[o:o + j]
            o += j
            out.append((W, b))
        return out

    def train(self, x, y, epochs, batch=256, lr=2e-3, seed=0, row_weight=None):
        x, y = _f32(x), _f32(y)
        rw = _f32(row_weight) if row_weight is not None else None
        losses = np.empty(epochs, dtype=np.float32)
        _check(self._lib.hom_mlp_train(self._h, _fptr(x), _fptr(y), x.shape[0], epochs, batch, lr, seed,
                                       _fptr(rw) if rw is not None else None, _fptr(losses)), self.error)
        return losses

    def forward_device(self, x_dev, y_dev, precise=False, stream=None):
        n = x_dev.shape[0]
        _check(self._lib.hom_mlp_forward(self._h, ct.c_void_p(x_dev.data_ptr()), ct.c_void_p(y_dev.data_ptr()), n,
                                         int(precise), stream), self.error)

    def forward(self, x, precise=False):
        import torch
        xd = torch.as_tensor(_f32(x), device="cuda")
        yd = torch.empty((xd.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        self.forward_device(xd, yd, precise, ct.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        return yd.cpu().numpy()

    def loss_grad(self, x, y, precise=True):
        x, y = _f32(x), _f32(y)
        g = np.empty(self.param_count, dtype=np.float32)
        L = ct.c_double()
        _check(self._lib.hom_mlp_loss_grad(self._h, _fptr(x), _fptr(y), x.shape[0], int(precise), ct.byref(L),
                                           _fptr(g)), self.error)
        return L.value, g


def mlp_ensemble_infer(nets, x_dev, threshold, floor_scale):
    """Ensemble inference with acceptance (2 .. 16 networks) on device tensors;
    returns (y, spread, accept) tensors."""
    import torch
    n = x_dev.shape[0]
    y = torch.empty((n, nets[0].n_out), dtype=torch.float32, device=x_dev.device)
    spread = torch.empty(n, dtype=torch.float32, device=x_dev.device)
    acc = torch.empty(n, dtype=torch.uint8, device=x_dev.device)
    handles = (ct.c_void_p * len(nets))(*[net._h.value if isinstance(net._h, ct.c_void_p) else net._h for net in nets])
    lib = library()
    _check(lib.hom_mlp_ensemble_infer(handles, len(nets), ct.c_void_p(x_dev.data_ptr()), ct.c_void_p(y.data_ptr()),
                                     ct.c_void_p(spread.data_ptr()), ct.c_void_p(acc.data_ptr()), n, threshold,
                                     floor_scale, ct.c_void_p(torch.cuda.current_stream().cuda_stream)),
           nets[0].error)
    return y, spread, acc


STATIC_SCRATCH_FLOATS = 8388608   # HOM_STATIC_SCRATCH_FLOATS


def mlp_ensemble_infer_static(nets, x_dev, threshold, floor_scale, y, spread, accept):
    """mlp_ensemble_infer into caller-owned device tensors y [n, n_out] (float32),
    spread [n] (float32), accept [n] (uint8), with the per-network outputs in
    the library's static device array: no device memory is allocated here or
    in the library."""
    import torch
    n = x_dev.shape[0]
    handles = (ct.c_void_p * len(nets))(*[net._h.value if isinstance(net._h, ct.c_void_p) else net._h for net in nets])
    lib = library()
    _check(lib.hom_mlp_ensemble_infer_static(handles, len(nets), ct.c_void_p(x_dev.data_ptr()),
                                             ct.c_void_p(y.data_ptr()), ct.c_void_p(spread.data_ptr()),
                                             ct.c_void_p(accept.data_ptr()), n, threshold, floor_scale,
                                             ct.c_void_p(torch.cuda.current_stream().cuda_stream)),
           nets[0].error)


# ---------------------------------------------------------------------------
# surrogate with FFT fallback
# ---------------------------------------------------------------------------
def surrogate_config(**kw) -> SurrogateConfig:
    c = SurrogateConfig()
    library().hom_surrogate_default_config(ct.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _histories(strain, theta, grad, dt):
    """(count, steps, strain [c, s, 6], theta [c, s], grad [c, s, 3], dt [c, s]) as
    contiguous float64; theta / dt may be given per history [c], grad per
    history [c, 3]."""
    e = _f64(strain)
    count, steps = e.shape[0], e.shape[1]
    t = _f64(np.broadcast_to(np.asarray(theta, dtype=np.float64).reshape(count, -1), (count, steps)))
    g = np.asarray(grad, dtype=np.float64)
    g = _f64(np.broadcast_to(g.reshape(count, 1, 3) if g.ndim == 2 else g, (count, steps, 3)))
    d = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64).reshape(count, -1), (count, steps)))
    return count, steps, e, t, g, d


def surrogate_features(strain, theta, grad, dt, fft, theta_init=293.15):
    """hom_surrogate_features: input rows X [count*steps, 32], targets Y
    [count*steps, 10] and denominators [count*steps] of histories with their
    FFT answers (a RESULT_DTYPE array [count, steps])."""
    count, steps, e, t, g, d = _histories(strain, theta, grad, dt)
    f = np.ascontiguousarray(fft, dtype=RESULT_DTYPE)
    X = np.empty((count * steps, 32), dtype=np.float32)
    Y = np.empty((count * steps, 10), dtype=np.float32)
    den = np.empty(count * steps)
    lib = library()
    _check(lib.hom_surrogate_features(count, steps, _dptr(e), _dptr(t), _dptr(g), _dptr(d),
                                      f.ctypes.data_as(ct.c_void_p), float(theta_init), _fptr(X), _fptr(Y),
                                      _dptr(den)), lambda: lib.hom_surrogate_last_error(None).decode())
    return X, Y, den


class Surrogate(_Handle):
    """hom_surrogate_*: the ensemble, its calibrated threshold and the FFT
    solver of one microstructure."""

    def __init__(self, phases, laws, config: SurrogateConfig | None = None, options: Options | None = None,
                 lengths=(1.0, 1.0, 1.0), **cfg_kw):
        lib = library()
        self._lib = lib
        self._phases = np.ascontiguousarray(phases, dtype=np.uint8)
        self._grid = make_grid(self._phases.shape, lengths)
        self._laws = (Law * len(laws))(*[make_law(p) for p in laws])
        self.options = options if options is not None else make_options()
        self.config = config if config is not None else surrogate_config(**cfg_kw)
        h = ct.c_void_p()
        _check(lib.hom_surrogate_create(ct.byref(self._grid), self._phases.ctypes.data_as(ct.c_void_p), self._laws,
                                        len(laws), ct.byref(self.options), ct.byref(self.config), ct.byref(h)),
               lambda: lib.hom_surrogate_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return self._lib.hom_surrogate_last_error(self._h).decode()

    def solve_histories(self, strain, theta, grad, dt):
        """Batched FFT answers [count, steps] (RESULT_DTYPE) and (solve, setup) seconds."""
        count, steps, e, t, g, d = _histories(strain, theta, grad, dt)
        out = np.empty((count, steps), dtype=RESULT_DTYPE)
        sec = np.zeros(2)
        _check(self._lib.hom_surrogate_solve_histories(self._h, count, steps, _dptr(e), _dptr(t), _dptr(g), _dptr(d),
                                                       out.ctypes.data_as(ct.c_void_p), _dptr(sec)), self.error)
        return out, (float(sec[0]), float(sec[1]))

    def train(self, strain, theta, grad, dt, fft=None):
        count, steps, e, t, g, d = _histories(strain, theta, grad, dt)
        f = None if fft is None else np.ascontiguousarray(fft, dtype=RESULT_DTYPE)
        rep = SurrogateReport()
        _check(self._lib.hom_surrogate_train(self._h, count, steps, _dptr(e), _dptr(t), _dptr(g), _dptr(d),
                                             None if f is None else f.ctypes.data_as(ct.c_void_p), ct.byref(rep)),
               self.error)
        return rep.as_dict(self.config.n_nets)

    def calibrate(self, strain, theta, grad, dt, fft, target, quantile=1.0):
        count, steps, e, t, g, d = _histories(strain, theta, grad, dt)
        f = np.ascontiguousarray(fft, dtype=RESULT_DTYPE)
        rep = SurrogateReport()
        _check(self._lib.hom_surrogate_calibrate(self._h, count, steps, _dptr(e), _dptr(t), _dptr(g), _dptr(d),
                                                 f.ctypes.data_as(ct.c_void_p), float(target), float(quantile),
                                                 ct.byref(rep)), self.error)
        return rep.as_dict(self.config.n_nets)

    @property
    def threshold(self):
        return self._lib.hom_surrogate_threshold(self._h)

    @threshold.setter
    def threshold(self, value):
        _check(self._lib.hom_surrogate_set_threshold(self._h, float(value)), self.error)

    def infer(self, x_dev, y=None, accepted=None):
        """Device rows x [n, 32] -> (y [n, 10], accepted [n]) device tensors."""
        import torch
        n = x_dev.shape[0]
        if y is None:
            y = torch.empty((n, 10), dtype=torch.float32, device=x_dev.device)
        if accepted is None:
            accepted = torch.empty(n, dtype=torch.uint8, device=x_dev.device)
        _check(self._lib.hom_surrogate_infer(self._h, ct.c_void_p(x_dev.data_ptr()), ct.c_void_p(y.data_ptr()),
                                             ct.c_void_p(accepted.data_ptr()), n,
                                             ct.c_void_p(torch.cuda.current_stream().cuda_stream)), self.error)
        return y, accepted

    def points(self, n_points):
        return SurrogatePoints(self, n_points)


class SurrogatePoints(_Handle):
    """hom_surrogate_points_*: Gauss points advanced increment by increment,
    with the FFT fallback executed for rejected points."""

    def __init__(self, sur: Surrogate, n_points):
        self._lib = sur._lib
        self._sur = sur            # the point set uses the surrogate: keep it alive
        self.n = int(n_points)
        h = ct.c_void_p()
        _check(self._lib.hom_surrogate_points_create(sur._h, self.n, ct.byref(h)), sur.error)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_surrogate_points_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, strain, theta, grad, dt, check=True):
        """One increment at every point. Returns (RESULT_DTYPE [n], accepted bool
        [n], info dict)."""
        e = _f64(strain).reshape(self.n, 6)
        t = _f64(np.broadcast_to(theta, (self.n,)))
        g = _f64(np.broadcast_to(np.asarray(grad, dtype=np.float64), (self.n, 3)))
        d = _f64(np.broadcast_to(dt, (self.n,)))
        out = np.empty(self.n, dtype=RESULT_DTYPE)
        acc = np.empty(self.n, dtype=np.uint8)
        info = SurrogateStepInfo()
        rc = self._lib.hom_surrogate_points_step(self._h, _dptr(e), _dptr(t), _dptr(g), _dptr(d),
                                                 out.ctypes.data_as(ct.c_void_p), acc.ctypes.data_as(ct.c_void_p),
                                                 ct.byref(info))
        if check:
            _check(rc, lambda: self._lib.hom_surrogate_points_last_error(self._h).decode() or f"status {rc}")
        return out, acc.astype(bool), info.as_dict()


# ---------------------------------------------------------------------------
# direct deep material network
# ---------------------------------------------------------------------------
def dmn_train_opts(**kw) -> DmnTrainOpts:
    o = DmnTrainOpts()
    library().hom_dmn_default_train_opts(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _mats(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 36)
    if n is not None and a.shape[0] != n:
        raise HomError(HOM_E_ARG, "stiffness arrays differ in length")
    return a


class Dmn(_Handle):
    """hom_dmn_*: a direct DMN of depth K (parameters m (2^K - 1, 3), v (2^K,))."""

    def __init__(self, K, seed=0):
        lib = library()
        self._lib = lib
        self.K = int(K)
        h = ct.c_void_p()
        _check(lib.hom_dmn_create(self.K, seed, ct.byref(h)), lambda: lib.hom_dmn_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_dmn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return self._lib.hom_dmn_last_error(self._h).decode()

    def params(self):
        m = np.empty((2 ** self.K - 1, 3))
        v = np.empty(2 ** self.K)
        _check(self._lib.hom_dmn_get_params(self._h, _dptr(m), _dptr(v)), self.error)
        return m, v

    def set_params(self, m, v):
        _check(self._lib.hom_dmn_set_params(self._h, _dptr(_f64(m)), _dptr(_f64(v))), self.error)

    def homogenize(self, C1, C2):
        a = _mats(C1)
        b = _mats(C2, a.shape[0])
        out = np.empty_like(a)
        _check(self._lib.hom_dmn_homogenize(self._h, a.shape[0], _dptr(a), _dptr(b), _dptr(out)), self.error)
        return out.reshape(-1, 6, 6)

    def loss_grad(self, C1, C2, Ceff, **opts):
        a = _mats(C1)
        b = _mats(C2, a.shape[0])
        c = _mats(Ceff, a.shape[0])
        o = dmn_train_opts(**opts)
        J = ct.c_double()
        gm = np.empty((2 ** self.K - 1, 3))
        gv = np.empty(2 ** self.K)
        _check(self._lib.hom_dmn_loss_grad(self._h, a.shape[0], _dptr(a), _dptr(b), _dptr(c), ct.byref(o),
                                           ct.byref(J), _dptr(gm), _dptr(gv)), self.error)
        return J.value, gm, gv

    def train(self, C1, C2, Ceff, epochs, batch=32, seed=0, **opts):
        a = _mats(C1)
        b = _mats(C2, a.shape[0])
        c = _mats(Ceff, a.shape[0])
        o = dmn_train_opts(**opts)
        hist = np.empty(max(int(epochs), 1))
        _check(self._lib.hom_dmn_train(self._h, a.shape[0], _dptr(a), _dptr(b), _dptr(c), int(epochs), int(batch),
                                       seed, ct.byref(o), _dptr(hist)), self.error)
        return hist[:epochs]


class DmnOnline(_Handle):
    """hom_dmn_online_*: a trained DMN at n_points macroscopic points with the
    laws of its two phases."""

    def __init__(self, net: Dmn, law1: dict, law2: dict, n_points, tol=1e-10, maxit=50, predictor=False):
        lib = library()
        self._lib = lib
        self.n = int(n_points)
        self._laws = (Law * 2)(make_law(law1), make_law(law2))
        h = ct.c_void_p()
        _check(lib.hom_dmn_online_create(net._h, self._laws, self.n, float(tol), int(maxit), ct.byref(h)),
               lambda: lib.hom_dmn_online_last_error(None).decode())
        self._h = h
        if predictor:
            self.set_predictor(True)

    def set_predictor(self, on: bool):
        """hom_dmn_online_set_predictor: extrapolated Newton starts."""
        _check(self._lib.hom_dmn_online_set_predictor(self._h, int(bool(on))),
               lambda: self._lib.hom_dmn_online_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hom_dmn_online_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, strains, thetas, dts, what=0, trial=False):
        """One increment at every point (theta, dt scalar or per point). Returns a
        record array of DMN_RESULT_DTYPE, one record per point."""
        e = _f64(strains).reshape(self.n, 6)
        t = _f64(np.broadcast_to(thetas, (self.n,)))
        d = _f64(np.broadcast_to(dts, (self.n,)))
        out = np.empty(self.n, dtype=DMN_RESULT_DTYPE)
        _check(self._lib.hom_dmn_online_step(self._h, _dptr(e), _dptr(t), _dptr(d), int(what), int(bool(trial)),
                                             out.ctypes.data_as(ct.POINTER(DmnResult))),
               lambda: self._lib.hom_dmn_online_last_error(self._h).decode())
        return out
