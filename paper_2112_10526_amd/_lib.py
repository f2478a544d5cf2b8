"""ctypes declarations of the libnqs C ABI (include/nqs.h).  Argument
marshalling only: every step of the method runs in the library's kernels."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnqs.so")

NQS_OK, NQS_EINVAL, NQS_ENOMEM, NQS_EDEVICE, NQS_ENUMERIC, NQS_ENOTCONV, NQS_ESTATE = range(7)
STATUS_NAMES = {0: "NQS_OK", 1: "NQS_EINVAL", 2: "NQS_ENOMEM", 3: "NQS_EDEVICE",
                4: "NQS_ENUMERIC", 5: "NQS_ENOTCONV", 6: "NQS_ESTATE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "c128": 3}
RK_SCHEMES = {"euler": 0, "heun": 1}
DENSE_SOLVERS = {"cg": 0, "cholesky": 1}
PROBES = {"fp32_fma": 0, "fp64_fma": 1, "fp32_exp": 2, "fp64_mfma": 3, "bf16_mfma": 4}
RULES = {"local": 0, "exchange": 1}
QGTS = {"onthefly": 0, "jacobian_dense": 1}

# every exported entry point of include/nqs.h
EXPORTS = [
    "nqs_create", "nqs_destroy", "nqs_last_error", "nqs_set_stream", "nqs_set_tfim",
    "nqs_set_heisenberg", "nqs_set_rbm", "nqs_set_rbm_symm", "nqs_set_dense_solver",
    "nqs_probe_rate",
    "nqs_num_params", "nqs_set_sampler", "nqs_set_qgt",
    "nqs_workspace_bytes", "nqs_bind_workspace", "nqs_set_params", "nqs_get_params",
    "nqs_reset_chains", "nqs_get_chains", "nqs_set_chains", "nqs_proposal_count",
    "nqs_get_state", "nqs_set_state", "nqs_sample", "nqs_thermalize", "nqs_load_samples", "nqs_local_energy",
    "nqs_local_energy_noalloc",
    "nqs_log_psi", "nqs_log_psi_vjp", "nqs_jacobian", "nqs_expect_and_grad", "nqs_sr_update",
    "nqs_vmc_step", "nqs_tdvp_step", "nqs_batch_step", "nqs_step_begin", "nqs_step_poll",
    "nqs_profile_enable", "nqs_profile_read",
    "nqs_profile_class_name", "nqs_set_cg_graphs", "nqs_set_cg_grouping",
]
PROF_CLASSES = ["sample", "theta", "eloc", "stats", "qgt_w", "outer", "reduce", "cg_vec",
                "jacobian", "gram", "dense_matvec", "update", "prepare"]


class NqsStats(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_double), ("variance", ctypes.c_double),
                ("error", ctypes.c_double), ("acceptance", ctypes.c_double)]


class NqsSrInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double)]


class NqsStepCfg(ctypes.Structure):
    _fields_ = [("qgt", ctypes.c_int), ("diag_shift", ctypes.c_double), ("lr", ctypes.c_double),
                ("cg_tol", ctypes.c_double), ("cg_maxiter", ctypes.c_int)]


class NqsStepReport(ctypes.Structure):
    _fields_ = [("energy", NqsStats), ("sr", NqsSrInfo), ("status", ctypes.c_int)]


class NqsTdvpCfg(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("dt", ctypes.c_double), ("gamma_re", ctypes.c_double),
                ("gamma_im", ctypes.c_double), ("diag_shift", ctypes.c_double),
                ("cg_tol", ctypes.c_double), ("cg_maxiter", ctypes.c_int)]


class NqsTdvpReport(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int), ("energy", NqsStats * 2),
                ("energy_im", ctypes.c_double * 2), ("solve", NqsSrInfo * 2),
                ("status", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libnqs and declare its signatures; raises if the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnqs is not built ({path} missing); run "
                           "`python -m paper_2112_10526_amd.build`")
    L = ctypes.CDLL(path)
    V, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    I64, U64, SZ = ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "nqs_create": (I, [ctypes.POINTER(V), I, V]),
        "nqs_destroy": (None, [V]),
        "nqs_last_error": (ctypes.c_char_p, [V]),
        "nqs_set_stream": (I, [V, V]),
        "nqs_set_tfim": (I, [V, I, I, V, D, D]),
        "nqs_set_heisenberg": (I, [V, I, I, V, D, V]),
        "nqs_set_rbm": (I, [V, I, I, I, I]),
        "nqs_set_rbm_symm": (I, [V, I, V, I, I, I, I]),
        "nqs_set_dense_solver": (I, [V, I]),
        "nqs_probe_rate": (I, [V, I, ctypes.POINTER(ctypes.c_double)]),
        "nqs_num_params": (SZ, [V]),
        "nqs_set_sampler": (I, [V, I, I, I, I, U64, I]),
        "nqs_set_qgt": (I, [V, I]),
        "nqs_workspace_bytes": (SZ, [V]),
        "nqs_bind_workspace": (I, [V, V, SZ]),
        "nqs_set_params": (I, [V, V, I]),
        "nqs_get_params": (I, [V, V, I]),
        "nqs_reset_chains": (I, [V]),
        "nqs_get_chains": (I, [V, V, I]),
        "nqs_set_chains": (I, [V, V, I]),
        "nqs_proposal_count": (U64, [V]),
        "nqs_get_state": (I, [V, V, ctypes.POINTER(SZ)]),
        "nqs_set_state": (I, [V, V, SZ]),
        "nqs_sample": (I, [V, I, V, V, ctypes.POINTER(D)]),
        "nqs_thermalize": (I, [V, I]),
        "nqs_load_samples": (I, [V, V, I64]),
        "nqs_local_energy": (I, [V, V, I64, V]),
        "nqs_local_energy_noalloc": (I, [V, V, I64, V]),
        "nqs_log_psi": (I, [V, V, I64, V]),
        "nqs_log_psi_vjp": (I, [V, V, I64, V, V]),
        "nqs_jacobian": (I, [V, V, I64, V, I]),
        "nqs_expect_and_grad": (I, [V, ctypes.POINTER(NqsStats), V]),
        "nqs_sr_update": (I, [V, I, D, D, D, I, V, ctypes.POINTER(NqsSrInfo)]),
        "nqs_vmc_step": (I, [V, ctypes.POINTER(NqsStepCfg), ctypes.POINTER(NqsStepReport)]),
        "nqs_tdvp_step": (I, [V, ctypes.POINTER(NqsTdvpCfg), ctypes.POINTER(NqsTdvpReport)]),
        "nqs_batch_step": (I, [ctypes.POINTER(V), I, ctypes.POINTER(NqsStepCfg),
                               ctypes.POINTER(NqsStepReport)]),
        "nqs_step_begin": (I, [V, ctypes.POINTER(NqsStepCfg)]),
        "nqs_step_poll": (I, [ctypes.POINTER(V), I, I, ctypes.POINTER(NqsStepReport),
                              ctypes.POINTER(ctypes.c_int32)]),
        "nqs_profile_enable": (I, [V, ctypes.c_uint32]),
        "nqs_profile_read": (I, [V, V, V, I]),
        "nqs_profile_class_name": (ctypes.c_char_p, [I]),
        "nqs_set_cg_graphs": (I, [V, I]),
        "nqs_set_cg_grouping": (I, [V, I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class NqsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
