"""ctypes binding of libdnb.so (argument marshalling only).

Every computation runs in the library's HIP kernels on the GPU; this module
checks tensor shapes, dtypes and devices, passes raw device pointers and the
current torch stream, and turns a non-zero status into an exception.  If the
library is not built, importing raises: there is no fallback path.
"""
import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdnb.so")

DNB_OK, DNB_ERR_ARG, DNB_ERR_HIP, DNB_ERR_NOMEM, DNB_ERR_STATE = 0, -1, -2, -3, -4
DNB_FP64, DNB_FP32C = 0, 1
PRECISIONS = {"fp64": DNB_FP64, "fp32c": DNB_FP32C}


class DnbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libdnb status {status}: {msg}")
        self.status = status


class dnb_pot(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("G", "eps", "m_nfw", "rs_nfw", "m_mn", "a_mn", "b_mn")]


class dnb_track_model(ctypes.Structure):
    _fields_ = [("w_now", ctypes.c_double * 6), ("G", ctypes.c_double),
                ("dt_total", ctypes.c_double), ("n_steps", ctypes.c_int64),
                ("sigma", ctypes.c_double * 3)]


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2511_22468_amd.build`")
    lib = ctypes.CDLL(path)
    P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    POT = ctypes.POINTER(dnb_pot)
    TM = ctypes.POINTER(dnb_track_model)
    sig = {
        "dnb_create": ([ctypes.POINTER(P), I64, I], I),
        "dnb_destroy": ([P], None),
        "dnb_last_error": ([], ctypes.c_char_p),
        "dnb_version": ([], ctypes.c_char_p),
        "dnb_accelerations": ([P, I64, P, P, POT, I, P, P], I),
        "dnb_accelerations_rows": ([P, I64, P, P, POT, I, I64, I64, P, P], I),
        "dnb_accelerations_noalloc": ([I64, P, P, POT, I, I, P, P], I),
        "dnb_accelerations_vjp": ([P, I64, P, P, POT, I, P, I64, I64, P, P, P], I),
        "dnb_step": ([P, I64, P, P, P, POT, D, P], I),
        "dnb_tape_doubles": ([I64, I64, I64], I64),
        "dnb_vjp_workspace_doubles": ([I64, I64], I64),
        "dnb_simulate": ([P, I64, P, P, P, POT, D, I64, I64, P, P], I),
        "dnb_check_state": ([P, I64, P, P, P, ctypes.POINTER(I64), P], I),
        "dnb_set_checks": ([P, I], I),
        "dnb_simulate_resume": ([P, I64, P, I64, I64, I64, P, P, P, POT, D, I64, I64, P, P], I),
        "dnb_simulate_vjp": ([P, I64, P, POT, D, I64, I64, P, P, P, P, P, P, P, P, P, P], I),
        "dnb_vjp_reversed_workspace_doubles": ([I64], I64),
        "dnb_simulate_vjp_reversed": ([P, I64, P, POT, D, I64, I64, P, P, P, P, P, P, P, P, P,
                                       P, P], I),
        "dnb_mmd": ([P, I64, P, I64, P, D, P, P, P], I),
        "dnb_energy": ([P, I64, P, P, P, POT, P, P], I),
        "dnb_orbit": ([P, P, POT, D, I64, P, P, P], I),
        "dnb_orbit_vjp": ([P, P, POT, D, I64, P, P, P, P], I),
        "dnb_place_plummer": ([P, I64, P, P, P, D, D, D, P, P, P, P], I),
        "dnb_place_plummer_vjp": ([P, I64, P, D, D, D, P, P, P, P, P, P], I),
        "dnb_simulate_batch": ([P, I64, I64, P, P, P, ctypes.POINTER(ctypes.c_double), I64, P, P],
                               I),
        "dnb_batch_tape_doubles": ([I64, I64, I64], I64),
        "dnb_simulate_batch_vjp": ([P, I64, I64, P, ctypes.POINTER(ctypes.c_double), I64, P, P, P,
                                    P, P, P, P, P, P], I),
        "dnb_batch_capacity": ([P, I64], I64),
        "dnb_place_plummer_batch": ([P, I64, I64, P, P, P, P, D, D, P, P, P, P], I),
        "dnb_mmd_batch": ([P, I64, I64, P, I64, P, ctypes.c_int, D, P, P, P], I),
        "dnb_mmd_batch_targets": ([P, I64, I64, P, I64, I64, P, D, P, P], I),
        "dnb_orbit_batch": ([P, I64, P, ctypes.POINTER(ctypes.c_double), I64, P, P, P], I),
        "dnb_orbit_batch_vjp": ([P, I64, P, ctypes.POINTER(ctypes.c_double), I64, P, P, P, P], I),
        "dnb_place_plummer_batch_vjp": ([P, I64, I64, P, P, D, D, P, P, P, P, P], I),
        "dnb_profile": ([P, I], I),
        "dnb_profile_read": ([P, ctypes.POINTER(ctypes.c_double)], I),
        # learned surrogate (include/dnb_surrogate.h)
        "dnb_mlp_param_count": ([], I64),
        "dnb_mlp_workspace_bytes": ([I64], I64),
        "dnb_mlp_to_bf16": ([I64, P, P, P], I),
        "dnb_mlp_forward": ([P, P, I64, P, P, P, P], I),
        "dnb_mlp_backward": ([P, I64, P, P, P, P, P], I),
        "dnb_mlp_mse": ([I64, P, P, P, P, P], I),
        "dnb_mlp_adam": ([I64, P, P, P, P, P, D, D, D, D, I64, P], I),
        "dnb_mlp_invert_workspace_bytes": ([I64], I64),
        "dnb_mlp_invert": ([P, P, I64, P, P, I64, D, P, P], I),
        "dnb_grid_workspace_bytes": ([], I64),
        # orbit fit (include/dnb_orbitfit.h)
        "dnb_track_observe": ([P, TM, I64, P, P, P, P], I),
        "dnb_track_chi2": ([P, TM, I64, P, I64, P, P, P, P, P], I),
        "dnb_track_hessian": ([P, TM, I64, P, I64, P, P, P, P], I),
        "dnb_track_lm": ([P, TM, I64, P, I64, P, I64, D, P, P], I),
        "dnb_density_grid": ([I64, P, ctypes.POINTER(ctypes.c_double), P, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def check(status):
    if status != DNB_OK:
        raise DnbError(status, lib().dnb_last_error().decode())


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
