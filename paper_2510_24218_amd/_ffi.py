"""ctypes mirror of include/pws.h and the loader of the in-tree libpws.so."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpws.so")

PWS_OK, PWS_ERR_ARG, PWS_ERR_UNSUPPORTED, PWS_ERR_NOMEM, PWS_ERR_PLAN, PWS_ERR_DEVICE, PWS_ERR_NUMERIC = range(7)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_UNSUPPORTED", "ERR_NOMEM", "ERR_PLAN", "ERR_DEVICE", "ERR_NUMERIC"]
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
PWS_PLAN_HOST_ONLY, PWS_PLAN_DENSE = 1, 2
GATE_KIND = {"H": 0, "X": 1, "RX": 2, "RZ": 3, "RZZ": 4, "CNOT": 5, "CZ": 6, "U1": 7, "U2": 8,
             "CRX": 9, "FSIM": 10}
NOISE_KIND = {"DEPOL1": 0, "DEPOL2": 1, "AMPDAMP": 2, "PHASEDAMP": 3, "PAULI1": 4}


class pws_gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32), ("param", C.c_int32),
                ("coeff", C.c_double), ("offset", C.c_double),
                ("param2", C.c_int32), ("_pad", C.c_int32),
                ("coeff2", C.c_double), ("offset2", C.c_double),
                ("matrix", C.POINTER(C.c_double))]


class pws_circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_gates", C.c_int32), ("n_params", C.c_int32),
                ("_pad", C.c_int32), ("gates", C.POINTER(pws_gate)), ("theta", C.POINTER(C.c_double))]


class pws_noise_site(C.Structure):
    _fields_ = [("after_gate", C.c_int32), ("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("p", C.c_double * 3)]


class pws_noise(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("_pad", C.c_int32), ("sites", C.POINTER(pws_noise_site)),
                ("readout", C.POINTER(C.c_double))]


class pws_tree(C.Structure):
    _fields_ = [("n_pairs", C.c_int32), ("_pad", C.c_int32), ("ssa_pairs", C.POINTER(C.c_int32))]


class pws_option(C.Structure):
    _fields_ = [("key", C.c_int32), ("value", C.c_int32)]


class pws_slices(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("n_sliced", C.c_int32), ("flags", C.c_int32),
                ("sliced_edges", C.POINTER(C.c_int32)), ("max_chains", C.c_int64),
                ("precision", C.c_int32), ("planner", C.c_int32),
                ("n_options", C.c_int32), ("_pad", C.c_int32), ("options", C.POINTER(pws_option))]


# plan option keys (PWS_OPT_*), by name
OPTIONS = {"grid": 1, "sweep_width": 2, "graph": 3, "lds_block": 4, "lds_bytes": 5, "waves_per_cu": 6,
           "coop4_width": 7, "coop8_width": 8, "range_width": 9, "cpw8": 10, "cpw10": 11, "window": 12,
           "fuse": 13, "keep": 14, "fresh": 15, "merge": 16, "lds_form": 17, "dense_range": 18,
           "dense_cpw2_width": 19}
# the environment variables the Python binding reads as option defaults
ENV_OPTIONS = {"PWS_GRID": "grid", "PWS_SWEEP": "sweep_width", "PWS_GRAPH": "graph", "PWS_BLOCK": "lds_block",
               "PWS_LDS_BYTES": "lds_bytes", "PWS_SWEEP_WPC": "waves_per_cu", "PWS_SWEEP_COOP": "coop4_width",
               "PWS_SWEEP_COOP8": "coop8_width", "PWS_SWEEP_RANGE": "range_width", "PWS_SWEEP_CPW8": "cpw8",
               "PWS_SWEEP_CPW10": "cpw10", "PWS_SWEEP_MTCAP": "window", "PWS_SWEEP_FUSE": "fuse",
               "PWS_SWEEP_CACHE": "keep", "PWS_FRESH": "fresh", "PWS_SWEEP_MERGE": "merge",
               "PWS_DENSE_RANGE": "dense_range", "PWS_DENSE_CPW2": "dense_cpw2_width"}


class pws_bits(C.Structure):
    _fields_ = [("n", C.c_int64), ("words", C.c_int32), ("on_device", C.c_int32),
                ("data", C.POINTER(C.c_uint64))]


EXPORTED = [
    "pws_plan", "pws_amplitudes", "pws_sample", "pws_grad", "pws_set_stream", "pws_workspace_bytes",
    "pws_bind_workspace", "pws_plan_stats", "pws_step_count", "pws_step_info", "pws_step_amplitudes",
    "pws_sample_trace", "pws_last_timing", "pws_plan_export", "pws_last_error", "pws_destroy",
    "pws_autotune", "pws_set_theta", "pws_plan_sweep_stats", "pws_sample_batch",
    "pws_sample_noalloc", "pws_sample_probe",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpws.so; raises loudly when the HIP engine has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP engine not built: {path} is missing (run paper_2510_24218_amd/build.py)")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.pws_plan.argtypes = [C.POINTER(pws_circuit), C.POINTER(pws_noise), C.POINTER(pws_tree),
                             C.POINTER(pws_slices), C.POINTER(P)]
    lib.pws_amplitudes.argtypes = [P, C.POINTER(pws_bits), C.c_void_p, C.c_void_p]
    lib.pws_sample.argtypes = [P, C.c_int64, C.c_uint64, C.POINTER(pws_bits)]
    lib.pws_sample_probe.argtypes = [P, C.c_int64, C.c_uint64, C.c_int32, C.POINTER(pws_bits), C.c_void_p,
                                     C.c_void_p]
    lib.pws_sample_noalloc.argtypes = [P, C.c_int64, C.c_uint64, C.POINTER(pws_bits)]
    lib.pws_sample_batch.argtypes = [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_uint64), C.POINTER(pws_bits)]
    lib.pws_grad.argtypes = [P, C.POINTER(pws_bits), C.c_void_p]
    lib.pws_set_stream.argtypes = [P, C.c_void_p]
    lib.pws_workspace_bytes.argtypes = [P, C.c_int64, C.POINTER(C.c_uint64)]
    lib.pws_bind_workspace.argtypes = [P, C.c_void_p, C.c_uint64]
    lib.pws_plan_stats.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    lib.pws_step_count.argtypes = [P, C.POINTER(C.c_int32)]
    lib.pws_step_info.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
    lib.pws_step_amplitudes.argtypes = [P, C.c_int32, C.POINTER(pws_bits), C.c_void_p, C.c_void_p]
    lib.pws_sample_trace.argtypes = [P, C.c_int64, C.c_uint64, C.POINTER(pws_bits), C.c_void_p]
    lib.pws_last_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.pws_autotune.argtypes = [P, C.c_int64, C.c_uint64, C.c_char_p, C.c_char_p, C.c_int64]
    lib.pws_set_theta.argtypes = [P, C.POINTER(C.c_double), C.c_int32]
    lib.pws_plan_sweep_stats.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.pws_plan_export.argtypes = [P, C.c_int32, C.c_char_p, C.POINTER(C.c_int64)]
    lib.pws_last_error.restype = C.c_char_p
    lib.pws_last_error.argtypes = []
    lib.pws_destroy.argtypes = [P]
    lib.pws_destroy.restype = None
    for name in EXPORTED:
        if name not in ("pws_last_error", "pws_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
