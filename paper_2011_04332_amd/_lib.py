"""ctypes binding of libnpfem.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/npfem.h; all
numerical work happens in the HIP library. Loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpfem.so")

NPFEM_OK = 0
ERR_INVALID_ARG = -1
ERR_MESH_OPEN = -2
ERR_MESH_NONMANIFOLD = -3
ERR_DEGENERATE_TRI = -4
ERR_NOT_SPD = -5
ERR_NONFINITE = -6
ERR_HIP = -7
ERR_OOM = -8

FP64, FP32, BF16_REFINE, FP16_REFINE = 0, 1, 2, 3

OPT_ENERGY = 1
OPT_NO_GRAPH = 2
OPT_AUTOTUNE = 4
OPT_SYNC_CHECK = 8
OPT_KERNEL_TIMING = 16

KERNEL_KINDS = ("predict", "local", "global", "residual", "update")

EXPORTED = [
    "npfem_create_mesh",
    "npfem_mesh_info",
    "npfem_mesh_system_matrix",
    "npfem_create_batch",
    "npfem_step",
    "npfem_run",
    "npfem_set_weights",
    "npfem_set_damping",
    "npfem_set_contacts",
    "npfem_set_quasi_newton",
    "npfem_ibm_interpolate",
    "npfem_ibm_spread",
    "npfem_rollout",
    "npfem_rollout_adjoint",
    "npfem_sync_status",
    "npfem_get_energy",
    "npfem_get_volume",
    "npfem_get_volume_noalloc",
    "npfem_batch_config",
    "npfem_set_batch_config",
    "npfem_kernel_times",
    "npfem_free",
    "npfem_last_error",
]


class Material(ctypes.Structure):
    _fields_ = [
        ("w_stretch", ctypes.c_double),
        ("w_area", ctypes.c_double),
        ("w_bend", ctypes.c_double),
        ("w_volume", ctypes.c_double),
        ("vertex_mass", ctypes.c_double),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("n_refine", ctypes.c_int32),
        ("max_vol_iter", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
    ]


class NpfemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"npfem error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2011_04332_amd.build`"
        )
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.npfem_create_mesh.argtypes = [P, I32, P, I32, ctypes.POINTER(Material), ctypes.POINTER(P)]
    lib.npfem_mesh_info.argtypes = [P, P, P, P, P]
    lib.npfem_mesh_system_matrix.argtypes = [P, P, D, P]
    lib.npfem_create_batch.argtypes = [P, I32, P, I32, P, P, P, ctypes.POINTER(Options),
                                       ctypes.POINTER(P)]
    lib.npfem_step.argtypes = [P, P, D, I32]
    lib.npfem_run.argtypes = [P, P, D, I32, I32]
    lib.npfem_set_weights.argtypes = [P, P]
    lib.npfem_set_damping.argtypes = [P, I32, D, D]
    lib.npfem_set_contacts.argtypes = [P, D, P, P, P, ctypes.c_int64]
    lib.npfem_set_quasi_newton.argtypes = [P, I32, I32]
    lib.npfem_ibm_interpolate.argtypes = [P, P, P, P, D, P, P]
    lib.npfem_ibm_spread.argtypes = [P, P, P, P, D, P, P]
    lib.npfem_rollout.argtypes = [P, P, D, I32, I32, I32]
    lib.npfem_rollout_adjoint.argtypes = [P, P, P, P, P, P, P]
    lib.npfem_sync_status.argtypes = [P]
    lib.npfem_get_energy.argtypes = [P, P, I32, P]
    lib.npfem_get_volume.argtypes = [P, P]
    lib.npfem_get_volume_noalloc.argtypes = [P, P]
    lib.npfem_kernel_times.argtypes = [P, P, P, I32]
    lib.npfem_batch_config.argtypes = [P, I32, P]
    lib.npfem_set_batch_config.argtypes = [P, I32, P]
    lib.npfem_free.argtypes = [P]
    lib.npfem_last_error.argtypes = []
    lib.npfem_last_error.restype = ctypes.c_char_p
    for name in EXPORTED[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != NPFEM_OK:
        msg = load().npfem_last_error().decode(errors="replace")
        raise NpfemError(rc, msg)
