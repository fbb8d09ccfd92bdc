"""ctypes binding of libgreen_gw.so (argument marshalling only).

Every step of the GW path runs in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw pointers and the current HIP stream,
and turns status codes into exceptions.  PyTorch provides device memory and
streams.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgreen_gw.so")

GREEN_OK = 0
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
STATUS = {0: "GREEN_OK", -1: "GREEN_EINVAL", -2: "GREEN_ENOMEM", -3: "GREEN_EHIP", -4: "GREEN_ESINGULAR",
          -5: "GREEN_ENOCONV", -6: "GREEN_ENAN", -7: "GREEN_EUNSUPPORTED"}


class GreenError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_strerror(code)})")


class Dims(ctypes.Structure):
    _fields_ = [("kmesh", ctypes.c_int32 * 3), ("nao", ctypes.c_int32), ("naux", ctypes.c_int32),
                ("ntau", ctypes.c_int32), ("nw_f", ctypes.c_int32), ("nw_b", ctypes.c_int32),
                ("nspin", ctypes.c_int32), ("beta", ctypes.c_double)]


class GridC(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_void_p), ("wf", ctypes.c_void_p), ("wb", ctypes.c_void_p),
                ("TF_t2w", ctypes.c_void_p), ("TF_w2t", ctypes.c_void_p), ("TB_t2w", ctypes.c_void_p),
                ("TB_w2t", ctypes.c_void_p)]


class Report(ctypes.Structure):
    _fields_ = [("e_1b", ctypes.c_double), ("e_hf", ctypes.c_double), ("e_corr", ctypes.c_double),
                ("e_tot", ctypes.c_double), ("n_elec", ctypes.c_double), ("mu", ctypes.c_double),
                ("max_dsigma", ctypes.c_double), ("herm_err", ctypes.c_double), ("mu_evals", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("ms", ctypes.c_float * 8), ("kern_ms", ctypes.c_double * 2),
                ("kern_flops", ctypes.c_double * 2), ("kern_launches", ctypes.c_int32 * 2)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("ms", "pad", "kern_ms", "kern_flops",
                                                                         "kern_launches")}
        d["ms"] = list(self.ms)
        d["kern_ms"] = list(self.kern_ms)
        d["kern_flops"] = list(self.kern_flops)
        d["kern_launches"] = list(self.kern_launches)
        return d


class System(ctypes.Structure):
    _fields_ = [("V", ctypes.c_void_p), ("H0", ctypes.c_void_p), ("S", ctypes.c_void_p), ("G", ctypes.c_void_p),
                ("Sinf", ctypes.c_void_p), ("Sigma", ctypes.c_void_p), ("mu", ctypes.c_double),
                ("n_target", ctypes.c_double), ("ws", ctypes.c_void_p)]


class Diis(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("start", ctypes.c_int32), ("count", ctypes.c_int32),
                ("next", ctypes.c_int32), ("iter", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("B", (ctypes.c_double * 16) * 16), ("coef", ctypes.c_double * 16)]


OPT_TUNE = 1
OPT_GRAPH = 2
OPT_P0_TILE = 3
OPT_STAGE1_TILE = 4
OPT_SIGMA_FUSED = 5
OPT_GF2 = 6
OPT_TIME_REVERSAL = 7
OPT_V_HALF = 8
OPT_SIGMA_TILE = 9

EXPORTS = ["green_plan_create", "green_plan_destroy", "green_workspace_bytes", "green_gw_polarization",
           "green_gw_screen", "green_gw_selfenergy", "green_hf_static", "green_dyson", "green_gw_iterate",
           "green_plan_set_option", "green_plan_tuning_report", "green_batch_workspace_bytes",
           "green_gw_iterate_batched", "green_batch_create", "green_batch_iterate", "green_batch_destroy",
           "green_diis_history_bytes", "green_gw_iterate_diis", "green_kpath_interpolate",
           "green_gf2_selfenergy", "green_dyson_noalloc", "green_check_status", "green_plan_set_kpoint_symmetry",
           "green_build_info", "green_strerror"]

NOALLOC_MAX_BYTES = 64 << 20  # GREEN_NOALLOC_MAX_BYTES
MAX_KPOINT_OPS = 192  # GREEN_MAX_KPOINT_OPS


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2406_18479_amd.build` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.green_plan_create.argtypes = [ctypes.POINTER(Dims), ctypes.POINTER(GridC), i32, ctypes.c_size_t,
                                      ctypes.POINTER(vp)]
    lib.green_plan_create.restype = i32
    lib.green_plan_destroy.argtypes = [vp]
    lib.green_plan_destroy.restype = None
    lib.green_workspace_bytes.argtypes = [vp]
    lib.green_workspace_bytes.restype = ctypes.c_size_t
    lib.green_gw_polarization.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.green_gw_polarization.restype = i32
    lib.green_gw_screen.argtypes = [vp, vp, vp, vp, vp]
    lib.green_gw_screen.restype = i32
    lib.green_gw_selfenergy.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.green_gw_selfenergy.restype = i32
    lib.green_gf2_selfenergy.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.green_gf2_selfenergy.restype = i32
    lib.green_hf_static.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.green_hf_static.restype = i32
    lib.green_dyson.argtypes = [vp, vp, vp, vp, vp, dbl, ctypes.POINTER(dbl), vp, ctypes.POINTER(dbl),
                                ctypes.POINTER(ctypes.c_int32), vp, vp]
    lib.green_dyson.restype = i32
    lib.green_dyson_noalloc.argtypes = [vp, vp, vp, vp, vp, dbl, ctypes.POINTER(dbl), vp, ctypes.POINTER(dbl),
                                        ctypes.POINTER(ctypes.c_int32), vp]
    lib.green_dyson_noalloc.restype = i32
    lib.green_check_status.argtypes = [vp, vp, vp]
    lib.green_check_status.restype = i32
    lib.green_kpath_interpolate.argtypes = [vp, ctypes.POINTER(dbl), i32, vp, vp, vp, vp, vp, vp]
    lib.green_kpath_interpolate.restype = i32
    lib.green_gw_iterate.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), dbl, dbl,
                                     ctypes.POINTER(Report), vp, vp]
    lib.green_gw_iterate.restype = i32
    lib.green_plan_set_option.argtypes = [vp, i32, i32]
    lib.green_plan_set_option.restype = i32
    lib.green_plan_set_kpoint_symmetry.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), i32,
                                                   ctypes.POINTER(ctypes.c_int32)]
    lib.green_plan_set_kpoint_symmetry.restype = i32
    lib.green_plan_tuning_report.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.green_plan_tuning_report.restype = i32
    lib.green_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(vp)]
    lib.green_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.green_gw_iterate_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(System), dbl,
                                             ctypes.POINTER(Report), vp, ctypes.c_size_t, vp]
    lib.green_gw_iterate_batched.restype = i32
    lib.green_batch_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(System), dbl, i32, vp,
                                       ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.green_batch_create.restype = i32
    lib.green_batch_iterate.argtypes = [vp, ctypes.POINTER(System), ctypes.POINTER(Report), vp]
    lib.green_batch_iterate.restype = i32
    lib.green_batch_destroy.argtypes = [vp]
    lib.green_batch_destroy.restype = None
    lib.green_diis_history_bytes.argtypes = [vp, i32]
    lib.green_diis_history_bytes.restype = ctypes.c_size_t
    lib.green_gw_iterate_diis.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), dbl, dbl,
                                          ctypes.POINTER(Diis), vp, ctypes.c_size_t, ctypes.POINTER(Report), vp, vp]
    lib.green_gw_iterate_diis.restype = i32
    lib.green_strerror.argtypes = [i32]
    lib.green_strerror.restype = ctypes.c_char_p
    lib.green_build_info.argtypes = []
    lib.green_build_info.restype = ctypes.c_char_p
    return lib


LIB = _load()
BUILD_INFO = LIB.green_build_info().decode()


def _check_provenance() -> None:
    """The library must have been built from the sources beside it (a stale build would run other kernels)."""
    from .build import source_digest
    want = source_digest()
    got = dict(kv.split("=", 1) for kv in BUILD_INFO.split()).get("sources")
    if got != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (library {got}, sources {want}); rebuild with "
                          "`python -m paper_2406_18479_amd.build`")


_check_provenance()


def _strerror(code: int) -> str:
    return LIB.green_strerror(code).decode()


def check(code: int, where: str) -> None:
    if code != GREEN_OK:
        raise GreenError(code, where)
