"""ctypes declarations of the C ABI in include/gp.h (argument marshalling only).

The shared library ``libgp_mi355x.so`` is built in-tree by
``paper_2003_03590_amd.build``.  There is no fallback: importing this module
without the library raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgp_mi355x.so")

GP_OK, GP_ERR_ARG, GP_ERR_UNSUPPORTED, GP_ERR_HIP, GP_ERR_NOMEM, GP_ERR_NONFINITE, GP_ERR_STATE = range(7)
GP_C128, GP_C64 = 0, 1
STATUS_NAMES = {0: "GP_OK", 1: "GP_ERR_ARG", 2: "GP_ERR_UNSUPPORTED", 3: "GP_ERR_HIP", 4: "GP_ERR_NOMEM",
                5: "GP_ERR_NONFINITE", 6: "GP_ERR_STATE"}


class gp_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("alpha", C.c_double), ("beta", C.c_double), ("dt", C.c_double),
                ("prec", C.c_int32), ("flags", C.c_uint32)]


class gp_energy(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gp_argle_report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("crit_sup", C.c_double), ("crit_energy", C.c_double), ("e_v", C.c_double),
                ("converged", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
ST = C.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "gp_plan": (ST, [C.POINTER(gp_desc), P, C.POINTER(P)]),
    "gp_plan_batch": (ST, [C.POINTER(gp_desc), C.c_int32, P, C.POINTER(P)]),
    "gp_plan_destroy": (ST, [P]),
    "gp_state_bytes": (C.c_size_t, [P, C.c_int32]),
    "gp_work_bytes": (C.c_size_t, [P]),
    "gp_nshell": (C.c_int32, [P]),
    "gp_init_phase": (ST, [P, P, P]),
    "gp_init_rvr": (ST, [P, C.POINTER(C.c_double), C.c_int32, C.c_double, P]),
    "gp_substep_linear": (ST, [P, P, C.c_int32, C.c_double]),
    "gp_substep_nonlinear": (ST, [P, P, C.c_double]),
    "gp_step_n": (ST, [P, P, C.c_int64]),
    "gp_step_literal_n": (ST, [P, P, C.c_int64]),
    "gp_fft3": (ST, [P, P, P, C.c_int32]),
    "gp_copy_state": (ST, [P, P, P]),
    "gp_energies": (ST, [P, P, P, C.POINTER(gp_energy)]),
    "gp_energies_static": (ST, [P, P, C.POINTER(gp_energy)]),
    "gp_spectra": (ST, [P, P, P, C.POINTER(C.c_double), C.c_int32, C.POINTER(gp_energy)]),
    "gp_structure_fn": (ST, [P, P, P, C.c_int32, C.POINTER(C.c_double)]),
    "gp_loss_ekin_i_shells": (ST, [P, P, P, C.c_int32, C.c_int32, C.POINTER(C.c_double), P]),
    "gp_adjoint_step_n": (ST, [P, P, P, C.c_int64, P]),
    "gp_phase_grad": (ST, [P, P, P, P]),
    "gp_argle_step": (ST, [P, P, P, C.c_double, C.c_int64, P]),
    "gp_argle_energy": (ST, [P, P, P, P, C.POINTER(C.c_double)]),
    "gp_structure_fn_velocity": (ST, [P, P, P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gp_mach": (ST, [P, P, P, C.POINTER(C.c_double)]),
    "gp_helicity_work_bytes": (C.c_size_t, [P]),
    "gp_helicity": (ST, [P, P, P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32]),
    "gp_argle_run": (ST, [P, P, P, C.c_double, C.c_int64, C.c_int64, C.c_double, P, C.POINTER(gp_argle_report)]),
    "gp_step_n_batch": (ST, [P, PP, C.c_int64]),
    "gp_energies_batch": (ST, [P, PP, P, C.POINTER(C.c_double)]),
    "gp_last_error": (C.c_char_p, []),
    "gp_schedule_name": (C.c_char_p, [P, C.c_int32]),
    "gp_variant_count": (C.c_int32, [C.c_int32, C.c_int32]),
    "gp_select_variant": (ST, [P, C.c_int32, C.c_int32]),
    "gp_autotune": (ST, [P, P, C.c_int32, C.c_char_p]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2003_03590_amd.build); there is no CPU fallback")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class GPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
