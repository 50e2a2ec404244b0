"""ctypes declarations of the demrx C-ABI (include/demrx.h).

Argument marshalling only: every step of the particle path runs in the HIP
kernels of libdemrx.so.  Importing this module fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdemrx.so")

DEMRX_OK = 0
DEMRX_EINVAL = -1
ERRORS = {-1: "EINVAL", -2: "EHIP", -3: "EOVERFLOW", -4: "EDOMAIN", -5: "ENONFINITE", -6: "ENOMEM", -7: "ESKIN"}
DEM_FP64, DEM_MIXED = 0, 1
DEM_WALL_BOX, DEM_WALL_CYL = 0, 1
DEM_MAX_NBR = 48


class DemBed(C.Structure):
    _fields_ = [("wall_kind", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("R", C.c_double),
                ("origin", C.c_double * 3), ("h", C.c_double), ("n", C.c_int32 * 3), ("refine", C.c_int32),
                ("theta", C.c_double * 6), ("mu_override", C.c_double)]


class DemOre(C.Structure):
    _fields_ = [("xi0", C.c_double), ("d_pore_cm", C.c_double), ("tau", C.c_double),
                ("rho_true", C.c_double * 4), ("kind", C.c_int32), ("psi", C.c_double)]


class DemParams(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_beds", C.c_int32), ("beds", C.POINTER(DemBed)),
                ("n_ores", C.c_int32), ("ores", C.POINTER(DemOre)),
                ("kn", C.c_double), ("e_p", C.c_double), ("mu_s", C.c_double), ("mu_r", C.c_double),
                ("kt_over_kn", C.c_double), ("gt_over_gn", C.c_double), ("eps_min", C.c_double),
                ("skin", C.c_double), ("dt", C.c_double), ("g", C.c_double * 3),
                ("max_nbr", C.c_int32), ("check_every", C.c_int32), ("ergun_printed", C.c_int32),
                ("drag_on", C.c_int32), ("energy_on", C.c_int32)]


PARCEL_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz", "d", "k", "ore", "bed", "nh", "nm", "nw", "nfe",
                 "Tp")


class DemParcels(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in PARCEL_FIELDS]


class DemContacts(C.Structure):
    _fields_ = [("cap", C.c_int64), ("count", C.c_int64), ("ids", C.POINTER(C.c_uint32)),
                ("xi", C.POINTER(C.c_double)), ("wall_on", C.POINTER(C.c_uint8)),
                ("wall_xi", C.POINTER(C.c_double))]


GAS_FIELDS = ("ug", "vg", "wg", "p", "dpdx", "dpdy", "dpdz", "T", "xH2", "xH2O", "xN2")


class DemGas(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in GAS_FIELDS]


SOURCE_FIELDS = ("eps", "np", "sumK", "sumKu", "sumKv", "sumKw", "sumKs", "mdotH2", "mdotH2O", "sumEQ", "sumES",
                 "hA", "hAT", "Qrm", "Hr")


class DemSources(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in SOURCE_FIELDS]


class DemGradSpec(C.Structure):
    _fields_ = [("n_substeps", C.c_int32), ("dt_react", C.c_double), ("dyn_every", C.c_int32),
                ("ckpt_every", C.c_int32), ("state_fp32", C.c_int32)]


class DemStats(C.Structure):
    _fields_ = [("n_parcels", C.c_int64), ("n_contacts", C.c_int64), ("n_wall_contacts", C.c_int64),
                ("rebuilds", C.c_int64), ("steps", C.c_int64), ("clamps", C.c_int64),
                ("mean_coordination", C.c_double), ("max_nbr_used", C.c_int32), ("status", C.c_uint32),
                ("step_kernel_ms", C.c_double), ("step_kernel_launches", C.c_int64),
                ("step_block", C.c_int32), ("step_xcd", C.c_int32), ("build_grid", C.c_int32),
                ("check_period", C.c_int32), ("build_threads", C.c_int32), ("build_tile", C.c_int32),
                ("build_item_x", C.c_int32), ("tune_cached", C.c_int32)]


EXPORTS = ("dem_init", "dem_step", "dem_couple", "dem_react", "dem_gas_species", "dem_gas_momentum", "dem_grad",
           "dem_forces",
           "dem_get_state", "dem_set_state", "dem_pairs", "dem_pairs_noalloc", "dem_get_contacts", "dem_set_contacts", "dem_get_stats", "dem_run", "dem_autotune", "dem_set_launch", "dem_set_build",
           "dem_profile",
           "dem_sync",
           "dem_last_error", "dem_destroy")

_lib = None


class DemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libdemrx.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built; run __graft_entry__.build() (hipcc, gfx950)")
    # PyTorch brings its own HIP runtime; loading it first makes the library
    # bind to that same runtime, so that device pointers and streams are shared.
    import torch  # noqa: F401

    L = C.CDLL(path)
    vp = C.c_void_p
    L.dem_init.argtypes = [C.POINTER(DemParams), C.POINTER(DemParcels), C.c_int32, vp, C.POINTER(vp)]
    L.dem_step.argtypes = [vp, C.c_int32, C.POINTER(DemGas)]
    L.dem_couple.argtypes = [vp, C.POINTER(DemGas), C.POINTER(DemSources)]
    L.dem_react.argtypes = [vp, C.c_double, C.POINTER(DemGas), C.POINTER(DemSources), C.POINTER(C.c_double), vp]
    L.dem_gas_species.argtypes = [vp, C.c_double, C.POINTER(DemGas), vp, vp, C.POINTER(C.c_double), vp, vp, vp]
    L.dem_gas_momentum.argtypes = [vp, C.c_double, C.POINTER(DemGas)] + [vp] * 7
    L.dem_grad.argtypes = [vp, C.POINTER(DemGradSpec), C.POINTER(DemGas), C.POINTER(C.c_double),
                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.dem_forces.argtypes = [vp, C.POINTER(DemGas), vp, vp]
    L.dem_get_state.argtypes = [vp, C.POINTER(DemParcels)]
    L.dem_set_state.argtypes = [vp, C.POINTER(DemParcels)]
    L.dem_pairs.argtypes = [vp, C.POINTER(C.c_uint32), C.c_int64, C.POINTER(C.c_int64)]
    L.dem_pairs_noalloc.argtypes = [vp, C.POINTER(C.c_uint32), C.c_int64, C.POINTER(C.c_int64)]
    L.dem_get_contacts.argtypes = [vp, C.POINTER(DemContacts)]
    L.dem_set_contacts.argtypes = [vp, C.POINTER(DemContacts)]
    L.dem_get_stats.argtypes = [vp, C.POINTER(DemStats)]
    L.dem_run.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(DemGas), C.POINTER(DemSources),
                          C.POINTER(C.c_double)]
    L.dem_autotune.argtypes = [vp, C.POINTER(DemGas)]
    L.dem_set_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.dem_set_build.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.dem_profile.argtypes = [vp, C.c_int32]
    L.dem_sync.argtypes = [vp]
    L.dem_last_error.argtypes = [vp]
    L.dem_last_error.restype = C.c_char_p
    L.dem_destroy.argtypes = [vp]
    for f in EXPORTS:
        if f not in ("dem_last_error", "dem_destroy"):
            getattr(L, f).restype = C.c_int
    L.dem_destroy.restype = None
    _lib = L
    return L
