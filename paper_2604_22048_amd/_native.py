"""ctypes view of the C ABI in include/bsi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsi.so")

BSI_OK = 0
ERRORS = {-1: "BSI_EINVAL", -2: "BSI_ENOMEM", -3: "BSI_EHIP", -4: "BSI_EUNSUPPORTED", -5: "BSI_ENODEV"}

STATUS_OUT_OF_SUPPORT = 1
STATUS_NONFINITE = 2
STATUS_DIVERGENT = 4

PROFILE_EXPONENTIAL = 0
PROFILE_GAUSSIAN = 1
PROFILE_SPERGEL = 2
SPERGEL_NU_MIN = -0.85
SPERGEL_NU_MAX = 4.0
MAX_EXPOSURES = 16
NOALLOC_SCRATCH_BYTES = 16 << 20
LIK_KSPACE = 0
LIK_PIXEL = 1
METRIC_GIVEN = 0
METRIC_FISHER = 1
SAMPLER_HMC = 0
SAMPLER_NUTS = 1
NUTS_MAX_DEPTH = 10
TRANSFORM_DEFAULT = 0
TRANSFORM_DIRECT = 1
TRANSFORM_MFMA = 2
FORM_BATCHED = 0
FORM_PLAIN = 1
E_BA14 = 0
E_TRUNC_GAUSS = 1


class Batch(C.Structure):
    _fields_ = [("n_gal", C.c_int32), ("n", C.POINTER(C.c_int32)), ("off", C.POINTER(C.c_int64)),
                ("psf_fwhm", C.c_void_p), ("sigma", C.c_void_p), ("pixel_scale", C.c_float),
                ("profile", C.c_int32), ("spergel_nu", C.c_float), ("n_exp", C.c_int32),
                ("noise_ps", C.c_void_p)]


class Interim(C.Structure):
    _fields_ = [("log10f_lo", C.c_float), ("log10f_hi", C.c_float), ("log10s_lo", C.c_float),
                ("log10s_hi", C.c_float), ("sigma_d", C.c_float), ("sigma_e", C.c_float)]


class HmcCfg(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_leapfrog", C.c_int32), ("n_warmup", C.c_int32),
                ("n_samples", C.c_int32), ("adapt", C.c_int32), ("metric", C.c_int32),
                ("step_size", C.c_float), ("target_accept", C.c_float), ("jitter", C.c_float),
                ("form", C.c_int32), ("iters_per_launch", C.c_int32), ("use_graph", C.c_int32),
                ("seed", C.c_uint64), ("uid_base", C.c_uint64), ("trace", C.c_void_p),
                ("waves_per_chain", C.c_int32), ("sampler", C.c_int32), ("max_tree_depth", C.c_int32)]


class TruePrior(C.Structure):
    _fields_ = [("e_kind", C.c_int32), ("e_max", C.c_float), ("size_term", C.c_int32),
                ("flux_term", C.c_int32), ("mu_ln_f", C.c_double), ("sigma_ln_f", C.c_double)]


class ShearHmcCfg(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_leapfrog", C.c_int32), ("n_warmup", C.c_int32),
                ("n_samples", C.c_int32), ("adapt", C.c_int32), ("step_size", C.c_float),
                ("target_accept", C.c_float), ("jitter", C.c_float), ("inv_mass", C.c_double * 5),
                ("seed", C.c_uint64), ("uid_base", C.c_uint64), ("use_graph", C.c_int32),
                ("trace", C.c_void_p)]


class SlotsCfg(C.Structure):
    _fields_ = [("n_sizes", C.c_int32), ("sizes", C.POINTER(C.c_int32)), ("hbm_budget", C.c_int64),
                ("max_slots", C.c_int32), ("hmc", HmcCfg), ("interim", Interim),
                ("pixel_scale", C.c_float), ("profile", C.c_int32),
                ("spergel_nu", C.c_float), ("pace", C.c_int32),
                ("ess_target", C.c_float), ("ess_every", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("id", C.c_uint64), ("n", C.c_int32), ("stamp", C.c_void_p), ("psf_fwhm", C.c_float),
                ("sigma", C.c_float), ("ref_x", C.c_float), ("ref_y", C.c_float),
                ("init", C.POINTER(C.c_float))]


class ReserveCfg(C.Structure):
    _fields_ = [("max_stamps", C.c_int64), ("max_n", C.c_int32), ("max_chains", C.c_int32),
                ("weighted", C.c_int32), ("pixel_method", C.c_int32), ("max_shear_gal", C.c_int64),
                ("max_points", C.c_int32), ("bias", C.c_int32), ("max_boot", C.c_int32)]


class SlotsInfo(C.Structure):
    _fields_ = [("resident", C.c_int32), ("finished", C.c_int32), ("pending", C.c_int32),
                ("max_slots", C.c_int32), ("budget", C.c_int64), ("slot_fixed_bytes", C.c_int64),
                ("arena_bytes", C.c_int64), ("arena_free", C.c_int64),
                ("arena_largest_free", C.c_int64)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "bsi_version": (C.c_int, []),
    "bsi_device_count": (C.c_int, [C.POINTER(C.c_int32)]),
    "bsi_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_char_p]),
    "bsi_destroy": (None, [C.c_void_p]),
    "bsi_last_error": (C.c_char_p, [C.c_void_p]),
    "bsi_reserve": (C.c_int, [C.c_void_p, C.POINTER(ReserveCfg)]),
    "bsi_render_stamps": (C.c_int, [C.c_void_p, C.POINTER(Batch), C.c_void_p, C.c_void_p, C.c_void_p]),
    "bsi_loglik_grad": (C.c_int, [C.c_void_p, C.POINTER(Batch), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "bsi_hmc_sample": (C.c_int, [C.c_void_p, C.POINTER(Batch), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.POINTER(Interim), C.POINTER(HmcCfg), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "bsi_shear_posterior": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.POINTER(TruePrior),
                                      C.POINTER(Interim), C.c_int32, C.c_void_p, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "bsi_shear_posterior_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.POINTER(TruePrior),
                                              C.POINTER(Interim), C.c_int32, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p]),
    "bsi_shear_galaxy_loglik": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.POINTER(TruePrior),
                                          C.POINTER(Interim), C.c_int32, C.c_void_p, C.c_int32,
                                          C.c_void_p, C.c_void_p]),
    "bsi_shear_bias": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "bsi_shear_hmc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.POINTER(TruePrior), C.POINTER(Interim),
                                C.POINTER(ShearHmcCfg), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    "bsi_slots_create": (C.c_int, [C.c_void_p, C.POINTER(SlotsCfg), C.c_void_p, C.POINTER(C.c_void_p)]),
    "bsi_slots_destroy": (None, [C.c_void_p]),
    "bsi_slots_footprint": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    "bsi_slots_admit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_int32)]),
    "bsi_slots_admit_many": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int32)]),
    "bsi_slots_advance": (C.c_int, [C.c_void_p, C.c_int32]),
    "bsi_slots_poll": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "bsi_slots_harvest": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_uint64), C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "bsi_slots_get_info": (C.c_int, [C.c_void_p, C.POINTER(SlotsInfo)]),
    "bsi_set_plan": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "bsi_get_plan": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "bsi_set_transform": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "bsi_get_transform": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "bsi_autotune_transform": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "bsi_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                               C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "bsi_ess": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


def load():
    """Load libbsi.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2604_22048_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
