"""ctypes binding of the C ABI in include/moff.h: same names, argument marshalling only.

Every compute step runs in the HIP library; this module only converts Python
arguments to C types.  Loading fails loudly when the library has not been built:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoff.so")

MOFF_OK = 0
STATUS_NAMES = {0: "MOFF_OK", 1: "MOFF_ERR_INVALID_ARG", 2: "MOFF_ERR_GRID_NOT_POW2",
                3: "MOFF_ERR_FOOTPRINT_OVERFLOW", 4: "MOFF_ERR_UNSUPPORTED", 5: "MOFF_ERR_NOMEM",
                6: "MOFF_ERR_HIP"}
MOFF_IN_C64 = 0
MOFF_IN_CI4 = 1
MOFF_AUTOCORR_NONE = 2
MOFF_NORM_PAIRS = 4
MOFF_MFMA_F16 = 8
MOFF_MFMA_BF16 = 16
MOFF_AUTOCORR_UV = 32

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_u32p = ctypes.POINTER(ctypes.c_uint32)
c_u16p = ctypes.POINTER(ctypes.c_uint16)
c_f32p = ctypes.POINTER(ctypes.c_float)
c_f64p = ctypes.POINTER(ctypes.c_double)


class moff_geometry(ctypes.Structure):
    _fields_ = [
        ("n_ant", ctypes.c_int32),
        ("ant_xy_m", c_f64p),
        ("n_ktypes", ctypes.c_int32),
        ("ktype_k", c_i32p),
        ("ktype_vals", c_f32p),
        ("ant_ktype", c_i32p),
        ("n_chan", ctypes.c_int32),
        ("freq_hz", c_f64p),
        ("grid_n", ctypes.c_int32),
        ("cell_m", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


# name -> (restype, argtypes); the order of arguments follows include/moff.h
SIGNATURES = {
    "moff_abi_version": (ctypes.c_int, []),
    "moff_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "moff_plan_create": (ctypes.c_int, [ctypes.POINTER(moff_geometry), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "moff_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "moff_plan_query": (ctypes.c_int, [ctypes.c_void_p, c_i32p, c_f64p, c_f64p, c_i32p]),
    "moff_plan_power_pattern": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, c_f64p]),
    "moff_plan_gather_program": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, c_u32p, c_f32p,
                                                c_i32p, c_i32p, c_i32p, c_i32p, c_i32p]),
    "moff_plan_mfma_tables": (ctypes.c_int, [ctypes.c_void_p, c_u32p, c_u16p, c_i32p, c_i32p, c_i32p, c_i32p,
                                             c_i32p]),
    "moff_plan_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "moff_plan_set_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "moff_plan_get_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, c_i32p, c_i32p, c_i32p, c_i32p, c_i32p,
                                            c_i32p]),
    "moff_plan_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "moff_plan_last_kernel_ms": (ctypes.c_int, [ctypes.c_void_p, c_f64p]),
    "moff_image": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "moff_image_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "moff_accumulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "moff_finalize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "moff_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]),
    "moff_self_power": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "moff_fft2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "moff_detect_accumulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "moff_gain_vjp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "moff_gain_vjp_staged": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "moff_image_staged": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "moff_image_fx": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "moff_plan_set_adjoint_waves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "moff_plan_get_adjoint_waves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


class MoffError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({_status_text(status)})")


def _status_text(s):
    try:
        return lib().moff_status_str(s).decode()
    except Exception:  # pragma: no cover - only while reporting a load failure
        return "?"


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_1510_08318_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, where):
    if status != MOFF_OK:
        raise MoffError(status, where)


def _call(name, *args):
    check(getattr(lib(), name)(*args), name)


# ---- same-name wrappers (pointers are ints: device addresses or host buffers) ----

def moff_abi_version():
    return lib().moff_abi_version()


def moff_status_str(s):
    return lib().moff_status_str(s).decode()


def moff_plan_create(geom: moff_geometry, hip_device: int):
    out = ctypes.c_void_p()
    _call("moff_plan_create", ctypes.byref(geom), hip_device, ctypes.byref(out))
    return out.value


def moff_plan_destroy(plan):
    _call("moff_plan_destroy", plan)


def moff_plan_query(plan, cells=None, cell_m=None, lm_per_pixel=None, grid_n=None):
    _call("moff_plan_query", plan, cells, cell_m, lm_per_pixel, grid_n)


def moff_plan_power_pattern(plan, ktype, out):
    _call("moff_plan_power_pattern", plan, ktype, out)


def moff_plan_gather_program(plan, variant, w, out, weights, prog_len, n_threads, n_classes, row_pitch, n_weights):
    _call("moff_plan_gather_program", plan, variant, w, out, weights, prog_len, n_threads, n_classes, row_pitch,
          n_weights)


def moff_plan_mfma_tables(plan, prog, dft, prog_len, n_threads, row_pitch, grid_base, dft_len):
    _call("moff_plan_mfma_tables", plan, prog, dft, prog_len, n_threads, row_pitch, grid_base, dft_len)


def moff_plan_autotune(plan, E, n_time, gains, stream):
    _call("moff_plan_autotune", plan, E, n_time, gains, stream)


def moff_plan_set_config(plan, variant, slices):
    _call("moff_plan_set_config", plan, variant, slices)


def moff_plan_get_config(plan, n_time):
    vals = [ctypes.c_int32() for _ in range(6)]
    _call("moff_plan_get_config", plan, n_time, *[ctypes.byref(v) for v in vals])
    return dict(zip(("variant", "slices", "grid", "threads", "n_variants", "tuned"), (v.value for v in vals)))


def moff_plan_set_timing(plan, enable):
    _call("moff_plan_set_timing", plan, int(enable))


def moff_plan_last_kernel_ms(plan):
    v = ctypes.c_double()
    _call("moff_plan_last_kernel_ms", plan, ctypes.byref(v))
    return v.value


def moff_image(plan, E, n_time, gains, image, stream):
    _call("moff_image", plan, E, n_time, gains, image, stream)


def moff_image_noalloc(plan, E, n_time, gains, image, stream):
    _call("moff_image_noalloc", plan, E, n_time, gains, image, stream)


def moff_accumulate(plan, E, n_time, gains, S, A, stream):
    _call("moff_accumulate", plan, E, n_time, gains, S, A, stream)


def moff_finalize(plan, S, A, n_time_total, image, stream):
    _call("moff_finalize", plan, S, A, n_time_total, image, stream)


def moff_grid(plan, E, n_time, gains, eg, stream):
    _call("moff_grid", plan, E, n_time, gains, eg, stream)


def moff_self_power(plan, E, n_time, gains, A, stream):
    _call("moff_self_power", plan, E, n_time, gains, A, stream)


def moff_fft2(plan, eg, n_frames, y, stream):
    _call("moff_fft2", plan, eg, n_frames, y, stream)


def moff_detect_accumulate(plan, y, n_time, S, stream):
    _call("moff_detect_accumulate", plan, y, n_time, S, stream)


def moff_image_staged(plan, E, n_time, gains, image, stream):
    _call("moff_image_staged", plan, E, n_time, gains, image, stream)


def moff_image_fx(plan, E, n_time, gains, image, stream):
    _call("moff_image_fx", plan, E, n_time, gains, image, stream)


def moff_gain_vjp_staged(plan, E, n_time, gains, dL_dimage, dL_dgains, stream):
    _call("moff_gain_vjp_staged", plan, E, n_time, gains, dL_dimage, dL_dgains, stream)


def moff_gain_vjp(plan, E, n_time, gains, dL_dimage, dL_dgains, stream):
    _call("moff_gain_vjp", plan, E, n_time, gains, dL_dimage, dL_dgains, stream)


def moff_plan_set_adjoint_waves(plan, waves):
    _call("moff_plan_set_adjoint_waves", plan, waves)


def moff_plan_get_adjoint_waves(plan, waves, max_waves):
    _call("moff_plan_get_adjoint_waves", plan, waves, max_waves)
