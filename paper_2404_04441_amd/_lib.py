"""ctypes binding of libwave (argument marshalling only).

Loads ``libwave.so`` from this package directory.  There is no fallback: if
the library is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwave.so")

WAVE_OK, WAVE_EINVAL, WAVE_EUNSTABLE, WAVE_ENOSPC, WAVE_EHIP, WAVE_ESTATE = 0, -1, -2, -3, -4, -5
WAVE_F32, WAVE_F16, WAVE_BF16 = 0, 1, 2
WAVE_FLAG_NONFINITE = 1
WAVE_STATIC_BYTES = 64 << 20  # size of the static workspace of wave_create_static
STORAGE = {"f32": WAVE_F32, "f16": WAVE_F16, "bf16": WAVE_BF16}

# Every symbol include/wave.h declares.
EXPORTS = (
    "wave_params_init", "wave_stable_dt", "wave_workspace_bytes", "wave_create", "wave_create_static",
    "wave_reset", "wave_step", "wave_run",
    "wave_adjoint", "wave_read_field", "wave_write_field", "wave_time_index", "wave_state_bytes", "wave_save_state", "wave_load_state",
    "wave_sync_status", "wave_destroy", "wave_tiling",
    "wave_variant_count", "wave_variant_info", "wave_status_string",
)


class WaveParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("sponge_width", ctypes.c_int32),
        ("sponge_alpha", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("src", ctypes.c_int32 * 3),
        ("nrec", ctypes.c_int32),
        ("rec", ctypes.POINTER(ctypes.c_int32)),
        ("adjoint", ctypes.c_int32),
        ("nt_max", ctypes.c_int32),
        ("ckpt_interval", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("zchunk", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32),
        ("tune", ctypes.c_int32),
        ("cpml_width", ctypes.c_int32),
        ("cpml_reflection", ctypes.c_double),
        ("cpml_f0", ctypes.c_double),
        ("cache_hint", ctypes.c_int32),
        ("model_bits", ctypes.c_int32),
        ("time_block", ctypes.c_int32),
    ]


class WaveError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libwave is not built ({LIB_PATH} missing); run "
                               "`python -m paper_2404_04441_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
        L.wave_params_init.argtypes = [P(WaveParams)]
        L.wave_params_init.restype = None
        L.wave_workspace_bytes.argtypes = [P(WaveParams), P(sz)]
        L.wave_stable_dt.argtypes = [P(WaveParams), ctypes.c_double, P(ctypes.c_double)]
        L.wave_create.argtypes = [P(WaveParams), vp, vp, sz, vp, P(vp)]
        L.wave_create_static.argtypes = [P(WaveParams), vp, vp, P(vp)]
        L.wave_reset.argtypes = [vp]
        L.wave_step.argtypes = [vp, i32, vp, vp]
        L.wave_run.argtypes = [vp, i32, vp, vp]
        L.wave_adjoint.argtypes = [vp, i32, vp, vp, vp]
        L.wave_read_field.argtypes = [vp, i32, vp]
        L.wave_write_field.argtypes = [vp, i32, vp]
        L.wave_time_index.argtypes = [vp, P(i32)]
        L.wave_state_bytes.argtypes = [vp, P(ctypes.c_size_t)]
        L.wave_save_state.argtypes = [vp, vp]
        L.wave_load_state.argtypes = [vp, vp]
        L.wave_sync_status.argtypes = [vp, P(u32)]
        L.wave_tiling.argtypes = [vp, P(i32)]
        L.wave_destroy.argtypes = [vp]
        L.wave_variant_count.argtypes = []
        L.wave_variant_info.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.wave_status_string.argtypes = [ctypes.c_int]
        L.wave_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("wave_params_init", "wave_status_string"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().wave_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != WAVE_OK:
        raise WaveError(status, where)
