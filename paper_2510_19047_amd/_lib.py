"""ctypes view of include/tfsc.h.  Loads the in-tree libtfsc.so and fails loudly if it is missing."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtfsc.so")

c_int32, c_int64, c_double, c_void_p, c_size_t = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t

TFSC_OK = 0
TFSC_ERR_SCRATCH = 7
ABI_VERSION = 4
MAX_HARMONICS = 4
FRESNEL_PAPER, FRESNEL_ACCURATE = 0, 1
NOALLOC_MAX_TRANCHES = 16384
F64, F32, BF16, F16, I16 = 0, 1, 2, 3, 4
LAYER_MAJOR, TRANCHE_MAJOR, LAYER_MAJOR_CI = 0, 1, 2
SCHED_THREAD, SCHED_WAVE = 0, 1
WS_LAYOUT, WS_STATISTIC, WS_VJP, WS_TRANSFORM, WS_ORDER = 0, 1, 2, 3, 4
FLAG_INVALID, FLAG_EMPTY, FLAG_BAND_END, FLAG_MERGE_END, FLAG_ALL_EXCLUDED = 1, 2, 4, 8, 16


class Grid(ctypes.Structure):
    _fields_ = [("n_channels", c_int32), ("tranche_len", c_int32), ("n_tranches", c_int32), ("n_fresnel", c_int32),
                ("dt", c_double), ("tukey_alpha", c_double)]


class Pixels(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("layout", ctypes.c_int), ("pix", c_void_p), ("layer_scale", c_void_p),
                ("inv_asd", c_void_p), ("tranche_w", c_void_p), ("rho", c_void_p), ("orbit", c_void_p),
                ("links", c_void_p), ("tdi_generation", c_int32)]


class Bank(ctypes.Structure):
    _fields_ = [("n", c_int64), ("mc", c_void_p), ("eta", c_void_p), ("f0", c_void_p), ("cos_theta", c_void_p),
                ("phi", c_void_p), ("psi", c_void_p), ("cos_iota", c_void_p), ("ln_mc", c_void_p)]


class Segments(ctypes.Structure):
    _fields_ = [("nseg_fixed", c_int32), ("nseg", c_void_p), ("seg_offset", c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("schedule", c_int32), ("block_waves", c_int32), ("groups_per_cu", c_int32),
                ("order", c_void_p), ("fresnel", c_int32), ("tune_key", ctypes.c_char_p)]


EXPORTS = ("tfsc_abi_version", "tfsc_status_string", "tfsc_workspace_bytes", "tfsc_transform", "tfsc_transform_tf",
           "tfsc_segment_layout", "tfsc_bank_statistic", "tfsc_bank_statistic_noalloc", "tfsc_bank_statistic_multi",
           "tfsc_statistic_vjp",
           "tfsc_follow_up_step",
           "tfsc_processing_order", "tfsc_tile_max", "tfsc_track", "tfsc_bank_statistic_harmonics",
           "tfsc_orbit_positions", "tfsc_link_lengths", "tfsc_tune_statistic", "tfsc_interleave_store")

_lib = None


class TfscError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load libtfsc.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2510_19047_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.tfsc_abi_version.restype = ctypes.c_int
    L.tfsc_abi_version.argtypes = []
    L.tfsc_status_string.restype = ctypes.c_char_p
    L.tfsc_status_string.argtypes = [ctypes.c_int]
    L.tfsc_workspace_bytes.restype = c_size_t
    L.tfsc_workspace_bytes.argtypes = [P(Grid), c_int64, P(Options), ctypes.c_int]
    L.tfsc_transform.restype = ctypes.c_int
    L.tfsc_transform.argtypes = [P(Grid), c_void_p, ctypes.c_int, c_void_p, c_void_p, c_void_p, P(Pixels),
                                 c_void_p, c_size_t, c_void_p]
    L.tfsc_transform_tf.restype = ctypes.c_int
    L.tfsc_transform_tf.argtypes = [P(Grid), c_void_p, ctypes.c_int, c_void_p, c_void_p, P(Pixels), c_void_p,
                                    c_size_t, c_void_p]
    L.tfsc_segment_layout.restype = ctypes.c_int
    L.tfsc_segment_layout.argtypes = [P(Grid), P(Bank), P(Segments), c_void_p, c_size_t, c_void_p]
    L.tfsc_bank_statistic.restype = ctypes.c_int
    L.tfsc_bank_statistic.argtypes = [P(Grid), P(Pixels), P(Bank), P(Segments), P(Options), c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.tfsc_bank_statistic_noalloc.restype = ctypes.c_int
    L.tfsc_bank_statistic_noalloc.argtypes = [P(Grid), P(Pixels), P(Bank), P(Segments), P(Options), c_void_p,
                                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tfsc_statistic_vjp.restype = ctypes.c_int
    L.tfsc_statistic_vjp.argtypes = [P(Grid), P(Pixels), P(Bank), P(Segments), P(Options), c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.tfsc_follow_up_step.restype = ctypes.c_int
    L.tfsc_follow_up_step.argtypes = [P(Grid), P(Bank), P(Segments), c_void_p, c_void_p, c_void_p, ctypes.c_double,
                                      ctypes.c_int, c_void_p]
    L.tfsc_processing_order.restype = ctypes.c_int
    L.tfsc_processing_order.argtypes = [P(Grid), P(Bank), c_void_p, c_void_p, c_size_t, c_void_p]
    L.tfsc_bank_statistic_multi.restype = ctypes.c_int
    L.tfsc_bank_statistic_multi.argtypes = [P(Grid), P(Pixels), ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                            P(Bank), P(Segments),
                                            P(Options), ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                            c_void_p, c_size_t, c_void_p]
    L.tfsc_tile_max.restype = ctypes.c_int
    L.tfsc_tile_max.argtypes = [c_void_p, c_void_p, ctypes.c_int64, ctypes.c_int32, c_void_p, c_void_p, c_void_p]
    L.tfsc_track.restype = ctypes.c_int
    L.tfsc_track.argtypes = [P(Grid), P(Bank), c_void_p, c_void_p]
    L.tfsc_bank_statistic_harmonics.restype = ctypes.c_int
    L.tfsc_bank_statistic_harmonics.argtypes = [P(Grid), P(Pixels), P(Bank), P(Segments), P(Options), c_int32,
                                                P(c_int32), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                                c_void_p, c_void_p, c_size_t, c_void_p]
    L.tfsc_orbit_positions.restype = ctypes.c_int
    L.tfsc_orbit_positions.argtypes = [P(Grid), c_void_p, c_void_p]
    L.tfsc_link_lengths.restype = ctypes.c_int
    L.tfsc_link_lengths.argtypes = [P(Grid), c_void_p, c_void_p, c_void_p]
    L.tfsc_interleave_store.restype = ctypes.c_int
    L.tfsc_interleave_store.argtypes = [P(Grid), P(Pixels), c_int32, c_int32, P(Pixels), c_void_p]
    L.tfsc_tune_statistic.restype = ctypes.c_int
    L.tfsc_tune_statistic.argtypes = [P(Grid), P(Pixels), P(Bank), P(Segments), P(Options), ctypes.c_char_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, P(c_int32),
                                      P(c_int32)]
    _lib = L
    return L


def check(status: int, what: str):
    if status != TFSC_OK:
        msg = load().tfsc_status_string(status).decode()
        raise TfscError(f"{what} failed: status {status} ({msg})")
