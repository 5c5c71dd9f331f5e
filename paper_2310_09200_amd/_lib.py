"""ctypes binding of libbluebild.so: argument marshalling only, same names as the C ABI."""

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbluebild.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p
POINTER = ctypes.POINTER

STATUS = {
    0: "BB_OK", 1: "BB_ERR_INVALID_ARG", 2: "BB_ERR_SHAPE", 3: "BB_ERR_NOT_POSDEF", 4: "BB_ERR_EIGEN",
    5: "BB_ERR_WORKSPACE", 6: "BB_ERR_DEVICE", 7: "BB_ERR_STATE",
}
BB_OK, BB_ERR_INVALID_ARG, BB_ERR_SHAPE, BB_ERR_NOT_POSDEF, BB_ERR_EIGEN, BB_ERR_WORKSPACE, BB_ERR_DEVICE, \
    BB_ERR_STATE = range(8)
BB_PREC_FP32, BB_PREC_BF16X3, BB_PREC_FP32_3M, BB_PREC_BF16X3_3M = 0, 1, 2, 3
BB_FILTER_LSQ, BB_FILTER_STD = 0, 1
BB_GRAM_SINC, BB_GRAM_IDENTITY = 0, 1
BB_K_CLASSES, BB_MAX_TILES = 4, 12


class bb_options(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("n_slots", c_int32), ("n_ant_max", c_int32), ("k_max", c_int32),
                ("precision", c_int32), ("filter", c_int32), ("gram", c_int32), ("reserved", c_int32)]


class bb_nufft_options(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("n_ant_max", c_int32), ("k_max", c_int32), ("transform", c_int32),
                ("epsilon", c_double), ("frame", c_double * 9), ("uvw_max", c_double * 3),
                ("partitions", c_int32), ("uvw_partitions", c_int32)]


class bb_instance(ctypes.Structure):
    _fields_ = [("n_ant", c_int32), ("n_eig", c_int32), ("slot", c_int32), ("reserved", c_int32),
                ("wavelength_m", c_double), ("ant_off", c_int64), ("w_off", c_int64), ("eig_off", c_int64)]


# name -> (restype, argtypes); every symbol declared in include/bluebild.h
PROTOS = {
    "bb_context_create": (c_int32, [c_int32, c_void_p, POINTER(c_void_p)]),
    "bb_context_set_stream": (c_int32, [c_void_p, c_void_p]),
    "bb_context_destroy": (c_int32, [c_void_p]),
    "bb_status_string": (c_char_p, [c_int32]),
    "bb_last_error": (c_char_p, [c_void_p]),
    "bb_workspace_size": (c_int32, [c_void_p, POINTER(bb_options), c_int64, POINTER(c_size_t)]),
    "bb_synth_create": (c_int32, [c_void_p, POINTER(bb_options), c_int64, c_void_p, c_void_p, c_void_p, c_size_t,
                                  POINTER(c_void_p)]),
    "bb_synth_collect": (c_int32, [c_void_p, c_int32, c_int32, c_double, c_void_p, c_void_p, c_int32,
                                   POINTER(c_double)]),
    "bb_synth_collect_beamformed": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_double, c_void_p, c_void_p,
                                              c_void_p, c_int32, POINTER(c_double)]),
    "bb_synth_collect_energy": (c_int32, [c_void_p, c_int32, c_int32, c_double, c_void_p, c_void_p, c_double,
                                          POINTER(c_double), POINTER(c_int32)]),
    "bb_synth_prestep": (c_int32, [c_void_p, c_int32, c_double, c_void_p, c_void_p, c_int32, POINTER(c_double),
                                   c_void_p, c_void_p, c_void_p, c_void_p]),
    "bb_synth_collect_eig": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_double, c_void_p, c_void_p,
                                       c_void_p, c_void_p]),
    "bb_synth_collect_eig_noalloc": (c_int32, [c_void_p, c_int32, c_int32, c_int64, c_void_p, c_void_p, c_int32,
                                               c_int32, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "bb_tile_info": (c_int32, [c_int32, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                               POINTER(c_int32)]),
    "bb_tune_cache_lookup": (c_int32, [c_char_p, c_int32, c_int64, POINTER(c_int32)]),
    "bb_synth_get_tiles": (c_int32, [c_void_p, POINTER(c_int32)]),
    "bb_synth_set_tiles": (c_int32, [c_void_p, POINTER(c_int32)]),
    "bb_synth_autotune_batched": (c_int32, [c_void_p, c_int32, POINTER(bb_instance), c_int64, c_int64, c_int64,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                            c_int32, POINTER(c_double)]),
    "bb_batched_workspace_size": (c_int32, [c_void_p, c_int32, POINTER(bb_instance), POINTER(c_size_t)]),
    "bb_synth_collect_eig_batched": (c_int32, [c_void_p, c_int32, POINTER(bb_instance), c_int64, c_int64, c_int64,
                                               c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    "bb_backward_workspace_size": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_size_t)]),
    "bb_synth_eig_backward": (c_int32, [c_void_p, c_int32, c_int32, c_double, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    "bb_prestep_batched_workspace_size": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "bb_synth_prestep_batched": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_double), c_void_p,
                                           c_void_p, POINTER(c_double), c_void_p, c_void_p, c_void_p, c_void_p,
                                           c_void_p, c_size_t]),
    "bb_synth_levels_kmeans": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p]),
    "bb_synth_uniform_weighting": (c_int32, [c_void_p, c_int32, c_double, c_void_p, POINTER(c_double),
                                             POINTER(c_double), c_double, c_void_p]),
    "bb_nufft_workspace_size": (c_int32, [c_void_p, POINTER(bb_nufft_options), c_int64, c_void_p, POINTER(c_size_t)]),
    "bb_nufft_create": (c_int32, [c_void_p, POINTER(bb_nufft_options), c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_size_t, POINTER(c_void_p)]),
    "bb_nufft_shape": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "bb_nufft_batched_workspace_size": (c_int32, [c_void_p, c_int32, c_void_p, POINTER(c_size_t)]),
    "bb_nufft_collect_eig_batched": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_int64, c_int64, c_void_p,
                                               c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    "bb_nufft_emit": (c_int32, [c_void_p]),
    "bb_nufft_sync": (c_int32, [c_void_p]),
    "bb_nufft_timings": (c_int32, [c_void_p, POINTER(c_double), c_int32]),
    "bb_nufft_destroy": (c_int32, [c_void_p]),
    "bb_synth_sync": (c_int32, [c_void_p]),
    "bb_synth_reset": (c_int32, [c_void_p]),
    "bb_synth_get_count": (c_int32, [c_void_p, POINTER(c_int64)]),
    "bb_synth_set_count": (c_int32, [c_void_p, c_int64]),
    "bb_synth_timings": (c_int32, [c_void_p, POINTER(c_double), c_int32]),
    "bb_phase_probe": (c_int32, [c_void_p, c_int32, c_double, c_void_p, c_int64, c_void_p, c_int32, c_void_p]),
    "bb_synth_destroy": (c_int32, [c_void_p]),
}

_lib = None


class BluebildError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {message}")


def load(path=None):
    """Load libbluebild.so (built in-tree); raises if it is missing -- there is no fallback."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2310_09200_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(status, ctx=None):
    if status != BB_OK:
        msg = ""
        if ctx is not None:
            m = load().bb_last_error(ctx)
            msg = m.decode() if m else ""
        raise BluebildError(status, msg)
