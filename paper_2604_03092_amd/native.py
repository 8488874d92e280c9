"""ctypes mirror of include/fm2dgs.h and loader of the in-tree libfm2dgs.so.

Argument marshalling only: every step of the rasterizer runs in the HIP
library.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfm2dgs.so")

c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_float = ctypes.c_float

FM_OK = 0
FM_ERR_INVALID_ARG = 1
FM_ERR_CAPACITY = 2
FM_ERR_HIP = 3
FM_ERR_UNSUPPORTED = 4
FM_ERR_WORKSPACE = 5
# bytes of the static scratch array behind fm_fwd_bwd_l1_noalloc
FM_NOALLOC_SCRATCH_BYTES = 128 << 20


class FmSurfels(ctypes.Structure):
    _fields_ = [("n", c_int32), ("mean", c_void_p), ("quat", c_void_p), ("scale", c_void_p),
                ("opacity", c_void_p), ("color", c_void_p)]


class FmSurfelGrads(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("opacity", c_void_p),
                ("color", c_void_p)]


class FmViewShape(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("submap", c_int32)]


class FmBatch(ctypes.Structure):
    _fields_ = [("n_submaps", c_int32), ("submaps", ctypes.POINTER(FmSurfels)), ("n_views", c_int32),
                ("views", ctypes.POINTER(FmViewShape)), ("intr", c_void_p), ("viewmat", c_void_p)]


class FmRasterParams(ctypes.Structure):
    _fields_ = [("alpha_min", c_float), ("alpha_max", c_float), ("t_min", c_float), ("rho_max", c_float),
                ("near_plane", c_float), ("bg", c_float * 3), ("tile_w", c_int32), ("tile_h", c_int32),
                ("deterministic", c_int32), ("overwrite", c_int32),
                ("tile_order", c_int32), ("tile_waves", c_int32), ("lds_depth", c_int32)]


class FmOutputs(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p), ("normal", c_void_p), ("alpha", c_void_p)]


class FmGradOutputs(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p), ("normal", c_void_p), ("alpha", c_void_p)]


class FmL1Loss(ctypes.Structure):
    _fields_ = [("target_rgb", c_void_p), ("target_depth", c_void_p), ("mask", c_void_p),
                ("w_rgb", c_float), ("w_depth", c_float)]


FM_PARAM_LINEAR = 0
FM_PARAM_LOG = 1
FM_PARAM_LOGIT = 2


class FmAdamTensor(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("m", c_void_p), ("v", c_void_p), ("n", c_int64),
                ("lr", c_float), ("kind", c_int32)]


class FmAdamConfig(ctypes.Structure):
    _fields_ = [("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("zero_grad", c_int32)]


class FmPixelMap(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("mean", c_void_p), ("quat", c_void_p),
                ("scale", c_void_p), ("opacity", c_void_p), ("color", c_void_p)]


class FmSim3(ctypes.Structure):
    _fields_ = [("s", c_float), ("q", c_float * 4), ("t", c_float * 3)]


class FmFusionParams(ctypes.Structure):
    _fields_ = [("tau_depth", c_float), ("tau_accum", c_float)]


class FmSurfelBuffer(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("opacity", c_void_p),
                ("color", c_void_p), ("capacity", c_int64)]


class FmPruneSpec(ctypes.Structure):
    _fields_ = [("target_rgb", c_void_p), ("target_depth", c_void_p), ("mask_in", c_void_p),
                ("mask_out", c_void_p), ("tau_rgb", c_float), ("tau_depth", c_float)]


P = ctypes.POINTER
SIGNATURES = {
    "fm_create": (c_int32, [P(c_void_p), c_int32]),
    "fm_destroy": (None, [c_void_p]),
    "fm_status_string": (ctypes.c_char_p, [c_int32]),
    "fm_last_error": (ctypes.c_char_p, [c_void_p]),
    "fm_default_params": (None, [P(FmRasterParams)]),
    "fm_version": (c_int32, []),
    "fm_workspace_size": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), c_int64, P(ctypes.c_size_t)]),
    "fm_forward": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), FmOutputs, c_void_p, ctypes.c_size_t,
                             c_int64, c_void_p]),
    "fm_backward": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), FmOutputs, FmGradOutputs, c_void_p,
                              ctypes.c_size_t, c_int64, P(FmSurfelGrads), c_void_p, c_void_p]),
    "fm_fwd_bwd_l1": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), P(FmL1Loss), FmOutputs, c_void_p,
                                P(FmSurfelGrads), c_void_p, c_void_p, ctypes.c_size_t, c_int64, c_void_p]),
    "fm_fwd_bwd_l1_noalloc": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), P(FmL1Loss), FmOutputs,
                                        c_void_p, P(FmSurfelGrads), c_void_p, c_int64, c_void_p, c_void_p]),
    "fm_prune_scores": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), P(FmPruneSpec), FmOutputs,
                                  P(c_void_p), c_void_p, ctypes.c_size_t, c_int64, c_void_p]),
    "fm_prune_compact_workspace_size": (ctypes.c_size_t, [c_int64]),
    "fm_prune_compact": (c_int32, [c_void_p, P(FmSurfels), c_void_p, c_float, FmSurfelBuffer, c_void_p, c_void_p,
                                   ctypes.c_size_t, c_void_p]),
    "fm_query_status": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), c_void_p, c_int64, P(c_int64),
                                  P(c_int64)]),
    "fm_debug_pairs": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), c_void_p, c_int64, c_void_p,
                                 c_void_p, c_void_p, c_int64, P(c_int64), c_void_p, c_void_p, c_int64]),
    "fm_tile_count": (c_int32, [P(FmBatch), P(FmRasterParams), P(c_int64)]),
    "fm_debug_pixel_state": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), c_void_p, c_int64, c_void_p,
                                       c_void_p, c_int64]),
    "fm_debug_counts": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), c_void_p, c_int64, P(c_int64),
                                  P(c_int64)]),
    "fm_bench_lds": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, P(ctypes.c_double), c_void_p]),
    "fm_set_timing": (c_int32, [c_void_p, c_int32]),
    "fm_phase_times": (c_int32, [c_void_p, P(c_float), c_int32]),
    "fm_autotune": (c_int32, [c_void_p, P(FmBatch), P(FmRasterParams), P(FmL1Loss), FmOutputs, c_void_p,
                              P(FmSurfelGrads), c_void_p, c_void_p, ctypes.c_size_t, c_int64, ctypes.c_char_p,
                              P(FmRasterParams), c_void_p]),
    "fm_adam_step": (c_int32, [c_void_p, P(FmAdamTensor), c_int32, P(FmAdamConfig), c_void_p, c_void_p]),
    "fm_fusion_workspace_size": (ctypes.c_size_t, [c_int32, c_int32]),
    "fm_warp_keyframes": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int32,
                                    c_void_p]),
    "fm_voxelize_fuse": (c_int32, [c_void_p, P(FmPixelMap), P(FmSim3), P(FmFusionParams), c_void_p,
                                   FmSurfelBuffer, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "fm_fusion_batch_workspace_size": (ctypes.c_size_t, [P(FmPixelMap), c_int32]),
    "fm_voxelize_fuse_batch": (c_int32, [c_void_p, P(FmPixelMap), P(FmSim3), c_int32, P(FmFusionParams),
                                         c_void_p, FmSurfelBuffer, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libfm2dgs.so (built by paper_2604_03092_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2604_03092_amd.build` "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fm2dgs status {status}: {msg}")
        self.status = status
