"""ctypes binding of liblens.so (include/lens.h).

Argument marshalling only: torch tensors are passed as device pointers, the
stream is torch's current stream.  Every computation runs in the HIP library;
there is no fallback -- a missing library or GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblens.so")

LENS_OK, LENS_ERR_INVALID, LENS_ERR_DEVICE, LENS_ERR_CAPACITY, LENS_ERR_SCRATCH = 0, 1, 2, 3, 4
NOALLOC_SCRATCH_BYTES = 512 << 20
LENS_FP64, LENS_FP32, LENS_MIXED = 0, 1, 2
STAT_HITS, STAT_FLAGGED, STAT_TILE_PASS, STAT_BBOX_PASS, STAT_STATUS, STAT_FB_HITS, STAT_TESTS = range(7)
STAT_N = 8

EXPORTS = ("lens_create", "lens_destroy", "lens_dls_dos", "lens_deflect", "lens_deflect_mixed",
           "lens_deflect_nfw", "lens_source_positions", "lens_image_chi2", "lens_image_chi2_noalloc",
           "lens_image_chi2_batched",
           "lens_deflect_backward", "lens_src_chi2", "lens_src_chi2_backward", "lens_hmc_step",
           "lens_mh_step_batched", "lens_autotune_chi2", "lens_autotune_chi2_batched", "lens_autotune_lookup",
           "lens_autotune_save", "lens_autotune_load", "lens_set_timing", "lens_field_timing", "lens_strerror")


class LensPotentials(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("y", C.c_void_p), ("eps", C.c_void_p),
                ("phi", C.c_void_p), ("r_core", C.c_void_p), ("r_cut", C.c_void_p), ("sigma_v", C.c_void_p)]


class LensGrid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("h", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32)]


class LensObs(C.Structure):
    _fields_ = [("n_sys", C.c_int32), ("n_img", C.c_int32), ("sys_off", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("sigma", C.c_void_p), ("dls_dos", C.c_void_p)]


class LensNfw(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("y", C.c_void_p), ("eps", C.c_void_p), ("phi", C.c_void_p),
                ("r_s", C.c_void_p), ("kappa_s", C.c_void_p)]


class LensMixedOpts(C.Structure):
    _fields_ = [("n_cluster", C.c_int32), ("patch_cluster", C.c_int32), ("patch_galaxy", C.c_int32),
                ("t12", C.c_double), ("t34", C.c_double)]


class LensChi2Opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("fb_mode", C.c_int32), ("fb_tau", C.c_double), ("hit_capacity", C.c_int32),
                ("field_npl", C.c_int32), ("tile", C.c_int32)]


class LensChi2Out(C.Structure):
    _fields_ = [("chi2", C.c_void_p), ("chi2_sys", C.c_void_p), ("n_pred", C.c_void_p), ("hits", C.c_void_p),
                ("img_xy", C.c_void_p), ("match", C.c_void_p), ("stats", C.c_void_p)]


class LensBatchOut(C.Structure):
    _fields_ = [("chi2", C.c_void_p), ("chi2_sys", C.c_void_p), ("n_pred", C.c_void_p), ("status", C.c_void_p),
                ("stats", C.c_void_p), ("n_hits", C.c_void_p), ("hits", C.c_void_p), ("img_xy", C.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load liblens.so (after torch has initialised its HIP runtime, so that both
    share one runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1902_03252_amd.build`")
    lib = C.CDLL(path)
    vp, i32, d = C.c_void_p, C.c_int32, C.c_double
    lib.lens_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.lens_create.restype = C.c_int
    lib.lens_destroy.argtypes = [vp]
    lib.lens_destroy.restype = None
    lib.lens_dls_dos.argtypes = [vp, d, vp, i32, d, d, vp, vp]
    lib.lens_dls_dos.restype = C.c_int
    lib.lens_deflect.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensGrid), C.c_int, vp, vp, vp, vp]
    lib.lens_deflect.restype = C.c_int
    lib.lens_deflect_nfw.argtypes = [vp, C.POINTER(LensNfw), C.POINTER(LensGrid), C.c_int, vp, vp, vp, vp]
    lib.lens_deflect_nfw.restype = C.c_int
    lib.lens_deflect_mixed.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensGrid), C.POINTER(LensMixedOpts),
                                       vp, vp, vp, vp, vp]
    lib.lens_deflect_mixed.restype = C.c_int
    lib.lens_source_positions.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensObs), vp, vp, vp, vp, vp, vp]
    lib.lens_source_positions.restype = C.c_int
    lib.lens_image_chi2.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensGrid), C.POINTER(LensObs),
                                    C.POINTER(LensChi2Opts), C.POINTER(LensChi2Out), vp]
    lib.lens_image_chi2.restype = C.c_int
    lib.lens_image_chi2_noalloc.argtypes = [C.POINTER(LensPotentials), C.POINTER(LensGrid), C.POINTER(LensObs),
                                            C.POINTER(LensChi2Opts), C.POINTER(LensChi2Out), vp]
    lib.lens_image_chi2_noalloc.restype = C.c_int
    lib.lens_image_chi2_batched.argtypes = [vp, C.POINTER(LensPotentials), i32, C.POINTER(i32), C.POINTER(LensGrid),
                                            C.POINTER(LensObs), C.POINTER(LensChi2Opts), C.POINTER(LensBatchOut), vp]
    lib.lens_image_chi2_batched.restype = C.c_int
    lib.lens_deflect_backward.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensGrid), C.c_int, vp, vp, vp,
                                          vp, vp]
    lib.lens_deflect_backward.restype = C.c_int
    lib.lens_src_chi2.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensObs), vp, vp, vp]
    lib.lens_src_chi2.restype = C.c_int
    lib.lens_src_chi2_backward.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensObs), vp, vp, vp, vp]
    lib.lens_src_chi2_backward.restype = C.c_int
    pi32 = C.POINTER(i32)
    lib.lens_hmc_step.argtypes = [vp, vp, i32, C.POINTER(LensObs), vp, i32, vp, vp, vp, vp, vp]
    lib.lens_hmc_step.restype = C.c_int
    lib.lens_mh_step_batched.argtypes = [vp, vp, i32, i32, C.POINTER(LensGrid), C.POINTER(LensObs),
                                         C.POINTER(LensChi2Opts), vp, vp, vp, vp, vp, vp]
    lib.lens_mh_step_batched.restype = C.c_int
    lib.lens_autotune_chi2.argtypes = [vp, C.POINTER(LensPotentials), C.POINTER(LensGrid), C.POINTER(LensObs),
                                       C.POINTER(LensChi2Opts), C.POINTER(LensChi2Out), i32, pi32, pi32, vp]
    lib.lens_autotune_chi2.restype = C.c_int
    lib.lens_autotune_chi2_batched.argtypes = [vp, C.POINTER(LensPotentials), i32, pi32, C.POINTER(LensGrid),
                                               C.POINTER(LensObs), C.POINTER(LensChi2Opts), C.POINTER(LensBatchOut),
                                               i32, pi32, pi32, vp]
    lib.lens_autotune_chi2_batched.restype = C.c_int
    lib.lens_autotune_lookup.argtypes = [vp, C.c_int, i32, i32, i32, pi32, pi32]
    lib.lens_autotune_lookup.restype = C.c_int
    lib.lens_autotune_save.argtypes = [vp, C.c_char_p]
    lib.lens_autotune_save.restype = C.c_int
    lib.lens_autotune_load.argtypes = [vp, C.c_char_p]
    lib.lens_autotune_load.restype = C.c_int
    lib.lens_set_timing.argtypes = [vp, C.c_int]
    lib.lens_set_timing.restype = C.c_int
    lib.lens_field_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
    lib.lens_field_timing.restype = C.c_int
    lib.lens_strerror.argtypes = [C.c_int]
    lib.lens_strerror.restype = C.c_char_p
    _lib = lib
    return lib


def check(rc: int, what: str):
    if rc != LENS_OK:
        msg = load().lens_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} (code {rc})")


def ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def stream_handle(device: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
