"""ctypes declarations of libmatprobe.so (see include/matprobe.h).

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already has in the process (both name it
libamdhip64.so.7); a second runtime would make torch's stream handles and
allocations foreign to it.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede the dlopen below)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmatprobe.so")

MP_OK = 0
MP_EINVAL = -1
MP_ENOMEM = -2
MP_EDEVICE = -3
MP_ESTATE = -4
MP_ENUMERIC = -5
MP_EUNSUPPORTED = -6
MP_F32 = 1
MP_F64 = 2
MP_SNAP_FULL = 0
MP_SNAP_CKPT_F32 = 1
MP_SNAP_CKPT_BF16 = 2
MP_OP_F, MP_OP_FADJ, MP_OP_H, MP_OP_FIT, MP_OP_HINV = 1, 2, 3, 4, 5
SWEEP_KINDS = ("fused", "born", "background", "adjoint")

EXPORTS = [
    "mp_create", "mp_destroy", "mp_set_background", "mp_footprint", "mp_apply_F", "mp_model",
    "mp_apply_Fadj", "mp_apply_H", "mp_apply_H_batch", "mp_apply_batch", "mp_footprint_batch",
    "mp_release_cache", "mp_basis_create",
    "mp_basis_destroy", "mp_probe_fit", "mp_apply_Hinv", "mp_last_stats", "mp_strerror",
    "mp_last_error", "mp_curvelet_create", "mp_curvelet_destroy", "mp_curvelet_wedges", "mp_curvelet_norms",
    "mp_illumination", "mp_curvelet_synthesis", "mp_curvelet_analysis", "mp_curvelet_sign_threshold",
    "mp_vec_dot", "mp_vec_dot_noalloc", "mp_vec_axpby",
    "mp_velocity_update",
]


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("nb", ctypes.c_int)]


class Acq(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("src", ctypes.POINTER(ctypes.c_int)), ("nr", ctypes.c_int),
                ("rec", ctypes.POINTER(ctypes.c_int)), ("f_peak", ctypes.c_double),
                ("t0", ctypes.c_double), ("dt", ctypes.c_double), ("nt", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("snap", ctypes.c_int), ("ckpt_every", ctypes.c_int),
                ("budget_bytes", ctypes.c_size_t), ("sponge_R", ctypes.c_double),
                ("timing", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("cell_steps", ctypes.c_double), ("waves", ctypes.c_int),
                ("background_cached", ctypes.c_int), ("bytes_reserved", ctypes.c_size_t),
                ("ms_sweep", ctypes.c_double * 4), ("launches_sweep", ctypes.c_longlong * 4),
                ("steps_sweep", ctypes.c_longlong * 4)]


class BasisDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("na", ctypes.c_int), ("degs", ctypes.POINTER(ctypes.c_int)),
                ("nq", ctypes.c_int), ("qs", ctypes.POINTER(ctypes.c_int)), ("family", ctypes.c_int),
                ("modes", ctypes.POINTER(ctypes.c_int)), ("mults", ctypes.POINTER(ctypes.c_int)),
                ("order", ctypes.c_int), ("tl_scale", ctypes.c_double)]


class CurveletDesc(ctypes.Structure):
    _fields_ = [("nscales", ctypes.c_int), ("nangles", ctypes.c_int), ("mask_stride", ctypes.c_int),
                ("nfan", ctypes.c_int), ("max_steps", ctypes.c_int), ("ray_rtol", ctypes.c_double)]


class MatprobeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def _check_single_runtime():
    try:
        with open("/proc/self/maps") as f:
            paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return
    real = {os.path.realpath(p) for p in paths}
    if len(real) > 1:
        raise RuntimeError("two HIP runtimes are loaded in this process: " + ", ".join(sorted(real)))


def lib():
    """Load the shared library (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_1101_3615_amd.build` (needs hipcc)")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, i, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    L.mp_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Acq), ctypes.POINTER(Opts),
                            ctypes.POINTER(vp)]
    L.mp_destroy.argtypes = [vp]
    L.mp_destroy.restype = None
    L.mp_set_background.argtypes = [vp, vp, vp]
    L.mp_footprint.argtypes = [vp, i, i, ctypes.POINTER(ctypes.c_size_t)]
    L.mp_footprint_batch.argtypes = [vp, i, i, i, ctypes.POINTER(ctypes.c_size_t)]
    L.mp_apply_batch.argtypes = [vp, i, i, i, ctypes.POINTER(ctypes.c_int), vp, vp, vp]
    L.mp_apply_H_batch.argtypes = [vp, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    for name in ("mp_apply_F", "mp_apply_Fadj", "mp_apply_H"):
        getattr(L, name).argtypes = [vp, vp, vp, vp]
    L.mp_model.argtypes = [vp, vp, vp]
    L.mp_release_cache.argtypes = [vp]
    L.mp_basis_create.argtypes = [ctypes.POINTER(BasisDesc), ctypes.POINTER(vp)]
    L.mp_basis_destroy.argtypes = [vp]
    L.mp_basis_destroy.restype = None
    L.mp_probe_fit.argtypes = [vp, vp, i, ctypes.POINTER(vp), ctypes.POINTER(vp), dp, dp, vp]
    L.mp_apply_Hinv.argtypes = [vp, vp, dp, vp, vp, vp]
    L.mp_curvelet_create.argtypes = [ctypes.POINTER(CurveletDesc), ctypes.POINTER(vp)]
    L.mp_curvelet_destroy.argtypes = [vp]
    L.mp_curvelet_destroy.restype = None
    L.mp_curvelet_wedges.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.mp_curvelet_norms.argtypes = [vp, vp, dp, vp]
    L.mp_illumination.argtypes = [vp, vp, vp, vp, vp]
    L.mp_curvelet_synthesis.argtypes = [vp, vp, vp, vp, dp, vp, vp]
    L.mp_curvelet_analysis.argtypes = [vp, vp, vp, vp, vp]
    L.mp_curvelet_sign_threshold.argtypes = [vp, vp, vp, ctypes.c_double, vp]
    L.mp_vec_dot.argtypes = [vp, ctypes.c_longlong, vp, vp, dp, vp]
    L.mp_vec_dot_noalloc.argtypes = [vp, ctypes.c_longlong, vp, vp, vp, vp]
    L.mp_vec_axpby.argtypes = [vp, ctypes.c_longlong, ctypes.c_double, vp, ctypes.c_double, vp, vp]
    L.mp_velocity_update.argtypes = [vp, vp, vp, vp]
    L.mp_last_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.mp_strerror.argtypes = [ip]
    L.mp_strerror.restype = ctypes.c_char_p
    L.mp_last_error.argtypes = []
    L.mp_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("mp_destroy", "mp_basis_destroy", "mp_curvelet_destroy", "mp_strerror", "mp_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _check_single_runtime()
    _lib = L
    return L


def check(rc):
    if rc != MP_OK:
        L = lib()
        raise MatprobeError(rc, f"{L.mp_strerror(rc).decode()}: {L.mp_last_error().decode()}")
    return rc
