"""ctypes declarations of the C ABI in include/isogs.h (argument marshalling only).

The shared library is built in-tree (``paper_2403_14244_amd/libisogs.so``, see build.py);
importing this module without it raises ImportError: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisogs.so")

ISOGS_OK = 0
ISOGS_ERR_INVALID = -1
ISOGS_ERR_CAPACITY = -2
ISOGS_ERR_WORKSPACE = -3
ISOGS_ERR_DEVICE = -4

ISOGS_FWD_WIDE = 1
ISOGS_FWD_TIMES = 2
ISOGS_STATIC_SCRATCH_BYTES = 128 << 20

EXPORTED = ("isogs_project", "isogs_bin_sort", "isogs_bin_sort_static", "isogs_render_fwd", "isogs_render_fwd_ordered",
            "isogs_render_bwd", "isogs_checkpoint_bytes", "isogs_field2d_bin", "isogs_field2d_fwd",
            "isogs_field2d_bwd", "isogs_field2d_tree_init", "isogs_field2d_prune", "isogs_field2d_split",
            "isogs_ssim_fwd", "isogs_ssim_bwd", "isogs_l1_fwd", "isogs_l1_bwd", "isogs_aniso_project",
            "isogs_aniso_render_fwd", "isogs_aniso_render_bwd", "isogs_loss_fwd", "isogs_loss_bwd",
            "isogs_field2d_merge", "isogs_octree_init", "isogs_field2d_aniso_bin", "isogs_field2d_aniso_fwd",
            "isogs_field2d_aniso_bwd", "isogs_stream_create", "isogs_stream_destroy", "isogs_last_error",
            "isogs_version")


class Scene(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("opacity", ctypes.c_void_p),
                ("color", ctypes.c_void_p), ("n", ctypes.c_int32), ("sh_degree", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("eye", ctypes.c_float * 3),
                ("f", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("near_z", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Projected(ctypes.Structure):
    _fields_ = [("record", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("tile_count", ctypes.c_void_p)]


class AnisoScene(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("rot", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("color", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32)]


class AnisoProjected(ctypes.Structure):
    _fields_ = [("fp", Projected), ("conic", ctypes.c_void_p)]


class Bins(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("pidx", ctypes.c_void_p), ("ranges", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("count", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class Field2D(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("amp", ctypes.c_void_p),
                ("K", ctypes.c_int32)]


class Field2DAniso(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("theta", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("amp", ctypes.c_void_p), ("K", ctypes.c_int32)]


class OctreeGrid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 3), ("root_side", ctypes.c_float), ("roots", ctypes.c_int32 * 3),
                ("levels", ctypes.c_int32)]


class IsoGSError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"isogs error {code}: {message}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch has loaded, so one
        # process never holds two copies of the runtime
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2403_14244_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.isogs_project.argtypes = [P(Scene), P(Camera), ctypes.c_int32, P(Projected), vp]
        L.isogs_bin_sort.argtypes = [P(Projected), P(ctypes.c_int32), P(Camera), ctypes.c_int32, P(Bins), vp,
                                     P(ctypes.c_size_t), vp]
        L.isogs_bin_sort_static.argtypes = [P(Projected), P(ctypes.c_int32), P(Camera), ctypes.c_int32, P(Bins),
                                            vp]
        L.isogs_render_fwd.argtypes = [P(Projected), P(ctypes.c_int32), P(Bins), P(Camera), ctypes.c_int32,
                                       P(ctypes.c_float), vp, vp, vp, vp, vp]
        L.isogs_render_fwd_ordered.argtypes = [P(Projected), P(ctypes.c_int32), P(Bins), P(Camera),
                                               ctypes.c_int32, P(ctypes.c_float), vp, vp, vp, vp, ctypes.c_uint32,
                                               vp, P(ctypes.c_size_t), vp]
        L.isogs_render_bwd.argtypes = [P(Scene), P(Camera), ctypes.c_int32, P(Projected), P(Bins),
                                       P(ctypes.c_float), vp, vp, vp, vp, vp, P(Scene), vp, P(ctypes.c_size_t), vp]
        L.isogs_aniso_project.argtypes = [P(AnisoScene), P(Camera), ctypes.c_int32, P(AnisoProjected), vp]
        L.isogs_aniso_render_fwd.argtypes = [P(AnisoProjected), P(ctypes.c_int32), P(Bins), P(Camera),
                                             ctypes.c_int32, P(ctypes.c_float), vp, vp, vp, vp, ctypes.c_uint32,
                                             vp, P(ctypes.c_size_t), vp]
        L.isogs_aniso_render_bwd.argtypes = [P(AnisoScene), P(Camera), ctypes.c_int32, P(AnisoProjected), P(Bins),
                                             P(ctypes.c_float), vp, vp, vp, vp, vp, P(AnisoScene), vp,
                                             P(ctypes.c_size_t), vp]
        L.isogs_field2d_bin.argtypes = [P(Field2D), ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P(Projected),
                                        P(Bins), vp, P(ctypes.c_size_t), vp]
        L.isogs_field2d_fwd.argtypes = [P(Projected), ctypes.c_int32, P(Bins), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_float, vp, vp]
        L.isogs_field2d_bwd.argtypes = [P(Projected), ctypes.c_int32, P(Bins), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_float, vp, P(Field2D), vp, P(ctypes.c_size_t), vp]
        L.isogs_field2d_tree_init.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, ctypes.c_int32, P(Field2D), vp, vp, P(ctypes.c_size_t),
                                              vp]
        for name in ("isogs_field2d_prune", "isogs_field2d_split"):
            getattr(L, name).argtypes = [P(Field2D), ctypes.c_float, P(Field2D), vp, vp, P(ctypes.c_size_t), vp]
        L.isogs_l1_fwd.argtypes = [vp, vp, ctypes.c_int64, vp, vp, P(ctypes.c_size_t), vp]
        L.isogs_l1_bwd.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
        L.isogs_ssim_fwd.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                     P(ctypes.c_size_t), vp]
        L.isogs_ssim_bwd.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_size_t,
                                     vp, vp]
        L.isogs_loss_fwd.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, vp, vp,
                                     P(ctypes.c_size_t), vp]
        L.isogs_loss_bwd.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, vp, vp,
                                     ctypes.c_size_t, vp, vp]
        L.isogs_field2d_merge.argtypes = [P(Field2D), ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                          P(Field2D), vp, vp, P(ctypes.c_size_t), vp]
        L.isogs_octree_init.argtypes = [vp, vp, ctypes.c_int32, P(OctreeGrid), ctypes.c_float, ctypes.c_int32,
                                        ctypes.c_float, P(Scene), vp, vp, P(ctypes.c_size_t), vp]
        L.isogs_field2d_aniso_bin.argtypes = [P(Field2DAniso), ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                              P(Projected), vp, P(Bins), vp, P(ctypes.c_size_t), vp]
        L.isogs_field2d_aniso_fwd.argtypes = [P(Projected), vp, ctypes.c_int32, P(Bins), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, vp, vp]
        L.isogs_field2d_aniso_bwd.argtypes = [P(Field2DAniso), P(Projected), vp, P(Bins), ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_float, vp, P(Field2DAniso), vp,
                                              P(ctypes.c_size_t), vp]
        L.isogs_stream_create.argtypes = [P(ctypes.c_void_p)]
        L.isogs_stream_destroy.argtypes = [vp]
        L.isogs_checkpoint_bytes.argtypes = [ctypes.c_uint64]
        L.isogs_checkpoint_bytes.restype = ctypes.c_size_t
        for name in ("isogs_project", "isogs_bin_sort", "isogs_bin_sort_static", "isogs_render_fwd", "isogs_render_fwd_ordered",
                     "isogs_render_bwd", "isogs_field2d_bin", "isogs_field2d_fwd", "isogs_field2d_bwd",
                     "isogs_ssim_fwd", "isogs_ssim_bwd", "isogs_field2d_tree_init", "isogs_field2d_prune",
                     "isogs_field2d_split", "isogs_l1_fwd", "isogs_l1_bwd", "isogs_aniso_project",
                     "isogs_aniso_render_fwd", "isogs_aniso_render_bwd", "isogs_loss_fwd", "isogs_loss_bwd",
                     "isogs_field2d_merge", "isogs_octree_init", "isogs_field2d_aniso_bin",
                     "isogs_field2d_aniso_fwd", "isogs_field2d_aniso_bwd"):
            getattr(L, name).restype = ctypes.c_int
        L.isogs_last_error.restype = ctypes.c_char_p
        L.isogs_last_error.argtypes = []
        L.isogs_version.restype = ctypes.c_char_p
        L.isogs_version.argtypes = []
        _lib = L
    return _lib


def check(rc):
    if rc != ISOGS_OK:
        raise IsoGSError(rc, lib().isogs_last_error().decode())
    return rc


def camera_struct(cam) -> Camera:
    """Any object with R (3x3), t, eye, f, cx, cy, width, height and optionally near."""
    c = Camera()
    R = [float(x) for row in cam.R for x in row]
    c.R[:] = R
    c.t[:] = [float(x) for x in cam.t]
    c.eye[:] = [float(x) for x in cam.eye]
    c.f = float(cam.f)
    c.cx = float(cam.cx)
    c.cy = float(cam.cy)
    c.near_z = float(getattr(cam, "near", 0.2))
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
    return arr


def int_array(vals):
    arr = (ctypes.c_int32 * len(vals))()
    arr[:] = [int(v) for v in vals]
    return arr
