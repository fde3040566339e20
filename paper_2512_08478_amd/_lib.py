"""ctypes binding of libgs.so (argument marshalling only).

Names and argument orders mirror include/gs.h.  Loading fails loudly when
the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

GS_OK = 0
GS_ERR_INVALID_ARGUMENT = 1
GS_ERR_UNSUPPORTED = 2
GS_ERR_CAPACITY = 3
GS_ERR_HIP = 4
GS_ERR_MISALIGNED = 5
GS_ERR_WORKSPACE = 6

GS_STAGE_PREPROCESS = 0
GS_STAGE_SORT = 1
GS_STAGE_SORT_PAIRS = 2
GS_STAGE_BACKWARD = 3

SPLAT_BYTES = 48

EXPORTED = (
    "gs_version", "gs_status_string", "gs_last_hip_error", "gs_default_settings",
    "gs_workspace_size", "gs_sort_key_bits", "gs_preprocess", "gs_sort", "gs_sort_checked", "gs_sort_pairs",
    "gs_rasterize", "gs_rasterize_backward", "gs_trace_enable", "gs_trace_read",
    "gs_preprocess_assets", "gs_rasterize_backward_assets", "gs_rasterize_backward_2d",
    "gs_preprocess_backward_views", "gs_sort_pairs32", "gs_packed_sh_stride", "gs_prepack",
    "gs_preprocess_packed", "gs_rasterize_mesh", "gs_rasterize_backward_2d_mesh", "gs_lbs_deform",
    "gs_preprocess_noalloc", "gs_preprocess_noalloc_max_n", "gs_sort_plan",
    "gs_raster_grid", "gs_raster_unit",
    "gs_batch_create", "gs_batch_destroy", "gs_batch_pixels", "gs_batch_pixel_offset",
    "gs_batch_capacity", "gs_batch_workspace_size", "gs_batch_plan", "gs_batch_run",
    "gs_batch_capture", "gs_batch_launch", "gs_autotune",
)
BWD_VIEWS_PER_LAUNCH = 8
GRAD2D_STRIDE = 12  # floats per Gaussian in a 2-D gradient record
MAX_ASSETS = 64


class GsLibraryMissing(RuntimeError):
    pass


class GsError(RuntimeError):
    def __init__(self, status, what, hip_error=0):
        self.status = status
        self.hip_error = hip_error
        msg = f"{what}: {status_string(status)} (status {status}"
        if status == GS_ERR_HIP:
            msg += f", hipError {hip_error}"
        super().__init__(msg + ")")


class GsSortPass(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_int32), ("digit_bits", ctypes.c_int32), ("keys", ctypes.c_int32),
                ("partition_keys", ctypes.c_int32), ("grid_partitions", ctypes.c_int32)]


GS_PASS_KEYS_ALL, GS_PASS_KEYS_VISIBLE, GS_PASS_KEYS_INSTANCES = 0, 1, 2


class GsBatchDesc(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("cams", ctypes.c_void_p), ("n_assets", ctypes.c_int32),
                ("assets", ctypes.c_void_p), ("n", ctypes.c_int64), ("means", ctypes.c_void_p),
                ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity_logits", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("sh_degree", ctypes.c_int32), ("targets", ctypes.c_void_p)]


class GsAutotuneSpace(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("tiles", ctypes.c_int32 * 32),
                ("n_bits", ctypes.c_int32), ("bits", ctypes.c_int32 * 8),
                ("n_modes", ctypes.c_int32), ("modes", ctypes.c_int32 * 2),
                ("n_orders", ctypes.c_int32), ("orders", ctypes.c_int32 * 6)]


class GsCamera(ctypes.Structure):
    _fields_ = [("viewmat", ctypes.c_float * 16), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("znear", ctypes.c_float), ("reserved", ctypes.c_float)]


class GsSettings(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("eps2d", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("t_eps", ctypes.c_float), ("clip", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("radix_bits", ctypes.c_int32), ("sort_mode", ctypes.c_int32),
                ("raster_order", ctypes.c_int32), ("depth_bits", ctypes.c_int32)]


class GsAsset(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("count", ctypes.c_int64),
                ("model", ctypes.POINTER(ctypes.c_float))]


def asset_table(assets):
    """ctypes array of GsAsset from [(offset, count, model 3x4 or None)].
    Returns (array, keep-alive list of model buffers)."""
    arr = (GsAsset * max(1, len(assets)))()
    keep = []
    for a, (off, cnt, model) in enumerate(assets):
        arr[a].offset = int(off)
        arr[a].count = int(cnt)
        if model is not None:
            m = model_array(model)
            keep.append(m)
            arr[a].model = ctypes.cast(m, ctypes.POINTER(ctypes.c_float))
    return arr, keep


_lib = None


def load():
    """Load libgs.so (built in-tree by paper_2512_08478_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GsLibraryMissing(
            f"{LIB_PATH} is missing; build it with `python -m paper_2512_08478_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    CAM, SET = ctypes.POINTER(GsCamera), ctypes.POINTER(GsSettings)
    lib.gs_version.restype = ctypes.c_char_p
    lib.gs_version.argtypes = []
    lib.gs_status_string.restype = ctypes.c_char_p
    lib.gs_status_string.argtypes = [I32]
    lib.gs_last_hip_error.restype = I32
    lib.gs_last_hip_error.argtypes = []
    lib.gs_default_settings.restype = None
    lib.gs_default_settings.argtypes = [SET]
    lib.gs_workspace_size.restype = SZ
    lib.gs_workspace_size.argtypes = [I32, I64, I64, CAM, SET]
    lib.gs_sort_key_bits.restype = I32
    lib.gs_sort_key_bits.argtypes = [CAM, SET]
    lib.gs_preprocess.restype = I32
    lib.gs_preprocess.argtypes = [I64, P, P, P, P, P, I32, P, CAM, SET, P, P, P, P, P, SZ, P]
    lib.gs_preprocess_noalloc.restype = I32
    lib.gs_preprocess_noalloc.argtypes = [I64, P, P, P, P, P, I32, P, CAM, SET, P, P, P, P, P]
    lib.gs_batch_create.restype = I32
    lib.gs_batch_create.argtypes = [P, SET, P]
    lib.gs_batch_destroy.restype = None
    lib.gs_batch_destroy.argtypes = [P]
    for nm in ("gs_batch_pixels", "gs_batch_capacity"):
        getattr(lib, nm).restype = I64
        getattr(lib, nm).argtypes = [P]
    lib.gs_batch_pixel_offset.restype = I64
    lib.gs_batch_pixel_offset.argtypes = [P, I32]
    lib.gs_batch_workspace_size.restype = SZ
    lib.gs_batch_workspace_size.argtypes = [P, I64]
    lib.gs_batch_plan.restype = I32
    lib.gs_batch_plan.argtypes = [P, ctypes.c_float, P, SZ, P, P]
    for nm in ("gs_batch_run", "gs_batch_capture"):
        getattr(lib, nm).restype = I32
        getattr(lib, nm).argtypes = [P, P, SZ, P, P, P, P, P, P, P, P]
    lib.gs_batch_launch.restype = I32
    lib.gs_batch_launch.argtypes = [P, P]
    lib.gs_autotune.restype = I32
    lib.gs_autotune.argtypes = [P, SET, P, I32, ctypes.c_float, P, SZ, P, P, P, P, P, P, P, SET,
                                P, P, P]
    lib.gs_sort_plan.restype = I32
    lib.gs_sort_plan.argtypes = [I64, I64, CAM, SET, I32, P, P, P]
    lib.gs_raster_grid.restype = I64
    lib.gs_raster_grid.argtypes = [CAM, SET, I32]
    lib.gs_raster_unit.restype = I32
    lib.gs_raster_unit.argtypes = [CAM, SET, I32, P, I64, P]
    lib.gs_preprocess_noalloc_max_n.restype = I64
    lib.gs_preprocess_noalloc_max_n.argtypes = []
    lib.gs_sort.restype = I32
    lib.gs_sort.argtypes = [I64, P, P, P, P, CAM, SET, I64, P, P, P, P, P, SZ, P]
    lib.gs_sort_checked.restype = I32
    lib.gs_sort_checked.argtypes = [I64, P, P, P, P, CAM, SET, I64, P, P, P, P, P, SZ,
                                    ctypes.POINTER(I64), P]
    lib.gs_sort_pairs.restype = I32
    lib.gs_sort_pairs.argtypes = [I64, P, P, I32, P, P, SET, P, SZ, P]
    lib.gs_sort_pairs32.restype = I32
    lib.gs_sort_pairs32.argtypes = [I64, P, P, I32, P, P, SET, P, SZ, P]
    lib.gs_rasterize.restype = I32
    lib.gs_rasterize.argtypes = [P, P, P, CAM, SET, P, P, P, P, P]
    lib.gs_rasterize_backward.restype = I32
    lib.gs_rasterize_backward.argtypes = [I64, P, P, P, P, P, I32, P, CAM, SET, P, P, P, P, P, P,
                                          P, P, P, P, P, I32, P, SZ, P]
    AS = ctypes.POINTER(GsAsset)
    lib.gs_preprocess_assets.restype = I32
    lib.gs_preprocess_assets.argtypes = [I32, AS, I64, P, P, P, P, P, I32, CAM, SET, P, P, P, P,
                                         P, SZ, P]
    lib.gs_rasterize_backward_assets.restype = I32
    lib.gs_rasterize_backward_assets.argtypes = [I32, AS, I64, P, P, P, P, P, I32, CAM, SET, P, P,
                                                 P, P, P, P, P, P, P, P, P, I32, P, SZ, P]
    lib.gs_rasterize_backward_2d.restype = I32
    lib.gs_rasterize_backward_2d.argtypes = [P, P, P, CAM, SET, P, P, P, I64, P, P]
    lib.gs_preprocess_backward_views.restype = I32
    lib.gs_preprocess_backward_views.argtypes = [I32, CAM, ctypes.POINTER(ctypes.c_void_p), I32, AS,
                                                 I64, P, P, P, P, P, I32, SET, P, P, P, P, P, I32,
                                                 P]
    lib.gs_packed_sh_stride.restype = I32
    lib.gs_packed_sh_stride.argtypes = [I32]
    lib.gs_prepack.restype = I32
    lib.gs_prepack.argtypes = [I64, P, P, P, P, P, I32, P, P, P, P]
    lib.gs_preprocess_packed.restype = I32
    lib.gs_preprocess_packed.argtypes = [I32, AS, I64, P, P, P, I32, CAM, SET, P, P, P, P, P, SZ, P]
    lib.gs_rasterize_mesh.restype = I32
    lib.gs_rasterize_mesh.argtypes = [P, P, P, CAM, SET, P, P, P, P, P, P, P]
    lib.gs_rasterize_backward_2d_mesh.restype = I32
    lib.gs_rasterize_backward_2d_mesh.argtypes = [P, P, P, CAM, SET, P, P, P, P, I64, P, P]
    lib.gs_lbs_deform.restype = I32
    lib.gs_lbs_deform.argtypes = [I64, P, P, P, P, I32, P, P, P, P]
    lib.gs_trace_enable.restype = I32
    lib.gs_trace_enable.argtypes = [I32]
    lib.gs_trace_read.restype = I32
    lib.gs_trace_read.argtypes = [I32, P, P, P]
    _lib = lib
    return lib


def trace_enable(on: bool):
    check(load().gs_trace_enable(1 if on else 0), "gs_trace_enable")


def trace_read(max_entries: int = 512):
    """[(label, ms)] recorded since the last read (waits for the GPU)."""
    lib = load()
    labels = ctypes.create_string_buffer(32 * max_entries)
    ms = (ctypes.c_float * max_entries)()
    cnt = ctypes.c_int32(0)
    check(lib.gs_trace_read(max_entries, labels, ms, ctypes.byref(cnt)), "gs_trace_read")
    raw = labels.raw
    return [(raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode(), float(ms[i]))
            for i in range(cnt.value)]


def packed_sh_stride(sh_degree: int) -> int:
    """Halves per packed SH row (4, 12, 28, 48 for degrees 0..3)."""
    S = load().gs_packed_sh_stride(int(sh_degree))
    if S < 0:
        raise GsError(GS_ERR_UNSUPPORTED, "gs_packed_sh_stride")
    return S


def status_string(status: int) -> str:
    return load().gs_status_string(int(status)).decode()


def check(status: int, what: str):
    if status != GS_OK:
        raise GsError(status, what, load().gs_last_hip_error() if status == GS_ERR_HIP else 0)


def default_settings(**overrides) -> GsSettings:
    s = GsSettings()
    load().gs_default_settings(ctypes.byref(s))
    for k, v in overrides.items():
        if k == "bg":
            for i in range(3):
                s.bg[i] = float(v[i])
        else:
            setattr(s, k, v)
    return s


def make_camera(cam) -> GsCamera:
    """GsCamera from any object with viewmat (4x4), fx, fy, cx, cy, width,
    height, znear."""
    c = GsCamera()
    vm = [float(x) for row in cam.viewmat for x in row] if hasattr(cam.viewmat[0], "__len__") \
        else [float(x) for x in cam.viewmat]
    for i in range(16):
        c.viewmat[i] = vm[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def model_array(model):
    """Host float[12] for a 3x4 model transform, or None."""
    if model is None:
        return None
    flat = [float(x) for row in model for x in row] if hasattr(model[0], "__len__") \
        else [float(x) for x in model]
    if len(flat) != 12:
        raise ValueError("model transform must be 3x4")
    return (ctypes.c_float * 12)(*flat)


def sort_plan(n, capacity, cam, settings, max_passes=32):
    """gs_sort_plan: (list of pass dicts, look-back words)."""
    lib = load()
    c = make_camera(cam)
    out = (GsSortPass * max_passes)()
    cnt = ctypes.c_int32(0)
    words = ctypes.c_int64(0)
    check(lib.gs_sort_plan(n, capacity, ctypes.byref(c), ctypes.byref(settings), max_passes, out,
                           ctypes.byref(cnt), ctypes.byref(words)), "gs_sort_plan")
    return ([dict(index=o.pass_, digit_bits=o.digit_bits, keys=o.keys, partition_keys=o.partition_keys,
                  grid_partitions=o.grid_partitions) for o in out[:cnt.value]], words.value)
