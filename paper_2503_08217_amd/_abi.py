"""ctypes mirror of include/s3r.h and the loader of libs3r.so.

Argument marshalling only: every computation happens in the HIP library.  If
the library has not been built the import of the renderer fails loudly; there
is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libs3r.so")

S3R_OK = 0
S3R_E_NULL, S3R_E_ALIGN, S3R_E_SIZE, S3R_E_WORKSPACE, S3R_E_HIP, S3R_E_ARG = -1, -2, -3, -4, -5, -6
S3R_E_SCRATCH = -7
S3R_TEMPORAL, S3R_LOD, S3R_PLAIN, S3R_LOD_STOCHASTIC, S3R_GRAD_SPARSE = 1, 2, 4, 8, 16
S3R_SORT_TILES = 32
S3R_DETERMINISTIC_GRADS = 64
S3R_VIS_UPDATE, S3R_VIS_FOLD, S3R_VIS_RESET = 0, 1, 2
S3R_WS_PROJECT, S3R_WS_SORT, S3R_WS_BACKWARD = 0, 1, 2
S3R_TUNE_OFFSET_FUSE_MAX, S3R_TUNE_SCAN_FUSE_MAX, S3R_TUNE_BIN_MAX_TILES = 0, 1, 2
S3R_TUNE_RASTER_WAVES, S3R_TUNE_FINE_TILES = 3, 4
TUNE_KNOBS = {"offset_fuse_max": S3R_TUNE_OFFSET_FUSE_MAX, "scan_fuse_max": S3R_TUNE_SCAN_FUSE_MAX,
              "bin_max_tiles": S3R_TUNE_BIN_MAX_TILES, "raster_waves": S3R_TUNE_RASTER_WAVES,
              "fine_tiles": S3R_TUNE_FINE_TILES}
CNT_SURV, CNT_OVF_SURV, CNT_DUP, CNT_OVF_DUP, CNT_SPIN, CNT_PAIRS = 0, 1, 2, 3, 4, 7
BSTAT = 8  # ints per (256-Gaussian block, view) entry of S3RProjected.bstat

P = C.c_void_p


class S3RParams(C.Structure):
    _fields_ = [("tile", C.c_int32), ("flags", C.c_uint32), ("lod_r", C.c_float),
                ("z_near", C.c_float), ("z_far", C.c_float), ("eps2d", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("cutoff", C.c_float), ("jac_clamp", C.c_float), ("bg", C.c_float * 3),
                ("cap_surv", C.c_int64), ("cap_dup", C.c_int64), ("seed", C.c_uint64),
                ("lod_pmax", C.c_float), ("lod_D", C.c_float), ("step", C.c_uint32),
                ("pad_", C.c_uint32)]


class S3RScene(C.Structure):
    _fields_ = [("mean", P), ("scale", P), ("quat", P), ("opacity", P), ("sh", P), ("inst", P),
                ("vis_s", P), ("vis_e", P), ("pose", P), ("mean_w", P), ("rot_w", P),
                ("n", C.c_int64), ("sh_degree", C.c_int32), ("n_slots", C.c_int32),
                ("n_timesteps", C.c_int32), ("pad_", C.c_int32)]


class S3RViews(C.Structure):
    _fields_ = [("W", P), ("K", P), ("wh", P), ("tstep", P), ("tile_offset", P),
                ("px_offset", P), ("plain_slot", P), ("n_views", C.c_int32),
                ("total_tiles", C.c_int32), ("total_px", C.c_int64)]


class S3RProjected(C.Structure):
    _fields_ = [("cam", P), ("cen", P), ("t_norm", P), ("mask", P), ("rec_gid", P),
                ("rec_view", P), ("rec_geo", P), ("rec_conic", P), ("rec_rgb", P),
                ("rec_rect", P), ("counters", P), ("stats", P), ("rec_npairs", P), ("surv", P),
                ("bstat", P), ("rec_pair", P)]


class S3RBins(C.Structure):
    _fields_ = [("tile_count", P), ("tile_start", P), ("vals", P), ("tile_order", P)]


class S3RImage(C.Structure):
    _fields_ = [("color", P), ("T_final", P), ("last", P), ("m_raster", P), ("rec_taken", P),
                ("n", C.c_int64), ("census", P)]


class S3RGrads(C.Structure):
    _fields_ = [("mean", P), ("scale", P), ("quat", P), ("opacity", P), ("sh", P), ("pose", P),
                ("pose6", P), ("mean_w", P), ("rot_w", P), ("rows", P), ("n_rows", P)]


class S3RSizes(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_views", C.c_int32), ("total_tiles", C.c_int32),
                ("cap_surv", C.c_int64), ("cap_dup", C.c_int64), ("n_slots", C.c_int32),
                ("pad_", C.c_int32)]


SIGNATURES = {
    "s3r_abi_version": ([], C.c_int),
    "s3r_set_tuning": ([C.c_int32, C.c_int32], C.c_int),
    "s3r_get_tuning": ([C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "s3r_status_string": ([C.c_int], C.c_char_p),
    "s3r_workspace_size": ([C.POINTER(S3RSizes), C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "s3r_project_cull": ([C.POINTER(S3RScene), C.POINTER(S3RViews), C.POINTER(S3RParams),
                          C.POINTER(S3RProjected), P, C.c_size_t, P], C.c_int),
    "s3r_project_cull_noalloc": ([C.POINTER(S3RScene), C.POINTER(S3RViews), C.POINTER(S3RParams),
                                  C.POINTER(S3RProjected), P], C.c_int),
    "s3r_sort": ([C.POINTER(S3RScene), C.POINTER(S3RProjected), C.POINTER(S3RViews),
                  C.POINTER(S3RParams), C.POINTER(S3RBins), P, C.c_size_t, P], C.c_int),
    "s3r_raster_fwd": ([C.POINTER(S3RProjected), C.POINTER(S3RBins), C.POINTER(S3RViews),
                        C.POINTER(S3RParams), C.POINTER(S3RImage), P], C.c_int),
    "s3r_l1_loss": ([C.POINTER(S3RImage), P, C.POINTER(S3RViews), P, P, P], C.c_int),
    "s3r_raster_bwd": ([C.POINTER(S3RScene), C.POINTER(S3RViews), C.POINTER(S3RParams),
                        C.POINTER(S3RProjected), C.POINTER(S3RBins), C.POINTER(S3RImage), P,
                        C.POINTER(S3RGrads), P, C.c_size_t, P], C.c_int),
    "s3r_update_visibility": ([P, P, P, P, P, P, C.c_int32, C.c_int64, C.c_int32, C.c_float, P],
                              C.c_int),
    "s3r_plain_transform": ([C.POINTER(S3RScene), C.POINTER(C.c_int32), C.c_int32, P, P, P],
                            C.c_int),
    "s3r_plain_transform_bwd": ([C.POINTER(S3RScene), C.POINTER(C.c_int32), C.c_int32,
                                 C.POINTER(S3RGrads), P], C.c_int),
    "s3r_profile_enable": ([C.c_int], C.c_int),
    "s3r_profile_reset": ([], C.c_int),
    "s3r_profile_only": ([C.c_int32], C.c_int),
    "s3r_profile_read": ([C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "s3r_profile_name": ([C.c_int32], C.c_char_p),
    "s3r_profile_kernels": ([], C.c_int),
}


def profile_id(name):
    lib = load()
    for i in range(lib.s3r_profile_kernels()):
        if lib.s3r_profile_name(i).decode() == name:
            return i
    raise KeyError(name)


def profile_table():
    """{kernel name: (total ms, launches)} since the last reset."""
    lib = load()
    out = {}
    for i in range(lib.s3r_profile_kernels()):
        ms, n = C.c_double(0), C.c_int64(0)
        check(lib.s3r_profile_read(i, C.byref(ms), C.byref(n)), "s3r_profile_read")
        if n.value:
            out[lib.s3r_profile_name(i).decode()] = (ms.value, n.value)
    return out

_LIB = None


def load(path: str = LIB_PATH):
    """Load libs3r.so (once) and declare every entry point."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2503_08217_amd.build` "
            "(there is no non-HIP fallback)")
    lib = C.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


class S3RError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != S3R_OK:
        msg = load().s3r_status_string(rc).decode()
        raise S3RError(f"{what} failed with status {rc}: {msg}")


def set_tuning(**knobs):
    """Set launch-shape knobs by name (TUNE_KNOBS; a negative value restores
    the default).  Returns the previous values."""
    lib = load()
    old = {}
    for name, value in knobs.items():
        k = TUNE_KNOBS[name]
        cur = C.c_int32(0)
        check(lib.s3r_get_tuning(k, C.byref(cur)), "s3r_get_tuning")
        old[name] = cur.value
        check(lib.s3r_set_tuning(k, int(value)), f"s3r_set_tuning({name}={value})")
    return old


def get_tuning():
    lib = load()
    out = {}
    for name, k in TUNE_KNOBS.items():
        cur = C.c_int32(0)
        check(lib.s3r_get_tuning(k, C.byref(cur)), "s3r_get_tuning")
        out[name] = cur.value
    return out
