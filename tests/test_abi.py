"""The C-ABI library loads, exports every entry point of include/s3r.h, and
rejects bad arguments on the host with the documented status codes (no GPU
work is issued on these paths)."""

import ctypes as C
import os
import re

import pytest

from paper_2503_08217_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "s3r.h")


def header_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(s3r_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.fail("libs3r.so is not built (run __graft_entry__.build())")
    return A.load()


def test_every_header_symbol_is_exported(lib):
    syms = header_symbols()
    assert len(syms) >= 16
    for s in syms:
        assert hasattr(lib, s), s
        assert s in A.SIGNATURES, s


def test_version_and_status(lib):
    assert lib.s3r_abi_version() == 2
    assert lib.s3r_status_string(0) == b"ok"
    assert b"aligned" in lib.s3r_status_string(-2)


def test_struct_sizes_match_c_layout():
    assert C.sizeof(A.S3RParams) == 96
    assert C.sizeof(A.S3RScene) == 11 * 8 + 8 + 16
    assert C.sizeof(A.S3RViews) == 7 * 8 + 16
    assert C.sizeof(A.S3RProjected) == 16 * 8
    assert C.sizeof(A.S3RBins) == 4 * 8
    assert C.sizeof(A.S3RGrads) == 11 * 8
    assert C.sizeof(A.S3RImage) == 7 * 8
    assert C.sizeof(A.S3RSizes) == 40


def test_workspace_sizes(lib):
    z = A.S3RSizes(2_000_000, 1, 8160, 400_000, 2_000_000, 31, 0)
    got = {}
    for w in (0, 1, 2):
        nb = C.c_size_t(0)
        assert lib.s3r_workspace_size(C.byref(z), w, C.byref(nb)) == 0
        got[w] = nb.value
    assert got[1] >= 16 * 2_000_000         # two key buffers
    assert got[2] >= 48 * 400_000           # per-record 2D gradients
    nb = C.c_size_t(0)
    assert lib.s3r_workspace_size(C.byref(z), 7, C.byref(nb)) == -6
    bad = A.S3RSizes(10, 0, 1, 1, 1, 1, 0)
    assert lib.s3r_workspace_size(C.byref(bad), 0, C.byref(nb)) == -3


def _params(**kw):
    p = dict(tile=16, flags=0, lod_r=0.0, z_near=0.2, z_far=1e30, eps2d=0.3,
             alpha_min=1 / 255, alpha_max=0.99, t_min=1e-4, cutoff=4.5, jac_clamp=1.3)
    p.update(kw)
    return A.S3RParams(p["tile"], p["flags"], p["lod_r"], p["z_near"], p["z_far"], p["eps2d"],
                       p["alpha_min"], p["alpha_max"], p["t_min"], p["cutoff"], p["jac_clamp"],
                       (C.c_float * 3)(0, 0, 0), p.get("cap_surv", 16), p.get("cap_dup", 64))


def test_host_validation_codes(lib):
    buf = (C.c_float * 64)()
    base = C.addressof(buf)
    al = base + (16 - base % 16) % 16
    ptr = C.c_void_p(al)
    scene = A.S3RScene(*([ptr] * 9), C.c_void_p(0), C.c_void_p(0), 4, 0, 1, 1, 0)
    views = A.S3RViews(*([ptr] * 6), C.c_void_p(0), 1, 1, 64)
    proj = A.S3RProjected(*([ptr] * 16))
    p = _params()
    ws = C.c_void_p(al)
    # NULL scene
    assert lib.s3r_project_cull(None, C.byref(views), C.byref(p), C.byref(proj), ws, 1 << 20,
                                None) == -1
    # bad tile size
    p_bad = _params(tile=12)
    assert lib.s3r_project_cull(C.byref(scene), C.byref(views), C.byref(p_bad), C.byref(proj),
                                ws, 1 << 20, None) == -3
    # misaligned array
    scene_mis = A.S3RScene(C.c_void_p(al + 4), *([ptr] * 8), C.c_void_p(0), C.c_void_p(0),
                           4, 0, 1, 1, 0)
    assert lib.s3r_project_cull(C.byref(scene_mis), C.byref(views), C.byref(p), C.byref(proj),
                                ws, 1 << 20, None) == -2
    # SH degree out of range
    scene_deg = A.S3RScene(*([ptr] * 9), C.c_void_p(0), C.c_void_p(0), 4, 5, 1, 1, 0)
    assert lib.s3r_project_cull(C.byref(scene_deg), C.byref(views), C.byref(p), C.byref(proj),
                                ws, 1 << 20, None) == -3
    # workspace too small
    assert lib.s3r_project_cull(C.byref(scene), C.byref(views), C.byref(p), C.byref(proj), ws,
                                8, None) == -4
    # plain route without world-frame arrays
    p_plain = _params(flags=A.S3R_PLAIN)
    assert lib.s3r_project_cull(C.byref(scene), C.byref(views), C.byref(p_plain), C.byref(proj),
                                ws, 1 << 20, None) == -1
    # too many views
    views_many = A.S3RViews(*([ptr] * 6), C.c_void_p(0), 65, 1, 64)
    assert lib.s3r_project_cull(C.byref(scene), C.byref(views_many), C.byref(p), C.byref(proj),
                                ws, 1 << 20, None) == -3
    # visibility: bad mode, NULL mask for UPDATE
    assert lib.s3r_update_visibility(ptr, ptr, ptr, ptr, ptr, ptr, 1, 10, 9, 0.1, None) == -6
    assert lib.s3r_update_visibility(ptr, ptr, ptr, ptr, None, ptr, 1, 10, 0, 0.1, None) == -1
    # plain transform: timestep out of range
    ts = (C.c_int32 * 1)(5)
    assert lib.s3r_plain_transform(C.byref(scene), ts, 1, ptr, ptr, None) == -6


def test_noalloc_rejects_problem_beyond_its_scratch(lib):
    """s3r_project_cull_noalloc refuses, on the host and before anything is
    enqueued, a problem whose projection workspace exceeds its fixed 4 MiB
    scratch (60M Gaussians x 64 views), and validates arguments like
    s3r_project_cull."""
    buf = (C.c_float * 64)()
    base = C.addressof(buf)
    al = base + (16 - base % 16) % 16
    ptr = C.c_void_p(al)
    views = A.S3RViews(*([ptr] * 6), C.c_void_p(0), 64, 1, 64)
    proj = A.S3RProjected(*([ptr] * 16))
    p = _params()
    big = A.S3RScene(*([ptr] * 9), C.c_void_p(0), C.c_void_p(0), 60_000_000, 0, 1, 1, 0)
    z = A.S3RSizes(60_000_000, 64, 1, 16, 64, 1, 0)
    nb = C.c_size_t(0)
    assert lib.s3r_workspace_size(C.byref(z), A.S3R_WS_PROJECT, C.byref(nb)) == 0
    assert nb.value > 4 << 20
    assert lib.s3r_project_cull_noalloc(C.byref(big), C.byref(views), C.byref(p), C.byref(proj),
                                        None) == A.S3R_E_SCRATCH
    assert b"scratch" in lib.s3r_status_string(A.S3R_E_SCRATCH)
    assert lib.s3r_project_cull_noalloc(None, C.byref(views), C.byref(p), C.byref(proj),
                                        None) == A.S3R_E_NULL
    p_bad = _params(tile=12)
    assert lib.s3r_project_cull_noalloc(C.byref(big), C.byref(views), C.byref(p_bad),
                                        C.byref(proj), None) == A.S3R_E_SIZE


def test_tuning_knobs(lib):
    """Launch-shape knobs: defaults, range checks, restore with a negative
    value (host-side state only)."""
    v = C.c_int32(-1)
    assert lib.s3r_get_tuning(A.S3R_TUNE_BIN_MAX_TILES, C.byref(v)) == 0 and v.value == 12288
    assert lib.s3r_get_tuning(A.S3R_TUNE_RASTER_WAVES, C.byref(v)) == 0 and v.value == 1
    assert lib.s3r_set_tuning(99, 1) == A.S3R_E_ARG
    assert lib.s3r_get_tuning(99, C.byref(v)) == A.S3R_E_ARG
    assert lib.s3r_set_tuning(A.S3R_TUNE_BIN_MAX_TILES, 12289) == A.S3R_E_ARG
    assert lib.s3r_set_tuning(A.S3R_TUNE_RASTER_WAVES, 0) == A.S3R_E_ARG
    assert lib.s3r_set_tuning(A.S3R_TUNE_FINE_TILES, (1 << 20) + 1) == A.S3R_E_ARG
    assert lib.s3r_get_tuning(A.S3R_TUNE_FINE_TILES, C.byref(v)) == 0 and v.value == 160
    old = A.set_tuning(offset_fuse_max=0, bin_max_tiles=0, raster_waves=4)
    assert old == {"offset_fuse_max": 1024, "bin_max_tiles": 12288, "raster_waves": 1}
    assert A.get_tuning()["raster_waves"] == 4
    A.set_tuning(offset_fuse_max=-1, bin_max_tiles=-1, raster_waves=-1)
    assert A.get_tuning() == {"offset_fuse_max": 1024, "scan_fuse_max": 1024,
                              "bin_max_tiles": 12288, "raster_waves": 1, "fine_tiles": 160}
