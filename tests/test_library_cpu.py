"""The C-ABI library loads, exports every symbol include/hgeo.h declares, its
structs match the binding, and host-side validation errors come back as
status codes -- all without a GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1812_06060_amd import _hgeo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgeo.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_hgeo.LIB_PATH):
        from paper_1812_06060_amd import build
        build.build(verbose=False)
    return _hgeo.load_library()


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_hgeo.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", _hgeo.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "hgeo.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(hg_opts), sizeof(hg_info),'
                   ' sizeof(hg_mesh_stats), offsetof(hg_info, bytes_alg), offsetof(hg_opts, mu),'
                   ' sizeof(hg_result), offsetof(hg_result, info), sizeof(hg_server_stats_t),'
                   ' sizeof(hg_tune_report), offsetof(hg_tune_report, admm_us_per_iteration));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [C.sizeof(_hgeo.Opts), C.sizeof(_hgeo.Info), C.sizeof(_hgeo.MeshStats),
                   _hgeo.Info.bytes_alg.offset, _hgeo.Opts.mu.offset, C.sizeof(_hgeo.Result),
                   _hgeo.Result.info.offset, C.sizeof(_hgeo.ServerStats), C.sizeof(_hgeo.TuneReport),
                   _hgeo.TuneReport.admm_us_per_iteration.offset]


def test_defaults(lib):
    o = _hgeo.Opts()
    assert lib.hg_opts_default(C.byref(o)) == 0
    assert o.formulation == _hgeo.FORM_EDGE and o.mu == 0.0 and o.relax == 1.9 and o.m == 1.0
    assert o.source_paths == 1
    assert o.cycle_constraints == 1
    assert lib.hg_opts_default(None) == _hgeo.HG_E_INVALID_ARG


def _create(lib, v, f):
    v = np.ascontiguousarray(v, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.int32)
    h = C.c_void_p()
    st = lib.hg_mesh_create(v.ctypes.data_as(C.c_void_p), v.shape[0], f.ctypes.data_as(C.c_void_p),
                            f.shape[0], None, C.byref(h))
    return st, lib.hg_last_error().decode()


@pytest.mark.parametrize("tris, what", [
    ([[0, 1, 5]], "out of range"),
    ([[0, 1, 1]], "repeats"),
    ([[0, 1, 2], [0, 1, 3]], "inconsistent"),
    ([[0, 1, 2], [1, 0, 3], [0, 1, 4]], "non-manifold"),
])
def test_bad_meshes_rejected_before_any_device_work(lib, tris, what):
    v = np.random.default_rng(0).standard_normal((5, 3))
    st, msg = _create(lib, v, tris)
    assert st == _hgeo.HG_E_BAD_MESH and what in msg


@pytest.mark.parametrize("tris, what", [
    ([[0, 1, 5]], "out of range"),
    ([[0, 1, 1]], "repeats"),
    ([[0, 1, 2], [0, 1, 3]], "inconsistent"),
    ([[0, 1, 2], [1, 0, 3], [0, 1, 4]], "non-manifold"),
])
def test_bad_meshes_rejected_by_intrinsic_build(lib, tris, what):
    """The host edge-flip build validates its input before any device work."""
    v = np.random.default_rng(0).standard_normal((5, 3))
    f = np.ascontiguousarray(np.asarray(tris, dtype=np.int32))
    h = C.c_void_p()
    st = lib.hg_mesh_create_intrinsic(v.ctypes.data_as(C.c_void_p), v.shape[0], f.ctypes.data_as(C.c_void_p),
                                      f.shape[0], None, C.byref(h))
    assert st == _hgeo.HG_E_BAD_MESH and what in lib.hg_last_error().decode()


def test_mesh_readback_rejects_null_arguments(lib):
    buf_i = (C.c_int32 * 4)()
    buf_f = (C.c_float * 4)()
    buf_d = (C.c_double * 4)()
    assert lib.hg_mesh_cycles(None, _hgeo.FORM_EDGE, buf_i, buf_i, buf_f, 4) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_mesh_intrinsic(None, buf_i, buf_d) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_mesh_weights(None, buf_d, buf_d, None) == _hgeo.HG_E_INVALID_ARG


def test_null_and_empty_arguments(lib):
    h = C.c_void_p()
    assert lib.hg_mesh_create(None, 3, None, 1, None, C.byref(h)) == _hgeo.HG_E_INVALID_ARG
    v = np.zeros((3, 3))
    f = np.zeros((0, 3), dtype=np.int32)
    st, msg = _create(lib, v, f)
    assert st == _hgeo.HG_E_INVALID_ARG and "empty" in msg
    st, msg = _create(lib, np.full((3, 3), np.nan), [[0, 1, 2]])
    assert st == _hgeo.HG_E_INVALID_ARG


def test_server_rejects_null_arguments(lib):
    assert lib.hg_server_create(0, 0, C.byref(C.c_void_p())) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_server_create(4, 0, None) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_server_submit(None, None, None, 1, 0.0, None, None, None) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_server_wait(None, None, 0) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_server_stats(None, None) == _hgeo.HG_E_INVALID_ARG
    lib.hg_server_destroy(None)
    assert lib.hg_server_clock() > 0.0


def test_autotune_rejects_null_mesh(lib):
    assert lib.hg_mesh_autotune(None, None, 0, 0.0, None, None, None) == _hgeo.HG_E_INVALID_ARG


def test_batch_and_size_calls_reject_null_arguments(lib):
    """hg_geodesic_solve_batch, hg_mesh_bytes, hg_query_bytes and
    hg_bfs_noalloc refuse NULL or empty arguments before any device work."""
    one = (C.c_int32 * 1)(1)
    meshes = (C.c_void_p * 1)(None)
    srcs = (C.c_void_p * 1)(None)
    outs = (C.c_void_p * 1)(None)
    assert lib.hg_geodesic_solve_batch(None, 1, srcs, one, 0.0, None, outs, None, None) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_geodesic_solve_batch(meshes, 0, srcs, one, 0.0, None, outs, None, None) == _hgeo.HG_E_INVALID_ARG
    assert lib.hg_geodesic_solve_batch(meshes, 1, srcs, one, 0.0, None, outs, None, None) == _hgeo.HG_E_INVALID_ARG
    assert "batch query 0" in lib.hg_last_error().decode()
    assert lib.hg_mesh_bytes(None) == 0
    assert lib.hg_query_bytes(None, 1, None) == 0
    assert lib.hg_bfs_noalloc(None, one, 1, None, None, None, None) == _hgeo.HG_E_INVALID_ARG
