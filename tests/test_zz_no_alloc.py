"""hg_bfs_noalloc (the breadth-first search on the library's fixed device
array, no device allocation inside the call) against hg_bfs: levels,
pairing and depth bit-exact, on two calls in a row, the second on a smaller
mesh, so that a value left in the shared array by the first call would show;
and the size limits refused with HG_E_INVALID_ARG before anything runs."""
import ctypes as C

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def hg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06060_amd as hg
    hg.load_library()
    return hg


def _check_same(hg, mesh, sources):
    lev_ref, par_ref, depth_ref = mesh.bfs(sources)
    lev = torch.full((mesh.nv,), 12345, dtype=torch.int32, device="cuda")
    par = torch.full((mesh.nv,), 12345, dtype=torch.int32, device="cuda")
    _, _, depth = mesh.bfs_noalloc(sources, level=lev, parent=par)
    torch.cuda.synchronize()
    assert depth == depth_ref
    assert torch.equal(lev, lev_ref)
    assert torch.equal(par, par_ref)
    return depth


def test_noalloc_bfs_equals_bfs_on_two_calls_in_a_row(hg):
    v1, f1 = meshgen.icosphere(6)
    v1 = meshgen.harmonic_displacement(v1, seed=3)
    v2, f2 = meshgen.icosphere(4)
    v2 = meshgen.harmonic_displacement(v2, seed=5)
    big = hg.Mesh(v1, f1)
    small = hg.Mesh(v2, f2)
    try:
        _say("noalloc bfs: level 6, 3 sources")
        d1 = _check_same(hg, big, meshgen.random_sources(big.nv, 3, seed=1))
        _say("noalloc bfs: level 4, 1 source (after the larger call)")
        d2 = _check_same(hg, small, [7])
        assert d2 < d1
        _say("noalloc bfs: level 6 again, 64 sources")
        _check_same(hg, big, meshgen.random_sources(big.nv, 64, seed=2))
    finally:
        big.close()
        small.close()


def test_noalloc_bfs_refuses_sizes_beyond_its_limit(hg):
    v, f = meshgen.icosphere(3)
    mesh = hg.Mesh(v, f)
    try:
        lib = hg._hgeo._lib
        lev = torch.empty(mesh.nv, dtype=torch.int32, device="cuda")
        src = np.zeros(65537, dtype=np.int32)
        depth = C.c_int32(-7)
        _say("noalloc bfs: 65537 sources (refused)")
        st = lib.hg_bfs_noalloc(mesh._h, src.ctypes.data, src.size, C.c_void_p(lev.data_ptr()), None, None,
                                C.byref(depth))
        assert st == 1
        assert b"65536" in lib.hg_last_error()
        assert depth.value == -7
        one = np.array([mesh.nv], dtype=np.int32)
        st = lib.hg_bfs_noalloc(mesh._h, one.ctypes.data, 1, C.c_void_p(lev.data_ptr()), None, None, None)
        assert st == 1
    finally:
        mesh.close()
