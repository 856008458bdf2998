"""Host construction of the overlapping diffusion tiles, checked without a
GPU against a brute-force construction (tests/overlap_tiles_check.cpp,
linked against libhgeo.so): the overlap vertices and the fixed ring of each
tile are exactly the vertices at hop distance 1..rings and rings + 1 from
its core, every ELL row decodes to the vertex's neighbours in CSR order, and
no tile reads the core of a tile of its own colour.  A tile whose rings
would exceed the overlap limit gets fewer rings, and only then."""
import os
import subprocess

import numpy as np
import pytest

import meshgen
from paper_1812_06060_amd import _hgeo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1812_06060_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    if not os.path.exists(_hgeo.LIB_PATH):
        from paper_1812_06060_amd import build
        build.build(verbose=False)
    exe = str(tmp_path_factory.mktemp("otiles") / "overlap_tiles_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "overlap_tiles_check.cpp"), f"-L{PKG}", "-lhgeo", f"-Wl,-rpath,{PKG}",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(checker, tmp_path, v, f, rings, max_ov):
    path = str(tmp_path / "mesh.bin")
    with open(path, "wb") as fp:
        np.array([v.shape[0], f.shape[0]], dtype=np.int64).tofile(fp)
        np.ascontiguousarray(v, dtype=np.float64).tofile(fp)
        np.ascontiguousarray(f, dtype=np.int32).tofile(fp)
    r = subprocess.run([checker, path, str(rings), str(max_ov)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.split()


MESHES = {
    "grid64": lambda: meshgen.config_mesh("grid64")[:2],
    "bumpy6": lambda: meshgen.config_mesh("bumpy6")[:2],
    "torus": lambda: meshgen.torus(64, 32, seed=7),
    "two_parts": lambda: meshgen.disjoint_union([meshgen.grid(24, 0.2, seed=4), meshgen.icosphere(3)])[:2],
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("rings", [0, 1, 2, 4])
def test_overlap_tiles_match_brute_force(checker, tmp_path, name, rings):
    v, f = MESHES[name]()
    out = _run(checker, tmp_path, v, f, rings, 1024)
    assert out[0] == "OK", out
    assert int(out[2]) <= 1024
    if rings == 0:
        assert int(out[2]) == 0


def test_rings_cut_per_tile_to_fit(checker, tmp_path):
    """With at most 100 overlap vertices allowed, tiles get fewer rings
    (only where the next ring would exceed the limit), never a refusal."""
    v, f = MESHES["bumpy6"]()
    out = _run(checker, tmp_path, v, f, 4, 100)
    assert out[0] == "OK", out
    assert int(out[2]) <= 100 and int(out[4]) > 0
