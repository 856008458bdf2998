"""Host construction of the blocked edge-ADMM face tiles, checked without a
GPU against a brute-force construction (tests/edge_tiles_check.cpp, linked
against libhgeo.so): the tiles partition the faces, each region is exactly
the faces within K edge steps of its tile in ring order, and every record
names the right twin copy, the boundary or "outside", and the face's signs.
A region above the size limit is refused (also when a tile's own faces
exceed it) rather than built."""
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
    exe = str(tmp_path_factory.mktemp("tiles") / "edge_tiles_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "edge_tiles_check.cpp"), f"-L{PKG}", "-lhgeo", f"-Wl,-rpath,{PKG}",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(checker, tmp_path, v, f, rings, max_region):
    path = str(tmp_path / "mesh.bin")
    with open(path, "wb") as fp:
        np.array([v.shape[0], f.shape[0]], dtype=np.int64).tofile(fp)
        np.ascontiguousarray(v, dtype=np.float64).tofile(fp)
        np.ascontiguousarray(f, dtype=np.int32).tofile(fp)
    r = subprocess.run([checker, path, str(rings), str(max_region)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.split()


def _fan(n):
    """A disk: one centre vertex joined to n rim vertices."""
    a = 2 * np.pi * np.arange(n) / n
    v = np.vstack([[0.0, 0.0, 0.0], np.stack([np.cos(a), np.sin(a), 0 * a], 1)])
    f = np.array([[0, 1 + i, 1 + (i + 1) % n] for i in range(n)], dtype=np.int32)
    return v, f


MESHES = {
    "grid64": lambda: meshgen.config_mesh("grid64")[:2],
    "bumpy5": lambda: meshgen.config_mesh("bumpy5")[:2],
    "torus": lambda: meshgen.torus(64, 32, seed=7),
    "two_parts": lambda: meshgen.disjoint_union([meshgen.grid(24, 0.2, seed=4), meshgen.icosphere(3)])[:2],
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("rings", [1, 4, 6])
def test_regions_match_brute_force(checker, tmp_path, name, rings):
    v, f = MESHES[name]()
    out = _run(checker, tmp_path, v, f, rings, 4096)
    assert out[0] == "OK", out
    assert int(out[2]) <= 4096


def test_oversized_regions_refused(checker, tmp_path):
    v, f = MESHES["bumpy5"]()
    assert _run(checker, tmp_path, v, f, 6, 500) == ["DOES_NOT_FIT"]
    # one vertex is the smallest vertex of 200 faces: that tile's own faces
    # alone exceed a limit of 150
    v, f = _fan(200)
    assert _run(checker, tmp_path, v, f, 2, 150) == ["DOES_NOT_FIT"]
    assert _run(checker, tmp_path, v, f, 2, 4096)[0] == "OK"
