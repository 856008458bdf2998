"""Host construction of the mesh topology (build_topology: tiles, vertex and
face order, edges and their slots, signs and twins, canonical edge order,
CSR rows, halos and ELL slots), checked without a GPU by
tests/topology_check.cpp against plain restatements of each array, and the
same with one host worker thread and with several: the digests of every
array agree, and so do the messages of refused meshes."""
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
    exe = str(tmp_path_factory.mktemp("topo") / "topology_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "topology_check.cpp"), f"-L{PKG}", "-lhgeo", f"-Wl,-rpath,{PKG}",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(checker, tmp_path, v, f, threads):
    path = str(tmp_path / "mesh.bin")
    with open(path, "wb") as fp:
        np.array([v.shape[0], f.shape[0]], dtype=np.int64).tofile(fp)
        np.ascontiguousarray(v, dtype=np.float64).tofile(fp)
        np.ascontiguousarray(f, dtype=np.int32).tofile(fp)
    env = dict(os.environ, HG_HOST_THREADS=str(threads))
    r = subprocess.run([checker, path], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.strip()


def _fan(n):
    a = 2 * np.pi * np.arange(n) / n
    v = np.vstack([[0.0, 0.0, 0.0], np.stack([np.cos(a), np.sin(a), 0 * a], 1)])
    f = np.array([[0, 1 + i, 1 + (i + 1) % n] for i in range(n)], dtype=np.int32)
    return v, f


def _extra_face(v, f, fi):
    """A third face on an edge of face fi (a non-manifold edge)."""
    a, _, b = f[fi]
    v2 = np.vstack([v, v[a] + np.array([0.0, 0.0, 0.1])])
    return v2, np.vstack([f, [a, v2.shape[0] - 1, b]]).astype(np.int32)


def _flipped(f, fi):
    g = np.array(f, dtype=np.int32, copy=True)
    g[fi] = g[fi][::-1]
    return g


MESHES = {
    "bumpy6": lambda: (meshgen.harmonic_displacement(meshgen.icosphere(6)[0], seed=3), meshgen.icosphere(6)[1]),
    "grid": lambda: meshgen.grid(150, 0.2, seed=8),
    "torus": lambda: meshgen.torus(200, 100, seed=7),
    "parts": lambda: meshgen.disjoint_union([meshgen.icosphere(4), meshgen.annulus(60), meshgen.torus(40, 20)])[:2],
    # large enough for the merge rounds of the parallel sort and for every
    # per-element loop to split across workers
    "bumpy8": lambda: (meshgen.harmonic_displacement(meshgen.icosphere(8)[0], seed=3), meshgen.icosphere(8)[1]),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_topology_checks_and_thread_count(checker, tmp_path, name):
    v, f = MESHES[name]()
    one = _run(checker, tmp_path, v, f, 1)
    assert one.startswith("OK"), one
    for t in (3, 8):
        assert _run(checker, tmp_path, v, f, t) == one, t


def test_refused_meshes_same_message_for_any_thread_count(checker, tmp_path):
    v, f = meshgen.grid(150, 0.2, seed=8)
    f = np.asarray(f, dtype=np.int32)
    n = f.shape[0]
    cases = [
        (_extra_face(v, f, n - 10), "non-manifold edge"),
        ((v, _flipped(f, n - 10)), "inconsistently oriented faces"),
        # both faults: the one met first in the internal vertex order wins
        (_extra_face(v, _flipped(f, 5), n - 10), None),
        (_extra_face(v, _flipped(f, n - 10), 5), None),
        (_fan(300), "vertex valence above 255"),
    ]
    for (vv, ff), expect in cases:
        one = _run(checker, tmp_path, vv, ff, 1)
        assert one.startswith("ERROR"), one
        if expect:
            assert expect in one, one
        for t in (2, 5, 8):
            assert _run(checker, tmp_path, vv, ff, t) == one, (t, one)
