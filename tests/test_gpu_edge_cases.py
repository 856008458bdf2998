"""Degenerate and boundary cases of the whole solve, against the oracle:

  * a component without a source: +inf there, the rest as on its own;
  * the smallest meshes: one triangle, two triangles;
  * every vertex a source: d = 0 everywhere (with the source paths);
  * a vertex of valence 24 (a fan): the tiled diffusion does not take
    valences above 16, the solve falls back to global sweeps;
  * invalid source lists are refused before any device work.
"""
import numpy as np
import pytest

import meshgen
from oracle import metrics, pipeline

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


def _fan(n=24, jitter=0.1, seed=5):
    """A disk: a centre vertex joined to n rim vertices, then a second ring
    of 2n vertices, counter-clockwise triangles."""
    rng = np.random.default_rng(seed)
    a = 2 * np.pi * (np.arange(n) + rng.uniform(-jitter, jitter, n)) / n
    b = 2 * np.pi * (np.arange(2 * n) + 0.5 + rng.uniform(-jitter, jitter, 2 * n)) / (2 * n)
    v = np.vstack([[0.0, 0.0, 0.0], np.stack([np.cos(a), np.sin(a), 0 * a], 1),
                   2.0 * np.stack([np.cos(b), np.sin(b), 0 * b], 1)])
    f = [[0, 1 + i, 1 + (i + 1) % n] for i in range(n)]
    for i in range(n):
        r0, r1 = 1 + i, 1 + (i + 1) % n
        o0, o1, o2 = 1 + n + 2 * i, 1 + n + 2 * i + 1, 1 + n + (2 * i + 2) % (2 * n)
        f += [[r0, o0, o1], [r0, o1, r1], [r1, o1, o2]]
    return v, np.array(f, dtype=np.int32)


@pytest.mark.parametrize("form", ["edge", "face"])
def test_component_without_source(hg, form):
    (va, fa), (vb, fb) = meshgen.grid(20, 0.2, seed=4), meshgen.grid(16, 0.2, seed=5)
    v, f, st = meshgen.disjoint_union([(va, fa), (vb, fb)])
    s = [57]
    m = hg.Mesh(v, f)
    try:
        d, info = m.solve(s, 0.0, hg.default_opts(formulation=form, t_per_component=1))
    finally:
        m.close()
    d = d.cpu().numpy()
    assert np.all(np.isinf(d[st[1]:])) and np.all(np.isfinite(d[:st[1]]))
    ref = pipeline.heat_method(va, fa, s, form=form)
    mean, mx = metrics.parity(d[:st[1]], ref.d)
    _say("unreached component", form, mean, mx)
    assert mean <= 1e-4 and mx <= 1e-3


@pytest.mark.parametrize("form", ["edge", "face"])
@pytest.mark.parametrize("case", ["one_triangle", "two_triangles"])
def test_smallest_meshes(hg, form, case):
    if case == "one_triangle":
        v = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.9, 0.2]])
        f = np.array([[0, 1, 2]], dtype=np.int32)
    else:
        v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.1], [0.1, 1.0, 0.0], [1.1, 1.0, 0.3]])
        f = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    m = hg.Mesh(v, f)
    try:
        d, info = m.solve([0], 0.0, hg.default_opts(formulation=form))
    finally:
        m.close()
    d = d.cpu().numpy()
    ref = pipeline.heat_method(v, f, [0], form=form)
    _say(case, form, d.tolist(), ref.d.tolist())
    assert d[0] == 0.0 and np.abs(d - ref.d).max() <= 1e-4 * ref.d.max()


def test_every_vertex_a_source(hg):
    v, f = meshgen.grid(8, 0.2, seed=3)
    m = hg.Mesh(v, f)
    try:
        d, info = m.solve(np.arange(v.shape[0], dtype=np.int32), 0.0, hg.default_opts())
    finally:
        m.close()
    assert info.n_paths == v.shape[0] - 1
    assert np.all(d.cpu().numpy() == 0.0)


@pytest.mark.parametrize("form", ["edge", "face"])
def test_high_valence_falls_back_to_global_sweeps(hg, form):
    v, f = _fan(24)
    m = hg.Mesh(v, f)
    try:
        assert m.stats["max_valence"] == 24
        d, info = m.solve([0], 0.0, hg.default_opts(formulation=form))
        d2, _ = m.solve([1], 0.0, hg.default_opts(formulation=form))
    finally:
        m.close()
    for s, dd in ((0, d), (1, d2)):
        ref = pipeline.heat_method(v, f, [s], form=form)
        mean, mx = metrics.parity(dd.cpu().numpy(), ref.d)
        _say("fan valence 24", form, s, mean, mx)
        assert mean <= 1e-4 and mx <= 1e-3
    assert info.passes == info.sweeps     # the global schedule: one sweep per pass


def test_invalid_sources_refused(hg):
    v, f = meshgen.grid(6, 0.1, seed=2)
    m = hg.Mesh(v, f)
    try:
        with pytest.raises(RuntimeError):
            m.solve([v.shape[0]], 0.0, hg.default_opts())
        with pytest.raises(RuntimeError):
            m.solve([-1], 0.0, hg.default_opts())
        with pytest.raises(RuntimeError):
            m.solve(np.zeros(0, dtype=np.int32), 0.0, hg.default_opts())
        d, _ = m.solve([3], 0.0, hg.default_opts())      # the mesh still works
        assert d.cpu().numpy()[3] == 0.0
    finally:
        m.close()
