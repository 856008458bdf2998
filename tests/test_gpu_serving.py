"""The serving runtime (hg_server_*): queries run concurrently on worker slots
with private workspaces give exactly the result of the same query run alone
with hg_geodesic_solve, whatever else runs beside them and however memory
admission orders them; timestamps are consistent; one query is also checked
against the oracle."""
import numpy as np
import pytest

import meshgen
from oracle import metrics, pipeline

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06060_amd as hg
    hg.load_library()
    meshes = {}
    for name in ("bumpy4", "sphere5", "grid64", "bumpy5"):
        v, f, _ = meshgen.config_mesh(name)
        meshes[name] = (v, f, hg.Mesh(v, f))
    rng = np.random.default_rng(11)
    queries = []
    for i in range(16):
        name = ("bumpy4", "sphere5", "grid64", "bumpy5")[i % 4]
        nv = meshes[name][0].shape[0]
        k = int(rng.integers(1, 6))
        src = rng.choice(nv, size=k, replace=False).astype(np.int32)
        form = "edge" if i % 3 else "face"
        queries.append((name, src, form))
    alone = []
    for name, src, form in queries:
        d, info = meshes[name][2].solve(src, 0.0, hg.default_opts(formulation=form))
        alone.append(d.cpu().numpy())
    yield hg, meshes, queries, alone
    for _, _, m in meshes.values():
        m.close()


def _run_server(hg, meshes, queries, n_slots, budget):
    srv = hg.Server(n_slots, budget)
    tickets = {}
    for i, (name, src, form) in enumerate(queries):
        tk, _ = srv.submit(meshes[name][2], src, opts=hg.default_opts(formulation=form))
        tickets[tk] = i
    results = {}
    while len(results) < len(queries):
        r = srv.wait(60000)
        assert r is not None, "server stalled"
        results[tickets[r["ticket"]]] = r
    st = srv.stats()
    srv.close()
    return results, st


@pytest.mark.parametrize("n_slots, budget", [(4, 0), (3, 1), (2, 8 << 20)])
def test_results_same_alone_and_in_the_mix(setup, n_slots, budget):
    hg, meshes, queries, alone = setup
    _say("server slots", n_slots, "budget", budget)
    results, st = _run_server(hg, meshes, queries, n_slots, budget)
    _say("stats", st)
    for i, r in results.items():
        assert r["status"] == 0, (i, r["status"])
        assert r["t_submit"] <= r["t_start"] <= r["t_end"]
        assert r["info"].converged_u and r["info"].converged_admm
        assert np.array_equal(r["out"].cpu().numpy(), alone[i]), i
    assert st["pending"] == 0 and st["running"] == 0
    if budget == 1:
        # only one workspace can be held: every query ran alone
        assert st["workspaces_idle"] == 1


def test_served_result_matches_oracle(setup):
    hg, meshes, queries, alone = setup
    name, src, form = queries[1]
    v, f, mesh = meshes[name]
    _say("oracle", name, form, src.tolist())
    ref = pipeline.heat_method(v, f, src, form=form)
    srv = hg.Server(2)
    srv.submit(mesh, src, opts=hg.default_opts(formulation=form))
    r = srv.wait(60000)
    srv.close()
    mean, mx = metrics.parity(r["out"].cpu().numpy(), ref.d)
    assert mean <= 1e-4 and mx <= 1e-3
