"""Graph-captured launches (opts.use_graphs) give exactly the result of
plain launches: repeated solves replay the captured runs, with other device
work on the null stream in between, on the null stream (the solve then runs
on its workspace's own stream) and on an explicit stream, single- and
multi-source, both forms."""
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


CASES = {
    "bumpy4_1src": lambda: meshgen.config_mesh("bumpy4"),
    "bumpy4_5src": lambda: (*meshgen.config_mesh("bumpy4")[:2], meshgen.random_sources(2562, 5, seed=7)),
    "grid64": lambda: meshgen.config_mesh("grid64"),
}


@pytest.mark.parametrize("form", ["edge", "face"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_graph_replays_equal_plain_launches(hg, case, form):
    v, f, src = CASES[case]()
    _say("graphs", case, form)
    mesh = hg.Mesh(v, f)
    try:
        ref, ri = mesh.solve(src, 0.0, hg.default_opts(formulation=form, use_graphs=0))
        ref = ref.cpu().numpy()
        side = torch.cuda.Stream()
        for rep in range(3):
            junk = torch.arange(1 << 20, device="cuda", dtype=torch.float32).sum()   # other null-stream work
            d, info = mesh.solve(src, 0.0, hg.default_opts(formulation=form))
            torch.cuda.synchronize()
            assert info.admm_iters == ri.admm_iters and info.passes == ri.passes
            assert np.array_equal(d.cpu().numpy(), ref), (case, form, rep)
            with torch.cuda.stream(side):
                d2, _ = mesh.solve(src, 0.0, hg.default_opts(formulation=form), stream=side)
            side.synchronize()
            assert np.array_equal(d2.cpu().numpy(), ref), (case, form, rep, "stream")
            del junk
    finally:
        mesh.close()
