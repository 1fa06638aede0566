"""Steps captured in a HIP graph (through torch.cuda.graph) and replayed: the
launch-bound 800-site shock tube advanced by graph replays equals the same
steps launched one by one, replay after replay, with other GPU work and
synchronisations between the replays."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(precision):
    from paper_1703_04605_amd import rlbm
    from tests.helpers import to_dev
    st = workloads.STENCILS["zeta1"]
    fields, tau = workloads.riemann_1d(800)
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=1, precision=precision)
    s.init_fields(*to_dev(fields), bc=("outflow", "periodic"), tau=tau)
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_equal_eager_steps(precision):
    import torch
    eager = _solver(precision)
    graph = _solver(precision)
    eager.step(1)
    graph.step(1)           # every captured step then pulls from streamed populations
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graph.step(20)      # recorded, not run: 20 kernel nodes, an even count
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        eager.step(20)
        a = {k: v.cpu().numpy() for k, v in graph.moments(raw=True).items()}
        b = {k: v.cpu().numpy() for k, v in eager.moments(raw=True).items()}
        torch.cuda.synchronize()
        for k in ("n", "eps", "T", "ux", "raw9"):
            assert np.array_equal(a[k], b[k]), (r, k)
        assert np.abs(b["ux"]).max() > 0.01
    assert graph.health()["flags"] == 0
