"""HIP-graph capture of the projection step (fused: reset + persistent + FP64 tail + exact-check
tail; plain: one launch per geodesic). Each graph is replayed several times with eager work and
synchronisations in between (the outputs are overwritten before every replay), and every replay
must reproduce the eager result bit for bit."""
import numpy as np
import pytest

from parity import config_inputs, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    import paper_2604_13323_amd as M
    M.lib()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return M


def blank_like(mc, r):
    return mc.ProjectResult(q=torch.empty_like(r.q), status=torch.empty_like(r.status), iters=torch.empty_like(r.iters),
                            resid=torch.empty_like(r.resid), verdict=torch.empty_like(r.verdict), geo_ok=None)


@pytest.mark.parametrize("name,variant,cond", [("c3", "fused", 1e6), ("c2", "fused", 1e6), ("c1", "fused", 0.5),
                                               ("c3", "plain", 1e6)])
def test_graph_replays_match_eager(mc, name, variant, cond):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True)
    G = mc.Problem(sc.to_blob())
    qd = to_dev(q, torch.float32)
    offs_d = torch.from_numpy(offs).cuda()
    kw = dict(tol=tol, max_iter=mi, variant=variant, cond=cond, geo_offsets=offs_d, geo_offsets_host=offs)
    ref = G.project(qd, **kw)  # eager; also sizes the work queues
    torch.cuda.synchronize()
    out = blank_like(mc, ref)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        G.project(qd, out=out, **kw)
    torch.cuda.synchronize()
    for rep in range(3):
        out.q.fill_(float("nan"))
        out.status.fill_(-1)
        out.iters.fill_(-1)
        out.verdict.fill_(7)
        G.check(ref.q)  # unrelated eager work on the same problem between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.status, ref.status), rep
        assert torch.equal(out.iters, ref.iters), rep
        assert torch.equal(out.q, ref.q), rep
        assert torch.equal(out.resid, ref.resid), rep
        assert torch.equal(out.verdict, ref.verdict), rep
