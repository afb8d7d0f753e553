"""project_batch_noalloc (the allocation-free entry point) against project_batch through the C ABI:
identical outputs on two calls in a row, the second with a smaller batch, in a scene whose
obstacles are within reach (the exact-check queue is used) and with every configuration sent to
the FP64 continuation queue (cond below 1), both queues living in the library's scratch array;
and the size limit is an argument error raised before anything is enqueued."""
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


FIELDS = ("q", "status", "iters", "resid", "verdict", "geo_ok")


def same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        if x is None and y is None:
            continue
        assert torch.equal(x, y), f


@pytest.mark.parametrize("dt,cond", [(torch.float32, 1e6), (torch.float32, 0.5), (torch.float64, 1e6)])
def test_noalloc_matches_project_batch_on_two_calls(mc, dt, cond):
    sc, P, q, offs, tol, mi = config_inputs("c3near", small=True)
    G = mc.Problem(sc.to_blob())
    q1 = to_dev(q, dt)                       # 1,024 configurations, 32 geodesics
    q2 = to_dev(q[:517], dt)                 # a smaller, ragged batch next
    offs_d = torch.from_numpy(offs).cuda()
    for qq, oo in ((q1, offs_d), (q2, None)):
        kw = dict(tol=tol, max_iter=mi, cond=cond)
        if oo is not None:
            kw.update(geo_offsets=oo, geo_ok=True)
        ref = G.project(qq, **kw)
        na = G.project(qq, noalloc=True, **kw)
        torch.cuda.synchronize()
        same(ref, na)
        v = na.verdict[na.status == 0]
        assert (v == 1).any() and (v == 0).any()  # the exact check ran on both kinds
    if cond < 1:
        assert G.fallback_count() > 0


def test_noalloc_rejects_batches_beyond_its_scratch(mc):
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True, max_geo=1)
    G = mc.Problem(sc.to_blob())
    limit = (64 * 2 ** 20 - 1024) // (16 * 36 + 12)
    big = torch.zeros((36, limit + 1), dtype=torch.float32, device="cuda")
    with pytest.raises(mc.McError, match="scratch capacity"):
        G.project(big, noalloc=True)
    # at the limit it runs (every column at the origin of the configuration space)
    r = G.project(big[:, :limit], noalloc=True, max_iter=1, check=False)
    torch.cuda.synchronize()
    assert r.status.shape[0] == limit
