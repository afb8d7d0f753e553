"""GPU parity of project_vjp_exact (the exact derivative of the projection map at off-manifold inputs)
against the FP64 oracle's forward-mode derivative of the same map, against central finite
differences of the oracle's converged projection, and against closed forms (the sphere's
(I - q^ q^T) / ||q0||, the linear constraint's I - A^+ A). The GPU takes the output cotangent
through the tangent projector at its last iterate, so against the oracle's map converged to 1e-13
it is exact up to O(tol) plus the central differences of its Hessian-vector products (~1e-9
relative): the FP64 checks project to tol 1e-10 and ask for 1e-6 (2e-7 on the sphere); the FP32
checks run at the benchmark's tol 1e-6 and ask for 1e-4 (1e-5 on the sphere)."""
import numpy as np
import pytest

from parity import CONV, config_inputs, from_dev, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    import paper_2604_13323_amd as M
    M.lib()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return M


def rel_err(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def gpu_exact(G, q, g, dt, tol=1e-6, max_iter=50, **kw):
    qd = to_dev(q, dt)
    r = G.project(qd, tol=tol, max_iter=max_iter, check=False, **kw)
    gi = G.vjp_exact(qd, r.status, r.iters, to_dev(g, dt), alpha=kw.get("alpha", 1.0), lam=kw.get("lam", 0.0))
    torch.cuda.synchronize()
    return from_dev(gi).T, from_dev(r.status).astype(int), from_dev(r.iters).astype(int), r


@pytest.mark.parametrize("dt,rtol,tol", [(torch.float64, 2e-7, 1e-10), (torch.float32, 1e-5, 1e-6)])
def test_sphere_closed_form_off_manifold(mc, dt, rtol, tol):
    from paper_2604_13323_amd import scenes as S
    G = mc.Problem(S.sphere_scene(0).to_blob())
    rng = np.random.default_rng(31)
    u = rng.standard_normal((256, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q0 = u * rng.uniform(0.05, 4.0, (256, 1))
    g = rng.standard_normal(q0.shape)
    gi, st, it, _ = gpu_exact(G, q0, g, dt, tol=tol)
    assert (st == CONV).all() and (it > 0).all()
    r = np.linalg.norm(q0, axis=1, keepdims=True)
    want = (g - u * np.sum(u * g, axis=1, keepdims=True)) / r
    assert rel_err(gi, want).max() < rtol, rel_err(gi, want).max()


def test_linear_exact_projector_from_anywhere(mc):
    from paper_2604_13323_amd import scenes as S
    rng = np.random.default_rng(32)
    for m, d in ((2, 5), (6, 8)):
        A = rng.standard_normal((m, d))
        b = rng.standard_normal(m)
        G = mc.Problem(S.linear_scene(A, b).to_blob())
        q0 = 3.0 * rng.standard_normal((70, d))
        g = rng.standard_normal(q0.shape)
        gi, st, it, _ = gpu_exact(G, q0, g, torch.float64, tol=1e-9)
        Pr = np.eye(d) - np.linalg.pinv(A) @ A
        np.testing.assert_allclose(gi, g @ Pr.T, atol=1e-9)


@pytest.mark.parametrize("name", ["c3", "c4"])
@pytest.mark.parametrize("dt,rtol,ftol", [(torch.float64, 1e-6, 1e-10), (torch.float32, 1e-4, None)])
def test_humanoid_matches_oracle_exact_derivative(mc, name, dt, rtol, ftol):
    """The humanoid batches' raw interpolants (off the manifold, 1-3 Newton steps each)."""
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=2)
    G = mc.Problem(sc.to_blob())
    rng = np.random.default_rng(33)
    g = rng.standard_normal(q.shape)
    gi, st, it, r = gpu_exact(G, q, g, dt, tol=ftol or tol, max_iter=60 if ftol else mi)
    qin = from_dev(to_dev(q, dt)).T  # the inputs the GPU saw
    go, sto = P.vjp_exact(qin, g.astype(np.float32).astype(np.float64) if dt == torch.float32 else g)
    ok = (st == CONV) & (sto == CONV)
    assert ok.mean() > 0.95 and (it[ok] > 0).mean() > 0.9
    e = rel_err(gi[ok], go[ok])
    assert e.max() < rtol, e.max()
    # the tangent projector at the output is a different (first-order) answer off the manifold: its
    # median gap to the exact derivative on these inputs is ~1e-3
    gt = from_dev(G.vjp(r.q, r.status, to_dev(g, dt))).T
    assert np.median(rel_err(gt[ok], go[ok])) > 5 * rtol


def test_c4_against_fp64_central_differences(mc):
    """The differentiation batch's check at its own (off-manifold) inputs: FP64 central differences
    (h = 1e-6) of the oracle's projection converged to ||F|| < 1e-13, on configurations sampled from
    the converged ones (stream 3), relative error below 1e-3 in FP32 mode."""
    sc, P, q, offs, tol, mi = config_inputs("c4", small=True)
    G = mc.Problem(sc.to_blob())
    rng = np.random.default_rng([4, 3])
    idx = rng.choice(len(q), size=64, replace=False)
    q0 = q[idx]
    g = rng.standard_normal(q0.shape)
    gi, st, it, _ = gpu_exact(G, q0, g, torch.float32, tol=tol, max_iter=mi)
    q0 = from_dev(to_dev(q0, torch.float32)).T
    h, d = 1e-6, sc.d
    qp = np.repeat(q0, d, axis=0) + h * np.tile(np.eye(d), (len(q0), 1))
    qm = np.repeat(q0, d, axis=0) - h * np.tile(np.eye(d), (len(q0), 1))
    pp, sp, _, _ = P.project(qp, tol=1e-13, max_iter=100)
    pm, sm, _, _ = P.project(qm, tol=1e-13, max_iter=100)
    assert (sp == CONV).all() and (sm == CONV).all() and (st == CONV).all()
    dP = ((pp - pm) / (2 * h)).reshape(len(q0), d, d)
    g_fd = np.einsum("nij,nj->ni", dP, g.astype(np.float32).astype(np.float64))
    e = rel_err(gi, g_fd)
    assert e.max() < 1e-3, e.max()


def test_on_the_manifold_equals_the_tangent_projector(mc):
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True, max_geo=2)
    qs = P.project(q, tol=1e-12, max_iter=60)[0]
    G = mc.Problem(sc.to_blob())
    g = np.random.default_rng(34).standard_normal(qs.shape)
    qd = to_dev(qs, torch.float64)
    r = G.project(qd, tol=1e-6, max_iter=40, check=False)
    gi = G.vjp_exact(qd, r.status, r.iters, to_dev(g, torch.float64))
    gt = G.vjp(r.q, r.status, to_dev(g, torch.float64))
    torch.cuda.synchronize()
    assert (from_dev(r.iters) == 0).all()
    np.testing.assert_allclose(from_dev(gi), from_dev(gt), atol=1e-6)


def test_autograd_exact_option(mc):
    sc, P, q, offs, tol, mi = config_inputs("c4", small=True, max_geo=1)
    G = mc.Problem(sc.to_blob())
    q0 = to_dev(q, torch.float64).requires_grad_(True)
    qp, st = mc.project(q0, G, tol=tol, max_iter=mi, exact=True)
    w = torch.randn_like(qp)
    (qp * w).sum().backward()
    r = G.project(q0.detach(), tol=tol, max_iter=mi)
    gi = G.vjp_exact(q0.detach(), r.status, r.iters, w)
    torch.cuda.synchronize()
    assert torch.allclose(q0.grad, gi)
