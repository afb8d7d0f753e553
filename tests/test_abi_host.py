"""Host-side checks that need no GPU: the C-ABI library loads and exports every function that
include/mcproj.h declares, host-side argument validation returns the documented errors before
any device work, the input generator is deterministic, and the FLOP model is consistent with
the scenes' structure."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcproj.h")

MC_OK, MC_ERR_INVALID_ARG, MC_ERR_UNSUPPORTED = 0, 1, 2


@pytest.fixture(scope="module")
def L():
    from paper_2604_13323_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build(force=False)
    return binding.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("project_batch", "check_batch", "project_vjp", "mc_problem_create", "mc_problem_destroy",
              "mc_last_error", "mc_default_opts", "interpolate_geodesics", "path_length_grad",
              "mc_eval_residual_jacobian", "mc_fallback_count", "extend_batch", "mc_eval_condition",
              "mc_queue_counts", "mc_autotune_candidates", "mc_autotune_project", "mc_tuned_shape"):
        assert n in names, n


def test_library_exports_every_declared_symbol(L):
    from paper_2604_13323_amd import binding
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if " T " in line)
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared in mcproj.h but not exported: {missing}"


def test_default_options(L):
    from paper_2604_13323_amd import binding
    o = binding.Opts()
    L.mc_default_opts(ctypes.byref(o))
    assert o.dtype == 0 and o.tol == 1e-6 and o.max_iter == 50 and o.alpha == 1.0 and o.lambda_ == 0.0
    assert o.max_step == 0.0 and o.fp64_cond_threshold == 1e6 and o.check_collision == 1 and o.variant == 0
    assert o.mode == 0 and o.lanes_per_config == 0 and o.waves_per_block == 0 and o.blocks_per_cu == 0


def test_autotune_candidates_and_host_errors(L):
    from paper_2604_13323_amd import binding
    n = L.mc_autotune_candidates(None)
    shapes = (binding.LaunchShape * n)()
    assert L.mc_autotune_candidates(shapes) == n and n >= 7
    assert all(s.waves_per_block in (1, 2, 4) and s.lanes_per_config == 1 and s.check_lanes == 0 for s in shapes)
    out = binding.LaunchShape()
    assert L.mc_tuned_shape(None, 0, 0, ctypes.byref(out)) == MC_ERR_INVALID_ARG
    assert L.mc_queue_counts(None, (ctypes.c_uint32 * 4)()) == MC_ERR_INVALID_ARG
    assert L.mc_eval_condition(None, 1, None, 1, 0, 0.0, None, None) == MC_ERR_INVALID_ARG
    o = binding.Opts()
    L.mc_default_opts(ctypes.byref(o))
    assert L.mc_autotune_project(None, 1, None, 1, ctypes.byref(o), 1, None, None, None) == MC_ERR_INVALID_ARG
    assert L.mc_set_check_lanes(None, 4) == MC_ERR_INVALID_ARG


def test_create_rejects_malformed_blobs_on_the_host(L):
    from paper_2604_13323_amd import scenes as S
    h = ctypes.c_void_p()
    assert L.mc_problem_create(None, 0, ctypes.byref(h)) == MC_ERR_INVALID_ARG
    assert b"null" in L.mc_last_error() or len(L.mc_last_error()) > 0
    blob = bytearray(S.sphere_scene(0).to_blob())
    bad = bytes(blob)
    bad = b"XXXX" + bad[4:]
    assert L.mc_problem_create(bad, len(bad), ctypes.byref(h)) == MC_ERR_INVALID_ARG
    assert L.mc_problem_create(bytes(blob[:40]), 40, ctypes.byref(h)) == MC_ERR_INVALID_ARG
    assert h.value is None


def test_calls_reject_a_null_problem(L):
    from paper_2604_13323_amd import binding
    o = binding.Opts()
    L.mc_default_opts(ctypes.byref(o))
    assert L.project_batch(None, 8, None, 8, None, 8, None, None, None, None, None, None, 0, None,
                           ctypes.byref(o), None) == MC_ERR_INVALID_ARG
    assert L.check_batch(None, 8, None, 8, 0, None, None, None) == MC_ERR_INVALID_ARG
    assert L.project_vjp(None, 8, None, 8, None, None, None, ctypes.byref(o), None) == MC_ERR_INVALID_ARG
    xo = binding.ExtendOpts(r=0.5, delta=0.05, n=8)
    assert L.extend_batch(None, 8, None, None, 8, None, ctypes.byref(xo), ctypes.byref(o), None, 8, None, None, None,
                          None) == MC_ERR_INVALID_ARG
    assert L.mc_problem_dof(None) == -1 and L.mc_problem_rows(None) == -1


def test_generator_is_deterministic():
    from paper_2604_13323_amd import scenes as S
    for name in ("c0", "c1", "c2", "c3", "c4"):
        a = S.make_config(name, small=True)
        b = S.make_config(name, small=True)
        assert a["scene"].to_blob() == b["scene"].to_blob()
        for k in ("q", "endpoints"):
            if k in a:
                np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(a["geo_offsets"], b["geo_offsets"])


def test_flop_model_structure():
    from paper_2604_13323_amd import flops as F
    from paper_2604_13323_amd import scenes as S
    sc = S.make_config("c3", small=True)["scene"]
    Jp = F.jacobian_pattern(sc)
    assert Jp.shape == (20, 36)
    # feet rows (0..11) never depend on arm joints, hand rows (12..17) never on the base or legs:
    G = (Jp.astype(int) @ Jp.T.astype(int)) > 0
    assert not G[12:18, 0:12].any(), "hands x feet block of J J^T must be structurally zero"
    assert Jp[18:20].all(), "CoM rows depend on every joint"
    f = F.iteration_flops(sc)
    assert f["per_iter"] == sum(v for k, v in f["parts"].items() if k != "broad_once")
    # structural Gram is cheaper than dense, and both are positive
    dense_gram = 36 * 20 * 21
    assert 0 < f["parts"]["gram"] < dense_gram
    s0 = F.iteration_flops(S.sphere_scene(0))
    assert s0["per_iter"] > 0 and s0["final"] == 6


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message before touching a device."""
    r = subprocess.run([os.sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
