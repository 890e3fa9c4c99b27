"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/heat1d.h declares, and rejects invalid arguments
before touching the device (Section 2: 0 < r <= 1/2, N >= 3)."""
import os
import re

import pytest

from paper_1510_08982_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "heat1d.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(heat1d_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(abi.EXPORTED) == syms


def test_version_and_strerror():
    assert "gfx950" in abi.heat1d_version()
    assert abi.strerror(abi.HEAT1D_EINVAL) == "invalid argument"
    assert abi.strerror(abi.HEAT1D_ETIMEOUT).startswith("asynchronous")


@pytest.mark.parametrize("N,dtype", [(2, 0), (0, 1), (-5, 0), (100, 7)])
def test_plan_rejects_bad_shape(N, dtype):
    with pytest.raises(abi.Heat1dError) as e:
        abi.heat1d_plan_create(N, dtype)
    assert e.value.status == abi.HEAT1D_EINVAL


@pytest.mark.parametrize("opts", [dict(depth_t=-1), dict(waves=17), dict(max_delay=300),
                                  dict(sync_kernel=9), dict(sync_kernel=6), dict(sync_kernel=5), dict(pts_per_lane=65),
                                  dict(fuse_steps=3), dict(fuse_steps=-1), dict(jitter=-1),
                                  dict(jitter=65537)])
def test_plan_rejects_bad_options(opts):
    with pytest.raises(abi.Heat1dError):
        abi.heat1d_plan_create(1000, 0, opts)


def test_fused_plans():
    p = abi.heat1d_plan_create(1 << 20, abi.HEAT1D_F32,
                               dict(sync_kernel=abi.HEAT1D_SYNC_PIPELINED, depth_t=96,
                                    pts_per_lane=48, fuse_steps=4))
    try:
        assert abi.heat1d_plan_describe(p).startswith("pipelined") and "S=4" in \
            abi.heat1d_plan_describe(p)
    finally:
        abi.heat1d_plan_destroy(p)
    with pytest.raises(abi.Heat1dError) as e:     # no fused instance at 40 points per lane
        abi.heat1d_plan_create(1 << 20, abi.HEAT1D_F32,
                               dict(sync_kernel=abi.HEAT1D_SYNC_TILED, pts_per_lane=40,
                                    fuse_steps=2))
    assert e.value.status == abi.HEAT1D_EUNSUPPORTED


def test_plan_rejects_tile_without_output():
    # depth 512 with 16 points per lane leaves no interior to write
    with pytest.raises(abi.Heat1dError):
        abi.heat1d_plan_create(100000, 0, dict(sync_kernel=2, depth_t=256, pts_per_lane=8))


def test_plan_describe_and_workspace_sizes():
    p = abi.heat1d_plan_create(1 << 20, abi.HEAT1D_F32,
                               dict(sync_kernel=abi.HEAT1D_SYNC_TILED, depth_t=16, pts_per_lane=32))
    try:
        assert "tiled" in abi.heat1d_plan_describe(p) and "T=16" in abi.heat1d_plan_describe(p)
        # one state: the other half of the ping-pong pair
        assert abi.heat1d_sync_workspace_bytes(p) == 4 << 20
        # K=400: stride sqrt(400) = 20 rounded up to one 24-step sub-stretch,
        # 17 checkpoints + 1 sub-stretch start buffer + 1 lambda
        ws = abi.heat1d_adjoint_workspace_bytes(p, 400)
        assert 19 * (4 << 20) <= ws < 20 * (4 << 20)
    finally:
        abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_create(4096, abi.HEAT1D_F64)
    try:
        assert "resident" in abi.heat1d_plan_describe(p)
    finally:
        abi.heat1d_plan_destroy(p)


@pytest.mark.parametrize("r", [0.0, -0.1, 0.5000001, 1.0, float("nan")])
def test_run_sync_rejects_r_outside_stability_range(r):
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F32)
    try:
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_run_sync(p, 4096, 1 << 20, r, 0, 0, 10, 1 << 24, None)
        assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(p)


def test_run_sync_rejects_overlap_null_and_negative_K():
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F32, dict(sync_kernel=abi.HEAT1D_SYNC_TILED))
    try:
        for args in [(None, 1 << 20, 0.3, 10, 1 << 24),      # null input
                     (4096, 4096 + 100, 0.3, 10, 1 << 24),    # overlapping in/out
                     (4096, 1 << 20, 0.3, -1, 1 << 24),       # K < 0
                     (4096, 1 << 20, 0.3, 10, None),          # tiled needs a workspace
                     (4096, 1 << 20, 0.3, 10, 4096 + 8)]:     # workspace overlaps input
            u0, uK, r, K, ws = args
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_sync(p, u0, uK, r, 0, 0, K, ws, None)
            assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(p)


def test_run_sync_observed_rejects_bad_arguments():
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F32, dict(sync_kernel=abi.HEAT1D_SYNC_TILED))
    try:
        ws_sync = abi.heat1d_sync_workspace_bytes(p)
        ws_obs = abi.heat1d_observed_workspace_bytes(p)
        assert ws_obs >= ws_sync + 4000           # plus one more state and the partial sums
        base = dict(u0=4096, uK=1 << 20, K=10, every=3, norms=1 << 22, ws=1 << 24)
        for change in [dict(every=0), dict(every=-2), dict(K=-1), dict(norms=None),
                       dict(ws=None), dict(norms=4096 + 8),        # norms overlap u0
                       dict(norms=(1 << 24) + 64)]:                # norms inside the workspace
            a = dict(base, **change)
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_sync_observed(p, a["u0"], a["uK"], 0.3, 0, 0, a["K"], a["every"],
                                             a["norms"], a["ws"], None)
            assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(p)


def test_run_async_ensemble_rejects_bad_arguments():
    # every check happens before anything touches a device; the pointers are
    # fake addresses that are never dereferenced
    p = abi.heat1d_plan_create(100, abi.HEAT1D_F64, dict(nrods=4))
    try:
        base = dict(u0=1 << 20, uK=1 << 22, K=50, d=3, seeds=1 << 24, every=1,
                    norms=1 << 26, r=0.5)
        E_bytes = 4 * 100 * 8
        for change, status in [(dict(u0=None), abi.HEAT1D_EINVAL),
                               (dict(uK=None), abi.HEAT1D_EINVAL),
                               (dict(seeds=None), abi.HEAT1D_EINVAL),
                               (dict(r=0.6), abi.HEAT1D_EINVAL),
                               (dict(K=-1), abi.HEAT1D_EINVAL),
                               (dict(d=-1), abi.HEAT1D_EINVAL),
                               (dict(d=256), abi.HEAT1D_EINVAL),
                               (dict(every=0), abi.HEAT1D_EINVAL),
                               (dict(uK=(1 << 20) + E_bytes - 8), abi.HEAT1D_EINVAL),
                               (dict(norms=(1 << 22) + 8), abi.HEAT1D_EINVAL),
                               (dict(d=200), abi.HEAT1D_EUNSUPPORTED)]:   # ring exceeds LDS
            a = dict(base, **change)
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_ensemble(p, a["u0"], a["uK"], a["r"], 1.0, 0.0, a["K"],
                                              a["d"], a["seeds"], a["every"], a["norms"], None)
            assert e.value.status == status, change
    finally:
        abi.heat1d_plan_destroy(p)
    # P > N, and a rod too long for on-chip memory
    for N, opts, status in [(100, dict(nsub=101), abi.HEAT1D_EINVAL),
                            (1487, dict(), abi.HEAT1D_EUNSUPPORTED),
                            (1634, dict(nsub=16), abi.HEAT1D_EUNSUPPORTED)]:
        p = abi.heat1d_plan_create(N, abi.HEAT1D_F64, opts)
        try:
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_ensemble(p, 1 << 20, 1 << 24, 0.5, 1.0, 0.0, 10, 3, 1 << 28,
                                              1, None, None)
            assert e.value.status == status
        finally:
            abi.heat1d_plan_destroy(p)


def test_run_async_ensemble_adjoint_rejects_bad_arguments():
    p = abi.heat1d_plan_create(100, abi.HEAT1D_F64, dict(nrods=2))
    try:
        ws = abi.heat1d_ensemble_adjoint_workspace_bytes(p, 50)
        assert ws >= 51 * 100 * 2 * 8
        base = dict(u0=1 << 20, gK=1 << 22, seeds=1 << 24, uK=None, gu=1 << 26, gr=1 << 28,
                    g1=(1 << 28) + 256, gN=(1 << 28) + 512, ws=1 << 30, K=50, d=3)
        for change, status in [(dict(gK=None), abi.HEAT1D_EINVAL),
                               (dict(gr=None), abi.HEAT1D_EINVAL),
                               (dict(ws=None), abi.HEAT1D_EINVAL),
                               (dict(K=-1), abi.HEAT1D_EINVAL),
                               (dict(d=300), abi.HEAT1D_EINVAL),
                               (dict(gu=(1 << 20) + 8), abi.HEAT1D_EINVAL),    # overlaps u0
                               (dict(g1=(1 << 28) + 8), abi.HEAT1D_EINVAL),    # overlaps gr
                               (dict(uK=(1 << 30) + 64), abi.HEAT1D_EINVAL),   # inside workspace
                               (dict(d=100), abi.HEAT1D_EUNSUPPORTED)]:        # rings exceed LDS
            a = dict(base, **change)
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_ensemble_adjoint(p, a["u0"], a["gK"], 0.4, 0, 0, a["K"], a["d"],
                                                      a["seeds"], a["uK"], a["gu"], a["gr"],
                                                      a["g1"], a["gN"], a["ws"], None)
            assert e.value.status == status, change
    finally:
        abi.heat1d_plan_destroy(p)


def test_run_async_adjoint_rejects_bad_arguments():
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F64, dict(nsub=7))
    try:
        ws = abi.heat1d_async_adjoint_workspace_bytes(p, 100)
        # about sqrt(K) checkpoints and stretch states of the rod, plus the
        # edge records of u and lambda, 2 (K+1) P values each
        assert ws >= (10 + 9 + 3) * 1000 * 8 + 2 * 101 * 7 * 2 * 8
        assert abi.heat1d_async_adjoint_workspace_bytes(p, 400) > ws
        base = dict(u0=1 << 20, gK=1 << 22, uK=None, gu=1 << 26, gr=1 << 28,
                    g1=(1 << 28) + 256, gN=(1 << 28) + 512, ws=1 << 30, r=0.4, K=100, d=3)
        for change, status in [(dict(gK=None), abi.HEAT1D_EINVAL),
                               (dict(gN=None), abi.HEAT1D_EINVAL),
                               (dict(ws=None), abi.HEAT1D_EINVAL),
                               (dict(r=0.51), abi.HEAT1D_EINVAL),
                               (dict(K=-1), abi.HEAT1D_EINVAL),
                               (dict(d=256), abi.HEAT1D_EINVAL),
                               (dict(d=-1), abi.HEAT1D_EINVAL),
                               (dict(gu=(1 << 20) + 8), abi.HEAT1D_EINVAL),    # overlaps u0
                               (dict(g1=(1 << 28) + 4), abi.HEAT1D_EINVAL),    # overlaps gr
                               (dict(uK=(1 << 30) + 64), abi.HEAT1D_EINVAL),   # inside workspace
                               (dict(K=1 << 30), abi.HEAT1D_EUNSUPPORTED)]:
            a = dict(base, **change)
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_adjoint(p, a["u0"], a["gK"], a["r"], 0, 0, a["K"], a["d"], 5,
                                             a["uK"], a["gu"], a["gr"], a["g1"], a["gN"], a["ws"],
                                             None)
            assert e.value.status == status, change
    finally:
        abi.heat1d_plan_destroy(p)
    # one rod; on the ring at least two subdomains
    for opts in (dict(nsub=4, nrods=2), dict(nsub=1, boundary=abi.HEAT1D_BC_PERIODIC)):
        p = abi.heat1d_plan_create(1000, abi.HEAT1D_F32, opts)
        try:
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_adjoint(p, 1 << 20, 1 << 22, 0.4, 0, 0, 10, 2, 5, None, 1 << 26,
                                             1 << 28, (1 << 28) + 256, (1 << 28) + 512, 1 << 30,
                                             None)
            assert e.value.status == abi.HEAT1D_EUNSUPPORTED, opts
        finally:
            abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_batched([300, 400], [10, 10], abi.HEAT1D_F32, None)
    try:
        assert abi.heat1d_async_adjoint_workspace_bytes(p, 10) == 0
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_run_async_adjoint(p, 1 << 20, 1 << 22, 0.4, 0, 0, 10, 2, 5, None, 1 << 26,
                                         1 << 28, (1 << 28) + 256, (1 << 28) + 512, 1 << 30, None)
        assert e.value.status == abi.HEAT1D_EUNSUPPORTED
    finally:
        abi.heat1d_plan_destroy(p)


def test_adjoint_ends_rejects_bad_arguments():
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F32, dict(nrods=4))
    try:
        ws = abi.heat1d_adjoint_ends_workspace_bytes(p)
        assert ws >= 3 * 1000 * 4
        base = dict(g=1 << 20, r=0.3, K=10, g1=1 << 24, gN=(1 << 24) + 256, ws=1 << 26)
        for change in [dict(g=None), dict(g1=None), dict(ws=None), dict(r=0.0), dict(K=-1),
                       dict(gN=(1 << 24) + 8),          # overlaps grad_c1
                       dict(g1=(1 << 26) + 64),         # inside the workspace
                       dict(g1=(1 << 20) + 128)]:       # inside gK
            a = dict(base, **change)
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_adjoint_ends(p, a["g"], a["r"], a["K"], a["g1"], a["gN"], a["ws"], None)
            assert e.value.status == abi.HEAT1D_EINVAL, change
    finally:
        abi.heat1d_plan_destroy(p)


def test_periodic_plans_refuse_the_dirichlet_only_entry_points():
    with pytest.raises(abi.Heat1dError) as e:
        abi.heat1d_plan_create(100, abi.HEAT1D_F64, dict(boundary=2))
    assert e.value.status == abi.HEAT1D_EINVAL
    # the synchronous ring runs ring tiles, narrow or wide (or one launch per
    # step): no resident or pipelined ring, and only the wide tile shapes the
    # Dirichlet rod has
    for opts in (dict(sync_kernel=abi.HEAT1D_SYNC_RESIDENT),
                 dict(sync_kernel=abi.HEAT1D_SYNC_PIPELINED),
                 dict(sync_kernel=abi.HEAT1D_SYNC_TILED, waves=4, fuse_steps=2),
                 dict(sync_kernel=abi.HEAT1D_SYNC_TILED, waves=2, fuse_steps=4)):
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_plan_create(10000, abi.HEAT1D_F32,
                                   dict(boundary=abi.HEAT1D_BC_PERIODIC, **opts))
        assert e.value.status == abi.HEAT1D_EUNSUPPORTED
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F64, dict(boundary=abi.HEAT1D_BC_PERIODIC))
    assert abi.heat1d_plan_describe(p).startswith("tiled")
    abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_create(100000, abi.HEAT1D_F32,
                               dict(boundary=abi.HEAT1D_BC_PERIODIC,
                                    sync_kernel=abi.HEAT1D_SYNC_TILED, waves=8, depth_t=256,
                                    pts_per_lane=32, fuse_steps=8))
    assert abi.heat1d_plan_describe(p).split()[-4:] == ["T=256", "M=32", "S=8", "W=8"]
    abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F64, dict(boundary=abi.HEAT1D_BC_PERIODIC))
    try:
        calls = [
            # one subdomain (the default for N = 1000): nothing would be delayed
            lambda: abi.heat1d_run_async(p, 1 << 20, 1 << 22, 0.3, 0, 0, 10, 1, 1, 0, 1 << 24,
                                         None, None),
            lambda: abi.heat1d_forward_checkpointed(p, 1 << 20, 1 << 22, 0.3, 0, 0, 10, 1 << 24,
                                                    None),
        ]
        for call in calls:
            with pytest.raises(abi.Heat1dError) as e:
                call()
            assert e.value.status == abi.HEAT1D_EUNSUPPORTED
    finally:
        abi.heat1d_plan_destroy(p)
    with pytest.raises(abi.Heat1dError) as e:
        abi.heat1d_plan_batched([300, 400], [10, 10], abi.HEAT1D_F32,
                                dict(boundary=abi.HEAT1D_BC_PERIODIC))
    assert e.value.status == abi.HEAT1D_EUNSUPPORTED


def test_async_options_shape_the_async_kernel_only():
    """waves and pts_per_lane on a plan with nsub > 0 (and no explicit
    synchronous kernel) configure the asynchronous kernel; the plan's
    synchronous kernel keeps its defaults instead of refusing them."""
    for N, dt, o in [(4096, abi.HEAT1D_F64, dict(nsub=16, pts_per_lane=1, waves=4)),
                     (1 << 24, abi.HEAT1D_F32, dict(nsub=1024, pts_per_lane=64, waves=4)),
                     (4096, abi.HEAT1D_F64, dict(nsub=16, pts_per_lane=1, waves=4,
                                                 boundary=abi.HEAT1D_BC_PERIODIC))]:
        p = abi.heat1d_plan_create(N, dt, o)
        try:
            assert abi.heat1d_async_workspace_bytes(p) > 0
        finally:
            abi.heat1d_plan_destroy(p)
    # an explicit synchronous kernel still takes them (and refuses what it cannot run)
    with pytest.raises(abi.Heat1dError) as e:
        abi.heat1d_plan_create(1 << 20, abi.HEAT1D_F32,
                               dict(nsub=16, sync_kernel=abi.HEAT1D_SYNC_TILED, pts_per_lane=40,
                                    fuse_steps=2))
    assert e.value.status == abi.HEAT1D_EUNSUPPORTED


def test_run_async_rejects_bad_delay_and_mode():
    p = abi.heat1d_plan_create(4096, abi.HEAT1D_F64, dict(nsub=16, max_delay=4))
    try:
        for d, mode in [(-1, 0), (5, 0), (2, 7)]:
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async(p, 4096, 1 << 20, 0.4, 0, 1, 10, d, 1, mode, 1 << 24, None, None)
            assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_create(100, abi.HEAT1D_F64, dict(nsub=51))
    try:
        with pytest.raises(abi.Heat1dError):   # P > N/2
            abi.heat1d_run_async(p, 4096, 1 << 20, 0.4, 0, 1, 10, 1, 1, 0, 1 << 24, None, None)
    finally:
        abi.heat1d_plan_destroy(p)


def test_batched_plan_limits_and_order():
    with pytest.raises(abi.Heat1dError) as e:
        abi.heat1d_plan_batched([300, 70000], [10, 10], abi.HEAT1D_F32)
    assert e.value.status == abi.HEAT1D_EUNSUPPORTED
    with pytest.raises(abi.Heat1dError):
        abi.heat1d_plan_batched([300, 40000], [10, 10], abi.HEAT1D_F64)
    with pytest.raises(abi.Heat1dError):
        abi.heat1d_plan_batched([2, 400], [10, 10], abi.HEAT1D_F32)
    p = abi.heat1d_plan_batched([300, 65536, 5000, 100], [10, 20, 30, 0], abi.HEAT1D_F32)
    try:
        d = abi.heat1d_plan_describe(p)
        assert "wg_rods=1" in d and "group_rods=1" in d and "wave_rods=2" in d
        assert abi.heat1d_batched_workspace_bytes(p) > 0
    finally:
        abi.heat1d_plan_destroy(p)


def test_delay_schedule_rejects_bad_arguments():
    for P, K, d in [(0, 10, 1), (4, -1, 1), (4, 10, -1), (4, 10, 256)]:
        with pytest.raises(abi.Heat1dError):
            abi.heat1d_delay_schedule(P, K, d, 1, 4096, None)


def test_product_package_does_not_import_oracle():
    import ast
    pkg = os.path.join(ROOT, "paper_1510_08982_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, name)).read())
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    assert all(not a.name.startswith("oracle") for a in node.names), name
                if isinstance(node, ast.ImportFrom):
                    assert not (node.module or "").startswith("oracle"), name


def test_missing_library_fails_loudly(monkeypatch):
    # no CPU fallback: without libheat1d.so every entry point raises
    monkeypatch.setattr(abi, "_lib", None)
    monkeypatch.setattr(abi, "LIB_PATH", abi.LIB_PATH + ".absent")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        abi.heat1d_version()


def test_host_tensors_are_refused():
    import torch
    from paper_1510_08982_amd.heat import SyncPlan
    plan = SyncPlan(1000, torch.float32)
    with pytest.raises(ValueError, match="GPU only"):
        plan.run(torch.zeros(1000), 0.3, 0.0, 0.0, 10)


def test_bench_refuses_more_than_one_gpu():
    # the hot path is measured on one GPU; asking for more exits with a message
    # before touching any device
    import json
    import subprocess
    import sys
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _exact_s_step_weights(r, S):
    """Coefficients of (r, 1-2r, r)^S in exact rationals (S steps of Eq.3
    away from the ends), centre first."""
    from fractions import Fraction
    c = [Fraction(1)]
    for _ in range(S):
        n = [Fraction(0)] * (len(c) + 2)
        for i, x in enumerate(c):
            n[i] += r * x
            n[i + 1] += (1 - 2 * r) * x
            n[i + 2] += r * x
        c = n
    return [c[S + d] for d in range(S + 1)]


@pytest.mark.parametrize("dtype,name", [(abi.HEAT1D_F32, "f32"), (abi.HEAT1D_F64, "f64")])
def test_fused_weights_row_sum_is_exactly_one(dtype, name):
    """The weights of the fused S-step sweeps (Section 2, Eq.3 applied S times)
    must keep a constant state constant: the row sum w0 + 2(w1+..+wS) is
    exactly 1 in rational arithmetic, every weight is representable in the
    state precision, and each lies within half a grid step (2^-26 FP32,
    2^-55 FP64) of the exact coefficient of (r', 1-2r', r')^S for r' = r
    rounded to that precision -- the same r the single steps use (plus 2^-51
    for evaluating the polynomial in double before rounding)."""
    from fractions import Fraction
    import numpy as np
    ft = np.float32 if name == "f32" else np.float64
    half_grid = Fraction(1, 2 ** 26) if name == "f32" else Fraction(1, 2 ** 55)
    slack = half_grid + Fraction(1, 2 ** 51)
    rng = np.random.default_rng(3)
    rs = [0.05, 0.1, 0.25, 0.3, 0.37, 0.41, 0.43, 0.45, 0.5, 1e-3] + list(rng.uniform(1e-3, 0.5, 40))
    for S in (2, 4, 8):
        for r in rs:
            w = abi.heat1d_fused_weights(dtype, r, S)
            wf = [Fraction(x) for x in w]
            assert wf[0] + 2 * sum(wf[1:]) == 1, (r, S, w)
            for x in w:
                assert float(ft(x)) == x and x >= 0.0, (r, S, w)
            rr = Fraction(float(ft(r)))
            for got, exact in zip(wf[1:], _exact_s_step_weights(rr, S)[1:]):
                assert abs(got - exact) <= slack, (r, S)
            # the centre weight absorbs the off-centre rounding of both sides
            assert abs(wf[0] - _exact_s_step_weights(rr, S)[0]) <= 2 * S * slack


def test_fused_weights_reject_bad_arguments():
    for args in ((abi.HEAT1D_F32, 0.0, 2), (abi.HEAT1D_F32, 0.6, 2), (abi.HEAT1D_F32, 0.3, 3),
                 (abi.HEAT1D_F32, 0.3, 1), (abi.HEAT1D_F32, 0.3, 6), (abi.HEAT1D_F32, 0.3, 16),
                 (7, 0.3, 2)):
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_fused_weights(*args)
        assert e.value.status == abi.HEAT1D_EINVAL


def test_run_async_noalloc_checks_arguments_and_its_scratch_limit():
    # FP64, 1024 subdomains, max_delay 255: the halo ring alone is
    # 1024 x 2 x 512 slots x 16 bytes = 16 MiB, beyond the fixed 4 MiB array
    p = abi.heat1d_plan_create(1 << 20, abi.HEAT1D_F64, dict(nsub=1024, max_delay=255))
    try:
        assert abi.heat1d_async_workspace_bytes(p) > abi.HEAT1D_NOALLOC_SCRATCH_BYTES
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_run_async_noalloc(p, 1 << 24, 1 << 30, 0.4, 0, 1, 10, 3, 1, 0, None, None,
                                         None)
        assert e.value.status == abi.HEAT1D_ESCRATCH
    finally:
        abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_create(4096, abi.HEAT1D_F64, dict(nsub=16, max_delay=4))
    try:
        assert abi.heat1d_async_workspace_bytes(p) <= abi.HEAT1D_NOALLOC_SCRATCH_BYTES
        for d, mode, r, u0 in [(-1, 0, 0.4, 4096), (5, 0, 0.4, 4096), (2, 7, 0.4, 4096),
                               (2, 0, 0.6, 4096), (2, 0, 0.4, None)]:
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_noalloc(p, u0, 1 << 20, r, 0, 1, 10, d, 1, mode, None, None,
                                             None)
            assert e.value.status == abi.HEAT1D_EINVAL
        with pytest.raises(abi.Heat1dError) as e:      # status word inside the output
            abi.heat1d_run_async_noalloc(p, 1 << 24, 1 << 20, 0.4, 0, 1, 10, 2, 1, 0, None,
                                         (1 << 20) + 64, None)
        assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(p)
    assert "4 MiB" in abi.strerror(abi.HEAT1D_ESCRATCH)


def test_autotune_batched_rejects_bad_arguments():
    p = abi.heat1d_plan_batched([300, 400], [10, 10], abi.HEAT1D_F32)
    try:
        for bad in range(8):
            args = [1 << 20, 1 << 24, 1 << 26, 1 << 27, 1 << 28, 1 << 29, 1 << 30, 1 << 31]
            args[bad] = None
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_autotune_batched(p, *args, None)
            assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(p)
    q = abi.heat1d_plan_create(1000, abi.HEAT1D_F32)        # not a batched plan
    try:
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_autotune_batched(q, 1 << 20, 1 << 24, 1 << 26, 1 << 27, 1 << 28, 1 << 29,
                                        1 << 30, 1 << 31, None)
        assert e.value.status == abi.HEAT1D_EINVAL
    finally:
        abi.heat1d_plan_destroy(q)


def test_run_async_ensemble_snapshots_rejects_bad_step_lists():
    p = abi.heat1d_plan_create(100, abi.HEAT1D_F64, dict(nrods=4))
    try:
        S = 1 << 30            # snapshot buffer: 4 members x nsnap x 100 doubles
        for steps, snaps in [([], S), ([3, 3], S), ([5, 2], S), ([-1, 4], S), ([0, 51], S),
                             (list(range(65)), S), ([0, 10], None),
                             ([0, 10], (1 << 22) + 8)]:      # overlaps uK
            with pytest.raises(abi.Heat1dError) as e:
                abi.heat1d_run_async_ensemble_snapshots(p, 1 << 20, 1 << 22, 0.5, 1.0, 0.0, 50,
                                                        3, 1 << 24, 1, None, steps, snaps, None)
            assert e.value.status == abi.HEAT1D_EINVAL, steps
    finally:
        abi.heat1d_plan_destroy(p)


def test_delay_schedule_option_is_checked():
    """opts.delay_schedule: 0..2; the fixed schedules (1, 2) are refused where
    they are not implemented (the ensemble entry points and the ring)."""
    with pytest.raises(abi.Heat1dError) as e:
        abi.heat1d_plan_create(1000, abi.HEAT1D_F64, dict(nsub=4, delay_schedule=3))
    assert e.value.status == abi.HEAT1D_EINVAL
    p = abi.heat1d_plan_create(1000, abi.HEAT1D_F64, dict(nsub=4, boundary=abi.HEAT1D_BC_PERIODIC,
                                                          delay_schedule=1, max_delay=4))
    try:
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_run_async(p, 1 << 20, 1 << 22, 0.3, 0, 0, 10, 2, 1,
                                 abi.HEAT1D_ASYNC_EMULATED, 1 << 24, None, None)
        assert e.value.status == abi.HEAT1D_EUNSUPPORTED
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_run_async_adjoint(p, 1 << 20, 1 << 22, 0.4, 0, 0, 10, 2, 5, None, 1 << 26,
                                         1 << 28, (1 << 28) + 256, (1 << 28) + 512, 1 << 30, None)
        assert e.value.status == abi.HEAT1D_EUNSUPPORTED
    finally:
        abi.heat1d_plan_destroy(p)
    p = abi.heat1d_plan_create(100, abi.HEAT1D_F64, dict(nrods=2, delay_schedule=2))
    try:
        with pytest.raises(abi.Heat1dError) as e:
            abi.heat1d_run_async_ensemble(p, 1 << 20, 1 << 22, 0.3, 0, 0, 10, 2, 1 << 24, 1, None,
                                          None)
        assert e.value.status == abi.HEAT1D_EUNSUPPORTED
    finally:
        abi.heat1d_plan_destroy(p)
