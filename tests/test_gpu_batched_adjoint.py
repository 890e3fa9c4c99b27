"""GPU parity of the batched persistent kernel (ragged rods) and of the
discrete adjoint (dL/du0, dL/dr) against the FP64 oracle, plus the autograd
wrapper and the HIP-graph capture of the batched launch."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1510_08982_amd import abi
from paper_1510_08982_amd.heat import BatchedPlan, SyncPlan, AdjointPlan, HeatFn
from _helpers import normwise, tol_for, torch_dtype, np_dtype, print_case

pytestmark = pytest.mark.gpu
DEV = "cuda"


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def batch_inputs(batch, dt):
    f = np_dtype(dt)
    u0 = workloads.as_dtype(batch.u0, f)
    r = workloads.as_dtype(batch.r, f)
    c1 = workloads.as_dtype(batch.c1, f)
    cN = workloads.as_dtype(batch.cN, f)
    return u0, r, c1, cN


def run_batched(batch, dt, **opts):
    u0, r, c1, cN = batch_inputs(batch, dt)
    n = np.diff(batch.offsets)
    plan = BatchedPlan(n, batch.K, torch_dtype(dt), **opts)
    out = plan.run(dev(u0, np_dtype(dt)), dev(batch.offsets, np.int64), dev(r, np.float64),
                   dev(c1, np.float64), dev(cN, np.float64), dev(batch.K, np.int32))
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batched_matches_oracle_and_single_rods(dt):
    batch = workloads.ragged_batch(nrods=96, nmin=3, nmax=20000 if dt == "f32" else 12000,
                                   kmin=0, kmax=300, seed=1)
    got, plan = run_batched(batch, dt)
    print_case(test="batched", dt=dt, plan=plan.describe())
    u0, r, c1, cN = batch_inputs(batch, dt)
    ref = oracle.sync_batched(batch.offsets, u0, r, c1, cN, batch.K)
    for b in range(batch.nrods):
        s, e = batch.offsets[b], batch.offsets[b + 1]
        err = normwise(got[s:e], ref[s:e])
        assert err <= tol_for(dt), (b, e - s, batch.K[b], err)
    # bitwise equal to the single-rod kernels (same arithmetic per point)
    for b in range(0, batch.nrods, 7):
        s, e = batch.offsets[b], batch.offsets[b + 1]
        one = SyncPlan(int(e - s), torch_dtype(dt), sync_kernel=abi.HEAT1D_SYNC_STEP).run(
            dev(u0[s:e], np_dtype(dt)), r[b], c1[b], cN[b], int(batch.K[b])).cpu().numpy()
        assert np.array_equal(got[s:e], one), b


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batched_wave_group_and_workgroup_paths_agree(dt):
    batch = workloads.ragged_batch(nrods=60, nmin=200, nmax=20000 if dt == "f32" else 9000,
                                   kmin=50, kmax=200, seed=4)
    a, pa = run_batched(batch, dt)              # short rods on wavefronts, medium on groups
    b, pb = run_batched(batch, dt, waves=4)     # no single-wavefront rods
    c, pc = run_batched(batch, dt, waves=16)    # every rod on a whole workgroup
    assert "wave_rods=0" in pb.describe() and "wave_rods=0 " not in pa.describe()
    assert "group_rods=0" in pc.describe() and "group_rods=0" not in pa.describe()
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batched_autotune_keeps_results_bitwise(dt):
    """The autotuner re-splits the rods between the wavefront, group and
    workgroup queues and the small-first workgroups; every candidate runs each
    rod with the same arithmetic, so the tuned plan's results equal the
    untuned plan's bit for bit, and match the oracle."""
    batch = workloads.ragged_batch(nrods=300, nmin=64, nmax=20000 if dt == "f32" else 9000,
                                   kmin=20, kmax=400, seed=12)
    u0, r, c1, cN = batch_inputs(batch, dt)
    n = np.diff(batch.offsets)
    args = [dev(u0, np_dtype(dt)), dev(batch.offsets, np.int64), dev(r, np.float64),
            dev(c1, np.float64), dev(cN, np.float64), dev(batch.K, np.int32)]
    with BatchedPlan(n, batch.K, torch_dtype(dt)) as plan:
        before = plan.run(*args).clone()
        rule = plan.describe()
        ms = plan.autotune(*args)
        tuned = plan.describe()
        after = plan.run(*args)
        torch.cuda.synchronize()
    print_case(test="batched_autotune", dt=dt, rule=rule, tuned=tuned, ms=ms)
    assert ms > 0 and "tuned" in tuned and "tuned" not in rule
    assert torch.equal(before, after)
    ref = oracle.sync_batched(batch.offsets, u0, r, c1, cN, batch.K)
    assert normwise(after.cpu().numpy(), ref) <= tol_for(dt)


def test_batched_workload_full_size():
    """4096 rods, N log-uniform in [256, 65536], K in 500..5000, FP32, in the
    benchmark's launch: every rod, point by point, against the oracle."""
    batch = workloads.ragged_batch(seed=0)
    got, plan = run_batched(batch, "f32")
    print_case(test="batched_full", plan=plan.describe())
    assert np.isfinite(got).all()
    u0, r, c1, cN = batch_inputs(batch, "f32")
    ref = oracle.sync_batched(batch.offsets, u0, r, c1, cN, batch.K)
    worst = 0.0
    for b in range(batch.nrods):
        s, e = batch.offsets[b], batch.offsets[b + 1]
        err = normwise(got[s:e], ref[s:e])
        worst = max(worst, err)
        assert err <= 2e-5, (b, e - s, batch.K[b], err)
    print(f"  worst rod normwise error {worst:.3e} over {batch.nrods} rods")


def test_batched_graph_replays_match_eager():
    batch = workloads.ragged_batch(nrods=64, nmin=100, nmax=9000, kmin=10, kmax=200, seed=8)
    u0, r, c1, cN = batch_inputs(batch, "f32")
    n = np.diff(batch.offsets)
    plan = BatchedPlan(n, batch.K, torch.float32)
    args = [dev(u0, np.float32), dev(batch.offsets, np.int64), dev(r, np.float64),
            dev(c1, np.float64), dev(cN, np.float64), dev(batch.K, np.int32)]
    eager = plan.run(*args).clone()
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.run(*args, out=out)   # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            plan.run(*args, out=out)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        _ = plan.run(*args)          # eager work between replays
        torch.cuda.synchronize()


# ------------------------------------------------------------------ adjoint

def adjoint_case(dt, N, K, B, r=0.3, r_target=0.35, c1=0.2, cN=-0.4, seed=0):
    f = np_dtype(dt)
    rng = np.random.default_rng(seed)
    u0 = workloads.as_dtype(rng.uniform(-1, 1, (B, N)), f)
    rr, cc1, ccN = (workloads.as_dtype(x, f) for x in (r, c1, cN))
    target = np.stack([oracle.sync(u0[b], r_target, cc1, ccN, K) for b in range(B)])
    target = workloads.as_dtype(target, f)
    return u0, rr, cc1, ccN, target


@pytest.mark.parametrize("dt,N,K,B", [("f64", 1000, 300, 1), ("f64", 2500, 200, 3),
                                      ("f32", 5000, 400, 2), ("f64", 70, 1, 1),
                                      ("f32", 3000, 37, 1),
                                      # one full tile; a shifted last tile; ragged rods
                                      # (N not a multiple of 4: the unpipelined kernel)
                                      ("f32", 512, 60, 1), ("f32", 600, 30, 1),
                                      ("f32", 3001, 50, 2), ("f64", 257, 40, 2)])
def test_adjoint_matches_oracle(dt, N, K, B):
    u0, r, c1, cN, target = adjoint_case(dt, N, K, B)
    plan = AdjointPlan(N, K, torch_dtype(dt), nrods=B)
    x = dev(u0.reshape(-1), np_dtype(dt))
    uK = plan.forward(x, r, c1, cN)
    gK = uK - dev(target.reshape(-1), np_dtype(dt))
    gu, gr = plan.backward(gK, r, c1, cN)
    torch.cuda.synchronize()
    uK, gK, gu, gr = (t.cpu().numpy() for t in (uK, gK, gu, gr))
    print_case(test="adjoint", dt=dt, N=N, K=K, B=B)
    for b in range(B):
        sl = slice(b * N, (b + 1) * N)
        ref_u = oracle.sync(u0[b], r, c1, cN, K)
        assert normwise(uK[sl], ref_u) <= tol_for(dt)
        ref_gu, ref_gr = oracle.adjoint(u0[b], gK[sl], r, c1, cN, K)
        e_gu = normwise(gu[sl], ref_gu)
        e_gr = abs(gr[b] - ref_gr) / abs(ref_gr)
        print(f"  rod {b}: dL/du0 normwise {e_gu:.3e}, dL/dr relative {e_gr:.3e}")
        assert e_gu <= (1e-12 if dt == "f64" else 2e-5)
        assert e_gr <= (1e-10 if dt == "f64" else 2e-5)
        assert gu[sl][0] == 0 and gu[sl][-1] == 0


def test_adjoint_workload_fp32_full_geometry():
    """The differentiation workload as the benchmark runs it: 256 rods of 2^16
    FP32 points, r = 0.3, K = 2000, target = the oracle's run at r = 0.35 on
    the same u0.  K = 2000 puts the checkpoints 48 steps apart, so every
    stretch is two 24-step sub-stretches and the start of the second one is
    recomputed.  Eight rods (first, last and six drawn) against the oracle's
    adjoint: dL/du0 point by point, dL/dr per rod."""
    from concurrent.futures import ThreadPoolExecutor
    B, N, K = 256, 1 << 16, 2000
    rng = np.random.default_rng(0)
    u0 = workloads.as_dtype(rng.uniform(-1, 1, B * N), np.float32)
    r = workloads.as_dtype(0.3, np.float32)
    rt = workloads.as_dtype(0.35, np.float32)
    offs = np.arange(B + 1, dtype=np.int64) * N
    ones = np.ones(B)
    target = workloads.as_dtype(oracle.sync_batched(offs, u0, rt * ones, 0 * ones, 0 * ones,
                                                    np.full(B, K)), np.float32)
    print_case(test="adjoint_fp32_full", B=B, N=N, K=K)
    plan = AdjointPlan(N, K, torch.float32, nrods=B)
    assert abi.heat1d_adjoint_workspace_bytes(plan.handle, K) > 0
    x = dev(u0, np.float32)
    uK = plan.forward(x, r, 0.0, 0.0)
    gK = uK - dev(target, np.float32)
    gu, gr = plan.backward(gK, r, 0.0, 0.0)
    torch.cuda.synchronize()
    uK, gK, gu, gr = (t.cpu().numpy() for t in (uK, gK, gu, gr))
    del x, target
    picks = [0, B - 1] + [int(b) for b in rng.choice(np.arange(1, B - 1), 6, replace=False)]

    def ref(b):
        sl = slice(b * N, (b + 1) * N)
        ru = oracle.sync(u0[sl], r, 0.0, 0.0, K)
        rgu, rgr = oracle.adjoint(u0[sl], gK[sl], r, 0.0, 0.0, K, full_traj_bytes=0)
        return b, ru, rgu, rgr

    with ThreadPoolExecutor(max_workers=8) as ex:
        for b, ru, rgu, rgr in ex.map(ref, picks):
            sl = slice(b * N, (b + 1) * N)
            e_u = normwise(uK[sl], ru)
            e_gu = normwise(gu[sl], rgu)
            e_gr = abs(gr[b] - rgr) / abs(rgr)
            print(f"  rod {b}: u(K) {e_u:.3e}, dL/du0 normwise {e_gu:.3e}, "
                  f"dL/dr relative {e_gr:.3e} (dL/dr = {rgr:.6e})")
            assert e_u <= 2e-5 and e_gu <= 2e-5
            assert e_gr <= 2e-5
            assert gu[sl][0] == 0 and gu[sl][-1] == 0


def test_adjoint_deterministic_and_stride_independent():
    # The forward passes use fused multi-step sweeps grouped by pass length, so
    # u(K) depends on the checkpoint stride at the level of rounding.  Given the
    # same dL/du(K), lambda never reads the forward states: dL/du0 must be
    # bitwise the same at every stride; dL/dr sums the same terms over states
    # that differ only by rounding.
    u0, r, c1, cN, target = adjoint_case("f64", 4000, 500, 2)
    x = dev(u0.reshape(-1), np.float64)
    ref = AdjointPlan(4000, 500, torch.float64, nrods=2)
    gK = ref.forward(x, r, c1, cN) - dev(target.reshape(-1), np.float64)
    outs = []
    for stride in (0, 7, 64):
        plan = AdjointPlan(4000, 500, torch.float64, nrods=2, ckpt_stride=stride)
        plan.forward(x, r, c1, cN)
        gu, gr = plan.backward(gK, r, c1, cN)
        outs.append((gu.cpu().numpy(), gr.cpu().numpy()))
    again = ref.backward(ref.forward(x, r, c1, cN) - dev(target.reshape(-1), np.float64),
                         r, c1, cN)
    assert np.array_equal(again[1].cpu().numpy(), outs[0][1])   # same plan: same bits
    for gu, gr in outs[1:]:
        assert np.array_equal(gu, outs[0][0])
        assert np.allclose(gr, outs[0][1], rtol=1e-12, atol=0)


def test_heatfn_end_gradients_finite_differences_fp64():
    # the loss is quadratic in (c1, cN): central differences with h = 1e-3 are
    # exact up to rounding; two rods share c1 and cN, so their sensitivities add
    N, K, B = 200, 300, 2
    u0, r, _, _, target = adjoint_case("f64", N, K, B, c1=0.0, cN=0.0)
    c1, cN = 0.3, -0.7
    x = dev(u0.reshape(-1), np.float64)
    c1t = torch.tensor(c1, dtype=torch.float64, device=DEV, requires_grad=True)
    cNt = torch.tensor(cN, dtype=torch.float64, device=DEV, requires_grad=True)
    uK = HeatFn.apply(x, torch.tensor(r, dtype=torch.float64, device=DEV), c1t, cNt, K, B)
    loss = 0.5 * ((uK - dev(target.reshape(-1), np.float64)) ** 2).sum()
    loss.backward()

    def L(a, b):
        return sum(0.5 * float(np.sum((oracle.sync(u0[i], r, a, b, K) - target[i]) ** 2))
                   for i in range(B))

    h = 1e-3
    fd1 = (L(c1 + h, cN) - L(c1 - h, cN)) / (2 * h)
    fdN = (L(c1, cN + h) - L(c1, cN - h)) / (2 * h)
    assert abs(c1t.grad.item() - fd1) <= 1e-8 * max(1.0, abs(fd1))
    assert abs(cNt.grad.item() - fdN) <= 1e-8 * max(1.0, abs(fdN))


def test_adjoint_finite_differences_fp64():
    # central differences of the oracle's loss, h = 1e-6 (dL/dr) and exact for
    # the quadratic dependence on u0
    N, K = 300, 400
    u0, r, c1, cN, target = adjoint_case("f64", N, K, 1, c1=0.0, cN=0.0)
    u0 = u0[0]
    x = dev(u0, np.float64)
    uK = HeatFn.apply(x, torch.tensor(r, dtype=torch.float64, device=DEV, requires_grad=True),
                      c1, cN, K, 1)
    rt = torch.tensor(r, dtype=torch.float64, device=DEV, requires_grad=True)
    xg = x.clone().requires_grad_(True)
    uK = HeatFn.apply(xg, rt, c1, cN, K, 1)
    loss = 0.5 * ((uK - dev(target[0], np.float64)) ** 2).sum()
    loss.backward()

    def L(u, rr):
        return 0.5 * float(np.sum((oracle.sync(u, rr, c1, cN, K) - target[0]) ** 2))

    h = 1e-6
    fd_r = (L(u0, r + h) - L(u0, r - h)) / (2 * h)
    assert abs(rt.grad.item() - fd_r) <= 1e-6 * abs(fd_r)
    gu = xg.grad.cpu().numpy()
    for j in (1, 50, 151, N - 2):
        e = np.zeros(N)
        e[j] = 1e-3
        fd = (L(u0 + e, r) - L(u0 - e, r)) / 2e-3
        assert abs(gu[j] - fd) <= 1e-8 * max(abs(fd), 1e-12)


def test_adjoint_workload_fp64_rod():
    """The FP64 rod of the differentiation workload: N=2^20, r=0.3, K=2000,
    target from r=0.35; checked against the oracle adjoint."""
    N, K = 1 << 20, 2000
    u0, r, c1, cN, target = adjoint_case("f64", N, K, 1, c1=0.0, cN=0.0, seed=1)
    plan = AdjointPlan(N, K, torch.float64)
    gu, gr, uK = plan.adjoint(dev(u0[0], np.float64),
                              dev(oracle.sync(u0[0], r, c1, cN, K) - target[0], np.float64),
                              r, c1, cN, want_uK=True)
    torch.cuda.synchronize()
    ref_gu, ref_gr = oracle.adjoint(u0[0], oracle.sync(u0[0], r, c1, cN, K) - target[0], r, c1,
                                    cN, K, full_traj_bytes=0)
    e_gu = normwise(gu.cpu().numpy(), ref_gu)
    e_gr = abs(gr.item() - ref_gr) / abs(ref_gr)
    print(f"  N=2^20 FP64: dL/du0 normwise {e_gu:.3e}, dL/dr relative {e_gr:.3e}")
    assert e_gu <= 1e-12 and e_gr <= 1e-10


# ------------------------------------------- dL/dc1 and dL/dcN of the rods

def _check_ends(dt, g1, gN, gK, refs):
    # the response w to a unit left end lies in [0, 1] (maximum principle), so
    # an error of tol in w moves <gK, w> by at most tol * sum |gK|
    tol = tol_for(dt)
    for b, (r1, rN) in enumerate(refs):
        scale = float(np.abs(gK[b]).sum())
        assert abs(g1[b] - r1) <= tol * scale, (b, g1[b], r1)
        assert abs(gN[b] - rN) <= tol * scale, (b, gN[b], rN)


@pytest.mark.parametrize("dt,N,K,B", [("f64", 1000, 300, 3), ("f32", 1000, 300, 3),
                                      ("f64", 3, 20, 2), ("f64", 777, 0, 2), ("f64", 777, 1, 2),
                                      ("f32", 4099, 1000, 2)])
def test_adjoint_end_gradients_match_oracle(dt, N, K, B):
    rng = np.random.default_rng(N + K)
    f = np_dtype(dt)
    gK = workloads.as_dtype(rng.uniform(-1, 1, (B, N)), f)
    r = workloads.as_dtype(0.37, f)
    print_case(test="adjoint_ends", dt=dt, N=N, K=K, B=B)
    plan = AdjointPlan(N, K, torch_dtype(dt), nrods=B)
    g1, gN = plan.ends(torch.from_numpy(gK.astype(f)).to("cuda"), r)
    torch.cuda.synchronize()
    g1, gN = g1.cpu().numpy(), gN.cpu().numpy()
    u0 = rng.uniform(-1, 1, N)   # the end gradients do not depend on u0
    refs = [oracle.adjoint(u0, gK[b], r, 0.2, -0.1, K, with_ends=True)[2:] for b in range(B)]
    _check_ends(dt, g1, gN, gK, refs)


def test_adjoint_end_gradients_full_size_sampled():
    # the differentiation workload: 256 rods of 2^16 FP32, r = 0.3, K = 2000;
    # two sampled rods against the oracle
    B, N, K = 256, 1 << 16, 2000
    rng = np.random.default_rng(5)
    gK = workloads.as_dtype(rng.uniform(-1, 1, (B, N)), np.float32)
    r = workloads.as_dtype(0.3, np.float32)
    print_case(test="adjoint_ends_full", B=B, N=N, K=K)
    plan = AdjointPlan(N, K, torch.float32, nrods=B)
    g1, gN = plan.ends(torch.from_numpy(gK.astype(np.float32)).to("cuda"), r)
    torch.cuda.synchronize()
    g1, gN = g1.cpu().numpy(), gN.cpu().numpy()
    picks = [0, 201]
    refs = [oracle.adjoint(np.zeros(N), gK[b], r, 0.0, 0.0, K, with_ends=True,
                           full_traj_bytes=0)[2:] for b in picks]
    _check_ends("f32", g1[picks], gN[picks], gK[picks], refs)


@pytest.mark.parametrize("dt,N,K,B", [("f64", 3000, 300, 5), ("f32", 1 << 16, 500, 9),
                                      ("f64", 777, 0, 3)])
def test_grad_sum_plans_return_the_shared_parameter_gradient(dt, N, K, B):
    """opts.grad_sum: the rods share r, c1 and cN, and the library returns one
    dL/dr, dL/dc1, dL/dcN each -- the per-rod values summed in a fixed order
    (the same bits on every run), equal to their sum up to its rounding."""
    u0, r, c1, cN, target = adjoint_case(dt, N, K, B)
    x = dev(u0.reshape(-1), np_dtype(dt))
    t = dev(target.reshape(-1), np_dtype(dt))
    print_case(test="grad_sum", dt=dt, N=N, K=K, B=B)
    per = AdjointPlan(N, K, torch_dtype(dt), nrods=B)
    tot = AdjointPlan(N, K, torch_dtype(dt), nrods=B, grad_sum=True)
    gK = per.forward(x, r, c1, cN) - t
    gu_p, gr_p = per.backward(gK, r, c1, cN)
    g1_p, gN_p = per.ends(gK, r)
    outs = []
    for _ in range(2):
        tot.forward(x, r, c1, cN)
        gu_t, gr_t = tot.backward(gK, r, c1, cN)
        g1_t, gN_t = tot.ends(gK, r)
        outs.append([v.cpu().numpy() for v in (gu_t, gr_t, g1_t, gN_t)])
    torch.cuda.synchronize()
    assert all(np.array_equal(a, b) for a, b in zip(outs[0], outs[1]))
    gu_t, gr_t, g1_t, gN_t = outs[0]
    assert gr_t.shape == (1,) and g1_t.shape == (1,) and gN_t.shape == (1,)
    assert np.array_equal(gu_t, gu_p.cpu().numpy())        # dL/du0 is per point either way
    for got, per_rod in ((gr_t, gr_p), (g1_t, g1_p), (gN_t, gN_p)):
        v = per_rod.cpu().numpy()
        assert abs(got[0] - v.sum()) <= 1e-14 * np.abs(v).sum() + 1e-300, (got, v)


def test_heatfn_with_python_float_scalars():
    """HeatFn.apply with r, c1 and cN given as Python floats: gradients flow to
    u0 only (no gradient is returned for an input that is not a tensor)."""
    N, K = 2000, 250
    u0, r, c1, cN, target = adjoint_case("f64", N, K, 1)
    xg = dev(u0[0], np.float64).requires_grad_(True)
    uK = HeatFn.apply(xg, float(r), float(c1), float(cN), K, 1)
    loss = 0.5 * ((uK - dev(target[0], np.float64)) ** 2).sum()
    loss.backward()
    gK = oracle.sync(u0[0], r, c1, cN, K) - target[0]
    ref_gu, _ = oracle.adjoint(u0[0], gK, r, c1, cN, K)
    assert normwise(xg.grad.cpu().numpy(), ref_gu) <= 1e-12
