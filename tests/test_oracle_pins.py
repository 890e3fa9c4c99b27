"""Pins for the CPU oracle: each test checks it against something other than
itself -- a closed form, an invariant, exact rational arithmetic or a
published value -- so that a dropped term, a wrong sign or index, or an
off-by-one in the delay history fails at least one of them.

Paper passages: Eq.3 and the Dirichlet ends (Section 2), the stability range
of r (Section 2), Eq.4 and its buffer of length q (Section 3), unique steady
state regardless of asynchrony for Dirichlet ends (Section 5.3).
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest
import scipy.fft

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def linear_profile(N, c1, cN):
    i = np.arange(N, dtype=np.float64)
    return c1 + (cN - c1) * i / (N - 1)


def with_ends(u0, c1, cN):
    u = np.array(u0, dtype=np.float64)
    u[0] = c1
    u[-1] = cN
    return u


def spectral_solution(u0, r, c1, cN, K):
    """u(K) = s + sum_m a_m g_m^K phi_m: the linear profile s plus the decay of
    each discrete sine mode, with g_m = 1 - 4 r sin^2(pi m / (2 (N-1))).
    The coefficients come from a type-I discrete sine transform."""
    N = len(u0)
    s = linear_profile(N, c1, cN)
    e = with_ends(u0, c1, cN) - s
    M = N - 2
    m = np.arange(1, M + 1)
    g = 1.0 - 4.0 * r * np.sin(np.pi * m / (2.0 * (N - 1))) ** 2
    coef = scipy.fft.dst(e[1:-1], type=1)
    out = s.copy()
    out[1:-1] += scipy.fft.idst(coef * g ** K, type=1)
    return out


def normwise(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ----------------------------------------------------------------- sync (Eq.3)

@pytest.mark.parametrize("N,m,r,K", [(257, 7, 0.4, 500), (101, 1, 0.5, 300),
                                     (64, 62, 0.25, 200), (4096, 7, 0.4, 2000)])
def test_sine_mode_decays_by_exact_factor(N, m, r, K):
    i = np.arange(N)
    u0 = np.sin(np.pi * m * i / (N - 1))
    g = 1.0 - 4.0 * r * math.sin(math.pi * m / (2 * (N - 1))) ** 2
    got = oracle.sync(u0, r, 0.0, 0.0, K)
    want = g ** K * with_ends(u0, 0.0, 0.0)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(u0)))


@pytest.mark.parametrize("r", [0.1, 0.25, 0.4, 0.5])
def test_matches_spectral_solution(r):
    rng = np.random.default_rng(7)
    N, K = 1000, 300
    u0 = rng.uniform(-1, 1, N)
    got = oracle.sync(u0, r, 0.3, -0.7, K)
    want = spectral_solution(u0, r, 0.3, -0.7, K)
    assert normwise(got, want) < 1e-13


def test_matches_spectral_solution_on_small_rod_workload():
    rod = workloads.small_rod(seed=0, K=2000)
    got = oracle.sync(rod.u0, rod.r, rod.c1, rod.cN, rod.K)
    want = spectral_solution(rod.u0, rod.r, rod.c1, rod.cN, rod.K)
    assert normwise(got, want) < 1e-13


def test_linear_profile_is_steady():
    N = 333
    s = linear_profile(N, 2.0, -3.0)
    got = oracle.sync(s, 0.45, 2.0, -3.0, 1000)
    assert np.max(np.abs(got - s)) < 1e-13


def test_converges_to_linear_profile():
    # Section 5.3: unique steady state for Dirichlet ends.
    rng = np.random.default_rng(3)
    N = 16
    got = oracle.sync(rng.uniform(-1, 1, N), 0.4, 1.0, -1.0, 20000)
    assert np.max(np.abs(got - linear_profile(N, 1.0, -1.0))) < 1e-10


@pytest.mark.parametrize("r", [0.05, 0.3, 0.5])
def test_maximum_principle(r):
    # For 0 < r <= 1/2 each update is a convex combination (Section 2 range).
    rng = np.random.default_rng(11)
    N = 500
    u0 = rng.uniform(-2, 5, N)
    c1, cN = 0.5, 1.5
    lo = min(u0[1:-1].min(), c1, cN)
    hi = max(u0[1:-1].max(), c1, cN)
    for K in (1, 10, 100, 1000):
        u = oracle.sync(u0, r, c1, cN, K)
        assert u.min() >= lo - 1e-14 and u.max() <= hi + 1e-14


def test_flux_identity_each_step():
    # Telescoping Eq.3: the interior sum changes by r (c1 - u_1 - u_{N-2} + cN).
    rng = np.random.default_rng(5)
    N, r, c1, cN = 64, 0.35, 0.25, -0.5
    u = with_ends(rng.uniform(-1, 1, N), c1, cN)
    for _ in range(20):
        nxt = oracle.sync(u, r, c1, cN, 1)
        lhs = nxt[1:-1].sum() - u[1:-1].sum()
        rhs = r * (c1 - u[1] - u[-2] + cN)
        assert abs(lhs - rhs) < 1e-13
        u = nxt


def test_mirror_symmetry():
    rng = np.random.default_rng(9)
    u0 = rng.uniform(-1, 1, 777)
    a = oracle.sync(u0, 0.3, 0.2, 0.9, 400)
    b = oracle.sync(u0[::-1], 0.3, 0.9, 0.2, 400)[::-1]
    assert np.max(np.abs(a - b)) < 1e-14


def exact_sync(u0, r, c1, cN, K):
    u = [Fraction(x) for x in u0]
    u[0], u[-1] = Fraction(c1), Fraction(cN)
    w = 1 - 2 * r
    for _ in range(K):
        u = [u[0]] + [r * u[i + 1] + w * u[i] + r * u[i - 1] for i in range(1, len(u) - 1)] + [u[-1]]
    return u


@pytest.mark.parametrize("r", [Fraction(2, 5), Fraction(1, 2), Fraction(1, 8)])
def test_brute_force_exact_rationals(r):
    rng = np.random.default_rng(21)
    u0 = rng.uniform(-1, 1, 9)
    K = 40
    got = oracle.sync(u0, float(r), 0.25, -0.75, K)
    want = np.array([float(x) for x in exact_sync(u0, r, 0.25, -0.75, K)])
    assert np.max(np.abs(got - want)) < 1e-15


def test_dense_matrix_power():
    N, r, K = 200, 0.45, 150
    A = np.zeros((N, N))
    A[0, 0] = A[-1, -1] = 1.0
    for i in range(1, N - 1):
        A[i, i - 1] = A[i, i + 1] = r
        A[i, i] = 1 - 2 * r
    rng = np.random.default_rng(2)
    u0 = with_ends(rng.uniform(0, 1, N), 0.0, 1.0)
    want = np.linalg.matrix_power(A, K) @ u0
    got = oracle.sync(u0, r, 0.0, 1.0, K)
    assert normwise(got, want) < 1e-13


def test_segment_matches_whole_rod_away_from_cuts():
    rng = np.random.default_rng(4)
    N, K = 3000, 200
    u0 = rng.uniform(-1, 1, N)
    full = oracle.sync(u0, 0.4, 1.0, -1.0, K)
    a, b = 1000, 1700
    seg = oracle.sync(u0[a:b], 0.4, 1.0, -1.0, K, gofs=a, N=N)
    assert np.array_equal(seg[K:-K], full[a + K:b - K])
    # a segment that touches a rod end keeps the Dirichlet value there
    seg0 = oracle.sync(u0[:700], 0.4, 1.0, -1.0, K, gofs=0, N=N)
    assert np.array_equal(seg0[:700 - K], full[:700 - K])


@pytest.mark.parametrize("bad", [dict(r=0.0), dict(r=0.5000001), dict(r=-0.1), dict(K=-1)])
def test_rejects_invalid_arguments(bad):
    args = dict(r=0.3, K=10)
    args.update(bad)
    with pytest.raises(ValueError):
        oracle.sync(np.zeros(10), args["r"], 0, 0, args["K"])
    with pytest.raises(ValueError):
        oracle.sync(np.zeros(2), 0.3, 0, 0, 1)


# ------------------------------------------------------------ delay schedule

def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        want = [int(line, 16) for line in f.read().splitlines()
                if line.strip() and not line.startswith("#")]
    state, got = 0, []
    for _ in want:
        got.append(oracle.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) % 2**64
    assert got == want


@pytest.mark.parametrize("d", [0, 1, 3, 16])
def test_delay_schedule_is_bounded_and_uniform(d):
    sched = oracle.delay_schedule(1, 64, 2000, d).astype(np.int64)
    assert sched.min() >= 0 and sched.max() <= d
    if d == 0:
        assert sched.max() == 0
        return
    counts = np.bincount(sched.ravel(), minlength=d + 1)
    n = sched.size
    chi2 = float(np.sum((counts - n / (d + 1)) ** 2 / (n / (d + 1))))
    # chi-square with d degrees of freedom: a 1e-6 tail bound, generous
    assert chi2 < d + 12 * math.sqrt(2 * d) + 30
    # the two sides of one subdomain are not copies of each other
    assert np.mean(sched[:, :, 0] == sched[:, :, 1]) < 1.0 / (d + 1) + 0.05
    # pointwise function equals the dump
    assert oracle.delay(1, 17, 5, 1, 64, d) == sched[17, 5, 1]


# ------------------------------------------------------- emulated async (Eq.4)

@pytest.mark.parametrize("P", [1, 2, 16])
def test_async_with_zero_delay_is_sync(P):
    rng = np.random.default_rng(1)
    u0 = rng.uniform(0, 1, 256)
    a = oracle.async_emulated(u0, 0.4, 0.0, 1.0, 500, P, 0, 99)
    b = oracle.sync(u0, 0.4, 0.0, 1.0, 500)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("d", [1, 3, 7])
def test_async_with_one_subdomain_is_sync(d):
    rng = np.random.default_rng(1)
    u0 = rng.uniform(0, 1, 256)
    a = oracle.async_emulated(u0, 0.4, 0.0, 1.0, 500, 1, d, 5)
    b = oracle.sync(u0, 0.4, 0.0, 1.0, 500)
    assert np.array_equal(a, b)


def exact_async(u0, r, c1, cN, K, P, sched):
    """Eq.4 in exact rationals with an explicit delay table sched[k][p][side];
    keeps the whole history."""
    N = len(u0)
    lo = [(p * N) // P for p in range(P + 1)]
    owner = [max(p for p in range(P) if lo[p] <= g) for g in range(N)]
    hist = [[Fraction(x) for x in u0]]
    hist[0][0], hist[0][-1] = Fraction(c1), Fraction(cN)
    w = 1 - 2 * r
    for k in range(K):
        cur = hist[k]
        nxt = [cur[0]] + [None] * (N - 2) + [cur[-1]]
        for i in range(1, N - 1):
            p = owner[i]
            left, right = cur[i - 1], cur[i + 1]
            if p > 0 and i == lo[p]:
                left = hist[max(0, k - int(sched[k][p][0]))][i - 1]
            if p < P - 1 and i == lo[p + 1] - 1:
                right = hist[max(0, k - int(sched[k][p][1]))][i + 1]
            nxt[i] = r * right + w * cur[i] + r * left
        hist.append(nxt)
    return hist[K]


@pytest.mark.parametrize("N,P,d", [(12, 3, 2), (11, 4, 3), (10, 10, 1), (9, 2, 5)])
def test_async_brute_force_exact_rationals(N, P, d):
    rng = np.random.default_rng(N * 100 + P)
    u0 = rng.uniform(-1, 1, N)
    K, seed = 30, 1234
    sched = oracle.delay_schedule(seed, P, K, d)
    got = oracle.async_emulated(u0, 0.4, 0.5, -0.5, K, P, d, seed)
    want = np.array([float(x) for x in exact_async(u0, Fraction(2, 5), 0.5, -0.5, K, P, sched)])
    assert np.max(np.abs(got - want)) < 1e-15
    # and the delays actually mattered (not the synchronous answer)
    if d > 0 and P > 1:
        assert np.max(np.abs(got - oracle.sync(u0, 0.4, 0.5, -0.5, K))) > 1e-6


def test_async_maximum_principle_and_unique_steady_state():
    # Section 5.3: with Dirichlet ends every delay schedule reaches the same
    # steady state (the linear profile); values stay within the data bounds.
    rng = np.random.default_rng(8)
    N = 32
    u0 = rng.uniform(-1, 1, N)
    s = linear_profile(N, 1.0, -1.0)
    for seed in (1, 2, 3):
        for K in (50, 500):
            u = oracle.async_emulated(u0, 0.45, 1.0, -1.0, K, 8, 3, seed)
            assert u.min() >= -1 - 1e-14 and u.max() <= 1 + 1e-14
        u = oracle.async_emulated(u0, 0.45, 1.0, -1.0, 8000, 8, 3, seed)
        assert np.max(np.abs(u - s)) < 1e-9


def test_async_segment_matches_whole_rod_away_from_cuts():
    rng = np.random.default_rng(12)
    N, P, K, d = 4096, 16, 300, 3
    u0 = rng.uniform(-1, 1, N)
    full = oracle.async_emulated(u0, 0.45, 1.0, -1.0, K, P, d, 77)
    a, b = 900, 1900
    seg = oracle.async_emulated(u0[a:b], 0.45, 1.0, -1.0, K, P, d, 77, gofs=a, N=N)
    assert np.array_equal(seg[K:-K], full[a + K:b - K])


# --------------------------------------------------------------- adjoint

def loss_and_grad_target(u0, r, c1, cN, K, target):
    uK = oracle.sync(u0, r, c1, cN, K)
    return 0.5 * float(np.sum((uK - target) ** 2)), uK - target


def test_adjoint_dot_product():
    # <A^K x, y> = <x, (A^K)^T y> on the homogeneous part.
    rng = np.random.default_rng(31)
    N, r, K = 300, 0.35, 120
    x = with_ends(rng.uniform(-1, 1, N), 0.0, 0.0)
    # y keeps non-zero ends: u(K) is fixed there, so they must not leak in
    y = rng.uniform(-1, 1, N)
    Ax = oracle.sync(x, r, 0.0, 0.0, K)
    ATy, _ = oracle.adjoint(x, y, r, 0.0, 0.0, K)
    assert abs(float(Ax @ y) - float(x @ ATy)) < 1e-12 * abs(float(Ax @ y)) + 1e-14


def test_adjoint_matches_finite_differences():
    rng = np.random.default_rng(32)
    N, r, K, c1, cN = 40, 0.3, 300, 0.2, -0.4
    u0 = rng.uniform(-1, 1, N)
    target = oracle.sync(u0, 0.35, c1, cN, K)
    _, gK = loss_and_grad_target(u0, r, c1, cN, K, target)
    gu, gr = oracle.adjoint(u0, gK, r, c1, cN, K)
    assert gu[0] == 0.0 and gu[-1] == 0.0
    # L is quadratic in u0: central differences are exact up to rounding
    h = 1e-3
    for j in (1, 5, 17, N - 2):
        e = np.zeros(N)
        e[j] = h
        fd = (loss_and_grad_target(u0 + e, r, c1, cN, K, target)[0]
              - loss_and_grad_target(u0 - e, r, c1, cN, K, target)[0]) / (2 * h)
        assert abs(fd - gu[j]) <= 1e-8 * max(abs(fd), 1e-12)
    h = 1e-6
    fd_r = (loss_and_grad_target(u0, r + h, c1, cN, K, target)[0]
            - loss_and_grad_target(u0, r - h, c1, cN, K, target)[0]) / (2 * h)
    assert abs(fd_r - gr) <= 1e-6 * abs(fd_r)


def test_adjoint_dr_closed_form():
    # The Eq.3 matrix is I + r L with L the Dirichlet Laplacian (acting on the
    # deviation from the linear profile), and I + r L commutes with L, so
    # dL/dr = K <lambda(K), L u(K-1)>.
    rng = np.random.default_rng(33)
    N, r, K, c1, cN = 200, 0.3, 500, 1.0, -1.0
    u0 = rng.uniform(-1, 1, N)
    gK = with_ends(rng.uniform(-1, 1, N), 0.0, 0.0)
    _, gr = oracle.adjoint(u0, gK, r, c1, cN, K)
    um = oracle.sync(u0, r, c1, cN, K - 1)
    lap = np.zeros(N)
    lap[1:-1] = um[2:] - 2 * um[1:-1] + um[:-2]
    closed = K * float(gK @ lap)
    assert abs(gr - closed) <= 1e-10 * abs(closed)


def test_adjoint_checkpointed_equals_stored_trajectory():
    rng = np.random.default_rng(34)
    N, r, K = 120, 0.45, 333
    u0 = rng.uniform(-1, 1, N)
    gK = rng.uniform(-1, 1, N)
    a = oracle.adjoint(u0, gK, r, 0.1, 0.2, K)
    b = oracle.adjoint(u0, gK, r, 0.1, 0.2, K, full_traj_bytes=0)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_batched_equals_single_rods():
    batch = workloads.ragged_batch(nrods=12, nmin=16, nmax=300, kmin=5, kmax=80, seed=3)
    out = oracle.sync_batched(batch.offsets, batch.u0, batch.r, batch.c1, batch.cN, batch.K)
    for b in range(batch.nrods):
        s, e = batch.offsets[b], batch.offsets[b + 1]
        one = oracle.sync(batch.u0[s:e], batch.r[b], batch.c1[b], batch.cN[b], int(batch.K[b]))
        assert np.array_equal(out[s:e], one)


def test_paper_rod_initial_profile_matches_ends():
    # Section 5: cos^2(0) = 1 = c1 and cos^2(3 pi / 2) = 0 = c2.
    rod = workloads.paper_rod()
    assert abs(rod.u0[0] - rod.c1) < 1e-15 and abs(rod.u0[-1] - rod.cN) < 1e-15
    u = oracle.sync(rod.u0, rod.r, rod.c1, rod.cN, 20000)
    assert np.max(np.abs(u - linear_profile(rod.N, 1.0, 0.0))) < 1e-6


# ------------------------------------- ensemble of emulated async runs (Fig. 3)

def _norm_series(u0, r, c1, cN, K, every):
    return np.array([np.linalg.norm(spectral_solution(u0, r, c1, cN, k))
                     for k in range(0, K + 1, every)])


@pytest.mark.parametrize("P,d", [(100, 0), (1, 3), (1, 0)])
def test_ensemble_norms_follow_closed_form_without_asynchrony(P, d):
    # zero delays, or a single subdomain, reduce Eq.4 to Eq.3, whose states
    # have the closed form of the sine-mode expansion
    rod = workloads.paper_ensemble(members=3, K=300)
    uK, norms = oracle.async_ensemble(rod.u0, rod.r, rod.c1, rod.cN, 300, P, d,
                                      rod.extra["seeds"], every=7)
    want = _norm_series(rod.u0, rod.r, rod.c1, rod.cN, 300, 7)
    assert norms.shape == (3, 300 // 7 + 1)
    for e in range(3):
        assert np.max(np.abs(norms[e] - want) / want) < 1e-12
        assert normwise(uK[e], spectral_solution(rod.u0, rod.r, rod.c1, rod.cN, 300)) < 1e-12


def _exact_async_states(u0, r, c1, cN, K, P, sched):
    """All states u(0..K) of Eq.4 in exact rationals (explicit delay table)."""
    return [exact_async(u0, r, c1, cN, k, P, sched) for k in range(K + 1)]


@pytest.mark.parametrize("N,P,d,every", [(8, 8, 2, 3), (10, 4, 3, 1), (9, 9, 1, 5)])
def test_ensemble_norms_brute_force_exact_rationals(N, P, d, every):
    rng = np.random.default_rng(N + P)
    u0 = rng.uniform(0, 1, N)
    K, seeds = 20, [11, 12, 13]
    uK, norms = oracle.async_ensemble(u0, 0.5, 1.0, 0.0, K, P, d, seeds, every=every)
    finals = []
    for e, seed in enumerate(seeds):
        sched = oracle.delay_schedule(seed, P, K, d)
        states = _exact_async_states(u0, Fraction(1, 2), 1, 0, K, P, sched)
        want = np.array([math.sqrt(float(sum(x * x for x in states[k])))
                         for k in range(0, K + 1, every)])
        assert np.max(np.abs(norms[e] - want)) < 1e-14
        assert np.max(np.abs(uK[e] - np.array([float(x) for x in states[K]]))) < 1e-15
        finals.append(norms[e, -1])
    # different seeds give different trajectories
    assert len(set(np.round(finals, 15))) > 1


def test_ensemble_members_reach_the_common_steady_state():
    # Section 5.3: with Dirichlet ends every member converges to the linear
    # profile whatever its delays, so the ensemble collapses to one norm
    rod = workloads.paper_ensemble(members=6, N=16, K=3000)
    uK, norms = oracle.async_ensemble(rod.u0, rod.r, rod.c1, rod.cN, 3000, 16, 3,
                                      rod.extra["seeds"], every=100)
    s = linear_profile(16, 1.0, 0.0)
    assert np.max(np.abs(uK - s)) < 1e-10
    assert np.max(np.abs(norms[:, -1] - np.linalg.norm(s))) < 1e-10
    # early on the members differ (the delays matter)
    assert np.ptp(norms[:, 1]) > 1e-6


# ------------------------------- periodic boundary (Section 5.3, Fig. 6)

def periodic_solution(u0, r, K):
    """Eq.3 on a ring of N points: each discrete Fourier mode m is multiplied
    by g_m = 1 - 4 r sin^2(pi m / N) per step."""
    N = len(u0)
    g = 1.0 - 4.0 * r * np.sin(np.pi * np.arange(N) / N) ** 2
    return np.real(np.fft.ifft(np.fft.fft(u0) * g ** K))


@pytest.mark.parametrize("P,d", [(1, 3), (100, 0), (7, 0)])
def test_periodic_without_asynchrony_follows_fourier_closed_form(P, d):
    rod = workloads.paper_ensemble(members=2, K=400)
    uK, norms = oracle.async_ensemble(rod.u0, rod.r, 0.0, 0.0, 400, P, d, rod.extra["seeds"],
                                      every=9, periodic=True)
    for e in range(2):
        assert normwise(uK[e], periodic_solution(rod.u0, rod.r, 400)) < 1e-12
        want = np.array([np.linalg.norm(periodic_solution(rod.u0, rod.r, k))
                         for k in range(0, 401, 9)])
        assert np.max(np.abs(norms[e] - want) / want) < 1e-12
    # the synchronous ring conserves the total heat
    assert abs(uK[0].sum() - rod.u0.sum()) < 1e-11


def exact_async_periodic(u0, r, K, P, sched):
    """Eq.4 on a ring in exact rationals with an explicit delay table."""
    N = len(u0)
    lo = [(p * N) // P for p in range(P + 1)]
    owner = [max(p for p in range(P) if lo[p] <= g) for g in range(N)]
    hist = [[Fraction(x) for x in u0]]
    w = 1 - 2 * r
    for k in range(K):
        cur = hist[k]
        nxt = []
        for i in range(N):
            il, ir = (i - 1) % N, (i + 1) % N
            p = owner[i]
            left, right = cur[il], cur[ir]
            if P > 1 and i == lo[p]:
                left = hist[max(0, k - int(sched[k][p][0]))][il]
            if P > 1 and i == lo[p + 1] - 1:
                right = hist[max(0, k - int(sched[k][p][1]))][ir]
            nxt.append(r * right + w * cur[i] + r * left)
        hist.append(nxt)
    return hist


@pytest.mark.parametrize("N,P,d", [(8, 8, 2), (10, 3, 3), (9, 2, 1)])
def test_periodic_brute_force_exact_rationals(N, P, d):
    rng = np.random.default_rng(N * 3 + P)
    u0 = rng.uniform(-1, 1, N)
    K, seeds = 20, [4, 5]
    uK, norms = oracle.async_ensemble(u0, 0.5, 0.0, 0.0, K, P, d, seeds, every=4, periodic=True)
    for e, seed in enumerate(seeds):
        hist = exact_async_periodic(u0, Fraction(1, 2), K, P, oracle.delay_schedule(seed, P, K, d))
        assert np.max(np.abs(uK[e] - np.array([float(x) for x in hist[K]]))) < 1e-15
        want = np.array([math.sqrt(float(sum(x * x for x in hist[k]))) for k in range(0, K + 1, 4)])
        assert np.max(np.abs(norms[e] - want)) < 1e-14


def test_periodic_async_members_settle_on_different_constants():
    # Section 5.3, Fig. 6: on the ring every member flattens out (the maximum
    # principle keeps it bounded) but to a level that depends on its delays
    rod = workloads.paper_ensemble(members=6, N=16, K=3000)
    uK, norms = oracle.async_ensemble(rod.u0, rod.r, 0.0, 0.0, 3000, 16, 3, rod.extra["seeds"],
                                      every=3000, periodic=True)
    lo, hi = rod.u0.min(), rod.u0.max()
    assert uK.min() >= lo - 1e-14 and uK.max() <= hi + 1e-14
    assert np.max(np.ptp(uK, axis=1)) < 1e-9          # each member is flat
    assert np.ptp(uK[:, 0]) > 1e-4                     # at different levels
    # the synchronous ring keeps the mean of the initial profile; at r = 1/2 on
    # an even ring the alternating mode has factor -1 and never decays, so it
    # settles on the mean plus that mode, as the closed form says
    sync, _ = oracle.async_ensemble(rod.u0, rod.r, 0.0, 0.0, 3000, 16, 0, [1], every=3000,
                                    periodic=True)
    assert abs(sync[0].mean() - rod.u0.mean()) < 1e-14
    assert normwise(sync[0], periodic_solution(rod.u0, rod.r, 3000)) < 1e-12
    alt = np.dot(rod.u0, (-1.0) ** np.arange(16)) / 16
    assert np.max(np.abs(sync[0] - rod.u0.mean() - alt * (-1.0) ** np.arange(16))) < 1e-12


# ------------------------- adjoint of the emulated asynchronous iteration

def _loss(u0, gK, r, c1, cN, K, P, d, seed):
    return float(np.dot(gK, oracle.async_emulated(u0, r, c1, cN, K, P, d, seed)))


@pytest.mark.parametrize("P,d", [(1, 3), (16, 0)])
def test_async_adjoint_without_delays_is_the_sync_adjoint(P, d):
    rng = np.random.default_rng(21)
    u0, gK = rng.uniform(-1, 1, 200), rng.uniform(-1, 1, 200)
    gu, gr, _, _ = oracle.async_adjoint(u0, gK, 0.4, 0.3, -0.2, 150, P, d, 7)
    ref_gu, ref_gr = oracle.adjoint(u0, gK, 0.4, 0.3, -0.2, 150)
    assert normwise(gu, ref_gu) < 1e-12
    assert abs(gr - ref_gr) <= 1e-12 * abs(ref_gr)


@pytest.mark.parametrize("N,P,d", [(60, 60, 3), (200, 7, 5), (33, 4, 16)])
def test_async_adjoint_is_the_transpose_of_the_forward_map(N, P, d):
    # for a fixed r and schedule u(K) is linear in (interior of u0, c1, cN),
    # so the loss <gK, u(K)> equals <dL/du0, u0> + dL/dc1 c1 + dL/dcN cN
    rng = np.random.default_rng(N + d)
    gK = rng.uniform(-1, 1, N)
    K, r, seed = 120, 0.45, 99
    gu, _, g1, gN = oracle.async_adjoint(rng.uniform(-1, 1, N), gK, r, 0.0, 0.0, K, P, d, seed)
    for _ in range(3):
        v, c1, cN = rng.uniform(-1, 1, N), rng.uniform(-1, 1), rng.uniform(-1, 1)
        lhs = _loss(v, gK, r, c1, cN, K, P, d, seed)
        rhs = float(np.dot(gu, v)) + g1 * c1 + gN * cN
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # and the gradients do not depend on the point of evaluation (only r and
    # the schedule matter)
    gu2, _, g12, gN2 = oracle.async_adjoint(rng.uniform(-1, 1, N), gK, r, 0.5, 0.1, K, P, d, seed)
    assert normwise(gu2, gu) < 1e-14 and abs(g12 - g1) < 1e-13 and abs(gN2 - gN) < 1e-13


@pytest.mark.parametrize("N,P,d", [(60, 60, 3), (200, 7, 5)])
def test_async_adjoint_dr_matches_finite_differences(N, P, d):
    rng = np.random.default_rng(3 * N + d)
    u0, gK = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    K, r, seed, h = 150, 0.3, 5, 1e-6
    _, gr, _, _ = oracle.async_adjoint(u0, gK, r, 0.7, -0.4, K, P, d, seed)
    fd = (_loss(u0, gK, r + h, 0.7, -0.4, K, P, d, seed)
          - _loss(u0, gK, r - h, 0.7, -0.4, K, P, d, seed)) / (2 * h)
    assert abs(gr - fd) <= 1e-6 * abs(fd)


def _exact_async_dr(u0, gK, r, c1, cN, K, P, sched):
    """dL/dr of L = <gK, u(K)> in exact rationals: Eq.4 carried forward on
    (value, d/dr) pairs with an explicit delay table."""
    N = len(u0)
    lo = [(p * N) // P for p in range(P + 1)]
    owner = [max(p for p in range(P) if lo[p] <= g) for g in range(N)]
    val = [[Fraction(x) for x in u0]]
    der = [[Fraction(0)] * N]
    val[0][0], val[0][-1] = Fraction(c1), Fraction(cN)
    for k in range(K):
        v, dv = [val[k][0]] + [None] * (N - 2) + [val[k][-1]], [Fraction(0)] * N
        for i in range(1, N - 1):
            p = owner[i]
            sl = max(0, k - int(sched[k][p][0])) if (p > 0 and i == lo[p]) else k
            sr = max(0, k - int(sched[k][p][1])) if (p < P - 1 and i == lo[p + 1] - 1) else k
            a, da = val[sl][i - 1], der[sl][i - 1]
            b, db = val[sr][i + 1], der[sr][i + 1]
            c, dc = val[k][i], der[k][i]
            v[i] = c + r * (a + b - 2 * c)
            dv[i] = dc + (a + b - 2 * c) + r * (da + db - 2 * dc)
        val.append(v)
        der.append(dv)
    return sum(Fraction(g) * x for g, x in zip(gK, der[K]))


@pytest.mark.parametrize("N,P,d", [(9, 9, 2), (12, 3, 3)])
def test_async_adjoint_dr_exact_rationals(N, P, d):
    rng = np.random.default_rng(N * 5 + P)
    u0, gK = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    K, seed = 25, 31
    _, gr, _, _ = oracle.async_adjoint(u0, gK, 0.375, 0.5, -0.25, K, P, d, seed)
    want = float(_exact_async_dr(u0, gK, Fraction(3, 8), 0.5, -0.25, K, P,
                                 oracle.delay_schedule(seed, P, K, d)))
    assert abs(gr - want) <= 1e-13 * abs(want)


def test_async_adjoint_scales_bound_the_sums():
    # the magnitudes returned for the rounding bounds dominate the sums they bound
    rng = np.random.default_rng(44)
    u0, gK = rng.uniform(-1, 1, 80), rng.uniform(-1, 1, 80)
    gu, gr, g1, gN, (sr, s1, sN) = oracle.async_adjoint(u0, gK, 0.45, 0.5, -0.5, 100, 80, 3, 9,
                                                         with_scales=True)
    assert sr >= abs(gr) > 0 and s1 >= abs(g1 - gK[0]) and sN >= abs(gN - gK[-1])
    # and the lambda part of the c1 scale is r times a sum of K maxima, each at
    # most the l1 mass of gK (the transposed step moves mass, never creates it)
    assert s1 <= 0.45 * 100 * np.abs(gK[1:-1]).sum() + 1e-12


@pytest.mark.parametrize("N,K", [(50, 200), (301, 120)])
def test_adjoint_end_gradients_are_exact_sensitivities(N, K):
    # u(K) is linear in (c1, cN): L = <gK, u(K)> changes by exactly dL/dc1 per
    # unit of c1 (central differences with a large step are exact up to
    # rounding), and the same value comes out of the asynchronous adjoint with
    # no delays
    rng = np.random.default_rng(N)
    u0, gK = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    r, c1, cN = 0.37, 0.4, -0.6
    _, _, g1, gN = oracle.adjoint(u0, gK, r, c1, cN, K, with_ends=True)
    L = lambda a, b: float(np.dot(gK, oracle.sync(u0, r, a, b, K)))
    assert abs(g1 - (L(c1 + 0.5, cN) - L(c1 - 0.5, cN))) <= 1e-12 * max(1.0, abs(g1))
    assert abs(gN - (L(c1, cN + 0.5) - L(c1, cN - 0.5))) <= 1e-12 * max(1.0, abs(gN))
    _, _, a1, aN = oracle.async_adjoint(u0, gK, r, c1, cN, K, 1, 3, 5)
    assert abs(a1 - g1) <= 1e-12 * max(1.0, abs(g1)) and abs(aN - gN) <= 1e-12 * max(1.0, abs(gN))
    # the checkpointed path gives the same
    _, _, h1, hN = oracle.adjoint(u0, gK, r, c1, cN, K, with_ends=True, full_traj_bytes=0)
    assert h1 == g1 and hN == gN


# ------------------------------- adjoint of the asynchronous ring iteration

def _ring_loss(u0, gK, r, K, P, d, seed):
    uK, _ = oracle.async_ensemble(u0, r, 0.0, 0.0, K, P, d, [seed], every=max(K, 1),
                                  periodic=True)
    return float(np.dot(gK, uK[0]))


@pytest.mark.parametrize("P,d", [(1, 3), (12, 0)])
def test_ring_adjoint_without_delays_follows_fourier_closed_form(P, d):
    # the synchronous ring operator is a symmetric circulant: lambda(0) = A^K gK
    rng = np.random.default_rng(P + d)
    u0, gK = rng.uniform(-1, 1, 60), rng.uniform(-1, 1, 60)
    gu, _ = oracle.async_adjoint_periodic(u0, gK, 0.4, 150, P, d, 3)
    assert normwise(gu, periodic_solution(gK, 0.4, 150)) < 1e-12


@pytest.mark.parametrize("N,P,d", [(40, 40, 3), (90, 7, 5)])
def test_ring_adjoint_is_the_transpose_and_matches_finite_differences(N, P, d):
    rng = np.random.default_rng(N * 3 + d)
    gK = rng.uniform(-1, 1, N)
    K, r, seed = 100, 0.45, 21
    gu, gr = oracle.async_adjoint_periodic(rng.uniform(-1, 1, N), gK, r, K, P, d, seed)
    for _ in range(3):
        v = rng.uniform(-1, 1, N)
        lhs = _ring_loss(v, gK, r, K, P, d, seed)
        assert abs(lhs - float(np.dot(gu, v))) <= 1e-12 * max(1.0, abs(lhs))
    u0 = rng.uniform(-1, 1, N)
    _, gr = oracle.async_adjoint_periodic(u0, gK, r, K, P, d, seed)
    h = 1e-6
    fd = (_ring_loss(u0, gK, r + h, K, P, d, seed) - _ring_loss(u0, gK, r - h, K, P, d, seed)) / (2 * h)
    assert abs(gr - fd) <= 1e-6 * abs(fd)


# ------------------------------------------- adversarial delay schedules (Eq.4)

def fixed_schedule(kind, P, K, d):
    """The two adversarial schedules written out as delay tables
    sched[k][p][side]: every edge read at the largest delay d (kind 1), or
    delay d on odd steps and 0 on even ones (kind 2)."""
    if kind == 1:
        return [[[d, d] for _ in range(P)] for _ in range(K)]
    return [[[d if k % 2 else 0] * 2 for _ in range(P)] for k in range(K)]


@pytest.mark.parametrize("kind", [1, 2])
def test_adversarial_schedule_delays(kind):
    for k in range(7):
        for p, side in ((0, 1), (3, 0), (3, 1)):
            want = 4 if kind == 1 else (4 if k % 2 else 0)
            assert oracle.sched_delay(kind, 99, k, p, side, 5, 4) == want
    # kind 0 is the seeded draw
    assert oracle.sched_delay(0, 99, 6, 3, 1, 5, 4) == oracle.delay(99, 6, 3, 1, 5, 4)


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("N,P,d", [(12, 3, 2), (11, 4, 3), (10, 10, 1), (9, 2, 5)])
def test_adversarial_schedules_brute_force_exact_rationals(kind, N, P, d):
    rng = np.random.default_rng(N * 100 + P + kind)
    u0 = rng.uniform(-1, 1, N)
    K = 30
    got = oracle.async_emulated(u0, 0.4, 0.5, -0.5, K, P, d, 1234, schedule=kind)
    want = np.array([float(x) for x in exact_async(u0, Fraction(2, 5), 0.5, -0.5, K, P,
                                                   fixed_schedule(kind, P, K, d))])
    assert np.max(np.abs(got - want)) < 1e-15
    if d > 0 and P > 1:
        assert np.max(np.abs(got - oracle.sync(u0, 0.4, 0.5, -0.5, K))) > 1e-6
        # the seed plays no part in a fixed schedule
        assert np.array_equal(got, oracle.async_emulated(u0, 0.4, 0.5, -0.5, K, P, d, 7,
                                                         schedule=kind))


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("N,P,d", [(9, 9, 2), (12, 3, 3)])
def test_adversarial_schedules_adjoint_exact_rationals(kind, N, P, d):
    """dL/dr under the fixed schedules in exact rationals, and the transpose
    identity <gK, u(K)> = <dL/du0, u0> + dL/dc1 c1 + dL/dcN cN."""
    rng = np.random.default_rng(N * 5 + P + kind)
    u0, gK = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    K = 25
    gu, gr, g1, gN = oracle.async_adjoint(u0, gK, 0.375, 0.5, -0.25, K, P, d, 31, schedule=kind)
    want = float(_exact_async_dr(u0, gK, Fraction(3, 8), 0.5, -0.25, K, P,
                                 fixed_schedule(kind, P, K, d)))
    assert abs(gr - want) <= 1e-13 * abs(want)
    v = rng.uniform(-1, 1, N)
    lhs = float(np.dot(gK, oracle.async_emulated(v, 0.375, 0.5, -0.25, K, P, d, 31,
                                                 schedule=kind)))
    assert abs(lhs - (float(np.dot(gu, v)) + g1 * 0.5 + gN * -0.25)) <= 1e-12 * max(1.0, abs(lhs))
