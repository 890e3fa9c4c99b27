"""Seeded synthetic inputs for the 1D heat-equation rods.

This module only draws numbers: it holds none of the method's arithmetic, so
both the oracle side and the GPU side of a test may take their inputs from
here.  Every generator uses numpy's PCG64 (``default_rng(seed)``) and returns
float64 host arrays; a float32 run rounds them with :func:`as_dtype` and gives
the oracle the rounded values.

The shapes follow the workloads of the heat-equation study: one long rod
(sync), one long rod cut into workgroup-owned subdomains (async), thousands of
ragged rods (batched) and a set of equal rods with a target profile
(differentiation).  The paper's own experiment (Section 5: N = 100, r = 0.5,
cos^2 initial profile, ends 1 and 0) is :func:`paper_rod`; its ensemble of
asynchronous runs (Fig. 3) is :func:`paper_ensemble`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Rod:
    """One rod: initial state (all N points, ends are overwritten by c1/cN)."""
    u0: np.ndarray
    r: float
    c1: float
    cN: float
    K: int
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.u0.shape[0])


@dataclass
class Batch:
    """Ragged rods packed back to back: rod b is u0[offsets[b]:offsets[b+1]]."""
    offsets: np.ndarray  # int64 [nrods+1]
    u0: np.ndarray       # float64 [total]
    r: np.ndarray        # float64 [nrods]
    c1: np.ndarray
    cN: np.ndarray
    K: np.ndarray        # int64 [nrods]
    name: str = ""

    @property
    def nrods(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def lups(self) -> int:
        n = np.diff(self.offsets)
        return int(np.sum((n - 2) * self.K))


def as_dtype(x, dtype):
    """Round values to the run's precision and return them as float64 again
    (the values the oracle must see) -- for scalars and arrays."""
    if np.isscalar(x):
        return float(np.asarray(x, dtype=dtype))
    return np.asarray(np.asarray(x, dtype=dtype), dtype=np.float64)


def uniform_rod(N: int, r: float, c1: float, cN: float, K: int, lo: float, hi: float,
                seed: int = 0, name: str = "") -> Rod:
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(lo, hi, size=N)
    return Rod(u0=u0, r=r, c1=c1, cN=cN, K=K, name=name or f"uniform N={N}")


def small_rod(seed: int = 0, N: int = 4096, K: int = 20000) -> Rod:
    """Plain method, small: N=4096, r=0.4, c1=0, cN=1, interior u0 ~ U[0,1],
    K=20000; the async form uses 16 subdomains and delays in {0,1,2,3}."""
    rod = uniform_rod(N, 0.4, 0.0, 1.0, K, 0.0, 1.0, seed, name=f"small rod N={N} K={K}")
    rod.extra.update(P=16, d=3)
    return rod


def sine_modes_rod(N: int, seed: int = 0, K: int = 2000, r: float = 0.25,
                   modes=tuple(8 ** j for j in range(8))) -> Rod:
    """Synchronous large rod: u0_i = sum_j a_j sin(pi m_j i/(N-1)) + eta_i with
    a_j ~ U[-1,1], eta ~ U[-0.01, 0.01], mode numbers m_j = 8^j, c1 = cN = 0."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(-1.0, 1.0, size=len(modes))
    i = np.arange(N, dtype=np.float64)
    u0 = rng.uniform(-0.01, 0.01, size=N)
    for a, m in zip(amps, modes):
        if m >= N - 1:
            continue
        u0 += a * np.sin(math.pi * m * i / (N - 1))
    return Rod(u0=u0, r=r, c1=0.0, cN=0.0, K=K, name=f"sine-mode rod N={N} K={K}",
               extra=dict(amps=amps, modes=modes))


def async_rod(N: int = 1 << 24, P: int = 1024, K: int = 5000, seed: int = 0) -> Rod:
    """Asynchronous large rod: r=0.45, c1=1, cN=-1, u0 ~ U[-1,1], P subdomains."""
    rod = uniform_rod(N, 0.45, 1.0, -1.0, K, -1.0, 1.0, seed, name=f"async rod N={N} P={P} K={K}")
    rod.extra.update(P=P)
    return rod


def ragged_batch(nrods: int = 4096, nmin: int = 256, nmax: int = 65536, kmin: int = 500,
                 kmax: int = 5000, seed: int = 0) -> Batch:
    """Batched ragged rods: N log-uniform in [nmin, nmax], r ~ U[0.05, 0.5),
    K ~ U{kmin..kmax}, c1, cN ~ U[-1, 1], u0 ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=nrods))).astype(np.int64)
    n = np.clip(n, max(3, nmin), nmax)
    r = rng.uniform(0.05, 0.5, size=nrods)
    K = rng.integers(kmin, kmax + 1, size=nrods).astype(np.int64)
    c1 = rng.uniform(-1.0, 1.0, size=nrods)
    cN = rng.uniform(-1.0, 1.0, size=nrods)
    offsets = np.zeros(nrods + 1, dtype=np.int64)
    np.cumsum(n, out=offsets[1:])
    u0 = rng.uniform(-1.0, 1.0, size=int(offsets[-1]))
    return Batch(offsets=offsets, u0=u0, r=r, c1=c1, cN=cN, K=K,
                 name=f"ragged batch {nrods} rods N in [{nmin},{nmax}] K in [{kmin},{kmax}]")


def adjoint_rods(nrods: int = 256, N: int = 1 << 16, K: int = 2000, r: float = 0.3,
                 r_target: float = 0.35, seed: int = 0):
    """Differentiation workload: nrods rods of N points, u0 ~ U[-1,1], r=0.3,
    c1 = cN = 0.  The target profile is produced by the caller (the oracle run
    at r_target on the same u0); this function only draws u0."""
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-1.0, 1.0, size=(nrods, N))
    return dict(u0=u0, r=r, r_target=r_target, c1=0.0, cN=0.0, K=K)


def paper_rod(N: int = 100, K: int = 1000) -> Rod:
    """Section 5 set-up: r = alpha dt/dx^2 = 0.5*0.01/0.1^2 = 0.5, initial
    profile cos^2(3 pi i / (2 (N-1))) on 0-based i, ends 1 and 0."""
    i = np.arange(N, dtype=np.float64)
    u0 = np.cos(3.0 * math.pi * i / (2.0 * (N - 1))) ** 2
    return Rod(u0=u0, r=0.5, c1=1.0, cN=0.0, K=K, name=f"paper rod N={N}")


def paper_ensemble(members: int = 300, N: int = 100, K: int = 5000, d: int = 3,
                   seed: int = 1) -> Rod:
    """Section 5, Fig. 3: `members` emulated-async runs of :func:`paper_rod`
    with one grid point per subdomain (P = N, the paper's one point per PE),
    delays 0..d and one delay seed per member (drawn here)."""
    rod = paper_rod(N, K)
    rng = np.random.default_rng(seed)
    seeds = rng.integers(0, 2**63 - 1, size=members, dtype=np.int64).astype(np.uint64)
    rod.extra.update(P=N, d=d, seeds=seeds)
    rod.name = f"paper ensemble {members} members N={N} P={N} d={d} K={K}"
    return rod


def sample_points(N: int, count: int, seed: int = 123, include_ends: bool = True) -> np.ndarray:
    """Sorted distinct sample indices in [0, N), including both ends and points
    near them when include_ends is set."""
    rng = np.random.default_rng(seed)
    pts = set(int(x) for x in rng.integers(0, N, size=count))
    if include_ends:
        pts.update([0, 1, 2, N // 2, N - 3, N - 2, N - 1])
    return np.array(sorted(p for p in pts if 0 <= p < N), dtype=np.int64)
