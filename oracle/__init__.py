"""Plain FP64 CPU oracle for the 1D heat-equation hot path (arXiv:1510.08982).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
(`paper_1510_08982_amd`) never imports it, and it never imports the product.

The arithmetic lives in ``heat1d_oracle.c`` (plain C, compiled with
``-O2 -ffp-contract=off -fopenmp``); this module only builds it and marshals
numpy arrays.  Every function works in float64.

Functions and the passages they follow:

* :func:`sync` -- Eq.3 with the Dirichlet ends of Section 2, two buffers
  (Jacobi), optionally on a segment of a longer rod.
* :func:`async_emulated` -- Eq.4 (Section 3) with a seeded delay schedule.
* :func:`async_ensemble` -- many Eq.4 runs of one rod that differ only in the
  delay seed, with the 2-norm of each state every few steps (Section 5, Fig. 3),
  also with the periodic boundary of Section 5.3 (Fig. 6).
* :func:`delay_schedule` / :func:`splitmix64` -- the counter-based delay hash
  (SplitMix64 output function, Steele, Lea and Flood, OOPSLA 2014).
* :func:`adjoint` -- the discrete adjoint of Eq.3 (transposed stencil with zero
  ends) and the dL/dr accumulation; derived from Eq.3, not stated in the paper.
* :func:`sync_batched` -- independent rods, each as :func:`sync`.
* :func:`async_adjoint` -- the discrete adjoint of the emulated asynchronous
  iteration (the delay schedule reversed), with dL/dr, dL/dc1 and dL/dcN;
  derived from Eq.4; :func:`async_adjoint_periodic` the same on the ring.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heat1d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so and return its path."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    """Declare the argument and result types of every exported function."""
    i64, dbl, u64, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p
    lib.oracle_sync.argtypes = [i64, i64, i64, vp, dbl, dbl, dbl, i64, vp]
    lib.oracle_sync.restype = ctypes.c_int
    lib.oracle_sync_batched.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_sync_batched.restype = ctypes.c_int
    lib.oracle_splitmix64.argtypes = [u64]
    lib.oracle_splitmix64.restype = u64
    lib.oracle_delay.argtypes = [u64, i64, i64, ctypes.c_int, i64, ctypes.c_int]
    lib.oracle_delay.restype = ctypes.c_int
    lib.oracle_delay_schedule.argtypes = [u64, i64, i64, ctypes.c_int, vp]
    lib.oracle_delay_schedule.restype = None
    lib.oracle_async_emulated.argtypes = [i64, i64, i64, i64, vp, dbl, dbl, dbl, i64,
                                          ctypes.c_int, u64, vp]
    lib.oracle_async_emulated.restype = ctypes.c_int
    lib.oracle_async_ensemble.argtypes = [i64, i64, i64, vp, dbl, dbl, dbl, i64, ctypes.c_int,
                                          vp, i64, ctypes.c_int, vp, vp]
    lib.oracle_async_ensemble.restype = ctypes.c_int
    lib.oracle_adjoint.argtypes = [i64, vp, vp, dbl, dbl, dbl, i64, vp, vp, vp, vp, i64]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_async_adjoint.argtypes = [i64, i64, vp, vp, dbl, dbl, dbl, i64, ctypes.c_int, u64,
                                         vp, vp, vp, vp, vp]
    lib.oracle_async_adjoint.restype = ctypes.c_int
    lib.oracle_async_emulated_kind.argtypes = [i64, i64, i64, i64, vp, dbl, dbl, dbl, i64,
                                               ctypes.c_int, u64, ctypes.c_int, vp]
    lib.oracle_async_emulated_kind.restype = ctypes.c_int
    lib.oracle_async_adjoint_kind.argtypes = [i64, i64, vp, vp, dbl, dbl, dbl, i64, ctypes.c_int,
                                              u64, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.oracle_async_adjoint_kind.restype = ctypes.c_int
    lib.oracle_sched_delay.argtypes = [ctypes.c_int, u64, i64, i64, ctypes.c_int, i64, ctypes.c_int]
    lib.oracle_sched_delay.restype = ctypes.c_int
    lib.oracle_async_adjoint_periodic.argtypes = [i64, i64, vp, vp, dbl, i64, ctypes.c_int, u64,
                                                  vp, vp, vp]
    lib.oracle_async_adjoint_periodic.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def compile_variant(src_text: str, out_path: str) -> None:
    """Compile C source text with the oracle's own flags into out_path.  Used
    by the mutation test, which plants mistakes in a copy of the source."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-std=c11", "-o", out_path, src, "-lm"], check=True)


@contextlib.contextmanager
def using_library(path: str):
    """Route every function of this module through the library at `path`
    for the duration of the block (the mutation test's planted mistakes)."""
    global _lib
    saved = _load()
    _lib = _bind(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(status: int, what: str) -> None:
    if status != 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {status})")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def sync(u0, r: float, c1: float, cN: float, K: int, *, gofs: int = 0, N: int | None = None):
    """u(K) of Eq.3 from u0 (ends replaced by c1, cN).

    With ``gofs``/``N`` the array is the segment [gofs, gofs+len) of a rod of N
    points; cut ends are frozen, so only outputs at distance >= K from a cut
    end are exact.
    """
    u = _f64(u0)
    n = u.shape[0]
    N = n if N is None else int(N)
    out = np.empty_like(u)
    _check(_load().oracle_sync(n, int(gofs), N, u.ctypes.data, float(r), float(c1), float(cN),
                               int(K), out.ctypes.data), "sync")
    return out


def sync_batched(offsets, u0, r, c1, cN, K):
    """Independent rods packed back to back (rod b = u0[offsets[b]:offsets[b+1]])."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    u = _f64(u0)
    r, c1, cN = _f64(r), _f64(c1), _f64(cN)
    K = np.ascontiguousarray(K, dtype=np.int64)
    out = np.empty_like(u)
    nr = off.shape[0] - 1
    _check(_load().oracle_sync_batched(nr, off.ctypes.data, u.ctypes.data, r.ctypes.data,
                                       c1.ctypes.data, cN.ctypes.data, K.ctypes.data,
                                       out.ctypes.data), "sync_batched")
    return out


def splitmix64(state: int) -> int:
    return int(_load().oracle_splitmix64(ctypes.c_uint64(state & (2**64 - 1))))


def delay(seed: int, k: int, p: int, side: int, P: int, d: int) -> int:
    return int(_load().oracle_delay(seed & (2**64 - 1), k, p, side, P, d))


def delay_schedule(seed: int, P: int, K: int, d: int) -> np.ndarray:
    """uint8 array of shape (K, P, 2): delay of subdomain p's left (0) / right (1) edge at step k."""
    out = np.empty((K, P, 2), dtype=np.uint8)
    _load().oracle_delay_schedule(seed & (2**64 - 1), P, K, d, out.ctypes.data)
    return out


def async_emulated(u0, r: float, c1: float, cN: float, K: int, P: int, d: int, seed: int,
                   *, gofs: int = 0, N: int | None = None, schedule: int = 0):
    """u(K) of Eq.4 with P subdomains and delays 0..d: the seeded schedule
    (schedule 0), every edge read at delay d (1), or delay d on odd steps and
    0 on even ones (2)."""
    u = _f64(u0)
    n = u.shape[0]
    N = n if N is None else int(N)
    out = np.empty_like(u)
    _check(_load().oracle_async_emulated_kind(n, int(gofs), N, int(P), u.ctypes.data, float(r),
                                              float(c1), float(cN), int(K), int(d),
                                              seed & (2**64 - 1), int(schedule), out.ctypes.data),
           "async_emulated")
    return out


def sched_delay(schedule: int, seed: int, k: int, p: int, side: int, P: int, d: int) -> int:
    """The delay of edge read (k, p, side) under a schedule (see async_emulated)."""
    return int(_load().oracle_sched_delay(int(schedule), seed & (2**64 - 1), int(k), int(p),
                                          int(side), int(P), int(d)))


def async_ensemble(u0, r: float, c1: float, cN: float, K: int, P: int, d: int, seeds,
                   every: int = 1, periodic: bool = False):
    """E emulated-async runs (E = len(seeds)) of the rods u0 (shape (E, N), or
    (N,) for one rod shared by all members).  Returns (uK of shape (E, N),
    norms of shape (E, K // every + 1)): norms[e, j] = ||u_e(j * every)||_2.
    With periodic=True the rod is a ring (Section 5.3) and c1, cN are unused."""
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1))
    E = sd.shape[0]
    u = np.asarray(u0, dtype=np.float64)
    if u.ndim == 1:
        u = np.broadcast_to(u, (E, u.shape[0]))
    u = np.ascontiguousarray(u, dtype=np.float64)
    N = u.shape[1]
    out = np.empty_like(u)
    norms = np.empty((E, K // int(every) + 1), dtype=np.float64)
    _check(_load().oracle_async_ensemble(E, N, int(P), u.ctypes.data, float(r), float(c1),
                                         float(cN), int(K), int(d), sd.ctypes.data, int(every),
                                         int(bool(periodic)), out.ctypes.data, norms.ctypes.data),
           "async_ensemble")
    return out, norms


def async_adjoint(u0, gK, r: float, c1: float, cN: float, K: int, P: int, d: int, seed: int,
                  with_scales: bool = False, schedule: int = 0):
    """Gradients of L with dL/du(K) = gK through the emulated asynchronous run
    (P subdomains, delays 0..d from `seed`): (dL/du0, dL/dr, dL/dc1, dL/dcN),
    plus, with_scales, the magnitudes (S_r, S_c1, S_cN) that bound the
    rounding of the three scalar sums (see the C source)."""
    u = _f64(u0)
    g = _f64(gK)
    n = u.shape[0]
    gu = np.empty_like(u)
    gr, g1, gN = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    sc = np.zeros(3)
    _check(_load().oracle_async_adjoint_kind(n, int(P), u.ctypes.data, g.ctypes.data, float(r),
                                             float(c1), float(cN), int(K), int(d),
                                             seed & (2**64 - 1), int(schedule), gu.ctypes.data,
                                             ctypes.byref(gr), ctypes.byref(g1), ctypes.byref(gN),
                                             sc.ctypes.data), "async_adjoint")
    if with_scales:
        return gu, float(gr.value), float(g1.value), float(gN.value), tuple(float(x) for x in sc)
    return gu, float(gr.value), float(g1.value), float(gN.value)


def async_adjoint_periodic(u0, gK, r: float, K: int, P: int, d: int, seed: int,
                           with_scale: bool = False):
    """(dL/du0, dL/dr) through the emulated asynchronous run on the periodic
    ring (every point updated, neighbours wrap around); with_scale also the
    magnitude of the dL/dr sum."""
    u = _f64(u0)
    g = _f64(gK)
    n = u.shape[0]
    gu = np.empty_like(u)
    gr = ctypes.c_double(0.0)
    sc = np.zeros(1)
    _check(_load().oracle_async_adjoint_periodic(n, int(P), u.ctypes.data, g.ctypes.data, float(r),
                                                 int(K), int(d), seed & (2**64 - 1), gu.ctypes.data,
                                                 ctypes.byref(gr), sc.ctypes.data),
           "async_adjoint_periodic")
    if with_scale:
        return gu, float(gr.value), float(sc[0])
    return gu, float(gr.value)


def adjoint(u0, gK, r: float, c1: float, cN: float, K: int, *, full_traj_bytes: int = 1 << 31,
            with_ends: bool = False):
    """(dL/du0, dL/dr) for a loss whose gradient at u(K) is gK; with_ends also
    (dL/dc1, dL/dcN)."""
    u = _f64(u0)
    g = _f64(gK)
    n = u.shape[0]
    gu = np.empty_like(u)
    gr, g1, gN = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(_load().oracle_adjoint(n, u.ctypes.data, g.ctypes.data, float(r), float(c1), float(cN),
                                  int(K), gu.ctypes.data, ctypes.byref(gr), ctypes.byref(g1),
                                  ctypes.byref(gN), int(full_traj_bytes)),
           "adjoint")
    if with_ends:
        return gu, float(gr.value), float(g1.value), float(gN.value)
    return gu, float(gr.value)
