"""ctypes binding of libheat1d.so: the C ABI of include/heat1d.h, one Python
function per C entry point and with the same name.

Only argument marshalling happens here.  Pointers are plain integers (device
addresses, e.g. ``tensor.data_ptr()``), streams are ``hipStream_t`` handles as
integers (``torch.cuda.current_stream().cuda_stream``).  A non-zero status is
raised as :class:`Heat1dError`.  If the library is not built, loading fails
loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libheat1d.so")

HEAT1D_OK = 0
HEAT1D_EINVAL = 1
HEAT1D_EUNSUPPORTED = 2
HEAT1D_EOCCUPANCY = 3
HEAT1D_ETIMEOUT = 4
HEAT1D_EHIP = 5
HEAT1D_ESCRATCH = 6
HEAT1D_NOALLOC_SCRATCH_BYTES = 4 << 20

HEAT1D_F32 = 0
HEAT1D_F64 = 1

HEAT1D_SYNC_AUTO = 0
HEAT1D_SYNC_STEP = 1
HEAT1D_SYNC_TILED = 2
HEAT1D_SYNC_RESIDENT = 3
HEAT1D_SYNC_PIPELINED = 4

HEAT1D_ASYNC_EMULATED = 0
HEAT1D_ASYNC_HARDWARE = 1
HEAT1D_BC_DIRICHLET = 0
HEAT1D_BC_PERIODIC = 1

# every symbol include/heat1d.h declares
EXPORTED = [
    "heat1d_plan_create", "heat1d_plan_batched", "heat1d_plan_destroy",
    "heat1d_sync_workspace_bytes", "heat1d_async_workspace_bytes",
    "heat1d_adjoint_workspace_bytes", "heat1d_batched_workspace_bytes", "heat1d_strerror",
    "heat1d_plan_describe", "heat1d_run_sync", "heat1d_autotune_sync", "heat1d_run_async",
    "heat1d_observed_workspace_bytes", "heat1d_run_sync_observed",
    "heat1d_async_status", "heat1d_delay_schedule",
    "heat1d_run_async_ensemble", "heat1d_ensemble_adjoint_workspace_bytes",
    "heat1d_run_async_ensemble_adjoint", "heat1d_batched_prepare",
    "heat1d_run_batched", "heat1d_forward_checkpointed", "heat1d_backward_checkpointed",
    "heat1d_adjoint", "heat1d_adjoint_ends_workspace_bytes", "heat1d_adjoint_ends",
    "heat1d_last_kernel_ms", "heat1d_set_timing", "heat1d_fused_weights", "heat1d_version",
    "heat1d_run_async_noalloc", "heat1d_autotune_batched", "heat1d_run_async_ensemble_snapshots",
    "heat1d_async_adjoint_workspace_bytes", "heat1d_run_async_adjoint",
]


class Heat1dError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


class heat1d_opts(ctypes.Structure):
    _fields_ = [
        ("sync_kernel", ctypes.c_int32),
        ("depth_t", ctypes.c_int32),
        ("pts_per_lane", ctypes.c_int32),
        ("waves", ctypes.c_int32),
        ("nsub", ctypes.c_int32),
        ("max_delay", ctypes.c_int32),
        ("watchdog_polls", ctypes.c_int64),
        ("ckpt_stride", ctypes.c_int32),
        ("nrods", ctypes.c_int32),
        ("fuse_steps", ctypes.c_int32),
        ("jitter", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("grad_sum", ctypes.c_int32),
        ("delay_schedule", ctypes.c_int32),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libheat1d.so (built by paper_1510_08982_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1510_08982_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "heat1d_plan_create": (ctypes.c_int, [P(vp), i64, i32, P(heat1d_opts)]),
        "heat1d_plan_batched": (ctypes.c_int, [P(vp), i32, P(i64), P(i32), i32, P(heat1d_opts)]),
        "heat1d_plan_destroy": (None, [vp]),
        "heat1d_sync_workspace_bytes": (sz, [vp]),
        "heat1d_async_workspace_bytes": (sz, [vp]),
        "heat1d_adjoint_workspace_bytes": (sz, [vp, i64]),
        "heat1d_batched_workspace_bytes": (sz, [vp]),
        "heat1d_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "heat1d_plan_describe": (ctypes.c_char_p, [vp]),
        "heat1d_run_sync": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, vp, vp]),
        "heat1d_autotune_sync": (ctypes.c_int, [vp, vp, vp, dbl, i64, vp, vp, P(dbl)]),
        "heat1d_observed_workspace_bytes": (sz, [vp]),
        "heat1d_run_sync_observed": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, i64, vp, vp,
                                                    vp]),
        "heat1d_run_async": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, i32, u64, i32, vp,
                                            vp, vp]),
        "heat1d_run_async_noalloc": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, i32, u64,
                                                    i32, vp, vp, vp]),
        "heat1d_run_async_ensemble": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, i32, vp,
                                                     i32, vp, vp]),
        "heat1d_run_async_ensemble_snapshots": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64,
                                                               i32, vp, i32, vp, P(i64), i32, vp,
                                                               vp]),
        "heat1d_ensemble_adjoint_workspace_bytes": (sz, [vp, i64]),
        "heat1d_run_async_ensemble_adjoint": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, i32,
                                                             vp, vp, vp, vp, vp, vp, vp, vp]),
        "heat1d_async_adjoint_workspace_bytes": (sz, [vp, i64]),
        "heat1d_run_async_adjoint": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, i32, u64, vp,
                                                    vp, vp, vp, vp, vp, vp]),
        "heat1d_adjoint_ends_workspace_bytes": (sz, [vp]),
        "heat1d_adjoint_ends": (ctypes.c_int, [vp, vp, dbl, i64, vp, vp, vp, vp]),
        "heat1d_async_status": (ctypes.c_int, [vp, vp, vp]),
        "heat1d_delay_schedule": (ctypes.c_int, [i32, i64, i32, u64, vp, vp]),
        "heat1d_batched_prepare": (ctypes.c_int, [vp, vp, vp]),
        "heat1d_run_batched": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "heat1d_autotune_batched": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                                   P(dbl)]),
        "heat1d_forward_checkpointed": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, vp, vp]),
        "heat1d_backward_checkpointed": (ctypes.c_int, [vp, vp, dbl, dbl, dbl, i64, vp, vp, vp,
                                                        vp]),
        "heat1d_adjoint": (ctypes.c_int, [vp, vp, vp, dbl, dbl, dbl, i64, vp, vp, vp, vp, vp]),
        "heat1d_last_kernel_ms": (dbl, [vp, P(i64)]),
        "heat1d_set_timing": (ctypes.c_int, [vp, i32]),
        "heat1d_fused_weights": (ctypes.c_int, [i32, dbl, i32, P(dbl)]),
        "heat1d_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str) -> None:
    if status != HEAT1D_OK:
        raise Heat1dError(status, where)


def _opts(opts) -> "ctypes.POINTER(heat1d_opts)":
    if opts is None:
        return None
    if isinstance(opts, dict):
        o = heat1d_opts()
        for k, v in opts.items():
            setattr(o, k, int(v))
        opts = o
    return ctypes.pointer(opts)


def strerror(status: int) -> str:
    return load().heat1d_strerror(int(status)).decode()


def heat1d_version() -> str:
    return load().heat1d_version().decode()


def heat1d_plan_create(N: int, dtype: int, opts=None) -> int:
    h = ctypes.c_void_p()
    _check(load().heat1d_plan_create(ctypes.byref(h), int(N), int(dtype), _opts(opts)),
           "heat1d_plan_create")
    return h.value


def heat1d_plan_batched(N_host, K_host, dtype: int, opts=None) -> int:
    n = len(N_host)
    Na = (ctypes.c_int64 * n)(*[int(x) for x in N_host])
    Ka = (ctypes.c_int32 * n)(*[int(x) for x in K_host])
    h = ctypes.c_void_p()
    _check(load().heat1d_plan_batched(ctypes.byref(h), n, Na, Ka, int(dtype), _opts(opts)),
           "heat1d_plan_batched")
    return h.value


def heat1d_plan_destroy(plan: int) -> None:
    if plan:
        load().heat1d_plan_destroy(plan)


def heat1d_sync_workspace_bytes(plan: int) -> int:
    return int(load().heat1d_sync_workspace_bytes(plan))


def heat1d_async_workspace_bytes(plan: int) -> int:
    return int(load().heat1d_async_workspace_bytes(plan))


def heat1d_adjoint_workspace_bytes(plan: int, K: int) -> int:
    return int(load().heat1d_adjoint_workspace_bytes(plan, int(K)))


def heat1d_batched_workspace_bytes(plan: int) -> int:
    return int(load().heat1d_batched_workspace_bytes(plan))


def heat1d_plan_describe(plan: int) -> str:
    return load().heat1d_plan_describe(plan).decode()


def heat1d_strerror(status: int) -> str:
    return strerror(status)


def heat1d_run_sync(plan, u0, uK, r, c1, cN, K, workspace, stream) -> None:
    _check(load().heat1d_run_sync(plan, u0, uK, float(r), float(c1), float(cN), int(K),
                                  workspace, stream), "heat1d_run_sync")


def heat1d_observed_workspace_bytes(plan: int) -> int:
    return int(load().heat1d_observed_workspace_bytes(plan))


def heat1d_run_sync_observed(plan, u0, uK, r, c1, cN, K, every, norms, workspace,
                             stream) -> None:
    _check(load().heat1d_run_sync_observed(plan, u0, uK, float(r), float(c1), float(cN), int(K),
                                           int(every), norms, workspace, stream),
           "heat1d_run_sync_observed")


def heat1d_run_async_ensemble(plan, u0, uK, r, c1, cN, K, d, seeds, every, norms,
                              stream) -> None:
    _check(load().heat1d_run_async_ensemble(plan, u0, uK, float(r), float(c1), float(cN), int(K),
                                            int(d), seeds, int(every), norms, stream),
           "heat1d_run_async_ensemble")


def heat1d_run_async_ensemble_snapshots(plan, u0, uK, r, c1, cN, K, d, seeds, every, norms,
                                        steps, snaps, stream) -> None:
    st = (ctypes.c_int64 * len(steps))(*[int(x) for x in steps])
    _check(load().heat1d_run_async_ensemble_snapshots(plan, u0, uK, float(r), float(c1),
                                                      float(cN), int(K), int(d), seeds,
                                                      int(every), norms, st, len(steps), snaps,
                                                      stream),
           "heat1d_run_async_ensemble_snapshots")


def heat1d_ensemble_adjoint_workspace_bytes(plan: int, K: int) -> int:
    return int(load().heat1d_ensemble_adjoint_workspace_bytes(plan, int(K)))


def heat1d_run_async_ensemble_adjoint(plan, u0, gK, r, c1, cN, K, d, seeds, uK, grad_u0, grad_r,
                                      grad_c1, grad_cN, workspace, stream) -> None:
    _check(load().heat1d_run_async_ensemble_adjoint(plan, u0, gK, float(r), float(c1), float(cN),
                                                    int(K), int(d), seeds, uK, grad_u0, grad_r,
                                                    grad_c1, grad_cN, workspace, stream),
           "heat1d_run_async_ensemble_adjoint")


def heat1d_async_adjoint_workspace_bytes(plan: int, K: int) -> int:
    return int(load().heat1d_async_adjoint_workspace_bytes(plan, int(K)))


def heat1d_run_async_adjoint(plan, u0, gK, r, c1, cN, K, d, seed, uK, grad_u0, grad_r, grad_c1,
                             grad_cN, workspace, stream) -> None:
    _check(load().heat1d_run_async_adjoint(plan, u0, gK, float(r), float(c1), float(cN), int(K),
                                           int(d), int(seed) & (2**64 - 1), uK, grad_u0, grad_r,
                                           grad_c1, grad_cN, workspace, stream),
           "heat1d_run_async_adjoint")


def heat1d_adjoint_ends_workspace_bytes(plan: int) -> int:
    return int(load().heat1d_adjoint_ends_workspace_bytes(plan))


def heat1d_adjoint_ends(plan, gK, r, K, grad_c1, grad_cN, workspace, stream) -> None:
    _check(load().heat1d_adjoint_ends(plan, gK, float(r), int(K), grad_c1, grad_cN, workspace,
                                      stream), "heat1d_adjoint_ends")


def heat1d_autotune_sync(plan, u0, uK, r, K_probe, workspace, stream) -> float:
    best = ctypes.c_double(0.0)
    _check(load().heat1d_autotune_sync(plan, u0, uK, float(r), int(K_probe), workspace, stream,
                                       ctypes.byref(best)), "heat1d_autotune_sync")
    return best.value


def heat1d_run_async(plan, u0, uK, r, c1, cN, K, d, seed, mode, workspace, stats, stream) -> None:
    _check(load().heat1d_run_async(plan, u0, uK, float(r), float(c1), float(cN), int(K), int(d),
                                   int(seed) & (2**64 - 1), int(mode), workspace, stats, stream),
           "heat1d_run_async")


def heat1d_run_async_noalloc(plan, u0, uK, r, c1, cN, K, d, seed, mode, stats, status,
                             stream) -> None:
    _check(load().heat1d_run_async_noalloc(plan, u0, uK, float(r), float(c1), float(cN), int(K),
                                           int(d), int(seed) & (2**64 - 1), int(mode), stats,
                                           status, stream),
           "heat1d_run_async_noalloc")


def heat1d_async_status(plan, workspace, stream) -> int:
    return int(load().heat1d_async_status(plan, workspace, stream))


def heat1d_delay_schedule(P, K, d, seed, out, stream) -> None:
    _check(load().heat1d_delay_schedule(int(P), int(K), int(d), int(seed) & (2**64 - 1), out,
                                        stream), "heat1d_delay_schedule")


def heat1d_batched_prepare(plan, workspace, stream) -> None:
    _check(load().heat1d_batched_prepare(plan, workspace, stream), "heat1d_batched_prepare")


def heat1d_run_batched(plan, u0, uK, offsets, r, c1, cN, K, workspace, stream) -> None:
    _check(load().heat1d_run_batched(plan, u0, uK, offsets, r, c1, cN, K, workspace, stream),
           "heat1d_run_batched")


def heat1d_autotune_batched(plan, u0, uK, offsets, r, c1, cN, K, workspace, stream) -> float:
    best = ctypes.c_double(0.0)
    _check(load().heat1d_autotune_batched(plan, u0, uK, offsets, r, c1, cN, K, workspace, stream,
                                          ctypes.byref(best)), "heat1d_autotune_batched")
    return best.value


def heat1d_forward_checkpointed(plan, u0, uK, r, c1, cN, K, workspace, stream) -> None:
    _check(load().heat1d_forward_checkpointed(plan, u0, uK, float(r), float(c1), float(cN), int(K),
                                              workspace, stream), "heat1d_forward_checkpointed")


def heat1d_backward_checkpointed(plan, gK, r, c1, cN, K, grad_u0, grad_r, workspace,
                                 stream) -> None:
    _check(load().heat1d_backward_checkpointed(plan, gK, float(r), float(c1), float(cN), int(K),
                                               grad_u0, grad_r, workspace, stream),
           "heat1d_backward_checkpointed")


def heat1d_adjoint(plan, u0, gK, r, c1, cN, K, grad_u0, grad_r, uK, workspace, stream) -> None:
    _check(load().heat1d_adjoint(plan, u0, gK, float(r), float(c1), float(cN), int(K), grad_u0,
                                 grad_r, uK, workspace, stream), "heat1d_adjoint")


def heat1d_set_timing(plan, enable: bool) -> None:
    _check(load().heat1d_set_timing(plan, 1 if enable else 0), "heat1d_set_timing")


def heat1d_last_kernel_ms(plan):
    n = ctypes.c_int64(0)
    ms = load().heat1d_last_kernel_ms(plan, ctypes.byref(n))
    return float(ms), int(n.value)


def heat1d_fused_weights(dtype: int, r: float, S: int) -> list:
    w = (ctypes.c_double * (max(int(S), 0) + 1))()
    _check(load().heat1d_fused_weights(int(dtype), float(r), int(S), w), "heat1d_fused_weights")
    return [w[i] for i in range(int(S) + 1)]
