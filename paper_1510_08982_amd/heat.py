"""PyTorch-facing helpers around the C ABI.

PyTorch provides device memory and the current stream; every arithmetic step
runs in the HIP kernels of libheat1d.so.  Inputs must already be on the GPU
(torch 'cuda' device on ROCm); nothing here computes on the host.
"""
from __future__ import annotations

import sys

import torch

from . import abi

_DT = {torch.float32: abi.HEAT1D_F32, torch.float64: abi.HEAT1D_F64}


def _dtype_code(dtype) -> int:
    if dtype not in _DT:
        raise TypeError(f"unsupported dtype {dtype}; use torch.float32 or torch.float64")
    return _DT[dtype]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _require_gpu(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("heat1d runs on the GPU only: pass device tensors")
        if not t.is_contiguous():
            raise ValueError("heat1d needs contiguous tensors")


def _workspace(nbytes: int, device) -> torch.Tensor:
    # 256-byte aligned by the caching allocator
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class _Plan:
    """Owner of one library plan handle.  close() destroys it (and drops the
    workspace tensor); it is also called on garbage collection, except while
    the interpreter shuts down, when the HIP runtime may already be gone and
    the process exit releases everything anyway."""

    handle = None

    def close(self) -> None:
        h, self.handle = self.handle, None
        self._ws = None
        self._adj_ws = None
        if h:
            abi.heat1d_plan_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def describe(self) -> str:
        return abi.heat1d_plan_describe(self.handle)

    def set_timing(self, on: bool = True):
        abi.heat1d_set_timing(self.handle, on)

    def last_kernel_ms(self):
        return abi.heat1d_last_kernel_ms(self.handle)


class SyncPlan(_Plan):
    """Plan for `nrods` equal rods of N points (heat1d_plan_create)."""

    def __init__(self, N: int, dtype=torch.float32, nrods: int = 1, **opts):
        self.N, self.dtype, self.nrods = int(N), dtype, int(nrods)
        o = dict(opts)
        o["nrods"] = self.nrods
        self.handle = abi.heat1d_plan_create(self.N, _dtype_code(dtype), o)
        self._ws = None

    def workspace(self, device) -> torch.Tensor:
        n = abi.heat1d_sync_workspace_bytes(self.handle)
        if self._ws is None or self._ws.numel() < n or self._ws.device != device:
            self._ws = _workspace(n, device)
        return self._ws

    def run(self, u0: torch.Tensor, r: float, c1: float, cN: float, K: int,
            out: torch.Tensor | None = None) -> torch.Tensor:
        _require_gpu(u0)
        if u0.dtype != self.dtype or u0.numel() != self.N * self.nrods:
            raise ValueError("u0 does not match the plan (dtype or size)")
        out = torch.empty_like(u0) if out is None else out
        ws = self.workspace(u0.device)
        abi.heat1d_run_sync(self.handle, u0.data_ptr(), out.data_ptr(), r, c1, cN, K,
                            ws.data_ptr(), _stream())
        return out

    def run_observed(self, u0: torch.Tensor, r: float, c1: float, cN: float, K: int, every: int,
                     out: torch.Tensor | None = None):
        """run(), and the 2-norm of every rod's state after 0, every, 2*every, ... steps:
        returns (uK, norms) with norms of shape (nrods, K // every + 1), float64."""
        _require_gpu(u0)
        if u0.dtype != self.dtype or u0.numel() != self.N * self.nrods:
            raise ValueError("u0 does not match the plan (dtype or size)")
        out = torch.empty_like(u0) if out is None else out
        norms = torch.empty((self.nrods, int(K) // int(every) + 1), dtype=torch.float64,
                            device=u0.device)
        ws = _workspace(abi.heat1d_observed_workspace_bytes(self.handle), u0.device)
        abi.heat1d_run_sync_observed(self.handle, u0.data_ptr(), out.data_ptr(), r, c1, cN, K,
                                     every, norms.data_ptr(), ws.data_ptr(), _stream())
        return out, norms

    def autotune(self, u0: torch.Tensor, r: float, K_probe: int) -> float:
        _require_gpu(u0)
        scratch = torch.empty_like(u0)
        ws = self.workspace(u0.device)
        return abi.heat1d_autotune_sync(self.handle, u0.data_ptr(), scratch.data_ptr(), r,
                                        K_probe, ws.data_ptr(), _stream())


def run_sync(u0: torch.Tensor, r: float, c1: float, cN: float, K: int, nrods: int = 1,
             **opts) -> torch.Tensor:
    """u(K) of the synchronous iteration for one rod (or `nrods` stacked rods)."""
    plan = SyncPlan(u0.numel() // nrods, u0.dtype, nrods=nrods, **opts)
    return plan.run(u0, r, c1, cN, K)


class AsyncPlan(_Plan):
    """Asynchronous persistent kernel with P = nsub subdomains; with
    periodic=True the rod is a ring of N points (P >= 2)."""

    def __init__(self, N: int, nsub: int, dtype=torch.float32, max_delay: int = 16,
                 periodic: bool = False, **opts):
        self.N, self.dtype, self.P = int(N), dtype, int(nsub)
        o = dict(opts)
        o.update(nsub=self.P, max_delay=int(max_delay))
        if periodic:
            o["boundary"] = abi.HEAT1D_BC_PERIODIC
        self.handle = abi.heat1d_plan_create(self.N, _dtype_code(dtype), o)
        self._ws = None

    def workspace(self, device) -> torch.Tensor:
        n = abi.heat1d_async_workspace_bytes(self.handle)
        if self._ws is None or self._ws.numel() < n or self._ws.device != device:
            self._ws = _workspace(n, device)
        return self._ws

    def run(self, u0, r, c1, cN, K, d, seed=1, mode=abi.HEAT1D_ASYNC_EMULATED,
            stats: torch.Tensor | None = None, out=None) -> torch.Tensor:
        _require_gpu(u0)
        if u0.dtype != self.dtype or u0.numel() != self.N:
            raise ValueError("u0 does not match the plan (dtype or size)")
        out = torch.empty_like(u0) if out is None else out
        ws = self.workspace(u0.device)
        sp = 0
        if stats is not None:
            if stats.dtype != torch.int64 or stats.numel() < d + 3 or not stats.is_cuda:
                raise ValueError("stats must be an int64 device tensor of d+3 entries")
            sp = stats.data_ptr()
        abi.heat1d_run_async(self.handle, u0.data_ptr(), out.data_ptr(), r, c1, cN, K, d, seed,
                             mode, ws.data_ptr(), sp or None, _stream())
        return out

    def status(self) -> int:
        return abi.heat1d_async_status(self.handle, self._ws.data_ptr(), _stream())

    def adjoint(self, u0, gK, r, c1, cN, K, d, seed=1, out=None):
        """Gradients through the emulated run of `run` (heat1d_run_async_adjoint):
        returns (grad_u0, grad_r, grad_c1, grad_cN, uK), the three scalars as
        float64 device tensors of one element."""
        _require_gpu(u0, gK)
        for t in (u0, gK):
            if t.dtype != self.dtype or t.numel() != self.N:
                raise ValueError("u0 and gK must match the plan (dtype and size)")
        out = torch.empty_like(u0) if out is None else out
        n = abi.heat1d_async_adjoint_workspace_bytes(self.handle, K)
        ws = getattr(self, "_adj_ws", None)
        if ws is None or ws.numel() < n or ws.device != u0.device:
            self._adj_ws = None  # free the smaller one first
            self._adj_ws = ws = _workspace(n, u0.device)
        g_u0 = torch.empty_like(u0)
        scal = torch.empty(3, dtype=torch.float64, device=u0.device)
        abi.heat1d_run_async_adjoint(self.handle, u0.data_ptr(), gK.data_ptr(), r, c1, cN, K, d,
                                     seed, out.data_ptr(), g_u0.data_ptr(), scal[0:1].data_ptr(),
                                     scal[1:2].data_ptr(), scal[2:3].data_ptr(), ws.data_ptr(),
                                     _stream())
        return g_u0, scal[0:1], scal[1:2], scal[2:3], out


class EnsemblePlan(_Plan):
    """Many emulated-async runs of equal rods in one launch
    (heat1d_run_async_ensemble): `members` rods of N points, P = nsub
    subdomains each (0: one point per subdomain), Dirichlet ends or, with
    periodic=True, rings of N points."""

    def __init__(self, N: int, members: int, nsub: int = 0, dtype=torch.float32,
                 periodic: bool = False):
        self.N, self.E, self.P, self.dtype = int(N), int(members), int(nsub), dtype
        bc = abi.HEAT1D_BC_PERIODIC if periodic else abi.HEAT1D_BC_DIRICHLET
        self.handle = abi.heat1d_plan_create(self.N, _dtype_code(dtype),
                                             dict(nrods=self.E, nsub=self.P, boundary=bc))

    def run(self, u0, r, c1, cN, K, d, seeds, every: int = 1, with_norms: bool = True,
            out=None, norms=None, snap_steps=None):
        """u0: (members, N) device tensor; seeds: int64 device tensor of
        `members` seeds (their bits are the uint64 seeds).  Returns (uK, norms)
        with norms of shape (members, K // every + 1), or None without norms.
        With snap_steps (increasing steps in [0, K]) it returns (uK, norms,
        snaps), snaps of shape (members, len(snap_steps), N): each member's
        state at those steps (heat1d_run_async_ensemble_snapshots)."""
        _require_gpu(u0, seeds)
        if u0.dtype != self.dtype or u0.numel() != self.N * self.E:
            raise ValueError("u0 does not match the plan (dtype or size)")
        if seeds.dtype != torch.int64 or seeds.numel() != self.E:
            raise ValueError("seeds must be an int64 device tensor with one seed per member")
        out = torch.empty_like(u0) if out is None else out
        _require_gpu(out)
        if with_norms and norms is None:
            norms = torch.empty((self.E, K // every + 1), dtype=torch.float64, device=u0.device)
        if norms is not None:
            _require_gpu(norms)
            if norms.dtype != torch.float64 or norms.numel() != self.E * (K // every + 1):
                raise ValueError("norms must be a float64 device tensor of members*(K//every+1)")
        nptr = norms.data_ptr() if norms is not None else None
        if snap_steps is not None:
            steps = [int(x) for x in snap_steps]
            snaps = torch.empty((self.E, len(steps), self.N), dtype=self.dtype, device=u0.device)
            abi.heat1d_run_async_ensemble_snapshots(self.handle, u0.data_ptr(), out.data_ptr(), r,
                                                    c1, cN, K, d, seeds.data_ptr(), every, nptr,
                                                    steps, snaps.data_ptr(), _stream())
            return out, norms, snaps
        abi.heat1d_run_async_ensemble(self.handle, u0.data_ptr(), out.data_ptr(), r, c1, cN, K,
                                      d, seeds.data_ptr(), every, nptr, _stream())
        return out, norms

    def adjoint(self, u0, gK, r, c1, cN, K, d, seeds, want_uK: bool = False):
        """Gradients through every member's emulated run: returns (grad_u0
        (members, N), grad_r, grad_c1, grad_cN (members,) float64, uK or
        None)."""
        _require_gpu(u0, gK, seeds)
        if u0.dtype != self.dtype or u0.numel() != self.N * self.E or gK.dtype != self.dtype \
                or gK.numel() != self.N * self.E:
            raise ValueError("u0 / gK do not match the plan (dtype or size)")
        if seeds.dtype != torch.int64 or seeds.numel() != self.E:
            raise ValueError("seeds must be an int64 device tensor with one seed per member")
        nws = abi.heat1d_ensemble_adjoint_workspace_bytes(self.handle, K)
        ws = _workspace(nws, u0.device)
        gu = torch.empty_like(u0)
        g = torch.empty((3, self.E), dtype=torch.float64, device=u0.device)
        uK = torch.empty_like(u0) if want_uK else None
        abi.heat1d_run_async_ensemble_adjoint(
            self.handle, u0.data_ptr(), gK.data_ptr(), r, c1, cN, K, d, seeds.data_ptr(),
            uK.data_ptr() if uK is not None else None, gu.data_ptr(), g[0].data_ptr(),
            g[1].data_ptr(), g[2].data_ptr(), ws.data_ptr(), _stream())
        return gu, g[0], g[1], g[2], uK


def delay_schedule(P: int, K: int, d: int, seed: int, device="cuda") -> torch.Tensor:
    out = torch.empty((K, P, 2), dtype=torch.uint8, device=device)
    abi.heat1d_delay_schedule(P, K, d, seed, out.data_ptr(), _stream())
    return out


class BatchedPlan(_Plan):
    """Ragged batch of rods (heat1d_plan_batched); lengths and step counts are
    fixed at plan time."""

    def __init__(self, lengths, steps, dtype=torch.float32, device="cuda", **opts):
        self.lengths = [int(x) for x in lengths]
        self.steps = [int(x) for x in steps]
        self.dtype = dtype
        self.handle = abi.heat1d_plan_batched(self.lengths, self.steps, _dtype_code(dtype),
                                              opts or None)
        self.ws = _workspace(abi.heat1d_batched_workspace_bytes(self.handle), device)
        abi.heat1d_batched_prepare(self.handle, self.ws.data_ptr(), _stream())

    def close(self) -> None:
        self.ws = None
        super().close()

    @staticmethod
    def _check_args(u0, offsets, r, c1, cN, K):
        _require_gpu(u0, offsets, r, c1, cN, K)
        if offsets.dtype != torch.int64 or K.dtype != torch.int32:
            raise ValueError("offsets must be int64 and K int32")
        for t in (r, c1, cN):
            if t.dtype != torch.float64:
                raise ValueError("r, c1, cN must be float64 device tensors")

    def run(self, u0, offsets, r, c1, cN, K, out=None) -> torch.Tensor:
        self._check_args(u0, offsets, r, c1, cN, K)
        out = torch.empty_like(u0) if out is None else out
        abi.heat1d_run_batched(self.handle, u0.data_ptr(), out.data_ptr(), offsets.data_ptr(),
                               r.data_ptr(), c1.data_ptr(), cN.data_ptr(), K.data_ptr(),
                               self.ws.data_ptr(), _stream())
        return out

    def autotune(self, u0, offsets, r, c1, cN, K) -> float:
        """Time the candidate work orders on these buffers and keep the
        fastest (heat1d_autotune_batched); returns its time in ms."""
        self._check_args(u0, offsets, r, c1, cN, K)
        scratch = torch.empty_like(u0)
        return abi.heat1d_autotune_batched(self.handle, u0.data_ptr(), scratch.data_ptr(),
                                           offsets.data_ptr(), r.data_ptr(), c1.data_ptr(),
                                           cN.data_ptr(), K.data_ptr(), self.ws.data_ptr(),
                                           _stream())


class AdjointPlan(_Plan):
    """Forward with checkpoints and the discrete adjoint for `nrods` equal rods.
    With grad_sum=True the rods share the plan's r, c1 and cN: the library
    sums the per-rod sensitivities and every scalar gradient is one value."""

    def __init__(self, N: int, K: int, dtype=torch.float32, nrods: int = 1,
                 grad_sum: bool = False, **opts):
        self.N, self.K, self.dtype, self.nrods = int(N), int(K), dtype, int(nrods)
        self.nout = 1 if grad_sum else self.nrods
        o = dict(opts)
        o["nrods"] = self.nrods
        o["grad_sum"] = 1 if grad_sum else 0
        self.handle = abi.heat1d_plan_create(self.N, _dtype_code(dtype), o)
        self._ws = None

    def workspace(self, device) -> torch.Tensor:
        n = abi.heat1d_adjoint_workspace_bytes(self.handle, self.K)
        if self._ws is None or self._ws.numel() < n or self._ws.device != device:
            self._ws = _workspace(n, device)
        return self._ws

    def _check(self, *ts):
        _require_gpu(*ts)
        for t in ts:
            if t.dtype != self.dtype or t.numel() != self.N * self.nrods:
                raise ValueError("tensor does not match the plan (dtype or size)")

    def forward(self, u0, r, c1, cN, out=None):
        self._check(u0)
        out = torch.empty_like(u0) if out is None else out
        ws = self.workspace(u0.device)
        abi.heat1d_forward_checkpointed(self.handle, u0.data_ptr(), out.data_ptr(), r, c1, cN,
                                        self.K, ws.data_ptr(), _stream())
        return out

    def backward(self, gK, r, c1, cN):
        """(dL/du0, dL/dr) from the checkpoints of the preceding forward();
        dL/dr is float64 of shape (nrods,), or (1,) with grad_sum."""
        self._check(gK)
        if self._ws is None:
            raise RuntimeError("backward() needs the checkpoints of a forward() on this plan")
        gu = torch.empty_like(gK)
        gr = torch.empty(self.nout, dtype=torch.float64, device=gK.device)
        abi.heat1d_backward_checkpointed(self.handle, gK.data_ptr(), r, c1, cN, self.K,
                                         gu.data_ptr(), gr.data_ptr(), self._ws.data_ptr(),
                                         _stream())
        return gu, gr

    def adjoint(self, u0, gK, r, c1, cN, want_uK=False):
        self._check(u0, gK)
        ws = self.workspace(u0.device)
        gu = torch.empty_like(u0)
        gr = torch.empty(self.nout, dtype=torch.float64, device=u0.device)
        uK = torch.empty_like(u0) if want_uK else None
        abi.heat1d_adjoint(self.handle, u0.data_ptr(), gK.data_ptr(), r, c1, cN, self.K,
                           gu.data_ptr(), gr.data_ptr(), uK.data_ptr() if uK is not None else None,
                           ws.data_ptr(), _stream())
        return gu, gr, uK

    def ends(self, gK, r):
        """(dL/dc1, dL/dcN), float64 device tensors of shape (nrods,), or (1,)
        with grad_sum (heat1d_adjoint_ends)."""
        self._check(gK)
        ws = _workspace(abi.heat1d_adjoint_ends_workspace_bytes(self.handle), gK.device)
        g = torch.empty((2, self.nout), dtype=torch.float64, device=gK.device)
        abi.heat1d_adjoint_ends(self.handle, gK.data_ptr(), r, self.K, g[0].data_ptr(),
                                g[1].data_ptr(), ws.data_ptr(), _stream())
        return g[0], g[1]


class HeatFn(torch.autograd.Function):
    """u(K) = HeatFn.apply(u0, r, c1, cN, K, nrods): K synchronous steps of
    Eq.3 on `nrods` stacked rods, differentiable in u0, in the scalar r and in
    the end values c1, cN (floats, or 0-d tensors when their gradients are
    wanted).  The backward pass is the hand-written adjoint kernel with
    checkpoint recomputation; the rods share r, c1 and cN, so the plan is made
    with grad_sum and the library returns dL/dr, dL/dc1 and dL/dcN as single
    values (heat1d_adjoint_ends for the ends).  Nothing is computed here."""

    @staticmethod
    def forward(ctx, u0, r, c1, cN, K: int, nrods: int = 1):
        rv, c1v, cNv = float(r), float(c1), float(cN)
        plan = AdjointPlan(u0.numel() // nrods, K, u0.dtype, nrods=nrods, grad_sum=True)
        uK = plan.forward(u0.contiguous(), rv, c1v, cNv)
        ctx.plan, ctx.rv, ctx.c1, ctx.cN = plan, rv, c1v, cNv
        ctx.dtypes = [x.dtype if torch.is_tensor(x) else torch.float64 for x in (r, c1, cN)]
        return uK

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        need = ctx.needs_input_grad
        grad_u0 = grad_r = grad_c1 = grad_cN = None
        if need[0] or need[1]:
            gu, gr = ctx.plan.backward(g, ctx.rv, ctx.c1, ctx.cN)
            grad_u0 = gu if need[0] else None
            grad_r = gr.reshape(()).to(ctx.dtypes[0]) if need[1] else None
        if need[2] or need[3]:
            g1, gN = ctx.plan.ends(g, ctx.rv)
            grad_c1 = g1.reshape(()).to(ctx.dtypes[1]) if need[2] else None
            grad_cN = gN.reshape(()).to(ctx.dtypes[2]) if need[3] else None
        return grad_u0, grad_r, grad_c1, grad_cN, None, None
