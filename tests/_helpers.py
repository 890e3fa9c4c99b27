"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

F32_TOL = 2e-5   # normwise, FP32 kernels vs the FP64 oracle on FP32-rounded inputs
F64_TOL = 1e-12  # normwise, FP64 kernels vs the FP64 oracle


def normwise(got, ref):
    """max_i |got_i - ref_i| / max_i |ref_i|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(got - ref))) / scale


def tol_for(dtype_name):
    return F32_TOL if dtype_name == "f32" else F64_TOL


def torch_dtype(name):
    import torch
    return torch.float32 if name == "f32" else torch.float64


def np_dtype(name):
    return np.float32 if name == "f32" else np.float64


def windows_for_samples(N, idx, K):
    """[(a, b)] segments of the rod whose points at distance >= K from a cut
    end contain each sample index; merged when they overlap."""
    segs = []
    for i in sorted(set(int(x) for x in idx)):
        a = max(0, i - K - 1)
        b = min(N, i + K + 2)
        if segs and a <= segs[-1][1]:
            segs[-1] = (segs[-1][0], max(segs[-1][1], b))
        else:
            segs.append((a, b))
    return segs


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
