"""Shared helpers for the GPU parity tests."""
import numpy as np
import torch

from oracle import oracle as O
from paper_1708_08976_amd import inputs

# Tolerances (normwise relative error against the FP64 oracle):
# float32 path 1e-5 and float64 path 1e-12, the targets stated for the plain
# method; the split-bf16 path 1e-4.
TOL = {"f32": 1e-5, "f64": 1e-12, "bf16x2": 1e-4}


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    return num / den if den > 0 else num


def rel_err_abs(got, ref, ref_abs):
    """Normwise error scaled by the MTTKRP of |X| and |U_k|: the size of the
    terms being summed, which bounds rounding error whatever the
    cancellation in the sum (a result that happens to be tiny still has
    errors of the order of its largest terms)."""
    got = np.asarray(got, dtype=np.float64)
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref_abs), 1e-300)


def make_case(dims, R, seed, dtype=torch.float32):
    X = inputs.normal_tensor(dims, seed=seed, dtype=dtype)
    U = inputs.normal_factors(dims, R, seed=seed + 1, dtype=dtype)
    return X, U


def oracle_all_modes(X, dims, U):
    Xh = X.numpy().ravel()
    Uh = [u.numpy() for u in U]
    return [O.mttkrp(Xh, dims, Uh, n) for n in range(len(dims))]


def oracle_abs_all_modes(X, dims, U):
    Xh = np.abs(X.numpy().ravel())
    Uh = [np.abs(u.numpy()) for u in U]
    return [O.mttkrp(Xh, dims, Uh, n) for n in range(len(dims))]


def announce(*parts):
    print(" ".join(str(p) for p in parts), flush=True)
