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
    """Error scaled by the MTTKRP of |X| and |U_k| (the size of the summed
    terms) instead of by the result.  Used only for the named cases whose
    result is cancellation-small, where no float32 summation can meet a
    relative bound on the result itself (see CANCELLATION_CASES)."""
    got = np.asarray(got, dtype=np.float64)
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref_abs), 1e-300)


# (dims, R, mode) of sweep cases whose result is dominated by cancellation:
# the summed terms are over 1e3 times the result (checked where used).
# (1, 1, 1000) at R = 1, modes 0 and 1 (the same single output value, as
# I_0 = I_1 = 1): the sum of 1000 terms of total size 298 that comes to
# -0.0108 (a factor 2.8e4); a sequential float32 sum is off by 9e-4
# relative.
CANCELLATION_CASES = {((1, 1, 1000), 1, 0), ((1, 1, 1000), 1, 1)}
CANCELLATION_MIN_RATIO = 1e3


def make_case(dims, R, seed, dtype=torch.float32):
    X = inputs.normal_tensor(dims, seed=seed, dtype=dtype)
    U = inputs.normal_factors(dims, R, seed=seed + 1, dtype=dtype)
    return X, U


def oracle_all_modes(X, dims, U):
    Xh = X.numpy().ravel()
    Uh = [u.numpy() for u in U]
    return [O.mttkrp(Xh, dims, Uh, n) for n in range(len(dims))]


def announce(*parts):
    print(" ".join(str(p) for p in parts), flush=True)
