"""GPU parity of the split-bfloat16 path (CPM_BF16X2) against the FP64 oracle.

The tensor is handed over as its hi and lo bfloat16 planes.  The oracle
evaluates the same pair values (hi + lo) in float64, so the comparison
isolates the kernels' arithmetic: the Khatri-Rao values split into bf16
pairs, the three-product MFMA contraction and its float32 accumulation.  A
second check compares with the oracle on the float32 tensor the planes came
from, which adds the (about 2^-17 relative) representation error of the
pair.
"""
import numpy as np
import pytest
import torch

from bf16_variants import VARIANT_CASES
from gpu_cases import TOL, announce, make_case, rel_err
from oracle import oracle as O
from paper_1708_08976_amd import _abi, inputs

pytestmark = pytest.mark.gpu

# Every shape class: mode 0 and short left products (right-first kernel,
# 8-wide loads when the row length is a multiple of 8, single loads
# otherwise), left products of 32 or more (left-first kernel, one or several
# chunks), size-1 neighbours, ragged tails in every tiled dimension.
SHAPES = [
    (37, 29, 41),
    (64, 48, 80),
    (40, 24, 36),
    (5, 7, 3, 11, 13),
    (16, 33, 2, 9),
    (3, 130, 21),
    (1, 17, 1, 19),
    (200, 3),
    (3, 200),
    (12, 12, 12, 12, 12),
    (1000, 1, 1),
    (1, 1, 1000),
    (31, 1, 257),
    (1, 40, 1, 1),
    (33, 47, 3, 2),
    (1, 1, 1),
]


def pair_case(dims, R, seed):
    X, U = make_case(dims, R, seed)
    planes = inputs.split_bf16_planes(X)
    return X, U, planes


def oracle_pair_all_modes(planes, dims, U):
    P = planes.numpy().view(np.uint16)
    Uh = [u.numpy() for u in U]
    return [O.mttkrp(P, dims, Uh, n, xtype=O.BF16PAIR) for n in range(len(dims))]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 13, 32, 70, 128])
def test_mttkrp_split_bf16_all_modes(dims, R):
    announce("mttkrp bf16x2", dims, R)
    X, U, planes = pair_case(dims, R, seed=sum(dims) + 7 * R)
    refs = oracle_pair_all_modes(planes, dims, U)
    Pd, Ud = planes.cuda(), [u.cuda() for u in U]
    for n in range(len(dims)):
        out = torch.full((dims[n], R), float("nan"), device="cuda")
        _abi.mttkrp(Pd, dims, Ud, n, out=out, dtype=_abi.CPM_BF16X2)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.isfinite(got).all(), "unwritten output entries, mode %d" % n
        err = rel_err(got, refs[n])
        assert err <= TOL["bf16x2"], (dims, R, n, err)


@pytest.mark.parametrize("R", [200, 256])
def test_mttkrp_split_bf16_wide_rank(R):
    dims = (40, 36, 30)
    announce("mttkrp bf16x2 wide", dims, R)
    X, U, planes = pair_case(dims, R, seed=R + 1)
    refs = oracle_pair_all_modes(planes, dims, U)
    Pd, Ud = planes.cuda(), [u.cuda() for u in U]
    for n in range(3):
        got = _abi.mttkrp(Pd, dims, Ud, n, dtype=_abi.CPM_BF16X2).cpu().numpy()
        assert rel_err(got, refs[n]) <= TOL["bf16x2"], n


def test_split_bf16_against_float32_tensor():
    """Against the oracle on the original float32 tensor: kernel arithmetic
    plus the representation error of the pair, still within 1e-4."""
    dims = (64, 48, 80)
    R = 32
    X, U, planes = pair_case(dims, R, seed=3)
    Xh = X.numpy().ravel()
    Uh = [u.numpy() for u in U]
    Pd, Ud = planes.cuda(), [u.cuda() for u in U]
    for n in range(3):
        ref = O.mttkrp(Xh, dims, Uh, n)
        got = _abi.mttkrp(Pd, dims, Ud, n, dtype=_abi.CPM_BF16X2).cpu().numpy()
        assert rel_err(got, ref) <= TOL["bf16x2"], n


def test_split_bf16_device_split_matches_host_planes():
    """The planes the library makes from a float32 tensor give the same
    MTTKRP, bit for bit, as the planes made on the host."""
    dims = (33, 40, 24)
    X, U, planes = pair_case(dims, 16, seed=12)
    Pd = _abi.split_bf16(X.cuda())
    assert torch.equal(Pd.cpu(), planes)
    Ud = [u.cuda() for u in U]
    for n in range(3):
        a = _abi.mttkrp(Pd, dims, Ud, n, dtype=_abi.CPM_BF16X2)
        b = _abi.mttkrp(planes.cuda(), dims, Ud, n, dtype=_abi.CPM_BF16X2)
        assert torch.equal(a, b)


def test_split_bf16_bitwise_reproducible():
    dims = (64, 48, 80)
    X, U, planes = pair_case(dims, 32, seed=4)
    Pd, Ud = planes.cuda(), [u.cuda() for u in U]
    for n in range(3):
        a = _abi.mttkrp(Pd, dims, Ud, n, dtype=_abi.CPM_BF16X2)
        b = _abi.mttkrp(Pd, dims, Ud, n, dtype=_abi.CPM_BF16X2)
        assert torch.equal(a, b)


def test_split_bf16_exact_products():
    """Entries and factors that are bf16 values: the lo plane of X is zero
    and every Khatri-Rao value (a product of two bf16 values) splits into
    hi + lo exactly, so all MFMA products are exact and only the float32
    accumulation rounds.  The result must then agree with float64 far more
    closely than the 1e-4 target."""
    dims = (48, 40, 36)
    R = 24
    X = inputs.normal_tensor(dims, seed=31).to(torch.bfloat16).float()
    U = [u.to(torch.bfloat16).float() for u in inputs.normal_factors(dims, R, seed=32)]
    planes = inputs.split_bf16_planes(X)
    assert not planes[X.numel():].any()
    Xh = X.numpy().ravel()
    Pd, Ud = planes.cuda(), [u.cuda() for u in U]
    for n in range(3):
        ref = O.mttkrp(Xh, dims, [u.numpy() for u in U], n)
        got = _abi.mttkrp(Pd, dims, Ud, n, dtype=_abi.CPM_BF16X2).cpu().numpy()
        assert rel_err(got, ref) <= 2e-6, n


@pytest.mark.parametrize("dims,R,mode,name", VARIANT_CASES, ids=[c[3] for c in VARIANT_CASES])
def test_split_bf16_lo_plane_is_used_by_every_variant(dims, R, mode, name):
    """One case per kernel variant, chosen so that the tensor's lo plane
    carries more than the tolerance: the oracle's result with the lo plane
    zeroed differs from the pair result by over 10x the 1e-4 bound, so a
    variant that lost the lo products would fail the first check.  The
    kernel is then run on the hi plane alone and must match the oracle on
    those values (it reads what it is given, not a cached plane)."""
    announce("bf16x2 lo plane", name, dims, R, mode)
    X, U, planes = pair_case(dims, R, seed=sum(dims) + 3 * R + mode)
    I = X.numel()
    hi_only = planes.clone()
    hi_only[I:] = 0
    Uh = [u.numpy() for u in U]
    ref = O.mttkrp(planes.numpy().view(np.uint16), dims, Uh, mode, xtype=O.BF16PAIR)
    ref_hi = O.mttkrp(hi_only.numpy().view(np.uint16), dims, Uh, mode, xtype=O.BF16PAIR)
    assert rel_err(ref_hi, ref) > 10 * TOL["bf16x2"]
    Ud = [u.cuda() for u in U]
    got = _abi.mttkrp(planes.cuda(), dims, Ud, mode, dtype=_abi.CPM_BF16X2).cpu().numpy()
    assert rel_err(got, ref) <= TOL["bf16x2"], rel_err(got, ref)
    got_hi = _abi.mttkrp(hi_only.cuda(), dims, Ud, mode, dtype=_abi.CPM_BF16X2).cpu().numpy()
    assert rel_err(got_hi, ref_hi) <= TOL["bf16x2"]
    assert rel_err(got_hi, ref) > TOL["bf16x2"]
