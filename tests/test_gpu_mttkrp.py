"""GPU parity of MTTKRP against the FP64 oracle, through the C-ABI."""
import numpy as np
import pytest
import torch

from gpu_cases import (CANCELLATION_CASES, CANCELLATION_MIN_RATIO, TOL, announce, make_case, oracle_all_modes,
                       rel_err, rel_err_abs)
from oracle import oracle as O
from paper_1708_08976_amd import _abi, inputs

pytestmark = pytest.mark.gpu

# Shapes span several tiles with ragged tails, every shape class (mode 0,
# internal modes with short and long left products, last mode), unaligned
# rows (no 4-wide vector loads), single-index modes and N from 2 to 6.
# Size-1 modes next to mode n make the left or right Khatri-Rao product a
# single factor row rather than a row of ones.
SHAPES = [
    (37, 29, 41),
    (64, 48, 80),
    (96, 50, 70),
    (5, 7, 3, 11, 13),
    (16, 33, 2, 9),
    (3, 130, 21),
    (1, 17, 1, 19),
    (200, 3),
    (3, 200),
    (12, 12, 12, 12, 12),
    (6, 5, 4, 3, 2, 7),
    (1000, 1, 1),
    (1, 1, 1000),
    (31, 1, 257),
    (17, 19, 1),
    (1, 40, 1, 1),
    (20, 1, 30, 1),
    (1, 1, 1),
]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 13, 32, 70])
def test_mttkrp_f32_all_modes(dims, R):
    announce("mttkrp f32", dims, R)
    X, U = make_case(dims, R, seed=sum(dims) + R)
    refs = oracle_all_modes(X, dims, U)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(len(dims)):
        out = torch.full((dims[n], R), float("nan"), device="cuda")
        _abi.mttkrp(Xd, dims, Ud, n, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.isfinite(got).all(), "unwritten output entries, mode %d" % n
        if (dims, R, n) in CANCELLATION_CASES:
            absr = O.mttkrp(np.abs(X.numpy().ravel()), dims, [np.abs(u.numpy()) for u in U], n)
            assert np.linalg.norm(absr) >= CANCELLATION_MIN_RATIO * np.linalg.norm(refs[n])
            err = rel_err_abs(got, refs[n], absr)
        else:
            err = rel_err(got, refs[n])
        assert err <= TOL["f32"], (dims, R, n, err)


def test_config1_fp64_60x50x40_r8_every_mode():
    """The 60x50x40 FP64 workload (entries uniform[0,1), seed 1; factors
    N(0,1), seed 2): every mode within 1e-12 of the oracle, normwise."""
    dims, R = (60, 50, 40), 8
    X = inputs.uniform_tensor(dims, seed=1, dtype=torch.float64)
    U = inputs.normal_factors(dims, R, seed=2, dtype=torch.float64)
    refs = oracle_all_modes(X, dims, U)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(3):
        got = _abi.mttkrp(Xd, dims, Ud, n).cpu().numpy()
        err = rel_err(got, refs[n])
        print("60x50x40 fp64 mode %d: relative error %.3e" % (n, err), flush=True)
        assert err <= TOL["f64"], (n, err)


@pytest.mark.parametrize("dims", [(60, 50, 40), (7, 9, 11, 5), (23, 40, 3)])
@pytest.mark.parametrize("R", [8, 33, 128, 200, 256])
def test_mttkrp_f64_all_modes(dims, R):
    announce("mttkrp f64", dims, R)
    X, U = make_case(dims, R, seed=3 + R, dtype=torch.float64)
    refs = oracle_all_modes(X, dims, U)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(len(dims)):
        got = _abi.mttkrp(Xd, dims, Ud, n).cpu().numpy()
        assert rel_err(got, refs[n]) <= TOL["f64"], (dims, R, n)


@pytest.mark.parametrize("R", [200, 256])
def test_mttkrp_f32_wide_rank_column_blocks(R):
    dims = (40, 36, 30)
    announce("mttkrp wide", dims, R)
    X, U = make_case(dims, R, seed=R)
    refs = oracle_all_modes(X, dims, U)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(3):
        got = _abi.mttkrp(Xd, dims, Ud, n).cpu().numpy()
        assert rel_err(got, refs[n]) <= TOL["f32"], n


def test_long_left_product_uses_several_chunks():
    dims = (33, 47, 3, 2)  # IL for the last mode = 4653 > one l-chunk
    X, U = make_case(dims, 24, seed=77)
    refs = oracle_all_modes(X, dims, U)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(4):
        got = _abi.mttkrp(Xd, dims, Ud, n).cpu().numpy()
        assert rel_err(got, refs[n]) <= TOL["f32"]


def test_unaligned_base_pointer():
    dims = (20, 16, 12)
    X, U = make_case(dims, 8, seed=5)
    big = torch.zeros(X.numel() + 1, dtype=torch.float32)
    big[1:] = X.reshape(-1)
    Xd = big.cuda()[1:]  # 4-byte offset: 16-byte vector loads must be avoided
    Ud = [u.cuda() for u in U]
    refs = oracle_all_modes(X, dims, U)
    for n in range(3):
        got = _abi.mttkrp(Xd, dims, Ud, n).cpu().numpy()
        assert rel_err(got, refs[n]) <= TOL["f32"]


def test_bitwise_reproducible():
    dims = (64, 48, 80)
    X, U = make_case(dims, 32, seed=11)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(3):
        a = _abi.mttkrp(Xd, dims, Ud, n)
        b = _abi.mttkrp(Xd, dims, Ud, n)
        assert torch.equal(a, b)


def test_exact_rank_closed_form():
    """For X = [[U]] the result is U_n times the Hadamard product of the
    other Grams (a fact of the CP model, independent of both codes)."""
    dims = (48, 40, 36)
    R = 6
    U = inputs.normal_factors(dims, R, seed=21, dtype=torch.float64)
    X = inputs.cp_model_tensor(U)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    for n in range(3):
        H = torch.ones(R, R, dtype=torch.float64)
        for k in range(3):
            if k != n:
                H *= U[k].T @ U[k]
        want = (U[n] @ H).numpy()
        got = _abi.mttkrp(Xd, dims, Ud, n).cpu().numpy()
        assert rel_err(got, want) <= 1e-12


@pytest.mark.parametrize("Js,R", [((7,), 5), ((3, 4), 16), ((5, 2, 3), 33), ((2, 3, 2, 5), 8)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_krp_rows_matches_oracle(Js, R, dtype):
    mats = [torch.randn(J, R, dtype=dtype) for J in Js]
    ref = O.krp_rows([m.numpy() for m in mats])
    got = _abi.krp_rows([m.cuda() for m in mats]).cpu().numpy()
    tol = 1e-6 if dtype == torch.float32 else 1e-15
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol)
    j0 = 3 if ref.shape[0] > 4 else 1
    part = _abi.krp_rows([m.cuda() for m in mats], j0=j0, nrows=ref.shape[0] - j0 - 1).cpu().numpy()
    np.testing.assert_allclose(part, ref[j0:-1], rtol=tol, atol=tol)


@pytest.mark.parametrize("dims,offset", [((1000, 37), 0), ((999, 37), 0), ((1000, 37), 1), ((64, 64, 64), 4)])
def test_split_bf16_bit_exact_and_xnorm2(dims, offset):
    """Both helpers on 16-byte-aligned data whose size is a multiple of 8
    (vector loads) and on an odd size or a shifted start (scalar loads)."""
    announce("split/xnorm2", dims, offset)
    n = int(np.prod(dims))
    x = inputs.normal_tensor(dims, seed=9).reshape(-1)
    buf = torch.zeros(n + offset, device="cuda")
    buf[offset:] = x.cuda()
    xd = buf[offset:]
    pbuf = torch.zeros(2 * n + 2 * offset, dtype=torch.int16, device="cuda")
    planes_d = pbuf[2 * offset:]
    _abi.split_bf16(xd, planes=planes_d)
    want = inputs.split_bf16_planes(x)
    assert torch.equal(planes_d.cpu(), want)
    xh = x.numpy()
    # every square is exact in float64 (24- or 16-bit significands), so each
    # side's sum of n non-negative terms is within (n - 1) 2^-53 relative of
    # the exact value, whatever its order
    tol = 2 * n * 2.0 ** -53
    got = _abi.xnorm2(xd, dims).item()
    assert got == pytest.approx(O.xnorm2(xh, dims), rel=tol)
    # the pair tensor's squared norm: the oracle on the pair values
    gotp = _abi.xnorm2(planes_d, dims, dtype=_abi.CPM_BF16X2).item()
    refp = O.xnorm2(want.numpy().view(np.uint16), dims, xtype=O.BF16PAIR)
    assert gotp == pytest.approx(refp, rel=tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16x2"])
@pytest.mark.parametrize("R", [8, 40, 130])
def test_many_blocks_per_work_group(dtype, R):
    """A long outer range (40000 blocks for mode 1) gives every work-group
    more blocks than one scale table holds, so the table is refilled
    between chunks; every mode against the oracle."""
    dims = (32, 8, 40000)
    announce("many blocks", dtype, dims, R)
    X, U = make_case(dims, R, seed=R + 5)
    Ud = [u.cuda() for u in U]
    if dtype == "f32":
        Xd, code, xh, xt = X.cuda(), _abi.CPM_F32, X.numpy().ravel(), None
    else:
        planes = inputs.split_bf16_planes(X)
        Xd, code, xh, xt = planes.cuda(), _abi.CPM_BF16X2, planes.numpy().view(np.uint16), O.BF16PAIR
    for n in range(3):
        ref = O.mttkrp(xh, dims, [u.numpy() for u in U], n, xtype=xt)
        got = _abi.mttkrp(Xd, dims, Ud, n, dtype=code).cpu().numpy()
        assert rel_err(got, ref) <= TOL[dtype], (n, R)


@pytest.mark.parametrize("dims", [(4096, 300), (2048, 500, 3), (8192, 96, 2)])
@pytest.mark.parametrize("R", [8, 32, 64])
def test_wide_output_long_resident_chunk(dims, R):
    """Mode 0 with a wide output and one long contracted mode: split-K
    partials would rival X, so the float32 plan keeps the whole inner mode
    (up to 512 rows) as one resident chunk and writes the result directly."""
    announce("wide output", dims, R)
    X, U = make_case(dims, R, seed=R + len(dims))
    ref = O.mttkrp(X.numpy().ravel(), dims, [u.numpy() for u in U], 0)
    got = _abi.mttkrp(X.cuda(), dims, [u.cuda() for u in U], 0).cpu().numpy()
    assert rel_err(got, ref) <= TOL["f32"]
