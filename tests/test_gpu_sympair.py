"""GPU parity of MTTKRP on symmetric-pair packed storage (the triangle i <= j
of two symmetric modes) against the FP64 oracle's definition for packed
tensors, and against the ordinary MTTKRP of the unpacked tensor."""
import numpy as np
import pytest
import torch

from gpu_cases import TOL, announce, rel_err
from oracle import oracle as O
from paper_1708_08976_amd import _abi, inputs

pytestmark = pytest.mark.gpu

CODES = {"f32": _abi.CPM_F32, "f64": _abi.CPM_F64, "bf16x2": _abi.CPM_BF16X2}


def symmetric_normal(dims, seed, dtype=torch.float32):
    """N(0,1) entries made symmetric in modes 0 and 1 (random diagonal)."""
    x = inputs.normal_tensor(dims, seed=seed, dtype=dtype)
    return (x + x.transpose(-1, -2)).contiguous()


def packed_case(dims, R, seed, kind, correlation=False):
    tdt = torch.float64 if kind == "f64" else torch.float32
    if correlation:
        X = inputs.symmetric_pair_tensor(dims, seed=seed, dtype=tdt)
    else:
        X = symmetric_normal(dims, seed, dtype=tdt)
    U = inputs.normal_factors(dims, R, seed=seed + 1, dtype=tdt)
    Xp = inputs.pack_sympair(X, dims)
    if kind == "bf16x2":
        full_dev = inputs.split_bf16_planes(X)
        pk = inputs.split_bf16_planes(Xp)
        return X, U, pk, pk.numpy().view(np.uint16), O.BF16PAIR, full_dev
    return X, U, Xp, Xp.numpy().ravel(), None, X


SHAPES = [(5, 5, 7), (33, 33, 9), (64, 64, 3, 5), (1, 1, 40), (17, 17, 2, 3, 2), (40, 40, 1, 6), (130, 130, 4)]


@pytest.mark.parametrize("kind", ["f32", "f64", "bf16x2"])
@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 13, 32, 70])
def test_mttkrp_sympair_all_modes_match_oracle(kind, dims, R):
    announce("sympair", kind, dims, R)
    X, U, Xp, Xph, xt, full = packed_case(dims, R, seed=sum(dims) + R, kind=kind)
    Ud = [u.cuda() for u in U]
    outs = _abi.mttkrp_sympair(Xp.cuda(), dims, Ud, dtype=CODES[kind])
    torch.cuda.synchronize()
    Uh = [u.numpy() for u in U]
    fulld = full.cuda()
    for n in range(len(dims)):
        got = outs[n].cpu().numpy()
        assert np.isfinite(got).all(), n
        ref = O.mttkrp_sympair(Xph, dims, Uh, n, xtype=xt)
        err = rel_err(got, ref)
        assert err <= TOL[kind], (n, err)
        # the ordinary MTTKRP of the unpacked tensor agrees too
        plain = _abi.mttkrp(fulld, dims, Ud, n, dtype=CODES[kind]).cpu().numpy()
        assert rel_err(got, plain) <= 2 * TOL[kind], n


@pytest.mark.parametrize("kind", ["f32", "f64", "bf16x2"])
@pytest.mark.parametrize("dims", [(5, 5, 7), (64, 64, 3, 5), (130, 130, 4), (1, 1, 3)])
def test_pack_sympair_bit_exact(kind, dims):
    tdt = torch.float64 if kind == "f64" else torch.float32
    X = symmetric_normal(dims, 3, dtype=tdt)
    want = inputs.pack_sympair(X, dims)
    if kind == "bf16x2":
        got = _abi.pack_sympair(inputs.split_bf16_planes(X).cuda(), dims, dtype=_abi.CPM_BF16X2)
        assert torch.equal(got.cpu(), inputs.split_bf16_planes(want))
    else:
        got = _abi.pack_sympair(X.cuda(), dims)
        assert torch.equal(got.cpu(), want.reshape(-1))


def test_mttkrp_sympair_subsets_and_reproducible():
    dims, R = (33, 33, 9, 4), 16
    X, U, Xp, Xph, xt, _ = packed_case(dims, R, seed=7, kind="f32")
    Xd, Ud = Xp.cuda(), [u.cuda() for u in U]
    Uh = [u.numpy() for u in U]
    for modes in [(0,), (1,), (0, 1), (2,), (3,), (2, 3), (0, 3), (1, 2, 3)]:
        sentinel = [torch.full((d, R), 7.0, device="cuda") for d in dims]
        outs = [sentinel[n] if n in modes else None for n in range(4)]
        _abi.mttkrp_sympair(Xd, dims, Ud, outs=outs)
        torch.cuda.synchronize()
        for n in range(4):
            if n in modes:
                assert rel_err(sentinel[n].cpu().numpy(), O.mttkrp_sympair(Xph, dims, Uh, n)) <= TOL["f32"]
            else:
                assert bool((sentinel[n] == 7.0).all())
    a = _abi.mttkrp_sympair(Xd, dims, Ud)
    b = _abi.mttkrp_sympair(Xd, dims, Ud)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("R,kind", [(64, "f32"), (128, "bf16x2"), (128, "f32")])
def test_sympair_full_size_correlation_tensor(R, kind):
    """256x256x512x32 correlation-style tensor, packed: whole outputs against
    the unpacked tensor's MTTKRP (the same launches the benchmark times),
    and the closed form of a symmetric exact-rank model (U_0 = U_1) on the
    whole output."""
    dims = (256, 256, 512, 32)
    announce("sympair full", dims, R, kind)
    code = CODES[kind]
    X = inputs.symmetric_pair_tensor(dims, seed=6, device="cuda")
    U = inputs.normal_factors(dims, R, seed=7 if R == 64 else 8, device="cuda")
    full = X if kind == "f32" else _abi.split_bf16(X.reshape(-1))
    packed = _abi.pack_sympair(full, dims, dtype=code)
    del X
    got = _abi.mttkrp_sympair(packed, dims, U, dtype=code)
    for n in range(4):
        plain = _abi.mttkrp(full, dims, U, n, dtype=code)
        e = rel_err(got[n].cpu().numpy(), plain.cpu().numpy())
        print("sympair %s R=%d mode %d vs unpacked: %.3e" % (kind, R, n, e), flush=True)
        assert e <= 2 * TOL[kind], (n, e)
    del full, packed
    # symmetric exact-rank model: X = [[A, A, U_2, U_3]]
    U64 = inputs.normal_factors(dims, R, seed=R + 40, device="cuda", dtype=torch.float64)
    U64[1] = U64[0]
    Xm = inputs.cp_model_tensor(U64).float()
    Xm = Xm if kind == "f32" else _abi.split_bf16(Xm.reshape(-1))
    pm = _abi.pack_sympair(Xm, dims, dtype=code)
    del Xm
    got = _abi.mttkrp_sympair(pm, dims, [u.float() for u in U64], dtype=code)
    Uh = [u.cpu().numpy() for u in U64]
    for n in range(4):
        H = np.ones((R, R))
        for k in range(4):
            if k != n:
                H *= Uh[k].T @ Uh[k]
        e = rel_err(got[n].cpu().numpy(), Uh[n] @ H)
        print("sympair %s R=%d mode %d closed form: %.3e" % (kind, R, n, e), flush=True)
        assert e <= TOL[kind], (n, e)
