"""GPU parity of cpm_residual2, the squared residual ||X - [[U]]||_F^2 with
the model recomputed on the fly, against the oracle's entry-by-entry FP64
residual.

Tolerance, from the arithmetic: each model entry is a float32 sum of R
products of N float32 factors, so its error is at most
(R + N + 2) 2^-24 sum_c prod_k |U_k(i_k, c)|.  The Frobenius norm of that
majorant has a closed form, sqrt(sum of the Hadamard product of the Grams
of |U_k|), which gives a bound db on ||delta||; the squared residual is then
within 2 ||E|| db + db^2 of the exact value (the float64 sums add a
negligible I 2^-53 relative).
"""
import numpy as np
import pytest
import torch

from gpu_cases import announce, make_case
from oracle import oracle as O
from paper_1708_08976_amd import _abi, inputs

pytestmark = pytest.mark.gpu

SHAPES = [
    (37, 29, 41),
    (64, 48, 80),
    (5, 7, 3, 11, 13),
    (16, 33, 2, 9),
    (1, 17, 1, 19),
    (200, 3),
    (3, 200),
    (1000, 1, 1),
    (1, 1, 1000),
    (31, 1, 257),
    (1, 1, 1),
    (33, 47, 3, 2),
    (130, 130),
    (12, 12, 12, 12, 12),
]


def model_bound(U, R):
    """db = (R + N + 2) 2^-24 ||[[|U|]]||_F, the latter from the Grams."""
    H = np.ones((R, R))
    for u in U:
        a = np.abs(np.asarray(u, dtype=np.float64))
        H *= a.T @ a
    return (R + len(U) + 2) * 2.0 ** -24 * np.sqrt(H.sum())


def check(got, ref, U, R):
    db = model_bound(U, R)
    tol = 2 * np.sqrt(max(ref, 0.0)) * db + db * db + 1e-12 * ref
    assert abs(got - ref) <= tol, (got, ref, tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16x2"])
@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 13, 32, 33, 64, 70, 128])
def test_residual2_matches_oracle(dims, R, dtype):
    announce("residual2", dtype, dims, R)
    X, U = make_case(dims, R, seed=sum(dims) + 3 * R)
    Ud = [u.cuda() for u in U]
    Uh = [u.numpy() for u in U]
    if dtype == "f32":
        got = _abi.residual2(X.cuda(), dims, Ud).item()
        ref = O.residual2(X.numpy().ravel(), dims, Uh)
    else:
        planes = inputs.split_bf16_planes(X)
        got = _abi.residual2(planes.cuda(), dims, Ud, dtype=_abi.CPM_BF16X2).item()
        ref = O.residual2(planes.numpy().view(np.uint16), dims, Uh, xtype=O.BF16PAIR)
    check(got, ref, Uh, R)


@pytest.mark.parametrize("R", [8, 32])
def test_residual2_of_a_close_fit(R):
    """A rank-R model plus 1e-3 noise: the residual is 1e-6 of ||X||^2, where
    the identity form in float32 keeps about one digit; the fused residual
    still meets the bound against the oracle."""
    dims = (40, 36, 44)
    X, U = inputs.noisy_low_rank(dims, R, seed_factors=51, seed_noise=52, eta=1e-3)
    Uh = [u.numpy() for u in U]
    got = _abi.residual2(X.cuda(), dims, [u.cuda() for u in U]).item()
    ref = O.residual2(X.numpy().ravel(), dims, Uh)
    x2 = float(np.sum(X.numpy().astype(np.float64) ** 2))
    assert ref < 1e-5 * x2
    check(got, ref, Uh, R)


def test_residual2_bitwise_reproducible():
    dims, R = (64, 48, 80), 32
    X, U = make_case(dims, R, seed=61)
    Xd, Ud = X.cuda(), [u.cuda() for u in U]
    a = _abi.residual2(Xd, dims, Ud)
    b = _abi.residual2(Xd, dims, Ud)
    assert torch.equal(a, b)


@pytest.mark.slow
@pytest.mark.timeout(300)
def test_residual2_512cube_fp32_r32():
    """The 512^3 workload: rank-32 model with 1% noise and its true factors,
    and the same tensor against the N(0,1) starting factors."""
    dims, R = (512, 512, 512), 32
    announce("residual2 512^3")
    X, U = inputs.noisy_low_rank(dims, R, seed_factors=3, seed_noise=4, eta=0.01, device="cuda")
    Xh = X.cpu().numpy().ravel()
    for tag, F in [("true factors", U), ("start factors", inputs.normal_factors(dims, R, seed=5, device="cuda"))]:
        Fh = [f.cpu().numpy() for f in F]
        got = _abi.residual2(X, dims, F).item()
        ref = O.residual2(Xh, dims, Fh)
        print("512^3 residual2 (%s): gpu %.12e oracle %.12e rel %.2e" % (tag, got, ref, abs(got - ref) / ref),
              flush=True)
        check(got, ref, Fh, R)


def test_cploss_exact_forward_on_a_close_fit():
    """CPLoss with exact=True: the forward is 1/2 of the fused residual, so on
    a model that fits to 1e-3 it meets the oracle's direct loss within the
    float32-model bound, where the identity form may not; the backward is
    the same hand-written gradient either way."""
    from paper_1708_08976_amd import api
    dims, R = (40, 36, 44), 8
    X, U = inputs.noisy_low_rank(dims, R, seed_factors=71, seed_noise=72, eta=1e-3)
    Uh = [u.numpy() for u in U]
    ref = 0.5 * O.residual2(X.numpy().ravel(), dims, Uh)
    Xt = X.cuda()  # torch shape = reversed paper dims
    Ut = [u.cuda().requires_grad_(True) for u in reversed(U)]
    f = api.cp_loss(Xt, Ut, exact=True)
    db = model_bound(Uh, R)
    assert abs(f.item() - ref) <= 0.5 * (2 * np.sqrt(2 * ref) * db + db * db) + 1e-12 * ref
    f.backward()
    U64 = [u.astype(np.float64) for u in Uh]
    G, _, _ = O.cp_grad(X.numpy().ravel(), dims, U64)
    for n in range(3):
        # scale: the two terms U_n H_n and M_n whose difference is the gradient
        H = np.ones((R, R))
        for k in range(3):
            if k != n:
                H *= U64[k].T @ U64[k]
        scale = np.linalg.norm(U64[n] @ H) + np.linalg.norm(G[n] + U64[n] @ H)
        g = Ut[2 - n].grad.cpu().numpy()
        assert np.linalg.norm(g - G[n]) <= 1e-5 * scale, n
    # the torch-order helper is the same call
    assert api.residual2(Xt, [u.detach() for u in Ut]).item() == pytest.approx(2 * f.item(), rel=1e-15)


@pytest.mark.slow
@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype", ["f32", "bf16x2"])
def test_residual2_64p5_full_size(dtype):
    """The 64^5 workload (rank-32 model, 5% noise) with its true factors:
    every one of the 1.07e9 entries, against the oracle's direct residual."""
    dims, R = (64,) * 5, 32
    announce("residual2 64^5", dtype)
    X, U = inputs.noisy_low_rank(dims, R, seed_factors=9, seed_noise=10, eta=0.05, device="cuda")
    Uh = [u.cpu().numpy() for u in U]
    if dtype == "f32":
        got = _abi.residual2(X, dims, U).item()
        ref = O.residual2(X.cpu().numpy().ravel(), dims, Uh)
    else:
        P = _abi.split_bf16(X.reshape(-1))
        got = _abi.residual2(P, dims, U, dtype=_abi.CPM_BF16X2).item()
        ref = O.residual2(P.cpu().numpy().view(np.uint16), dims, Uh, xtype=O.BF16PAIR)
    print("64^5 residual2 %s: gpu %.12e oracle %.12e rel %.2e" % (dtype, got, ref, abs(got - ref) / ref), flush=True)
    check(got, ref, Uh, R)


@pytest.mark.slow
@pytest.mark.timeout(300)
def test_residual2_sym4d_fp32_r64_full_size():
    dims, R = (256, 256, 512, 32), 64
    announce("residual2 sym4d")
    X = inputs.symmetric_pair_tensor(dims, seed=6, device="cuda")
    U = inputs.normal_factors(dims, R, seed=7, device="cuda")
    Uh = [u.cpu().numpy() for u in U]
    got = _abi.residual2(X, dims, U).item()
    ref = O.residual2(X.cpu().numpy().ravel(), dims, Uh)
    print("sym4d residual2: gpu %.12e oracle %.12e rel %.2e" % (got, ref, abs(got - ref) / ref), flush=True)
    check(got, ref, Uh, R)
