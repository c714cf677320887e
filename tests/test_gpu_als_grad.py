"""GPU parity of the CP-ALS sweep, the CP gradient and the CPLoss autograd
function against the FP64 oracle, plus finite-difference checks."""
import numpy as np
import pytest
import torch

from gpu_cases import TOL, announce, rel_err
from oracle import oracle as O
from paper_1708_08976_amd import _abi, api, inputs

pytestmark = pytest.mark.gpu


def kappa_max(dims, U):
    """Largest condition number of the Hadamard-of-Grams matrices."""
    k = 1.0
    for n in range(len(dims)):
        H = np.ones((U[0].shape[1],) * 2)
        for m in range(len(dims)):
            if m != n:
                H *= U[m].T @ U[m]
        k = max(k, np.linalg.cond(H))
    return k


def test_als_sweep_fp64_config1():
    """60x50x40 FP64, entries uniform[0,1) (seed 1), R = 8 factors N(0,1)
    (seed 2): one sweep on the GPU against the oracle sweep."""
    dims, R = (60, 50, 40), 8
    announce("als fp64", dims, R)
    X = inputs.uniform_tensor(dims, seed=1, dtype=torch.float64)
    U = inputs.normal_factors(dims, R, seed=2, dtype=torch.float64)
    ref, fit_ref = O.cp_als_step(X.numpy().ravel(), dims, [u.numpy() for u in U])
    Ud = [u.cuda() for u in U]
    fit = _abi.cp_als_step(X.cuda(), dims, Ud)
    for g, r in zip(Ud, ref):
        assert rel_err(g.cpu().numpy(), r) <= 1e-10
    assert fit == pytest.approx(fit_ref, abs=1e-10)


def test_als_sweep_fp32_on_cast_tensor():
    dims, R = (60, 50, 40), 8
    X = inputs.uniform_tensor(dims, seed=1, dtype=torch.float32)
    U = inputs.normal_factors(dims, R, seed=2, dtype=torch.float32)
    Uh = [u.numpy().astype(np.float64) for u in U]
    ref, fit_ref = O.cp_als_step(X.numpy().ravel(), dims, Uh)
    kap = kappa_max(dims, ref)
    Ud = [u.cuda() for u in U]
    fit = _abi.cp_als_step(X.cuda(), dims, Ud)
    for g, r in zip(Ud, ref):
        assert rel_err(g.cpu().numpy(), r) <= 1e-5 * kap
    assert fit == pytest.approx(fit_ref, abs=1e-5)


@pytest.mark.parametrize("dims,R", [((30, 20, 25, 6), 5), ((40, 33, 17), 16), ((12, 10, 9, 8, 7), 3)])
def test_als_true_factors_fixed_point(dims, R):
    U = inputs.normal_factors(dims, R, seed=31, dtype=torch.float64)
    X = inputs.cp_model_tensor(U)
    Ud = [u.cuda().clone() for u in U]
    fit = _abi.cp_als_step(X.cuda(), dims, Ud)
    for g, u in zip(Ud, U):
        assert rel_err(g.cpu().numpy(), u.numpy()) <= 1e-9
    assert fit == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_als_not_positive_definite_restores_factors(dtype):
    dims, R = (20, 18, 16), 4
    X = inputs.normal_tensor(dims, seed=41, dtype=dtype).cuda()
    U = [u.cuda() for u in inputs.normal_factors(dims, R, seed=42, dtype=dtype)]
    U[2][:, 1] = 0.0  # makes the Hadamard of Grams singular for modes 0 and 1
    before = [u.clone() for u in U]
    with pytest.raises(_abi.CpmError) as e:
        _abi.cp_als_step(X, dims, U)
    assert e.value.status == _abi.CPM_ENOTPD
    for b, u in zip(before, U):
        assert torch.equal(b, u)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dims,R", [((130, 140, 150), 96), ((130, 140, 150), 128), ((24, 20, 18, 16), 96),
                                    ((24, 20, 18, 16), 128)])
def test_als_sweep_wide_rank(dtype, dims, R):
    """R above 64: the Cholesky factorisation keeps up to 128 KB of H in LDS
    and the row solves read L from memory with two entries per lane; one
    sweep against the oracle's sweep."""
    announce("als wide", dims, R, dtype)
    X = inputs.uniform_tensor(dims, seed=R + 1, dtype=dtype)
    U = inputs.normal_factors(dims, R, seed=R + 2, dtype=dtype)
    Uh = [u.numpy().astype(np.float64) for u in U]
    ref, fit_ref = O.cp_als_step(X.numpy().ravel(), dims, Uh)
    kap = kappa_max(dims, ref)
    Ud = [u.cuda() for u in U]
    fit = _abi.cp_als_step(X.cuda(), dims, Ud)
    tol = 1e-5 * kap if dtype == torch.float32 else max(1e-10, 1e-14 * kap)
    for n, (g, r) in enumerate(zip(Ud, ref)):
        e = rel_err(g.cpu().numpy(), r)
        print("als R=%d mode %d: relative error %.3e (kappa %.2e)" % (R, n, e, kap), flush=True)
        assert e <= tol, (n, e, tol)
    assert fit == pytest.approx(fit_ref, abs=1e-5 if dtype == torch.float32 else 1e-10)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_als_not_positive_definite_restores_factors_r128(dtype):
    """The 128 KB-LDS factorisation detects the zero pivot too, and every
    factor comes back unchanged."""
    dims, R = (40, 36, 30), 128
    X = inputs.normal_tensor(dims, seed=43, dtype=dtype).cuda()
    U = [u.cuda() for u in inputs.normal_factors(dims, R, seed=44, dtype=dtype)]
    U[2][:, 1] = 0.0
    before = [u.clone() for u in U]
    with pytest.raises(_abi.CpmError) as e:
        _abi.cp_als_step(X, dims, U)
    assert e.value.status == _abi.CPM_ENOTPD
    for b, u in zip(before, U):
        assert torch.equal(b, u)


def test_als_twenty_iterations_fit_tracks_oracle():
    """Short run of ALS on a noisy low-rank tensor: the fit after each sweep
    agrees with the oracle's (iterates diverge slowly by rounding, so the
    fit, not the factors, is compared over many sweeps)."""
    dims, R = (40, 36, 32), 4
    X, _ = inputs.noisy_low_rank(dims, R, seed_factors=3, seed_noise=4, eta=0.01)
    U0 = inputs.normal_factors(dims, R, seed=5)
    Uo = [u.numpy().astype(np.float64) for u in U0]
    Ud = [u.cuda() for u in U0]
    Xd = X.cuda()
    xn = float(np.sum(X.numpy().astype(np.float64) ** 2))
    for it in range(20):
        Uo, fo = O.cp_als_step(X.numpy().ravel(), dims, Uo)
        fg = _abi.cp_als_step(Xd, dims, Ud, xnorm2=xn)
        assert abs(fg - fo) <= 1e-4, (it, fg, fo)
    assert fo > 0.98


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dims,R", [((20, 24, 28), 8), ((9, 10, 11, 12), 20), ((12, 12, 12, 12, 12), 32),
                                    ((20, 24, 28), 200), ((9, 10, 11, 12), 256)])
def test_cp_grad_matches_oracle(dtype, dims, R):
    announce("cp_grad", dims, R, dtype)
    X, _ = inputs.noisy_low_rank(dims, R, seed_factors=9, seed_noise=10, eta=0.05, dtype=torch.float64)
    X = X.to(dtype)
    U = inputs.normal_factors(dims, R, seed=11, dtype=dtype)
    Xh = X.numpy().ravel()
    Uh = [u.numpy().astype(np.float64) for u in U]
    G, ld, li = O.cp_grad(Xh, dims, Uh)
    grads, loss = _abi.cp_grad(X.cuda(), dims, [u.cuda() for u in U])
    tol = TOL["f32"] if dtype == torch.float32 else 1e-11
    for n in range(len(dims)):
        # scale: the two terms U_n H_n and M_n whose difference is the gradient
        H = np.ones((R, R))
        for k in range(len(dims)):
            if k != n:
                H *= Uh[k].T @ Uh[k]
        scale = np.linalg.norm(Uh[n] @ H) + np.linalg.norm(G[n] + Uh[n] @ H)
        assert np.linalg.norm(grads[n].cpu().numpy() - G[n]) <= tol * scale, n
    x2 = float(np.sum(Xh.astype(np.float64) ** 2))
    assert abs(loss.item() - ld) <= (1e-5 if dtype == torch.float32 else 1e-12) * x2


def _slice_12p5(dtype=torch.float64):
    """12^5 instance of the 64^5 recipe: factor rows 0..11 of the rank-32
    N(0,1) model (seed 9) and 5% Gaussian noise (seed 10) on that slice."""
    dims = (12,) * 5
    full = inputs.normal_factors((64,) * 5, 32, seed=9, dtype=torch.float32)
    Us = [u[:12].contiguous().to(torch.float64) for u in full]
    Y = inputs.cp_model_tensor(Us)
    E = inputs.normal_tensor(dims, seed=10, dtype=torch.float64)
    X = Y + 0.05 * (Y.norm() / E.norm()) * E
    return dims, X.to(dtype)


def test_cploss_autograd_central_differences_fp64():
    """CPLoss forward + hand-written backward on the 12^5 slice in float64:
    the central difference with h = 1e-3 along a random direction in one
    factor equals <grad, direction> (f is quadratic in each factor), and the
    gradient matches the oracle's."""
    dims, X = _slice_12p5()
    Xt = X.cuda()  # torch layout: axes are paper modes reversed
    U = [u.cuda().requires_grad_(True) for u in
         inputs.normal_factors(tuple(reversed(dims)), 32, seed=12, dtype=torch.float64)]
    loss = api.cp_loss(Xt, U)
    loss.backward()
    h = 1e-3
    rng = np.random.default_rng(13)
    for m in range(5):
        E = torch.from_numpy(rng.standard_normal(U[m].shape)).cuda()
        with torch.no_grad():
            Up = [u.detach().clone() for u in U]
            Um = [u.detach().clone() for u in U]
            Up[m] += h * E
            Um[m] -= h * E
            fd = (api.cp_loss(Xt, Up).item() - api.cp_loss(Xt, Um).item()) / (2 * h)
        an = float((U[m].grad * E).sum())
        assert fd == pytest.approx(an, rel=1e-6, abs=1e-8), (m, fd, an)
    # oracle gradient (paper order = torch axes reversed)
    Uh = [u.detach().cpu().numpy() for u in reversed(U)]
    G, ld, _ = O.cp_grad(X.numpy().ravel(), dims, Uh)
    for m in range(5):
        assert rel_err(U[m].grad.cpu().numpy(), G[4 - m]) <= 1e-10
    assert loss.item() == pytest.approx(ld, rel=1e-9)


def test_cploss_autograd_fp32_matches_oracle():
    dims, X = _slice_12p5(torch.float32)
    Xt = X.cuda()
    U = [u.cuda().requires_grad_(True) for u in
         inputs.normal_factors(tuple(reversed(dims)), 32, seed=12, dtype=torch.float32)]
    api.cp_loss(Xt, U).backward()
    Uh = [u.detach().cpu().numpy().astype(np.float64) for u in reversed(U)]
    G, _, _ = O.cp_grad(X.numpy().ravel(), dims, Uh)
    for m in range(5):
        assert rel_err(U[m].grad.cpu().numpy(), G[4 - m]) <= 1e-4


def test_torch_order_api_matches_paper_order():
    shape = (7, 9, 11)  # torch axes
    X = inputs.normal_tensor(tuple(reversed(shape)), seed=3).cuda()  # torch shape == `shape`
    assert tuple(X.shape) == shape
    U = [torch.randn(s, 6, device="cuda") for s in shape]
    dims = tuple(reversed(shape))
    for m in range(3):
        a = api.mttkrp(X, U, m)
        b = _abi.mttkrp(X, dims, list(reversed(U)), 2 - m)
        assert torch.equal(a, b)
        # torch reference of the definition for this small case
        others = [k for k in range(3) if k != m]
        ref = torch.einsum(X.double(), [0, 1, 2], U[others[0]].double(), [others[0], 3],
                           U[others[1]].double(), [others[1], 3], [m, 3])
        assert rel_err(a.cpu().numpy(), ref.cpu().numpy()) <= 1e-5
