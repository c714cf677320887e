"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (same planner, same library calls).

The oracle cannot produce a whole MTTKRP of 1e9 entries in seconds, so it
computes sampled output rows one by one (first, middle, last of every mode:
the first and last tiles and a ragged tail), and properties that hold at any
size pin the rest: the closed form for an exactly rank-R tensor (the whole
output) and the pair symmetry of the correlation-style tensor.

Per-mode errors are printed (run with -s to see them).
"""
import numpy as np
import pytest
import torch

from gpu_cases import TOL, announce, rel_err
from oracle import oracle as O
from paper_1708_08976_amd import _abi, inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(300)]


def sample_rows(In):
    return sorted({0, 1, In // 2 + 1, In - 1} & set(range(In)))


def gpu_all_modes(X, dims, U, dtype=None):
    outs = []
    for n in range(len(dims)):
        announce("  mode", n, "dims", dims, "R", U[0].shape[1])
        out = torch.full((dims[n], U[0].shape[1]), float("nan"), device="cuda")
        _abi.mttkrp(X, dims, U, n, out=out, dtype=dtype)
        outs.append(out)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def check_sampled(got, Xh, dims, Uh, tol, tag, xtype=None):
    errs = []
    for n in range(len(dims)):
        rows = sample_rows(dims[n])
        ref = O.mttkrp_rows(Xh, dims, Uh, n, rows, xtype=xtype)
        assert np.isfinite(got[n]).all(), (tag, n)
        e = rel_err(got[n][rows], ref)
        errs.append(e)
        print("%s mode %d rows %s: relative error %.3e" % (tag, n, rows, e), flush=True)
    for n, e in enumerate(errs):
        assert e <= tol, (tag, n, e)
    return errs


def test_config2_512cube_fp32_sampled_rows():
    dims, R = (512, 512, 512), 32
    announce("512^3 fp32 R=32, noisy rank-32 model")
    X, _ = inputs.noisy_low_rank(dims, R, seed_factors=3, seed_noise=4, eta=0.01, device="cuda")
    U = inputs.normal_factors(dims, R, seed=5, device="cuda")
    got = gpu_all_modes(X, dims, U)
    check_sampled(got, X.cpu().numpy().ravel(), dims, [u.cpu().numpy() for u in U], TOL["f32"], "512^3 f32")


def test_config2_512cube_closed_form_whole_output():
    """X = [[U]] exactly (float64 model rounded to float32): every output
    row equals U_n times the Hadamard product of the other Grams."""
    dims, R = (512, 512, 512), 32
    announce("512^3 closed form")
    U64 = inputs.normal_factors(dims, R, seed=3, device="cuda", dtype=torch.float64)
    X = inputs.cp_model_tensor(U64).float()
    U = [u.float() for u in U64]
    got = gpu_all_modes(X, dims, U)
    Uh = [u.cpu().numpy() for u in U64]
    for n in range(3):
        H = np.ones((R, R))
        for k in range(3):
            if k != n:
                H *= Uh[k].T @ Uh[k]
        e = rel_err(got[n], Uh[n] @ H)
        print("512^3 closed form mode %d: relative error %.3e" % (n, e), flush=True)
        assert e <= TOL["f32"], (n, e)


@pytest.mark.timeout(600)
def test_config2_twenty_als_iterations_fit_trajectory():
    """20 CP-ALS sweeps on the 512^3 tensor from the same start: the fit
    after every sweep agrees with the oracle's to 1e-4."""
    dims, R = (512, 512, 512), 32
    announce("512^3 ALS x20")
    X, _ = inputs.noisy_low_rank(dims, R, seed_factors=3, seed_noise=4, eta=0.01, device="cuda")
    U0 = inputs.normal_factors(dims, R, seed=5)
    Xh = X.cpu().numpy().ravel()
    xn = O.xnorm2(Xh, dims)
    Uo = [u.numpy().astype(np.float64) for u in U0]
    Ud = [u.cuda() for u in U0]
    ws = torch.empty(_abi.cp_als_workspace_bytes(dims, R, _abi.CPM_F32), dtype=torch.uint8, device="cuda")
    for it in range(20):
        Uo, fo = O.cp_als_step(Xh, dims, Uo)
        fg = _abi.cp_als_step(X, dims, Ud, xnorm2=xn, workspace=ws)
        print("sweep %2d: fit gpu %.8f oracle %.8f" % (it, fg, fo), flush=True)
        assert abs(fg - fo) <= 1e-4, (it, fg, fo)


def test_config3_sym4d_fp32_r64_sampled_rows_and_symmetry():
    dims, R = (256, 256, 512, 32), 64
    announce("256x256x512x32 fp32 R=64")
    X = inputs.symmetric_pair_tensor(dims, seed=6, device="cuda")
    U = inputs.normal_factors(dims, R, seed=7, device="cuda")
    got = gpu_all_modes(X, dims, U)
    check_sampled(got, X.cpu().numpy().ravel(), dims, [u.cpu().numpy() for u in U], TOL["f32"], "sym4d f32")
    # X symmetric in modes 0 and 1: with U_1 = U_0, M_0 = M_1 (two
    # different kernels, right-first and left-first, must agree).
    Us = [U[0], U[0].clone(), U[2], U[3]]
    m0 = _abi.mttkrp(X, dims, Us, 0).cpu().numpy()
    m1 = _abi.mttkrp(X, dims, Us, 1).cpu().numpy()
    e = rel_err(m0, m1)
    print("sym4d symmetry M0 vs M1: %.3e" % e, flush=True)
    assert e <= TOL["f32"]


def test_config4_sym4d_split_bf16_r128_per_mode_error():
    dims, R = (256, 256, 512, 32), 128
    announce("256x256x512x32 split bf16 R=128")
    X = inputs.symmetric_pair_tensor(dims, seed=6, device="cuda")
    U = inputs.normal_factors(dims, R, seed=8, device="cuda")
    P = _abi.split_bf16(X.reshape(-1))
    got = gpu_all_modes(P, dims, U, dtype=_abi.CPM_BF16X2)
    Uh = [u.cpu().numpy() for u in U]
    # total error: against the oracle on the float32 tensor
    check_sampled(got, X.cpu().numpy().ravel(), dims, Uh, TOL["bf16x2"], "sym4d bf16x2 vs f32 X")
    # arithmetic error: against the oracle on the pair values
    check_sampled(got, P.cpu().numpy().view(np.uint16), dims, Uh, TOL["bf16x2"], "sym4d bf16x2 vs pair",
                  xtype=O.BF16PAIR)


def test_config5_64p5_fp32_sampled_rows_and_grad():
    dims, R = (64,) * 5, 32
    announce("64^5 fp32 R=32")
    X, _ = inputs.noisy_low_rank(dims, R, seed_factors=9, seed_noise=10, eta=0.05, device="cuda")
    U = inputs.normal_factors(dims, R, seed=11, device="cuda")
    Xh = X.cpu().numpy().ravel()
    Uh = [u.cpu().numpy().astype(np.float64) for u in U]
    got = gpu_all_modes(X, dims, U)
    check_sampled(got, Xh, dims, Uh, TOL["f32"], "64^5 f32")
    # gradient rows: G_n = U_n H_n - M_n, with M_n rows from the oracle
    xn = O.xnorm2(Xh, dims)
    grads, loss = _abi.cp_grad(X, dims, U, xnorm2=xn)
    torch.cuda.synchronize()
    for n in range(5):
        rows = sample_rows(dims[n])
        H = np.ones((R, R))
        for k in range(5):
            if k != n:
                H *= Uh[k].T @ Uh[k]
        ref = Uh[n][rows] @ H - O.mttkrp_rows(Xh, dims, Uh, n, rows)
        e = rel_err(grads[n].cpu().numpy()[rows], ref)
        print("64^5 grad mode %d: relative error %.3e" % (n, e), flush=True)
        assert e <= TOL["f32"], (n, e)
    ref_loss = 0.5 * O.residual2(Xh, dims, Uh)
    print("64^5 loss gpu %.10e oracle (direct) %.10e" % (loss.item(), ref_loss), flush=True)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-6)


def test_config3_sym4d_fp32_r128_sampled_rows():
    """The float32 side of the split-bf16 comparison (four 32-column blocks
    per work-group)."""
    dims, R = (256, 256, 512, 32), 128
    announce("256x256x512x32 fp32 R=128")
    X = inputs.symmetric_pair_tensor(dims, seed=6, device="cuda")
    U = inputs.normal_factors(dims, R, seed=8, device="cuda")
    got = gpu_all_modes(X, dims, U)
    check_sampled(got, X.cpu().numpy().ravel(), dims, [u.cpu().numpy() for u in U], TOL["f32"], "sym4d f32 R128")


@pytest.mark.parametrize("R", [32, 128])
def test_config5_64p5_split_bf16_sampled_rows_and_grad(R):
    """The split-bf16 MTTKRPs and gradient that the benchmark times on 64^5
    (the last mode's rows are 32 MB apart)."""
    dims = (64,) * 5
    announce("64^5 split bf16 R=%d" % R)
    X, _ = inputs.noisy_low_rank(dims, 32, seed_factors=9, seed_noise=10, eta=0.05, device="cuda")
    P = _abi.split_bf16(X.reshape(-1))
    U = inputs.normal_factors(dims, R, seed=11, device="cuda")
    Xh = X.cpu().numpy().ravel()
    Uh = [u.cpu().numpy().astype(np.float64) for u in U]
    got = gpu_all_modes(P, dims, U, dtype=_abi.CPM_BF16X2)
    check_sampled(got, Xh, dims, Uh, TOL["bf16x2"], "64^5 bf16x2 R%d" % R)
    if R == 32:
        xn = O.xnorm2(Xh, dims)
        grads, _ = _abi.cp_grad(P, dims, U, xnorm2=xn, dtype=_abi.CPM_BF16X2)
        torch.cuda.synchronize()
        for n in range(5):
            rows = sample_rows(dims[n])
            H = np.ones((R, R))
            for k in range(5):
                if k != n:
                    H *= Uh[k].T @ Uh[k]
            ref = Uh[n][rows] @ H - O.mttkrp_rows(Xh, dims, Uh, n, rows)
            e = rel_err(grads[n].cpu().numpy()[rows], ref)
            print("64^5 bf16x2 grad mode %d: relative error %.3e" % (n, e), flush=True)
            assert e <= TOL["bf16x2"], (n, e)


def test_config5_64p5_fp32_r128_sampled_rows():
    dims, R = (64,) * 5, 128
    announce("64^5 fp32 R=128")
    X, _ = inputs.noisy_low_rank(dims, 32, seed_factors=9, seed_noise=10, eta=0.05, device="cuda")
    U = inputs.normal_factors(dims, R, seed=11, device="cuda")
    got = gpu_all_modes(X, dims, U)
    check_sampled(got, X.cpu().numpy().ravel(), dims, [u.cpu().numpy().astype(np.float64) for u in U], TOL["f32"],
                  "64^5 f32 R128")


@pytest.mark.parametrize("dtype", ["f32", "bf16x2"])
def test_config5_64p5_mttkrp_all_with_reuse_sampled_rows(dtype):
    """All five MTTKRPs of the 64^5 tensor from the two passes of the
    cross-mode reuse (modes split 2 | 3), in the configuration the gradient
    benchmark runs; sampled rows against the oracle."""
    dims, R = (64,) * 5, 32
    announce("64^5 mttkrp_all", dtype)
    X, _ = inputs.noisy_low_rank(dims, 32, seed_factors=9, seed_noise=10, eta=0.05, device="cuda")
    U = inputs.normal_factors(dims, R, seed=11, device="cuda")
    code = _abi.CPM_F32 if dtype == "f32" else _abi.CPM_BF16X2
    Xd = X if dtype == "f32" else _abi.split_bf16(X.reshape(-1))
    outs = _abi.mttkrp_all(Xd, dims, U, dtype=code)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    check_sampled(got, X.cpu().numpy().ravel(), dims, [u.cpu().numpy().astype(np.float64) for u in U],
                  TOL[dtype], "64^5 mttkrp_all %s" % dtype)


@pytest.mark.parametrize("dims,R,dtype", [((64,) * 5, 32, "f32"), ((64,) * 5, 128, "f32"),
                                          ((64,) * 5, 128, "bf16x2"),
                                          ((256, 256, 512, 32), 64, "f32"),
                                          ((256, 256, 512, 32), 128, "bf16x2")])
@pytest.mark.timeout(600)
def test_closed_form_whole_output_full_size(dims, R, dtype):
    """X = [[U]] exactly (a float64 rank-R model, stored as float32 or as its
    bf16 pair): every row of every mode equals U_n times the Hadamard
    product of the other Grams, a fact of the CP model that needs no oracle
    pass, so the whole output -- every row tile, column block and split-K
    slice of the launches the benchmark times -- is checked.  The stored
    tensor differs from the model by its rounding (2^-24 relative per entry
    for float32, 2^-17 for the pair), which moves M by far less than the
    tolerance: the model's MTTKRP adds its terms coherently."""
    announce("closed form", dims, R, dtype)
    U64 = inputs.normal_factors(dims, R, seed=R + len(dims), device="cuda", dtype=torch.float64)
    X = inputs.cp_model_tensor(U64).float()
    if dtype == "bf16x2":
        Xd, code = _abi.split_bf16(X.reshape(-1)), _abi.CPM_BF16X2
        del X
    else:
        Xd, code = X, _abi.CPM_F32
    U = [u.float() for u in U64]
    Uh = [u.cpu().numpy() for u in U64]
    got = gpu_all_modes(Xd, dims, U, dtype=code)
    for n in range(len(dims)):
        H = np.ones((R, R))
        for k in range(len(dims)):
            if k != n:
                H *= Uh[k].T @ Uh[k]
        e = rel_err(got[n], Uh[n] @ H)
        print("closed form %s R=%d %s mode %d: relative error %.3e" % (dims, R, dtype, n, e), flush=True)
        assert e <= TOL[dtype], (n, e)
