"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own loops (CPU only)."""
import itertools

import numpy as np
import pytest

import brute
from oracle import oracle as O

rng = np.random.default_rng(20240601)

SHAPES = [
    (3, 4), (1, 5), (5, 1), (2, 3, 4), (3, 1, 2), (1, 1, 1), (2, 2, 3, 2),
    (3, 2, 1, 2, 2), (2, 1, 2, 2, 1, 3), (5, 3, 2),
]


def _factors(dims, R, seed):
    r = np.random.default_rng(seed)
    return [r.standard_normal((d, R)) for d in dims]


def _tensor(dims, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(int(np.prod(dims)))


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 3, 8])
def test_mttkrp_matches_unfolding_times_kron(dims, R):
    """Section 2.2 matrix form: X_(n) times the explicit KRP built from
    Kronecker products of columns (Section 2.1)."""
    X = _tensor(dims, 1 + R)
    U = _factors(dims, R, 2 + R)
    for n in range(len(dims)):
        got = O.mttkrp(X, dims, U, n)
        ref = brute.mttkrp(X, dims, U, n)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("dims", [(3, 4, 5, 2), (4, 3, 5), (2, 3, 2, 2, 3)])
def test_closed_form_exact_rank_R(dims):
    """For X = [[U]], MTTKRP_n = U_n * (Hadamard product of the other Grams)."""
    R = 4
    U = _factors(dims, R, 7)
    X = brute.cp_tensor(U)
    for n in range(len(dims)):
        H = np.ones((R, R))
        for k in range(len(dims)):
            if k != n:
                H *= U[k].T @ U[k]
        np.testing.assert_allclose(O.mttkrp(X, dims, U, n), U[n] @ H, rtol=1e-11, atol=1e-11)


def test_ones_tensor_closed_form():
    """X = all ones: M(i,c) = prod_{k!=n} sum_i U_k(i,c), for every row i."""
    dims = (3, 5, 2, 4)
    U = _factors(dims, 6, 11)
    X = np.ones(int(np.prod(dims)))
    for n in range(4):
        col = np.ones(6)
        for k in range(4):
            if k != n:
                col *= U[k].sum(axis=0)
        np.testing.assert_allclose(O.mttkrp(X, dims, U, n), np.tile(col, (dims[n], 1)), rtol=1e-12)


@pytest.mark.parametrize("dims", [(3, 5, 2, 4), (7, 2, 3)])
def test_single_entry_tensor(dims):
    """One nonzero entry v at multi-index a, stored at l = sum_k a_k prod_{j<k} I_j
    (natural linearisation, Section 2.1): row a_n of M_n is
    v * prod_{k!=n} U_k(a_k,:), every other row is zero.  Pins the index map."""
    N = len(dims)
    U = _factors(dims, 5, 13)
    for a in [tuple(d - 1 for d in dims), tuple(min(1, d - 1) for d in dims), (0,) * N]:
        l = 0
        stride = 1
        for k in range(N):
            l += a[k] * stride
            stride *= dims[k]
        X = np.zeros(int(np.prod(dims)))
        X[l] = 2.5
        for n in range(N):
            want = np.zeros((dims[n], 5))
            row = np.full(5, 2.5)
            for k in range(N):
                if k != n:
                    row = row * U[k][a[k]]
            want[a[n]] = row
            np.testing.assert_allclose(O.mttkrp(X, dims, U, n), want, rtol=1e-14, atol=0)


def test_multilinearity_and_independence_of_own_factor():
    dims = (4, 3, 5)
    U = _factors(dims, 3, 17)
    X1, X2 = _tensor(dims, 18), _tensor(dims, 19)
    for n in range(3):
        M1 = O.mttkrp(X1, dims, U, n)
        M2 = O.mttkrp(X2, dims, U, n)
        np.testing.assert_allclose(O.mttkrp(2.0 * X1 - 3.0 * X2, dims, U, n), 2 * M1 - 3 * M2,
                                   rtol=1e-12, atol=1e-12)
        V = [u.copy() for u in U]
        V[n] = rng.standard_normal(V[n].shape)
        np.testing.assert_array_equal(O.mttkrp(X1, dims, V, n), M1)
        k = (n + 1) % 3
        V = [u.copy() for u in U]
        V[k] = 0.5 * V[k]
        np.testing.assert_allclose(O.mttkrp(X1, dims, V, n), 0.5 * M1, rtol=1e-13, atol=1e-13)


def test_symmetric_pair_gives_equal_modes():
    """A tensor symmetric in modes 0 and 1 with U_0 = U_1 gives M_0 = M_1."""
    dims = (5, 5, 3, 2)
    A = np.random.default_rng(23).uniform(-1, 1, size=tuple(reversed(dims)))
    A = np.triu(A, 1)
    A = A + np.swapaxes(A, -1, -2)
    for idx in range(5):
        A[..., idx, idx] = 1.0
    U = _factors(dims, 4, 29)
    U[1] = U[0].copy()
    np.testing.assert_allclose(O.mttkrp(A, dims, U, 0), O.mttkrp(A, dims, U, 1), rtol=1e-13, atol=1e-13)


def test_rows_subset_and_thread_determinism():
    dims = (6, 4, 5, 3)
    X = _tensor(dims, 31)
    U = _factors(dims, 7, 37)
    for n in range(4):
        full = O.mttkrp(X, dims, U, n, nthreads=3)
        rows = np.arange(dims[n])[::-1].copy()
        np.testing.assert_allclose(O.mttkrp_rows(X, dims, U, n, rows), full[rows], rtol=1e-13, atol=1e-13)
        np.testing.assert_array_equal(O.mttkrp(X, dims, U, n, nthreads=3), full)
        np.testing.assert_allclose(O.mttkrp(X, dims, U, n, nthreads=1), full, rtol=1e-13, atol=1e-13)


def test_input_widening_is_exact():
    dims = (4, 3, 5)
    U = _factors(dims, 3, 41)
    x32 = np.random.default_rng(43).standard_normal(60).astype(np.float32)
    for n in range(3):
        np.testing.assert_array_equal(O.mttkrp(x32, dims, U, n),
                                      O.mttkrp(x32.astype(np.float64), dims, U, n))
    # bfloat16 pair: hi plane then lo plane; value hi + lo.
    bits = np.random.default_rng(47).integers(0, 2 ** 16, size=120, dtype=np.uint16)
    bits[(bits & 0x7F80) == 0x7F80] &= 0x3FFF  # keep every value finite
    as32 = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    val = as32[:60] + as32[60:]
    for n in range(3):
        np.testing.assert_array_equal(O.mttkrp(bits, dims, U, n, xtype=O.BF16PAIR),
                                      O.mttkrp(val, dims, U, n))


@pytest.mark.parametrize("Js", [(3,), (2, 3), (3, 1, 4), (2, 2, 3, 2)])
def test_krp_rows_column_and_row_definitions(Js):
    """Section 2.1: K(:,c) is the Kronecker product of the columns, and row
    r_B + r_A I_B of A kr B is A(r_A,:) * B(r_B,:)."""
    mats = [rng.standard_normal((J, 4)) for J in Js]
    K = O.krp_rows(mats)
    np.testing.assert_allclose(K, brute.krp_columns(mats), rtol=1e-14, atol=0)
    if len(mats) >= 2:
        A, B = mats[0], mats[1]
        AB = O.krp_rows([A, B])
        for ra, rb in itertools.product(range(A.shape[0]), range(B.shape[0])):
            np.testing.assert_array_equal(AB[rb + ra * B.shape[0]], A[ra] * B[rb])
    tail = O.krp_rows(mats, j0=1, nrows=K.shape[0] - 1)
    np.testing.assert_array_equal(tail, K[1:])


def _als_sweep_numpy(X, dims, U):
    """Section 2.2 update with library routines: M by unfolding times KRP and
    U_n = M H^+ with numpy's pseudo-inverse."""
    U = [u.copy() for u in U]
    for n in range(len(dims)):
        M = brute.mttkrp(X, dims, U, n)
        H = np.ones((U[0].shape[1],) * 2)
        for k in range(len(dims)):
            if k != n:
                H *= U[k].T @ U[k]
        U[n] = M @ np.linalg.pinv(H)
    return U


@pytest.mark.parametrize("dims,R", [((6, 5, 4), 3), ((4, 3, 5, 3), 2)])
def test_als_step_matches_pseudoinverse_update(dims, R):
    X = _tensor(dims, 53)
    U0 = _factors(dims, R, 59)
    got, fit = O.cp_als_step(X, dims, U0)
    want = _als_sweep_numpy(X, dims, U0)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=1e-9, atol=1e-9)
    Y = brute.cp_tensor(want)
    np.testing.assert_allclose(fit, 1 - np.linalg.norm(X - Y) / np.linalg.norm(X), rtol=1e-12)


def test_als_true_factors_are_a_fixed_point():
    dims = (5, 4, 6)
    U = _factors(dims, 3, 61)
    X = brute.cp_tensor(U)
    got, fit = O.cp_als_step(X, dims, U)
    for g, u in zip(got, U):
        np.testing.assert_allclose(g, u, rtol=1e-9, atol=1e-9)
    assert fit == pytest.approx(1.0, abs=1e-7)


def test_als_normal_equations_after_sweep():
    """After the sweep the last factor solves its least-squares problem, so
    the gradient with respect to it vanishes (Section 2.2)."""
    dims = (5, 6, 4)
    X = _tensor(dims, 67)
    U, _ = O.cp_als_step(X, dims, _factors(dims, 3, 71))
    G, _, _ = O.cp_grad(X, dims, U)
    scale = np.abs(O.mttkrp(X, dims, U, 2)).max()
    assert np.abs(G[2]).max() < 1e-10 * scale


def test_als_not_positive_definite_leaves_factors():
    dims = (4, 5, 3)
    X = _tensor(dims, 73)
    U = _factors(dims, 3, 79)
    U[2][:, 1] = 0.0  # zero column -> the Hadamard of Grams for modes 0 and 1 is singular
    before = [u.copy() for u in U]
    with pytest.raises(O.OracleError) as e:
        O.cp_als_step(X, dims, U)
    assert e.value.status == 3
    for b, u in zip(before, U):
        np.testing.assert_array_equal(b, u)


def test_grad_matches_matrix_form_and_losses_agree():
    dims = (4, 5, 3, 2)
    X = _tensor(dims, 83)
    U = _factors(dims, 3, 89)
    G, ld, li = O.cp_grad(X, dims, U)
    for n in range(4):
        H = np.ones((3, 3))
        for k in range(4):
            if k != n:
                H *= U[k].T @ U[k]
        np.testing.assert_allclose(G[n], U[n] @ H - brute.mttkrp(X, dims, U, n), rtol=1e-10, atol=1e-10)
    Y = brute.cp_tensor(U)
    assert ld == pytest.approx(0.5 * np.sum((X - Y) ** 2), rel=1e-12)
    assert li == pytest.approx(ld, rel=1e-10)


@pytest.mark.parametrize("h", [1e-3, 0.1, 1.0])
def test_grad_central_difference_is_exact(h):
    """f is quadratic in any single factor, so the central difference along a
    direction E in one factor equals <grad, E> for every step h."""
    dims = (3, 4, 2, 3)
    X = _tensor(dims, 97)
    U = _factors(dims, 2, 101)
    G, _, _ = O.cp_grad(X, dims, U, direct=False)
    for n in range(4):
        E = np.random.default_rng(103 + n).standard_normal(U[n].shape)
        Up = [u.copy() for u in U]
        Um = [u.copy() for u in U]
        Up[n] = U[n] + h * E
        Um[n] = U[n] - h * E
        fp = 0.5 * O.residual2(X, dims, Up)
        fm = 0.5 * O.residual2(X, dims, Um)
        fd = (fp - fm) / (2 * h)
        assert fd == pytest.approx(float(np.sum(G[n] * E)), rel=1e-8, abs=1e-10)


def test_grad_vanishes_at_true_factors():
    dims = (4, 3, 5)
    U = _factors(dims, 2, 107)
    X = brute.cp_tensor(U)
    G, ld, _ = O.cp_grad(X, dims, U)
    for g in G:
        assert np.abs(g).max() < 1e-10
    assert abs(ld) < 1e-20


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 3])
def test_residual2_matches_dense_model(dims, R):
    """||X - [[U]]||^2 against the dense CP tensor built from Kronecker
    products of factor columns (Section 2.1), and zero for X = [[U]]."""
    X = _tensor(dims, 301 + R)
    U = _factors(dims, R, 307 + R)
    Y = brute.cp_tensor(U)
    assert O.residual2(X, dims, U) == pytest.approx(float(np.sum((X - Y) ** 2)), rel=1e-12)
    assert O.residual2(Y, dims, U) <= 1e-24 * max(1.0, float(np.sum(Y ** 2)))


def test_residual2_widens_bf16_pairs_exactly():
    dims = (4, 3, 5)
    U = _factors(dims, 2, 311)
    bits = np.random.default_rng(313).integers(0, 2 ** 16, size=120, dtype=np.uint16)
    bits[(bits & 0x7F80) == 0x7F80] &= 0x3FFF  # keep every value finite
    as32 = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    val = as32[:60] + as32[60:]
    assert O.residual2(bits, dims, U, xtype=O.BF16PAIR) == O.residual2(val, dims, U)


# ---------------------------------------------------------------------------
# Symmetric-pair packed storage (Section 5.3.3 stores the symmetric region
# pair of its fMRI tensor as one linearised triangle).
# ---------------------------------------------------------------------------
def _symmetric_full(dims, seed):
    """A tensor symmetric in modes 0 and 1, in natural storage order."""
    r = np.random.default_rng(seed)
    A = r.standard_normal(tuple(reversed(dims)))  # torch layout: [..., j, i]
    return (A + np.swapaxes(A, -1, -2)).ravel()


def _pack(Xfull, dims):
    import torch
    from paper_1708_08976_amd import inputs
    x = torch.from_numpy(np.asarray(Xfull).reshape(tuple(reversed(dims))))
    return inputs.pack_sympair(x, dims).numpy().ravel()


def test_sympair_layout_by_hand():
    """n = 3: packed order (0,0), (0,1), (1,1), (0,2), (1,2), (2,2), pair
    index fastest, then the next mode."""
    dims = (3, 3, 2)
    vals = {}
    full = np.zeros(18)
    for r in range(2):
        for i in range(3):
            for j in range(i, 3):
                v = 100 * r + 10 * i + j
                full[i + 3 * j + 9 * r] = v
                full[j + 3 * i + 9 * r] = v
    want = [0, 1, 11, 2, 12, 22, 100, 101, 111, 102, 112, 122]
    assert list(_pack(full, dims)) == want


@pytest.mark.parametrize("dims", [(3, 3, 2), (4, 4, 3, 2), (2, 2, 1), (5, 5, 2, 1, 3), (1, 1, 4)])
@pytest.mark.parametrize("R", [1, 4])
def test_sympair_oracle_matches_brute_force_of_the_full_tensor(dims, R):
    """The packed-storage oracle equals the explicit unfolding times the
    explicit Khatri-Rao product of the unpacked symmetric tensor, every
    mode (pair modes included)."""
    X = _symmetric_full(dims, 5 + R)
    Xp = _pack(X, dims)
    U = _factors(dims, R, 6 + R)
    for n in range(len(dims)):
        got = O.mttkrp_sympair(Xp, dims, U, n)
        ref = brute.mttkrp(X, dims, U, n)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_sympair_ones_counts_the_diagonal_once():
    """All-ones packed tensor and factors: row i of mode n counts the full
    tensor's entries with index i in mode n, prod_{k != n} I_k; a diagonal
    pair counted twice (or an off-diagonal one once) changes the count."""
    dims = (4, 4, 3)
    P = 10
    Xp = np.ones(P * 3)
    U = [np.ones((d, 2)) for d in dims]
    for n in range(3):
        want = np.prod([d for k, d in enumerate(dims) if k != n])
        np.testing.assert_array_equal(O.mttkrp_sympair(Xp, dims, U, n), np.full((dims[n], 2), want))


def test_sympair_closed_form_symmetric_exact_rank():
    """X = [[A, A, U_2, U_3]] is symmetric in modes 0 and 1; its packed
    triangle gives MTTKRP_n = U_n * (Hadamard product of the other Grams)."""
    dims, R = (5, 5, 3, 4), 3
    U = _factors(dims, R, 17)
    U[1] = U[0]
    X = brute.cp_tensor(U)
    Xp = _pack(X, dims)
    for n in range(4):
        H = np.ones((R, R))
        for k in range(4):
            if k != n:
                H *= U[k].T @ U[k]
        np.testing.assert_allclose(O.mttkrp_sympair(Xp, dims, U, n), U[n] @ H, rtol=1e-11, atol=1e-11)


def test_sympair_rejects_unequal_pair_modes():
    with pytest.raises(O.OracleError):
        O.mttkrp_sympair(np.ones(12), (3, 4, 2), _factors((3, 4, 2), 2, 1), 0)
