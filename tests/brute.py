"""Independent brute-force forms used to pin the oracle.

These are NOT the oracle's element-by-element loop: MTTKRP is evaluated in
its matrix form (Section 2.2) as the explicit mode-n unfolding (Section 2.1)
times the explicit Khatri-Rao product assembled column by column with
Kronecker products (the column-wise definition of Section 2.1), using numpy.
"""
import numpy as np


def paper_view(X, dims):
    """numpy array indexed [i_0, i_1, ..., i_{N-1}] for a buffer stored in
    the natural linearisation (mode 0 fastest)."""
    a = np.asarray(X).reshape(tuple(reversed(dims)))
    return a.transpose(tuple(reversed(range(len(dims)))))


def unfold(X, dims, n):
    """Mode-n matricization X_(n): I_n x prod_{k!=n} I_k, columns ordered by
    the natural linearisation of the remaining modes."""
    Xp = paper_view(X, dims)
    return np.moveaxis(Xp, n, 0).reshape(dims[n], -1, order="F")


def krp_columns(mats):
    """mats[0] kr mats[1] kr ... (column c = kron of the columns)."""
    R = mats[0].shape[1]
    cols = []
    for c in range(R):
        v = np.ones(1)
        for A in mats:
            v = np.kron(v, A[:, c])
        cols.append(v)
    return np.stack(cols, axis=1)


def full_krp(factors, n):
    """U_{N-1} kr ... kr U_{n+1} kr U_{n-1} kr ... kr U_0."""
    N = len(factors)
    order = [factors[k] for k in reversed(range(N)) if k != n]
    return krp_columns(order)


def mttkrp(X, dims, factors, n):
    return unfold(X, dims, n) @ full_krp([np.asarray(u, np.float64) for u in factors], n)


def cp_tensor(factors):
    """Dense [[U_0..U_{N-1}]] in natural storage order, float64, built from
    the column-wise Kronecker form of its entries."""
    K = krp_columns([np.asarray(u, np.float64) for u in reversed(factors)])
    return K.sum(axis=1)
