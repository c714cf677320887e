"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers and arranges them; it computes no
MTTKRP, Khatri-Rao product, Gram matrix or solve.  Both the oracle and the
GPU library consume what it returns, and neither is imported here.

Dimension convention: ``dims`` lists I_0..I_{N-1} with mode 0 the fastest
index in memory (the natural linearisation of the paper's Section 2.1).  A
torch tensor holding such a tensor has shape ``tuple(reversed(dims))``.
Factor k is an I_k x R matrix.  Values depend on the generator's device
(CPU and GPU streams differ), so a test always draws once and hands the same
buffer to both sides.

The recipes follow the paper's workloads (Section 5): equal-sided tensors of
about 7.5e8 entries, the fMRI-shaped correlation tensor that is symmetric in
a pair of region modes (Section 5.3.3), and low-rank CP models plus
Gaussian noise.
"""
import torch


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def torch_shape(dims):
    return tuple(int(d) for d in reversed(dims))


def normal_factors(dims, R, seed, device="cpu", dtype=torch.float32):
    """i.i.d. N(0,1) factors U_k of shape (I_k, R)."""
    g = _gen(seed, device)
    base = torch.float64 if dtype == torch.float64 else torch.float32
    return [torch.randn((int(d), int(R)), generator=g, device=device, dtype=base).to(dtype)
            for d in dims]


def uniform_tensor(dims, seed, device="cpu", dtype=torch.float32, low=0.0, high=1.0):
    """Entries i.i.d. uniform on [low, high)."""
    g = _gen(seed, device)
    x = torch.rand(torch_shape(dims), generator=g, device=device,
                   dtype=torch.float64 if dtype == torch.float64 else torch.float32)
    if low != 0.0 or high != 1.0:
        x.mul_(high - low).add_(low)
    return x.to(dtype)


def normal_tensor(dims, seed, device="cpu", dtype=torch.float32):
    g = _gen(seed, device)
    return torch.randn(torch_shape(dims), generator=g, device=device,
                       dtype=torch.float64 if dtype == torch.float64 else torch.float32).to(dtype)


def cp_model_tensor(factors, dtype=None):
    """Dense tensor sum_c U_0(:,c) o U_1(:,c) o ... (outer products), built
    one rank-1 term at a time with broadcasting, in float64 when the factors
    are float64 and float32 otherwise.  Returned in torch layout."""
    N = len(factors)
    R = factors[0].shape[1]
    dt = factors[0].dtype
    shape = tuple(int(u.shape[0]) for u in reversed(factors))
    out = torch.zeros(shape, device=factors[0].device, dtype=dt)
    for c in range(R):
        term = None
        for pos, k in enumerate(reversed(range(N))):
            v = factors[k][:, c]
            view = [1] * N
            view[pos] = -1
            v = v.reshape(view)
            term = v if term is None else term * v
        out.add_(term)
    return out if dtype is None else out.to(dtype)


def noisy_low_rank(dims, R, seed_factors, seed_noise, eta, device="cpu", dtype=torch.float32):
    """X = Y + eta * (||Y|| / ||E||) * E with Y a rank-R CP model with N(0,1)
    factors and E i.i.d. N(0,1).  Returns (X, true_factors)."""
    U = normal_factors(dims, R, seed_factors, device=device, dtype=torch.float32)
    Y = cp_model_tensor(U)
    E = normal_tensor(dims, seed_noise, device=device, dtype=torch.float32)
    scale = float(eta) * float(torch.linalg.vector_norm(Y.double())) / float(torch.linalg.vector_norm(E.double()))
    Y.add_(E, alpha=scale)
    del E
    return Y.to(dtype), U


def symmetric_pair_tensor(dims, seed, device="cpu", dtype=torch.float32):
    """Correlation-style tensor symmetric in modes 0 and 1 (dims[0] ==
    dims[1]): X(i,j,...) = X(j,i,...) uniform on [-1,1) off the diagonal and
    X(i,i,...) = 1, like a region-by-region correlation array per time step
    and subject."""
    assert dims[0] == dims[1]
    x = uniform_tensor(dims, seed, device=device, dtype=torch.float32, low=-1.0, high=1.0)
    # torch layout: the last two axes are modes 1 and 0.
    up = torch.triu(x, diagonal=1)
    x = up + up.transpose(-1, -2)
    x.diagonal(dim1=-2, dim2=-1).fill_(1.0)
    return x.contiguous().to(dtype)


def sympair_count(n):
    """Pairs (i, j) with i <= j < n: the packed length of a symmetric pair
    of modes of size n."""
    return n * (n + 1) // 2


def sympair_indices(n, device="cpu"):
    """(i, j) of every packed pair index p = j (j + 1) / 2 + i, i <= j, in
    order of p: i fastest, then j (the natural linearisation restricted to
    the triangle)."""
    j = torch.repeat_interleave(torch.arange(n, device=device), torch.arange(1, n + 1, device=device))
    start = j * (j + 1) // 2
    i = torch.arange(sympair_count(n), device=device) - start
    return i, j


def pack_sympair(x, dims):
    """Packed triangle of a tensor symmetric in modes 0 and 1 (torch layout
    in, torch layout out): entry (p, i_2, ..., i_{N-1}) of the result is
    X(i_p, j_p, i_2, ...).  The result has torch shape
    (I_{N-1}, ..., I_2, P).  Pure data movement."""
    n = int(dims[0])
    assert int(dims[1]) == n
    i, j = sympair_indices(n, device=x.device)
    # torch layout: the last two axes are modes 1 and 0
    return x[..., j, i].contiguous()


def split_bf16_planes(x):
    """hi = bf16(x) and lo = bf16(x - hi), both round-to-nearest-even,
    returned as one uint16-compatible int16 tensor holding the hi plane
    followed by the lo plane (2 * numel entries)."""
    x = x.contiguous().float()
    hi = x.to(torch.bfloat16)
    lo = (x - hi.float()).to(torch.bfloat16)
    return torch.cat([hi.reshape(-1).view(torch.int16), lo.reshape(-1).view(torch.int16)])


# Named workloads: (dims, R) with dims in paper order (mode 0 fastest).
CONFIGS = {
    "fp64_60x50x40_r8": ((60, 50, 40), 8),
    "fp32_512cube_r32": ((512, 512, 512), 32),
    "fp32_sym_256x256x512x32_r64": ((256, 256, 512, 32), 64),
    "bf16x2_sym_256x256x512x32_r128": ((256, 256, 512, 32), 128),
    "fp32_64p5_r32": ((64, 64, 64, 64, 64), 32),
}

# Equal-sided tensors of about 7.5e8 entries used for the paper's MTTKRP
# scaling study (Section 5.3.1), rank 25, and the fMRI-shaped tensors of
# Section 5.3.3.
PAPER_SHAPES = {
    "900^3": (900, 900, 900),
    "165^4": (165, 165, 165, 165),
    "60^5": (60, 60, 60, 60, 60),
    "30^6": (30, 30, 30, 30, 30, 30),
    "fmri4d": (225, 59, 200, 200),
    "fmri3d": (225, 59, 19900),
}
