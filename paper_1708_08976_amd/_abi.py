"""Thin ctypes binding of libcpmttkrp.so: same names and argument order as
the C-ABI in include/cpmttkrp.h, marshalling only.  Tensors are torch
tensors on the GPU; dims and modes follow the paper's order (mode 0 is the
stride-1 index).  There is no fallback: if the library is missing or a call
fails, an exception is raised.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpmttkrp.so")

CPM_OK, CPM_EINVAL, CPM_EUNSUPPORTED, CPM_ENOTPD, CPM_EHIP, CPM_EWORKSPACE = range(6)
CPM_F32, CPM_F64, CPM_BF16X2 = 0, 1, 2
STATUS_NAMES = {0: "CPM_OK", 1: "CPM_EINVAL", 2: "CPM_EUNSUPPORTED", 3: "CPM_ENOTPD",
                4: "CPM_EHIP", 5: "CPM_EWORKSPACE"}

EXPORTS = ["cpm_version", "cpm_last_error", "cpm_mttkrp_workspace_bytes", "mttkrp", "mttkrp_scratch",
           "cpm_mttkrp_describe", "cpm_mttkrp_all_workspace_bytes", "mttkrp_all",
           "cpm_explicit_workspace_bytes", "mttkrp_explicit", "cpm_sympair_workspace_bytes", "mttkrp_sympair", "cpm_pack_sympair",
           "cpm_residual2_workspace_bytes", "cpm_residual2",
           "cpm_cp_als_workspace_bytes", "cpm_cp_grad_workspace_bytes", "cp_als_step", "cp_grad",
           "cpm_xnorm2_workspace_bytes", "cpm_xnorm2", "cpm_split_bf16", "cpm_krp_rows"]


class CpmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_lib = None


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcpmttkrp.so is not built; run paper_1708_08976_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_size_t
    ci, cd = ctypes.c_int, ctypes.c_double
    vpp = ctypes.POINTER(ctypes.c_void_p)
    lib.cpm_version.restype = ci
    lib.cpm_last_error.restype = ctypes.c_char_p
    lib.cpm_mttkrp_workspace_bytes.argtypes = [i64p, ci, ci, ci, ci]
    lib.cpm_mttkrp_workspace_bytes.restype = sz
    lib.mttkrp.argtypes = [vp, i64p, ci, vpp, ci, ci, vp, ci, vp, sz, vp]
    lib.mttkrp.restype = ci
    lib.mttkrp_scratch.argtypes = [vp, i64p, ci, vpp, ci, ci, vp, ci, vp]
    lib.mttkrp_scratch.restype = ci
    lib.cpm_mttkrp_describe.argtypes = [i64p, ci, ci, ci, ci, vp, ctypes.c_char_p, sz]
    lib.cpm_mttkrp_describe.restype = ci
    lib.cpm_mttkrp_all_workspace_bytes.argtypes = [i64p, ci, ci, ci]
    lib.cpm_mttkrp_all_workspace_bytes.restype = sz
    lib.mttkrp_all.argtypes = [vp, i64p, ci, vpp, ci, vpp, ci, vp, sz, vp]
    lib.mttkrp_all.restype = ci
    lib.cpm_explicit_workspace_bytes.argtypes = [i64p, ci, ci, ci, ci]
    lib.cpm_explicit_workspace_bytes.restype = sz
    lib.mttkrp_explicit.argtypes = [vp, i64p, ci, vpp, ci, ci, vp, ci, vp, sz, vp]
    lib.mttkrp_explicit.restype = ci
    lib.cpm_sympair_workspace_bytes.argtypes = [i64p, ci, ci, ci]
    lib.cpm_sympair_workspace_bytes.restype = sz
    lib.mttkrp_sympair.argtypes = [vp, i64p, ci, vpp, ci, vpp, ci, vp, sz, vp]
    lib.mttkrp_sympair.restype = ci
    lib.cpm_pack_sympair.argtypes = [vp, i64p, ci, ci, vp, vp]
    lib.cpm_pack_sympair.restype = ci
    lib.cpm_residual2_workspace_bytes.argtypes = [i64p, ci, ci, ci]
    lib.cpm_residual2_workspace_bytes.restype = sz
    lib.cpm_residual2.argtypes = [vp, i64p, ci, vpp, ci, ci, vp, vp, sz, vp]
    lib.cpm_residual2.restype = ci
    lib.cpm_cp_als_workspace_bytes.argtypes = [i64p, ci, ci, ci]
    lib.cpm_cp_als_workspace_bytes.restype = sz
    lib.cpm_cp_grad_workspace_bytes.argtypes = [i64p, ci, ci, ci]
    lib.cpm_cp_grad_workspace_bytes.restype = sz
    lib.cp_als_step.argtypes = [vp, i64p, ci, vpp, ci, ci, cd, ctypes.POINTER(cd), vp, sz, vp]
    lib.cp_als_step.restype = ci
    lib.cp_grad.argtypes = [vp, i64p, ci, vpp, ci, vpp, cd, vp, ci, vp, sz, vp]
    lib.cp_grad.restype = ci
    lib.cpm_xnorm2_workspace_bytes.argtypes = [i64p, ci, ci]
    lib.cpm_xnorm2_workspace_bytes.restype = sz
    lib.cpm_xnorm2.argtypes = [vp, i64p, ci, ci, vp, vp, sz, vp]
    lib.cpm_xnorm2.restype = ci
    lib.cpm_split_bf16.argtypes = [vp, ctypes.c_int64, vp, vp]
    lib.cpm_split_bf16.restype = ci
    lib.cpm_krp_rows.argtypes = [vpp, i64p, ci, ci, ctypes.c_int64, ctypes.c_int64, vp, ci, vp]
    lib.cpm_krp_rows.restype = ci
    _lib = lib
    return lib


def last_error():
    return load().cpm_last_error().decode()


def _check(status):
    if status != CPM_OK:
        raise CpmError(status, last_error())


def _dims(dims):
    arr = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    return arr


def _ptrs(tensors):
    return (ctypes.c_void_p * len(tensors))(*[0 if t is None else t.data_ptr() for t in tensors])


def _stream(device, stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(X, dtype):
    if dtype is not None:
        return dtype
    if X.dtype == torch.float32:
        return CPM_F32
    if X.dtype == torch.float64:
        return CPM_F64
    raise TypeError("X dtype %s needs an explicit dtype code (CPM_BF16X2 for bf16 planes)" % X.dtype)


def _require(t, name):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous GPU tensor" % name)


def _workspace(nbytes, device):
    if nbytes == 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def mttkrp_workspace_bytes(dims, R, mode, dtype):
    return load().cpm_mttkrp_workspace_bytes(_dims(dims), len(dims), int(R), int(mode), int(dtype))


def mttkrp(X, dims, factors, mode, out=None, dtype=None, workspace=None, stream=None):
    """Mode-`mode` MTTKRP of X (paper-order dims) -> out (I_mode x R)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(next(f for f in factors if f is not None).shape[1])
    fdt = torch.float64 if dt == CPM_F64 else torch.float32
    for k, f in enumerate(factors):
        if f is not None and k != mode:
            _require(f, "factors[%d]" % k)
    if out is None:
        out = torch.empty((int(dims[mode]), R), dtype=fdt, device=X.device)
    _require(out, "out")
    need = lib.cpm_mttkrp_workspace_bytes(_dims(dims), len(dims), R, int(mode), dt)
    if workspace is None:
        workspace = _workspace(need, X.device)
    ws_ptr = None if workspace is None else workspace.data_ptr()
    ws_len = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib.mttkrp(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, int(mode), out.data_ptr(), dt,
                      ws_ptr, ws_len, _stream(X.device, stream)))
    return out


def mttkrp_scratch(X, dims, factors, mode, out=None, dtype=None, stream=None):
    """mttkrp with the library's built-in scratch array for its partial
    results (no workspace, nothing allocated by the library)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(next(f for f in factors if f is not None).shape[1])
    fdt = torch.float64 if dt == CPM_F64 else torch.float32
    for k, f in enumerate(factors):
        if f is not None and k != mode:
            _require(f, "factors[%d]" % k)
    if out is None:
        out = torch.empty((int(dims[mode]), R), dtype=fdt, device=X.device)
    _require(out, "out")
    _check(lib.mttkrp_scratch(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, int(mode), out.data_ptr(),
                              dt, _stream(X.device, stream)))
    return out


def describe(dims, R, mode, dtype, X=None):
    """Kernel and launch shape mttkrp picks (X only for its alignment: a
    tensor, an integer address, or None for a 4096-byte aligned one)."""
    lib = load()
    addr = 4096 if X is None else (X if isinstance(X, int) else X.data_ptr())
    buf = ctypes.create_string_buffer(512)
    _check(lib.cpm_mttkrp_describe(_dims(dims), len(dims), int(R), int(mode), int(dtype), addr, buf, 512))
    return buf.value.decode()


def mttkrp_all_workspace_bytes(dims, R, dtype):
    return load().cpm_mttkrp_all_workspace_bytes(_dims(dims), len(dims), int(R), int(dtype))


def mttkrp_all(X, dims, factors, outs=None, modes=None, dtype=None, workspace=None, stream=None):
    """MTTKRPs of every mode in `modes` (default: all) with the same factors
    -> list of N outputs (None where a mode was not requested)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(factors[0].shape[1])
    for k, f in enumerate(factors):
        _require(f, "factors[%d]" % k)
    fdt = torch.float64 if dt == CPM_F64 else torch.float32
    if outs is None:
        want = set(range(len(dims))) if modes is None else set(modes)
        outs = [torch.empty((int(d), R), dtype=fdt, device=X.device) if n in want else None
                for n, d in enumerate(dims)]
    for n, o in enumerate(outs):
        if o is not None:
            _require(o, "outs[%d]" % n)
    need = lib.cpm_mttkrp_all_workspace_bytes(_dims(dims), len(dims), R, dt)
    if workspace is None:
        workspace = _workspace(need, X.device)
    _check(lib.mttkrp_all(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, _ptrs(outs), dt,
                          None if workspace is None else workspace.data_ptr(),
                          0 if workspace is None else workspace.numel() * workspace.element_size(),
                          _stream(X.device, stream)))
    return outs


def explicit_workspace_bytes(dims, R, mode, dtype):
    return load().cpm_explicit_workspace_bytes(_dims(dims), len(dims), int(R), int(mode), int(dtype))


def mttkrp_explicit(X, dims, factors, mode, out=None, dtype=None, workspace=None, stream=None):
    """The straightforward MTTKRP (explicit X_(n), explicit Khatri-Rao
    product, one GEMM) -> out (I_mode x R)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(next(f for f in factors if f is not None).shape[1])
    fdt = torch.float64 if dt == CPM_F64 else torch.float32
    for k, f in enumerate(factors):
        if f is not None and k != mode:
            _require(f, "factors[%d]" % k)
    if out is None:
        out = torch.empty((int(dims[mode]), R), dtype=fdt, device=X.device)
    _require(out, "out")
    need = lib.cpm_explicit_workspace_bytes(_dims(dims), len(dims), R, int(mode), dt)
    if workspace is None:
        workspace = _workspace(need, X.device)
    _check(lib.mttkrp_explicit(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, int(mode), out.data_ptr(),
                               dt, None if workspace is None else workspace.data_ptr(),
                               0 if workspace is None else workspace.numel() * workspace.element_size(),
                               _stream(X.device, stream)))
    return out


def sympair_workspace_bytes(dims, R, dtype):
    return load().cpm_sympair_workspace_bytes(_dims(dims), len(dims), int(R), int(dtype))


def pack_sympair(X, dims, dtype=None, out=None, stream=None):
    """Packed triangle (i <= j of modes 0 and 1) of a full symmetric tensor
    -> flat tensor of P * I_2 * ... entries (two planes for CPM_BF16X2)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    n = int(dims[0])
    count = n * (n + 1) // 2
    for d in dims[2:]:
        count *= int(d)
    if out is None:
        if dt == CPM_BF16X2:
            out = torch.empty(2 * count, dtype=torch.int16, device=X.device)
        else:
            out = torch.empty(count, dtype=torch.float64 if dt == CPM_F64 else torch.float32, device=X.device)
    _require(out, "out")
    _check(lib.cpm_pack_sympair(X.data_ptr(), _dims(dims), len(dims), dt, out.data_ptr(), _stream(X.device, stream)))
    return out


def mttkrp_sympair(Xp, dims, factors, outs=None, modes=None, dtype=None, workspace=None, stream=None):
    """MTTKRPs of the full symmetric tensor held packed in Xp, for every
    mode in `modes` (default: all) -> list of N outputs (None where skipped)."""
    lib = load()
    dt = _dtype_code(Xp, dtype)
    _require(Xp, "Xp")
    R = int(factors[0].shape[1])
    for k, f in enumerate(factors):
        _require(f, "factors[%d]" % k)
    fdt = torch.float64 if dt == CPM_F64 else torch.float32
    if outs is None:
        want = set(range(len(dims))) if modes is None else set(modes)
        outs = [torch.empty((int(d), R), dtype=fdt, device=Xp.device) if n in want else None
                for n, d in enumerate(dims)]
    for n, o in enumerate(outs):
        if o is not None:
            _require(o, "outs[%d]" % n)
    need = lib.cpm_sympair_workspace_bytes(_dims(dims), len(dims), R, dt)
    if workspace is None:
        workspace = _workspace(need, Xp.device)
    _check(lib.mttkrp_sympair(Xp.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, _ptrs(outs), dt,
                              None if workspace is None else workspace.data_ptr(),
                              0 if workspace is None else workspace.numel() * workspace.element_size(),
                              _stream(Xp.device, stream)))
    return outs


def residual2_workspace_bytes(dims, R, dtype):
    return load().cpm_residual2_workspace_bytes(_dims(dims), len(dims), int(R), int(dtype))


def residual2(X, dims, factors, dtype=None, out=None, workspace=None, stream=None):
    """||X - [[U]]||_F^2 into a float64 GPU scalar (allocated if None)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(factors[0].shape[1])
    for k, f in enumerate(factors):
        _require(f, "factors[%d]" % k)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=X.device)
    need = lib.cpm_residual2_workspace_bytes(_dims(dims), len(dims), R, dt)
    if workspace is None:
        workspace = _workspace(need, X.device)
    _check(lib.cpm_residual2(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, dt, out.data_ptr(),
                             None if workspace is None else workspace.data_ptr(),
                             0 if workspace is None else workspace.numel() * workspace.element_size(),
                             _stream(X.device, stream)))
    return out


def cp_als_workspace_bytes(dims, R, dtype):
    return load().cpm_cp_als_workspace_bytes(_dims(dims), len(dims), int(R), int(dtype))


def cp_grad_workspace_bytes(dims, R, dtype):
    return load().cpm_cp_grad_workspace_bytes(_dims(dims), len(dims), int(R), int(dtype))


def cp_als_step(X, dims, factors, dtype=None, xnorm2=-1.0, want_fit=True, workspace=None, stream=None):
    """One CP-ALS sweep, factors updated in place.  Returns the fit or None."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(factors[0].shape[1])
    for k, f in enumerate(factors):
        _require(f, "factors[%d]" % k)
    need = lib.cpm_cp_als_workspace_bytes(_dims(dims), len(dims), R, dt)
    if workspace is None:
        workspace = _workspace(need, X.device)
    fit = ctypes.c_double(float("nan"))
    _check(lib.cp_als_step(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, dt, float(xnorm2),
                           ctypes.byref(fit) if want_fit else None,
                           None if workspace is None else workspace.data_ptr(),
                           0 if workspace is None else workspace.numel(), _stream(X.device, stream)))
    return fit.value if want_fit else None


def cp_grad(X, dims, factors, grads=None, xnorm2=-1.0, loss=None, dtype=None, workspace=None, stream=None):
    """Gradients of 1/2||X - [[U]]||^2 into grads (allocated if None; pass
    grads=False for the loss only) and the loss into `loss` (a float64 GPU
    tensor of one element, allocated if None).  Returns (grads, loss)."""
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    R = int(factors[0].shape[1])
    for k, f in enumerate(factors):
        _require(f, "factors[%d]" % k)
    if grads is None:
        grads = [torch.empty_like(f) for f in factors]
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=X.device)
    need = lib.cpm_cp_grad_workspace_bytes(_dims(dims), len(dims), R, dt)
    if workspace is None:
        workspace = _workspace(need, X.device)
    gp = _ptrs(grads) if grads else None
    _check(lib.cp_grad(X.data_ptr(), _dims(dims), len(dims), _ptrs(factors), R, gp, float(xnorm2),
                       loss.data_ptr(), dt, None if workspace is None else workspace.data_ptr(),
                       0 if workspace is None else workspace.numel(), _stream(X.device, stream)))
    return grads, loss


def xnorm2(X, dims, dtype=None, out=None, stream=None):
    lib = load()
    dt = _dtype_code(X, dtype)
    _require(X, "X")
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=X.device)
    ws = _workspace(lib.cpm_xnorm2_workspace_bytes(_dims(dims), len(dims), dt), X.device)
    _check(lib.cpm_xnorm2(X.data_ptr(), _dims(dims), len(dims), dt, out.data_ptr(),
                          None if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel(),
                          _stream(X.device, stream)))
    return out


def split_bf16(x, planes=None, stream=None):
    """float32 tensor -> int16 tensor of 2*numel bf16 bit patterns (hi plane, lo plane)."""
    lib = load()
    _require(x, "x")
    if x.dtype != torch.float32:
        raise TypeError("split_bf16 takes float32")
    if planes is None:
        planes = torch.empty(2 * x.numel(), dtype=torch.int16, device=x.device)
    _require(planes, "planes")
    _check(lib.cpm_split_bf16(x.data_ptr(), x.numel(), planes.data_ptr(), _stream(x.device, stream)))
    return planes


def krp_rows(mats, j0=0, nrows=None, out=None, stream=None):
    """Rows [j0, j0+nrows) of mats[0] kr ... kr mats[-1] (last index fastest)."""
    lib = load()
    for k, m in enumerate(mats):
        _require(m, "mats[%d]" % k)
    R = int(mats[0].shape[1])
    J = [int(m.shape[0]) for m in mats]
    total = 1
    for j in J:
        total *= j
    if nrows is None:
        nrows = total - j0
    dt = CPM_F64 if mats[0].dtype == torch.float64 else CPM_F32
    if out is None:
        out = torch.empty((nrows, R), dtype=mats[0].dtype, device=mats[0].device)
    _check(lib.cpm_krp_rows(_ptrs(mats), _dims(J), len(mats), R, int(j0), int(nrows), out.data_ptr(), dt,
                            _stream(mats[0].device, stream)))
    return out
