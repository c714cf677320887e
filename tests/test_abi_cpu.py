"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_1708_08976_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x100000  # never dereferenced: validation fails before any device access


def header_functions():
    text = open(os.path.join(ROOT, "include", "cpmttkrp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", text)
    skip = {"defined", "if", "extern"}
    return sorted({n for n in names if n not in skip and not n.isupper()})


def test_library_exports_every_declared_function():
    lib = _abi.load()
    declared = header_functions()
    assert "mttkrp" in declared and "cp_als_step" in declared and "cp_grad" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_abi.EXPORTS) == declared


def test_version_and_error_string():
    lib = _abi.load()
    assert lib.cpm_version() >= 10000
    assert isinstance(_abi.last_error(), str)


def _dims(d):
    return (ctypes.c_int64 * len(d))(*d)


def _ptrs(n, null_at=None):
    return (ctypes.c_void_p * n)(*[None if k == null_at else FAKE for k in range(n)])


def call_mttkrp(dims, R=8, mode=0, X=FAKE, out=FAKE, dt=0, factors=None, ws=None, ws_len=0, N=None):
    lib = _abi.load()
    N = len(dims) if N is None else N
    f = factors if factors is not None else _ptrs(max(1, len(dims)))
    return lib.mttkrp(X, _dims(dims) if dims else None, N, f, R, mode, out, dt, ws, ws_len, None)


@pytest.mark.parametrize("case,expect", [
    (dict(dims=(4, 5, 6), N=0), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), N=13), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), mode=3), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), mode=-1), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), R=0), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), R=257), _abi.CPM_EUNSUPPORTED),
    (dict(dims=(4, 0, 6)), _abi.CPM_EINVAL),
    (dict(dims=(4, -3, 6)), _abi.CPM_EINVAL),
    (dict(dims=(1 << 31, 1 << 31, 2)), _abi.CPM_EUNSUPPORTED),
    (dict(dims=(4, 5, 6), X=None), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), out=None), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), dt=7), _abi.CPM_EINVAL),
    (dict(dims=(4, 5, 6), dt=1, R=257), _abi.CPM_EUNSUPPORTED),
    (dict(dims=(4,), N=1), _abi.CPM_EINVAL),
    # factor 0 spans 2^24 * 64 * 4 bytes = 4 GiB: beyond one buffer resource
    (dict(dims=(1 << 24, 4, 4), R=64, mode=1), _abi.CPM_EUNSUPPORTED),
    (dict(dims=(1 << 23, 4, 4), R=64, mode=1, dt=1), _abi.CPM_EUNSUPPORTED),
])
def test_mttkrp_rejects_bad_arguments(case, expect):
    assert call_mttkrp(**case) == expect
    assert _abi.last_error() != ""


def test_factor_reach_names_the_factor():
    assert call_mttkrp((1 << 24, 4, 4), R=64, mode=1) == _abi.CPM_EUNSUPPORTED
    assert "factor 0" in _abi.last_error()
    assert call_mttkrp((4, 1 << 24, 4), R=64, mode=0) == _abi.CPM_EUNSUPPORTED
    assert "factor 1" in _abi.last_error()


def test_mttkrp_rejects_null_factor_except_own_mode():
    assert call_mttkrp((4, 5, 6), mode=0, factors=_ptrs(3, null_at=1)) == _abi.CPM_EINVAL
    assert "factors[1]" in _abi.last_error()


def test_mttkrp_workspace_checked_before_launch():
    dims = (512, 512, 512)
    need = _abi.mttkrp_workspace_bytes(dims, 32, 2, _abi.CPM_F32)
    assert need > 0
    assert call_mttkrp(dims, R=32, mode=2, ws=None, ws_len=0) == _abi.CPM_EWORKSPACE
    assert call_mttkrp(dims, R=32, mode=2, ws=FAKE, ws_len=need - 1) == _abi.CPM_EWORKSPACE


def test_workspace_queries():
    lib = _abi.load()
    assert lib.cpm_mttkrp_workspace_bytes(_dims((4, 5)), 2, 8, 5, 0) == 0  # bad mode -> 0
    assert _abi.cp_als_workspace_bytes((60, 50, 40), 8, _abi.CPM_F64) > 0
    assert _abi.cp_grad_workspace_bytes((64,) * 5, 32, _abi.CPM_F32) > 0
    assert _abi.cp_als_workspace_bytes((60, 50, 40), 129, _abi.CPM_F32) == 0
    # the gradient needs no factorisation: R up to 256
    assert _abi.cp_grad_workspace_bytes((60, 50, 40), 256, _abi.CPM_F32) > 0
    assert _abi.cp_grad_workspace_bytes((60, 50, 40), 257, _abi.CPM_F32) == 0
    assert _abi.mttkrp_workspace_bytes((60, 50, 40), 256, 1, _abi.CPM_F64) > 0


def test_solver_entry_points_validate():
    lib = _abi.load()
    d = _dims((4, 5, 6))
    assert lib.cp_als_step(FAKE, d, 3, _ptrs(3), 129, 0, -1.0, None, FAKE, 1 << 30, None) == _abi.CPM_EUNSUPPORTED
    assert lib.cp_als_step(FAKE, d, 3, _ptrs(3, null_at=2), 8, 0, -1.0, None, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.cp_als_step(FAKE, d, 3, _ptrs(3), 8, 0, -1.0, None, FAKE, 16, None) == _abi.CPM_EWORKSPACE
    assert lib.cp_grad(FAKE, d, 3, _ptrs(3), 8, None, -1.0, None, 0, None, 0, None) == _abi.CPM_EWORKSPACE
    assert lib.cp_grad(None, d, 3, _ptrs(3), 8, None, -1.0, None, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.cpm_split_bf16(None, 10, FAKE, None) == _abi.CPM_EINVAL
    assert lib.cpm_split_bf16(FAKE, -1, FAKE, None) == _abi.CPM_EINVAL
    assert lib.cpm_krp_rows(_ptrs(2), _dims((3, 4)), 2, 5, 10, 5, FAKE, 0, None) == _abi.CPM_EINVAL
    assert lib.cpm_krp_rows(_ptrs(2), _dims((3, 4)), 0, 5, 0, 5, FAKE, 0, None) == _abi.CPM_EINVAL
    assert lib.cpm_xnorm2(FAKE, d, 3, 0, FAKE, None, 0, None) == _abi.CPM_EWORKSPACE
    # cp_grad: R = 256 passes validation (stops at the workspace), 257 does not
    assert lib.cp_grad(FAKE, d, 3, _ptrs(3), 256, None, -1.0, None, 0, None, 0, None) == _abi.CPM_EWORKSPACE
    assert lib.cp_grad(FAKE, d, 3, _ptrs(3), 257, None, -1.0, None, 0, FAKE, 1 << 30, None) == _abi.CPM_EUNSUPPORTED
    assert lib.cp_grad(FAKE, d, 1, _ptrs(1), 8, None, -1.0, None, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.cp_als_step(FAKE, d, 1, _ptrs(1), 8, 0, -1.0, None, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    big = _dims((1 << 24, 4, 4))
    assert lib.cp_grad(FAKE, big, 3, _ptrs(3), 64, None, -1.0, None, 0, FAKE, 1 << 40, None) == _abi.CPM_EUNSUPPORTED
    assert lib.cp_als_step(FAKE, big, 3, _ptrs(3), 64, 0, -1.0, None, FAKE, 1 << 40, None) == _abi.CPM_EUNSUPPORTED
    assert lib.cpm_residual2(FAKE, big, 3, _ptrs(3), 64, 0, FAKE, FAKE, 1 << 40, None) == _abi.CPM_EUNSUPPORTED


def test_mttkrp_scratch_validates_before_any_device_call():
    """The entry point without a workspace: bad arguments and shapes whose
    partial results exceed the built-in scratch array are rejected before
    any HIP call (so this runs without a GPU)."""
    lib = _abi.load()

    def call(dims, R=8, mode=0, X=FAKE, out=FAKE, dt=0, factors=None):
        f = factors if factors is not None else _ptrs(len(dims))
        return lib.mttkrp_scratch(X, _dims(dims), len(dims), f, R, mode, out, dt, None)

    assert call((4, 5, 6), X=None) == _abi.CPM_EINVAL
    assert call((4, 5, 6), out=None) == _abi.CPM_EINVAL
    assert call((4, 5, 6), mode=3) == _abi.CPM_EINVAL
    assert call((4, 5, 6), R=257) == _abi.CPM_EUNSUPPORTED
    assert call((4, 5, 6), factors=_ptrs(3, null_at=2)) == _abi.CPM_EINVAL
    need = _abi.mttkrp_workspace_bytes((4096, 4096, 64), 256, 0, _abi.CPM_F32)
    assert need > 64 << 20
    assert call((4096, 4096, 64), R=256, mode=0) == _abi.CPM_EUNSUPPORTED
    assert "scratch" in _abi.last_error()
    # every benchmark workload fits the scratch array
    for dims, R in [((512, 512, 512), 32), ((256, 256, 512, 32), 128), ((64,) * 5, 128)]:
        for dt in (_abi.CPM_F32, _abi.CPM_BF16X2):
            for n in range(len(dims)):
                assert _abi.mttkrp_workspace_bytes(dims, R, n, dt) <= 64 << 20


def test_describe_names_the_kernel_and_launch():
    d = _abi.describe((512, 512, 512), 32, 1, _abi.CPM_F32)
    assert d.startswith("k_left32<NC=1,WM=1>") and "grid=" in d
    assert _abi.describe((512, 512, 512), 32, 0, _abi.CPM_F32).startswith("k_right32<")
    assert _abi.describe((60, 50, 40), 8, 0, _abi.CPM_F64).startswith("k_contract_right<f64")
    assert _abi.describe((256, 256, 512, 32), 128, 0, _abi.CPM_BF16X2).startswith("k_contract_right_bf16<NB=8")
    # rows need only 4-byte alignment on the 32x32 kernels
    assert _abi.describe((60, 50, 40), 8, 1, _abi.CPM_F32, X=4100).startswith("k_left32<")
    assert _abi.describe((165, 165, 165, 165), 25, 2, _abi.CPM_F32).startswith("k_left32<")
    assert _abi.describe((165, 165, 165, 165), 25, 0, _abi.CPM_F32).startswith("k_right32<NC=1,TJ=1")
    # rows 31 * IL apart beyond one buffer resource: the 16x16 float kernels
    assert _abi.describe((40000000, 2, 2), 8, 1, _abi.CPM_F32).startswith("k_contract_left<f32")
    lib = _abi.load()
    buf = ctypes.create_string_buffer(8)
    assert lib.cpm_mttkrp_describe(_dims((4, 5, 6)), 3, 8, 3, 0, 4096, buf, 8) == _abi.CPM_EINVAL
    assert lib.cpm_mttkrp_describe(_dims((4, 5, 6)), 3, 8, 0, 0, 4096, None, 0) == _abi.CPM_EINVAL
    assert lib.cpm_mttkrp_describe(_dims((4, 5, 6)), 3, 8, 0, 0, 4096, buf, 8) == _abi.CPM_OK
    assert len(buf.value) == 7  # truncated, NUL-terminated


def call_mttkrp_all(dims, R=8, X=FAKE, dt=0, factors=None, outs=None, ws=None, ws_len=0):
    lib = _abi.load()
    N = len(dims)
    f = factors if factors is not None else _ptrs(N)
    o = outs if outs is not None else _ptrs(N)
    return lib.mttkrp_all(X, _dims(dims), N, f, R, o, dt, ws, ws_len, None)


def test_mttkrp_all_validates_before_launch():
    lib = _abi.load()
    d = (64,) * 5
    assert call_mttkrp_all(d, X=None) == _abi.CPM_EINVAL
    assert call_mttkrp_all(d, R=257) == _abi.CPM_EUNSUPPORTED
    assert call_mttkrp_all(d, R=257, dt=_abi.CPM_F64) == _abi.CPM_EUNSUPPORTED  # as for mttkrp
    assert call_mttkrp_all((1 << 24, 4, 4, 2), R=64) == _abi.CPM_EUNSUPPORTED  # factor 0 beyond 4 GiB
    assert call_mttkrp_all(d, dt=9) == _abi.CPM_EINVAL
    # every factor is read (each one belongs to some other mode's product)
    assert call_mttkrp_all(d, factors=_ptrs(5, null_at=3)) == _abi.CPM_EINVAL
    assert "factors[3]" in _abi.last_error()
    assert lib.mttkrp_all(FAKE, _dims(d), 5, _ptrs(5), 8, None, 0, FAKE, 1 << 40, None) == _abi.CPM_EINVAL
    need = _abi.mttkrp_all_workspace_bytes(d, 32, _abi.CPM_F32)
    assert call_mttkrp_all(d, R=32, ws=None) == _abi.CPM_EWORKSPACE
    assert call_mttkrp_all(d, R=32, ws=FAKE, ws_len=need - 1) == _abi.CPM_EWORKSPACE


def test_mttkrp_all_workspace_holds_the_group_intermediates():
    """64^5, R=32: the modes split 2 | 3, so the workspace holds the left
    group's 64^2 x 32 and the right group's 64^3 x 32 float32 intermediates;
    for a 3-way tensor each mode is an ordinary MTTKRP."""
    d5 = (64,) * 5
    inter = (64 ** 2 + 64 ** 3) * 32 * 4
    ws5 = _abi.mttkrp_all_workspace_bytes(d5, 32, _abi.CPM_F32)
    per_mode = max(_abi.mttkrp_workspace_bytes(d5, 32, n, _abi.CPM_F32) for n in range(5))
    assert inter + per_mode <= ws5 <= inter + per_mode + (64 << 20)
    assert _abi.mttkrp_all_workspace_bytes(d5, 32, _abi.CPM_F64) >= 2 * inter
    # 3-way 512^3 at R = 32: modes 0 and 1 share the pass over the
    # (512 * 512, 512) view, whose 262144 x 32 intermediate is reserved;
    # split bf16 (no such pass) keeps one ordinary MTTKRP per mode
    d3 = (512, 512, 512)
    per3 = max(_abi.mttkrp_workspace_bytes(d3, 32, n, _abi.CPM_F32) for n in range(3))
    assert _abi.mttkrp_all_workspace_bytes(d3, 32, _abi.CPM_F32) >= 512 * 512 * 32 * 4 + 512 * 32 * 4
    assert _abi.mttkrp_all_workspace_bytes(d3, 32, _abi.CPM_BF16X2) == max(
        _abi.mttkrp_workspace_bytes(d3, 32, n, _abi.CPM_BF16X2) for n in range(3))
    # small 3-way tensors: no reuse
    d3s = (40, 30, 20)
    assert _abi.mttkrp_all_workspace_bytes(d3s, 16, _abi.CPM_F32) == max(
        _abi.mttkrp_workspace_bytes(d3s, 16, n, _abi.CPM_F32) for n in range(3))
    assert per3 > 0
    # intermediates as large as X itself: no reuse, ordinary MTTKRPs
    d = (2, 2, 2, 100000)
    assert _abi.mttkrp_all_workspace_bytes(d, 32, _abi.CPM_F32) == max(
        _abi.mttkrp_workspace_bytes(d, 32, n, _abi.CPM_F32) for n in range(4))
    assert _abi.cp_grad_workspace_bytes(d5, 32, _abi.CPM_F32) >= inter


def test_residual2_validates_before_launch():
    lib = _abi.load()
    d = _dims((8, 9, 10))
    assert lib.cpm_residual2(None, d, 3, _ptrs(3), 4, 0, FAKE, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.cpm_residual2(FAKE, d, 3, _ptrs(3), 4, 0, None, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.cpm_residual2(FAKE, d, 3, _ptrs(3, null_at=0), 4, 0, FAKE, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.cpm_residual2(FAKE, d, 3, _ptrs(3), 4, 1, FAKE, FAKE, 1 << 30, None) == _abi.CPM_EUNSUPPORTED
    assert lib.cpm_residual2(FAKE, d, 3, _ptrs(3), 129, 0, FAKE, FAKE, 1 << 30, None) == _abi.CPM_EUNSUPPORTED
    assert lib.cpm_residual2(FAKE, d, 3, _ptrs(3), 4, 0, FAKE, None, 0, None) == _abi.CPM_EWORKSPACE
    assert _abi.residual2_workspace_bytes((512, 512, 512), 32, _abi.CPM_F32) > 0
    assert _abi.residual2_workspace_bytes((512, 512, 512), 32, _abi.CPM_F64) == 0


def test_mttkrp_all_with_no_requested_mode_is_a_no_op():
    """Every output pointer null: validation passes and nothing is launched
    (so this runs without a GPU)."""
    d = (64,) * 5
    need = _abi.mttkrp_all_workspace_bytes(d, 32, _abi.CPM_F32)
    nulls = (ctypes.c_void_p * 5)(*([None] * 5))
    assert call_mttkrp_all(d, R=32, outs=nulls, ws=FAKE, ws_len=need) == _abi.CPM_OK


def test_sympair_validates_before_launch():
    lib = _abi.load()
    d = _dims((6, 6, 5))
    f, o = _ptrs(3), _ptrs(3)
    assert lib.mttkrp_sympair(FAKE, _dims((6, 7, 5)), 3, f, 4, o, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_sympair(FAKE, _dims((6, 6)), 2, _ptrs(2), 4, _ptrs(2), 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_sympair(None, d, 3, f, 4, o, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_sympair(FAKE, d, 3, _ptrs(3, null_at=0), 4, o, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_sympair(FAKE, d, 3, f, 4, None, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_sympair(FAKE, d, 3, f, 257, o, 0, FAKE, 1 << 30, None) == _abi.CPM_EUNSUPPORTED
    assert lib.mttkrp_sympair(FAKE, d, 3, f, 4, o, 0, FAKE, 16, None) == _abi.CPM_EWORKSPACE
    assert lib.cpm_pack_sympair(FAKE, _dims((6, 7, 5)), 3, 0, FAKE, None) == _abi.CPM_EINVAL
    assert lib.cpm_pack_sympair(None, d, 3, 0, FAKE, None) == _abi.CPM_EINVAL
    # the workspace holds the pair factor and the pair intermediate (P x R each)
    P = 256 * 257 // 2
    ws = _abi.sympair_workspace_bytes((256, 256, 512, 32), 64, _abi.CPM_F32)
    assert ws >= 2 * P * 64 * 4
    assert _abi.sympair_workspace_bytes((6, 7, 5), 4, _abi.CPM_F32) == 0


def test_explicit_validates_before_launch():
    lib = _abi.load()
    d = _dims((6, 7, 5))
    f = _ptrs(3)
    assert lib.mttkrp_explicit(FAKE, d, 3, f, 4, 1, FAKE, 2, FAKE, 1 << 30, None) == _abi.CPM_EUNSUPPORTED
    assert lib.mttkrp_explicit(None, d, 3, f, 4, 1, FAKE, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_explicit(FAKE, d, 3, f, 4, 3, FAKE, 0, FAKE, 1 << 30, None) == _abi.CPM_EINVAL
    assert lib.mttkrp_explicit(FAKE, d, 3, f, 4, 1, FAKE, 0, FAKE, 16, None) == _abi.CPM_EWORKSPACE
    # internal modes hold the reordered tensor; external ones do not
    ws1 = _abi.explicit_workspace_bytes((512, 512, 512), 32, 1, _abi.CPM_F32)
    ws0 = _abi.explicit_workspace_bytes((512, 512, 512), 32, 0, _abi.CPM_F32)
    assert ws1 - ws0 >= 512 ** 3 * 4
    assert _abi.explicit_workspace_bytes((512, 512, 512), 32, 0, _abi.CPM_BF16X2) == 0
