"""Host-side planner checks (no GPU): the kernel variants that the parity
tests rely on are the ones the planner picks."""
import re

from bf16_variants import VARIANT_CASES
from paper_1708_08976_amd import _abi

import os

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel(dims, R, mode, dt, X=None):
    return _abi.describe(dims, R, mode, dt, X).split(" ")[0]


def test_variant_cases_reach_their_kernels():
    for dims, R, mode, name in VARIANT_CASES:
        assert kernel(dims, R, mode, _abi.CPM_BF16X2) == name, (dims, R, mode)


def test_variant_cases_cover_every_variant_of_the_bf16_sweeps():
    """Every split-bf16 kernel variant that the GPU sweeps reach (16-byte
    aligned planes, as torch allocates them) has a case in VARIANT_CASES."""
    src = open(os.path.join(HERE, "test_gpu_bf16.py")).read()
    shapes = eval(re.search(r"SHAPES = (\[.*?\])\n\n", src, re.S).group(1))
    ranks = eval(re.search(r'parametrize\("R", (\[[0-9, ]+\])\)\ndef test_mttkrp_split_bf16_all_modes', src).group(1))
    reached = set()
    for dims in shapes:
        for R in ranks:
            for n in range(len(dims)):
                reached.add(kernel(dims, R, n, _abi.CPM_BF16X2))
    for R in (200, 256):
        for n in range(3):
            reached.add(kernel((40, 36, 30), R, n, _abi.CPM_BF16X2))
    listed = {name for _, _, _, name in VARIANT_CASES}
    assert reached <= listed, sorted(reached - listed)


def launch(dims, R, mode, dt):
    """(kernel, work-groups, chunk, chunks, splits, outer blocks) of a plan."""
    d = _abi.describe(dims, R, mode, dt)
    g = [int(x) for x in re.search(r"grid=\((\d+),(\d+),(\d+)\)", d).groups()]
    f = {k: int(re.search(k + r"=(\d+)", d).group(1)) for k in ("chunk", "chunks", "splits", "outer_blocks")}
    return d.split(" ")[0], g[0] * g[1] * g[2], f


# Resident work-groups per CU of each kernel at these shapes (one wave per
# SIMD each; registers and LDS), times 256 CUs.
ROUNDS = [
    ((512, 512, 512), 32, _abi.CPM_F32, [512, 768, 768]),
    ((256, 256, 512, 32), 64, _abi.CPM_F32, [512, 512, 512, 512]),
    ((256, 256, 512, 32), 128, _abi.CPM_BF16X2, [512, 512, 512, 512]),
    ((900, 900, 900), 25, _abi.CPM_F32, [512, 768, 768]),
    ((165, 165, 165, 165), 25, _abi.CPM_F32, [1024, 768, 768, 768]),
    ((60, 60, 60, 60, 60), 25, _abi.CPM_F32, [768, 768, 768, 768, 768]),
]


def test_grids_fit_one_round_of_resident_work_groups():
    """A grid just past a round ran its last few work-groups as a second
    round of the same length; the split count is rounded down instead."""
    for dims, R, dt, slots in ROUNDS:
        for n, s in enumerate(slots):
            name, groups, f = launch(dims, R, n, dt)
            assert groups <= s, (dims, R, n, name, groups, s)
            if f["splits"] < f["outer_blocks"]:
                assert groups > s // 2, (dims, R, n, name, groups, s)


def test_chunks_are_even():
    """Chunks of equal step counts: 256 contracted rows at R = 128 in four
    chunks of 64 (not 96 + 96 + 64), 165 rows in two of 96 (not 128 + 37)."""
    _, _, f = launch((256, 256, 512, 32), 128, 0, _abi.CPM_BF16X2)
    assert (f["chunk"], f["chunks"]) == (64, 4)
    _, _, f = launch((165, 165, 165, 165), 25, 0, _abi.CPM_F32)
    assert (f["chunk"], f["chunks"]) == (96, 2)
    _, _, f = launch((512, 512, 512), 32, 0, _abi.CPM_F32)
    assert (f["chunk"], f["chunks"]) == (128, 4)


def test_underfilled_round_takes_more_splits():
    """257 tiles for 512 slots: one split would leave half the CUs idle, so
    the planner takes the split count with the shortest estimated time."""
    name, groups, f = launch((32896, 512, 32), 64, 2, _abi.CPM_F32)
    assert f["chunks"] == 257 and f["splits"] == 3 and groups == 771, (name, groups, f)
    name, groups, f = launch((32896, 512, 32), 128, 2, _abi.CPM_BF16X2)
    assert f["chunks"] == 257 and f["splits"] == 3 and groups == 771, (name, groups, f)
