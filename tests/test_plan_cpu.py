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
