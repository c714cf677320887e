"""Split-bf16 kernel variants and one small case that reaches each.

The planner picks a kernel and its template parameters (rank blocks NB,
row tiles MB, inner groups Q, 8-wide loads V8, wave row groups WM) from the
shape, the rank and the alignment.  VARIANT_CASES lists, for every variant
that the GPU parity sweeps reach, one case (dims, R, mode) that reaches it,
with the kernel the planner must report for it; a CPU test checks both
facts, and a GPU test runs each case with and without the tensor's lo plane.
"""

# (dims, R, mode, kernel with template parameters)
VARIANT_CASES = [
    ((5, 7, 3, 11, 13), 1, 3, "k_contract_left_bf16<NB=1,MB=1,Q=1,V8=0,WM=2>"),
    ((5, 7, 3, 11, 13), 1, 2, "k_contract_left_bf16<NB=1,MB=1,Q=1,V8=0,WM=4>"),
    ((200, 3), 1, 1, "k_contract_left_bf16<NB=1,MB=1,Q=1,V8=1,WM=1>"),
    ((16, 33, 2, 9), 1, 2, "k_contract_left_bf16<NB=1,MB=1,Q=1,V8=1,WM=4>"),
    ((1000, 1, 1), 1, 1, "k_contract_left_bf16<NB=1,MB=1,Q=2,V8=1,WM=1>"),
    ((37, 29, 41), 1, 1, "k_contract_left_bf16<NB=1,MB=2,Q=1,V8=0,WM=4>"),
    ((64, 48, 80), 1, 1, "k_contract_left_bf16<NB=1,MB=2,Q=1,V8=1,WM=2>"),
    ((40, 24, 36), 1, 1, "k_contract_left_bf16<NB=1,MB=2,Q=1,V8=1,WM=4>"),
    ((3, 130, 21), 1, 2, "k_contract_left_bf16<NB=1,MB=2,Q=2,V8=0,WM=1>"),
    ((8, 33, 64), 8, 2, "k_contract_left_bf16<NB=1,MB=2,Q=2,V8=1,WM=1>"),
    ((5, 7, 3, 11, 13), 32, 3, "k_contract_left_bf16<NB=2,MB=1,Q=1,V8=0,WM=2>"),
    ((5, 7, 3, 11, 13), 32, 2, "k_contract_left_bf16<NB=2,MB=1,Q=1,V8=0,WM=4>"),
    ((200, 3), 32, 1, "k_contract_left_bf16<NB=2,MB=1,Q=1,V8=1,WM=1>"),
    ((16, 33, 2, 9), 32, 2, "k_contract_left_bf16<NB=2,MB=1,Q=1,V8=1,WM=4>"),
    ((1000, 1, 1), 32, 1, "k_contract_left_bf16<NB=2,MB=1,Q=2,V8=1,WM=1>"),
    ((37, 29, 41), 32, 1, "k_contract_left_bf16<NB=2,MB=2,Q=1,V8=0,WM=4>"),
    ((64, 48, 80), 32, 1, "k_contract_left_bf16<NB=2,MB=2,Q=1,V8=1,WM=2>"),
    ((40, 24, 36), 32, 1, "k_contract_left_bf16<NB=2,MB=2,Q=1,V8=1,WM=4>"),
    ((3, 130, 21), 32, 2, "k_contract_left_bf16<NB=2,MB=2,Q=2,V8=0,WM=1>"),
    ((8, 64, 64), 32, 2, "k_contract_left_bf16<NB=2,MB=2,Q=2,V8=1,WM=1>"),
    ((16, 33, 64), 40, 2, "k_contract_left_bf16<NB=4,MB=1,Q=1,V8=1,WM=4>"),
    ((5, 7, 3, 11, 13), 70, 3, "k_contract_left_bf16<NB=8,MB=1,Q=1,V8=0,WM=2>"),
    ((37, 29, 41), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=1,V8=0,WM=4>"),
    ((200, 3), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=1,V8=1,WM=1>"),
    ((64, 48, 80), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=1,V8=1,WM=2>"),
    ((64, 48, 80), 70, 2, "k_contract_left_bf16<NB=8,MB=1,Q=1,V8=1,WM=4>"),
    ((260, 40, 20), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=2,V8=0,WM=2>"),
    ((260, 70, 20), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=2,V8=0,WM=4>"),
    ((256, 40, 20), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=2,V8=1,WM=2>"),
    ((256, 70, 20), 70, 1, "k_contract_left_bf16<NB=8,MB=1,Q=2,V8=1,WM=4>"),
    ((37, 29, 41), 1, 0, "k_contract_right_bf16<NB=1,V8=0>"),
    ((64, 48, 80), 1, 0, "k_contract_right_bf16<NB=1,V8=1>"),
    ((37, 29, 41), 32, 0, "k_contract_right_bf16<NB=2,V8=0>"),
    ((64, 48, 80), 32, 0, "k_contract_right_bf16<NB=2,V8=1>"),
    ((64, 48, 80), 40, 0, "k_contract_right_bf16<NB=4,V8=1>"),
    ((37, 29, 41), 70, 0, "k_contract_right_bf16<NB=8,V8=0>"),
    ((64, 48, 80), 70, 0, "k_contract_right_bf16<NB=8,V8=1>"),
]
