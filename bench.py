"""Benchmark of the dense MTTKRP path on one MI355X.

One step = the mode-0, mode-1 and mode-2 MTTKRP of a 512 x 512 x 512 float32
tensor (a rank-32 CP model with N(0,1) factors plus 1% Gaussian noise) with
rank R = 32, inputs resident in HBM, as one mttkrp_all call (modes 0 and 1
from one pass that contracts mode 2, mode 2 from an ordinary pass).
`value` is the MTTKRP throughput of the whole step in GFLOP/s (2*I*R flops
per mode).  The line also carries the roofline of the step's slowest pass
over X (HBM-bound at R = 32), the single-mode calls' figures, and the FP64
oracle timed on the host cores as a CPU baseline (all cores and one core).

Extra measurements (on by default, --quick skips them, --only picks
sections): the CP-ALS sweep and exact residual on the same tensor; the
256x256x512x32 correlation-style tensor at R = 64 in float32 and at R = 128
in split bf16 against float32, with the split form's per-mode error against
the FP64 oracle (sampled rows), unpacked and in packed symmetric-pair
storage; CP-gradient evaluations per second on the 64^5 tensor in float32
and split bf16; the straightforward explicit-unfolding baseline (reordered
tensor, explicit Khatri-Rao product, one hipBLASLt GEMM) beside the fused
kernels; and the paper-shaped tensors (equal-sided ~7.5e8 entries at rank
25, the fMRI shapes at ranks 10, 20, 30).  `rooflines` lists the roofline
of every graded workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="main workload only")
    ap.add_argument("--only", default="", help="comma-separated extra sections: als, residual, sym4d, "
                    "sympair, grad, explicit, paper (default: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 512 MiB device copy (known bytes) to scale HBM counters")
    return ap.parse_args()


KERNEL_FILES = ("device_common.hpp", "mttkrp32_kernels.hpp", "mttkrp_kernels.hpp")


def kernel_source_sha(launch=""):
    """Hash of the sources that define the MTTKRP contraction and reduction
    kernels, and of the launch the planner picks (its description)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1708_08976_amd", "csrc")
    for name in KERNEL_FILES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    h.update(launch.encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, launch):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources or the launch changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    shas = rec.get("kernel_source_sha")
    if not isinstance(shas, dict) or shas.get(kernel) != kernel_source_sha(launch):
        return None
    return rec.get("per_launch", {}).get(kernel)


class Timer:
    """HIP events on the stream the library launches on."""

    def __init__(self, torch, stream):
        self.torch = torch
        self.stream = stream

    def event(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e


def algo_bytes(dims, R, mode, xbytes):
    I = 1
    for d in dims:
        I *= d
    fb = sum(d * R * 4 for k, d in enumerate(dims) if k != mode)
    return I * xbytes + fb + dims[mode] * R * 4


def time_modes(torch, _abi, X, dims, U, outs, ws, dt, steps, warmup, stream):
    """Whole-step time (ms): `steps` passes over all modes between two HIP
    events.  Per-mode time (ms per call): each mode's call repeated `steps`
    times back to back between two events, so the figure is the launches'
    own duration (contraction plus split reduction) without event records
    in between."""
    timer = Timer(torch, stream)
    N = len(dims)

    def call(n):
        _abi.mttkrp(X, dims, U, n, out=outs[n], dtype=dt, workspace=ws)

    for _ in range(warmup):
        for n in range(N):
            call(n)
    torch.cuda.synchronize()
    t0 = timer.event()
    for _ in range(steps):
        for n in range(N):
            call(n)
    t1 = timer.event()
    torch.cuda.synchronize()
    step_ms = t0.elapsed_time(t1) / steps
    per_mode = []
    for n in range(N):
        call(n)
        a = timer.event()
        for _ in range(steps):
            call(n)
        b = timer.event()
        torch.cuda.synchronize()
        per_mode.append(a.elapsed_time(b) / steps)
    return step_ms, per_mode


def shape_class(dims, n):
    if n == 0:
        return "mode0 (contiguous output index, right-first)"
    if n == len(dims) - 1:
        return "last mode (contracted index contiguous, left-first)"
    return "internal (fused 2-step)"


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, dims, U, min_seconds=10.0, max_reps=40):
    """The FP64 oracle on the host cores: all modes of the main tensor,
    repeated until at least `min_seconds` of CPU work (bounded); then mode 1
    once on one core."""
    import numpy as np

    from oracle import oracle as O
    Xh = X.cpu().numpy().ravel()
    Uh = [u.cpu().numpy().astype(np.float64) for u in U]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    reps = 0
    t0 = time.perf_counter()
    while reps < max_reps:
        for n in range(len(dims)):
            O.mttkrp(Xh, dims, Uh, n, nthreads=threads)
        reps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    I = Xh.size
    R = Uh[0].shape[1]
    flops = reps * len(dims) * 2.0 * I * R
    t1 = time.perf_counter()
    O.mttkrp(Xh, dims, Uh, 1, nthreads=1)
    d1 = time.perf_counter() - t1
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "all %d modes of the full %s float32 tensor, R=%d, repeated %d times (%.1f s)" % (
                len(dims), "x".join(map(str, dims)), R, reps, dt),
            "cpu_model": cpu_model(),
            "one_core": {"value": round(2.0 * I * R / d1 / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                         "sample": "mode 1 of the same tensor once (%.1f s)" % d1}}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d (WORLD_SIZE=%d) is not supported"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1708_08976_amd import _abi, inputs
    _abi.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    if args.calibrate_copy:
        # 512 MiB read + 512 MiB written per launch, three launches.
        src = torch.randn(128 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------- main workload: 512^3 float32, R = 32 ----------------
    # One step = the MTTKRP of every mode, one mttkrp_all call: modes 0 and 1
    # come from one pass over the (512*512, 512) view that contracts mode 2
    # (the cross-mode reuse), mode 2 from an ordinary pass.
    dims, R = (512, 512, 512), 32
    X, _ = inputs.noisy_low_rank(dims, R, seed_factors=3, seed_noise=4, eta=0.01, device="cuda")
    U = inputs.normal_factors(dims, R, seed=5, device="cuda")
    outs = [torch.empty((d, R), device=dev) for d in dims]
    ws = torch.empty(max(_abi.mttkrp_workspace_bytes(dims, R, n, _abi.CPM_F32) for n in range(3)) + 256,
                     dtype=torch.uint8, device=dev)
    wsa = torch.empty(max(256, _abi.mttkrp_all_workspace_bytes(dims, R, _abi.CPM_F32)), dtype=torch.uint8, device=dev)
    reuse = _abi.mttkrp_all_workspace_bytes(dims, R, _abi.CPM_F32) > ws.numel()
    timer = Timer(torch, stream)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.warmup):
        _abi.mttkrp_all(X, dims, U, outs=outs, workspace=wsa)
    torch.cuda.synchronize()
    t0 = timer.event()
    for _ in range(args.steps):
        _abi.mttkrp_all(X, dims, U, outs=outs, workspace=wsa)
    t1 = timer.event()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    step_ms = t0.elapsed_time(t1) / args.steps
    # the single-mode calls (what a caller wanting one mode gets), timed after
    _, per_mode = time_modes(torch, _abi, X, dims, U, outs, ws, _abi.CPM_F32, args.steps, 1, stream)
    I = 512 ** 3
    flops_mode = 2.0 * I * R
    value = 3 * flops_mode / (step_ms / 1e3) / 1e9
    modes = []
    for n in range(3):
        b = algo_bytes(dims, R, n, 4)
        gbs = b / (per_mode[n] / 1e3) / 1e9
        modes.append({"mode": n, "class": shape_class(dims, n), "kernel": _abi.describe(dims, R, n, _abi.CPM_F32, X),
                      "us": round(per_mode[n] * 1e3, 2),
                      "GFLOP/s": round(flops_mode / (per_mode[n] / 1e3) / 1e9, 1),
                      "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
    # the step's two passes over X, each timed as the same library call on
    # its own (the wide pass is mode 0 of the (512*512, 512) view)
    L = dims[0] * dims[1]
    wide = torch.empty((L, R), device=dev)
    launches = []
    if reuse:
        wide_us = timed(torch, stream, lambda: _abi.mttkrp(X, (L, dims[2]), [None, U[2]], 0, out=wide, workspace=ws),
                        args.steps) * 1e3
        launches.append(("wide_pass", "modes 0-1 pass: mode 0 of the (512*512, 512) view, %s" % _abi.describe(
            (L, dims[2]), R, 0, _abi.CPM_F32, X), wide_us, I * 4 + dims[2] * R * 4 + L * R * 4,
            _abi.describe((L, dims[2]), R, 0, _abi.CPM_F32, X)))
        launches.append(("mttkrp_mode2", "mode 2 pass, %s" % modes[2]["kernel"], per_mode[2] * 1e3,
                         algo_bytes(dims, R, 2, 4), modes[2]["kernel"]))
    else:
        for n in range(3):
            launches.append(("mttkrp_mode%d" % n, modes[n]["kernel"], per_mode[n] * 1e3, algo_bytes(dims, R, n, 4),
                             modes[n]["kernel"]))
    dom = max(launches, key=lambda x: x[2])
    achieved = dom[3] / (dom[2] / 1e6) / 1e9
    roofline = {"bound": "hbm", "kernel": dom[0] + " (" + dom[1] + "; one C-ABI call)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes": dom[3],
                "traffic": measured_traffic("fp32_512cube_r32", dom[0], dom[4])}

    line = {"metric": "MTTKRP GFLOP/s (all modes) + HBM GB/s, % of roofline", "value": round(value, 1),
            "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(step_ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "512x512x512 float32 tensor (rank-32 CP model, N(0,1) factors, 1% noise), "
                                   "R=32, MTTKRP of modes 0,1,2 per step (one mttkrp_all call: modes 0 and 1 "
                                   "from one pass that contracts mode 2, mode 2 from an ordinary pass)",
                       "dims": list(dims), "R": R},
            "roofline": roofline, "per_mode": modes,
            "step_components_us": {name: round(us, 2) for name, _, us, _, _ in launches},
            "ms_per_step_three_single_mode_calls": round(sum(per_mode), 4),
            "wall_s_timed": round(wall, 3)}
    # context for the fraction above: what PyTorch's own streaming kernels
    # reach on the same 512 MiB tensor on this GPU (a reduction reads it
    # once; a copy reads and writes it)
    dst = torch.empty_like(X)
    t_sum = timed(torch, stream, lambda: X.sum(), args.steps)
    t_copy = timed(torch, stream, lambda: dst.copy_(X), args.steps)
    line["read_probe"] = {"torch_sum_GB/s": round(I * 4 / (t_sum / 1e3) / 1e9, 1),
                          "torch_copy_GB/s": round(2 * I * 4 / (t_copy / 1e3) / 1e9, 1)}
    del dst
    rooflines = [dict(roofline, workload="512^3 float32 R=32, slowest pass of the step")]

    if not args.quick:
        want = set(x for x in args.only.split(",") if x) or set(SECTIONS)
        extra = {}
        for name in SECTIONS:
            if name in want:
                print("bench: section %s" % name, file=sys.stderr, flush=True)
                try:
                    SECTIONS[name](torch, _abi, inputs, X, dims, U, stream, extra, rooflines)
                except Exception as e:  # a failed extra section is reported, not fatal to the line
                    extra["error_" + name] = "%s: %s" % (type(e).__name__, e)
                    torch.cuda.synchronize()
                    torch.cuda.empty_cache()
        line["extra"] = extra
    line["rooflines"] = rooflines

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(X, dims, U)
    print(json.dumps(line), flush=True)


def timed(torch, stream, fn, reps, warm=1):
    """ms per call of fn, `reps` calls between two HIP events."""
    timer = Timer(torch, stream)
    for _ in range(warm):
        fn()
    a = timer.event()
    for _ in range(reps):
        fn()
    b = timer.event()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def sec_als(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """CP-ALS sweep on the main tensor (MTTKRP x3 + FP64 Grams/Cholesky/solves)."""
    dev = X2.device
    Ua = [u.clone() for u in U2]
    ws = torch.empty(_abi.cp_als_workspace_bytes(dims2, 32, _abi.CPM_F32), dtype=torch.uint8, device=dev)
    xn = float(_abi.xnorm2(X2, dims2).item())
    res = {}
    ms = timed(torch, stream, lambda: res.__setitem__(
        "fit", _abi.cp_als_step(X2, dims2, Ua, xnorm2=xn, want_fit=True, workspace=ws)), 5, warm=2)
    out["cp_als_sweep_512cube_r32"] = {"ms": round(ms, 3), "fit": round(res["fit"], 6)}
    # 20 CP-ALS sweeps from the N(0,1) start (seed 5), as in the 512^3 workload
    Ub = inputs.normal_factors(dims2, 32, seed=5, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        fit = _abi.cp_als_step(X2, dims2, Ub, xnorm2=xn, want_fit=True, workspace=ws)
    out["cp_als_20_sweeps_512cube_r32"] = {"ms": round((time.perf_counter() - t0) * 1e3, 3),
                                           "final_fit": round(fit, 6)}


def sec_residual(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """Exact squared residual ||X - [[U]]||^2 (one pass over X, the model
    formed on the fly), float32 and split bf16."""
    dev = X2.device
    P2 = _abi.split_bf16(X2.reshape(-1))
    r2 = torch.empty((), dtype=torch.float64, device=dev)
    rec = {}
    for dt, tag, Xin in [(_abi.CPM_F32, "fp32", X2), (_abi.CPM_BF16X2, "bf16x2", P2)]:
        wsr = torch.empty(max(1, _abi.residual2_workspace_bytes(dims2, 32, dt)), dtype=torch.uint8, device=dev)
        us = timed(torch, stream, lambda: _abi.residual2(Xin, dims2, U2, dtype=dt, out=r2, workspace=wsr), 20,
                   warm=2) * 1e3
        nbytes = 4 * 512 ** 3
        rec[tag] = {"us": round(us, 1), "GB/s": round(nbytes / us / 1e3, 1),
                    "hbm_frac": round(nbytes / us / 1e3 / HBM_PEAK_GBS, 4)}
    out["residual2_512cube_r32"] = rec


def sampled_errors(O, got, Xh, dims, Uh, xtype=None):
    """Normwise error of rows {0, 1, mid+1, last} of every mode against the
    FP64 oracle (rows computed one by one)."""
    import numpy as np
    errs = []
    for n in range(len(dims)):
        rows = sorted({0, 1, dims[n] // 2 + 1, dims[n] - 1} & set(range(dims[n])))
        ref = O.mttkrp_rows(Xh, dims, Uh, n, rows, xtype=xtype)
        g = np.asarray(got[n], dtype=np.float64)[rows]
        errs.append(float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
    return errs


def sec_sym4d(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """256x256x512x32 correlation-style tensor: float32 at R=64 and R=128,
    split bf16 at R=128 (same tensor, same factors), one call per mode and
    all four modes with the cross-mode reuse; split bf16's per-mode error
    against the FP64 oracle."""
    import numpy as np

    from oracle import oracle as O
    dev = X2.device
    dims3 = (256, 256, 512, 32)
    I3 = 256 * 256 * 512 * 32
    X3 = inputs.symmetric_pair_tensor(dims3, seed=6, device="cuda")
    P3 = _abi.split_bf16(X3.reshape(-1))
    runs = {}
    for R, dt, tag in [(64, _abi.CPM_F32, "fp32_r64"), (128, _abi.CPM_F32, "fp32_r128"),
                       (128, _abi.CPM_BF16X2, "bf16x2_r128")]:
        U3 = inputs.normal_factors(dims3, R, seed=7 if R == 64 else 8, device="cuda")
        outs = [torch.empty((d, R), device=dev) for d in dims3]
        ws3 = torch.empty(max(_abi.mttkrp_workspace_bytes(dims3, R, n, dt) for n in range(4)) + 256,
                          dtype=torch.uint8, device=dev)
        Xin = P3 if dt == _abi.CPM_BF16X2 else X3
        step_ms, per_mode = time_modes(torch, _abi, Xin, dims3, U3, outs, ws3, dt, 5, 1, stream)
        fl = 2.0 * I3 * R
        rec = {"ms_all_modes": round(step_ms, 3),
               "per_mode_us": [round(t * 1e3, 1) for t in per_mode],
               "per_mode_TFLOP/s": [round(fl / (t / 1e3) / 1e12, 2) for t in per_mode],
               "per_mode_hbm_frac": [round(algo_bytes(dims3, R, n, 4) / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                     for n, t in enumerate(per_mode)],
               "kernels": [_abi.describe(dims3, R, n, dt, Xin).split(" ")[0] for n in range(4)]}
        if dt == _abi.CPM_BF16X2:
            # three bf16 MFMA products per multiply-add of the method
            rec["per_mode_bf16_mfma_frac"] = [round(3 * fl / (t / 1e3) / 1e12 / BF16_PEAK_TFLOPS, 4)
                                              for t in per_mode]
            torch.cuda.synchronize()
            got = [o.cpu().numpy() for o in outs]
            Uh = [u.cpu().numpy() for u in U3]
            rec["per_mode_rel_err_vs_fp64_oracle"] = {
                "float32_tensor": [float("%.3e" % e) for e in sampled_errors(O, got, X3.cpu().numpy().ravel(),
                                                                            dims3, Uh)],
                "pair_values": [float("%.3e" % e) for e in sampled_errors(O, got, P3.cpu().numpy().view(np.uint16),
                                                                         dims3, Uh, xtype=O.BF16PAIR)],
                "rows": "0, 1, I_n/2+1, I_n-1 of every mode (all columns), normwise"}
            slow = max(range(4), key=lambda n: per_mode[n])
            b = algo_bytes(dims3, R, slow, 4)
            rooflines.append({"workload": "256x256x512x32 split bf16 R=128, slowest mode %d" % slow,
                              "bound": "hbm", "achieved": round(b / (per_mode[slow] / 1e3) / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(b / (per_mode[slow] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)})
        else:
            rec["per_mode_fp32_peak_frac"] = [round(fl / (t / 1e3) / 1e12 / FP32_PEAK_TFLOPS, 4)
                                              for t in per_mode]
            if R == 64:
                slow = max(range(4), key=lambda n: per_mode[n])
                ach = fl / (per_mode[slow] / 1e3) / 1e12
                rooflines.append({"workload": "256x256x512x32 float32 R=64, slowest mode %d" % slow,
                                  "bound": "mfma", "achieved": round(ach, 2), "peak": FP32_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4)})
        # all four modes at once with the cross-mode reuse (modes split 2 | 2)
        wsa = torch.empty(max(1, _abi.mttkrp_all_workspace_bytes(dims3, R, dt)), dtype=torch.uint8, device=dev)
        rec["ms_all_modes_cross_mode_reuse"] = round(timed(torch, stream, lambda: _abi.mttkrp_all(
            Xin, dims3, U3, outs=outs, dtype=dt, workspace=wsa), 3), 3)
        rec["cross_mode_reuse_speedup"] = round(step_ms / rec["ms_all_modes_cross_mode_reuse"], 3)
        runs[tag] = rec
        out["sym4d_" + tag] = rec
        del U3, outs, ws3, wsa
    out["sym4d_r128_split_bf16_speedup_over_fp32"] = {
        "all_modes": round(runs["fp32_r128"]["ms_all_modes"] / runs["bf16x2_r128"]["ms_all_modes"], 3),
        "per_mode": [round(a / b, 3) for a, b in zip(runs["fp32_r128"]["per_mode_us"],
                                                       runs["bf16x2_r128"]["per_mode_us"])]}
    del X3, P3
    torch.cuda.empty_cache()


def sec_sympair(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """The same correlation tensor in packed symmetric-pair storage (the
    triangle i <= j of modes 0 and 1, P = 32896 pairs): every mode of the
    unpacked tensor, per mode and all four in one call, against the packed
    tensor's bytes."""
    dev = X2.device
    dims3 = (256, 256, 512, 32)
    P = 256 * 257 // 2
    Ip = P * 512 * 32
    X3 = inputs.symmetric_pair_tensor(dims3, seed=6, device="cuda")
    for R, dt, tag in [(64, _abi.CPM_F32, "fp32_r64"), (128, _abi.CPM_BF16X2, "bf16x2_r128")]:
        full = X3 if dt == _abi.CPM_F32 else _abi.split_bf16(X3.reshape(-1))
        packed = _abi.pack_sympair(full, dims3, dtype=dt)
        if dt != _abi.CPM_F32:
            del full
        U3 = inputs.normal_factors(dims3, R, seed=7 if R == 64 else 8, device="cuda")
        outs = [torch.empty((d, R), device=dev) for d in dims3]
        ws = torch.empty(_abi.sympair_workspace_bytes(dims3, R, dt), dtype=torch.uint8, device=dev)
        per = []
        for n in range(4):
            o = [outs[k] if k == n else None for k in range(4)]
            per.append(timed(torch, stream, lambda: _abi.mttkrp_sympair(packed, dims3, U3, outs=o, dtype=dt,
                                                                        workspace=ws), 5))
        t_all = timed(torch, stream, lambda: _abi.mttkrp_sympair(packed, dims3, U3, outs=outs, dtype=dt,
                                                                 workspace=ws), 5)
        nbytes = Ip * 4
        fl = 2.0 * 256 * 256 * 512 * 32 * R  # the unpacked tensor's MTTKRP flops (same result)
        rec = {"packed_entries": Ip, "packed_bytes": nbytes,
               "per_mode_us": [round(t * 1e3, 1) for t in per],
               "per_mode_hbm_frac_packed_bytes": [round(nbytes / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4) for t in per],
               "per_mode_unpacked_equivalent_TFLOP/s": [round(fl / (t / 1e3) / 1e12, 2) for t in per],
               "ms_all_modes_one_call": round(t_all, 3)}
        unpacked = out.get("sym4d_" + tag)
        if unpacked:
            rec["per_mode_speedup_over_unpacked"] = [round(u / (t * 1e3), 3)
                                                     for u, t in zip(unpacked["per_mode_us"], per)]
        out["sympair_" + tag] = rec
        slow = max(range(4), key=lambda n: per[n])
        ach = nbytes / (per[slow] / 1e3) / 1e9
        rooflines.append({"workload": "256x256x512x32 packed symmetric pair %s, slowest mode %d" % (tag, slow),
                          "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ach / HBM_PEAK_GBS, 4)})
        del packed, U3, outs, ws
    del X3
    torch.cuda.empty_cache()


def sec_grad(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """CP gradient evaluations per second on 64^5: float32 and split bf16."""
    dev = X2.device
    dims5 = (64,) * 5
    X5, _ = inputs.noisy_low_rank(dims5, 32, seed_factors=9, seed_noise=10, eta=0.05, device="cuda")
    P5 = _abi.split_bf16(X5.reshape(-1))
    x5 = float(_abi.xnorm2(X5, dims5).item())
    for R5 in (32, 128):
        U5 = inputs.normal_factors(dims5, R5, seed=11, device="cuda")
        grads = [torch.empty_like(u) for u in U5]
        loss = torch.empty((), dtype=torch.float64, device=dev)
        res = {}
        for dt, tag, Xin in [(_abi.CPM_F32, "fp32", X5), (_abi.CPM_BF16X2, "bf16x2", P5)]:
            ws5 = torch.empty(_abi.cp_grad_workspace_bytes(dims5, R5, dt), dtype=torch.uint8, device=dev)
            ms = timed(torch, stream, lambda: _abi.cp_grad(Xin, dims5, U5, grads=grads, xnorm2=x5, loss=loss,
                                                           dtype=dt, workspace=ws5), 5, warm=2)
            res[tag] = ms
            outs5 = [torch.empty_like(u) for u in U5]
            wsa = torch.empty(max(1, _abi.mttkrp_all_workspace_bytes(dims5, R5, dt)), dtype=torch.uint8, device=dev)
            wsm = torch.empty(max(1, max(_abi.mttkrp_workspace_bytes(dims5, R5, n, dt) for n in range(5))),
                              dtype=torch.uint8, device=dev)

            def one_by_one():
                for n in range(5):
                    _abi.mttkrp(Xin, dims5, U5, n, out=outs5[n], dtype=dt, workspace=wsm)

            t_reuse = timed(torch, stream, lambda: _abi.mttkrp_all(Xin, dims5, U5, outs=outs5, dtype=dt,
                                                                   workspace=wsa), 5)
            t_per = timed(torch, stream, one_by_one, 5)
            # algorithmic bytes: X twice, each group intermediate written
            # once and read by every leaf of its group (s = 2 of 5 modes)
            inter = (64 ** 2 * 3 + 64 ** 3 * 4) * R5 * 4
            two_pass = 2 * 4 * 64 ** 5 + inter
            roof = HBM_PEAK_GBS * 1e9 / two_pass
            out["cp_grad_64p5_r%d_%s" % (R5, tag)] = {
                "ms_per_eval": round(ms, 3), "evals_per_s": round(1e3 / ms, 2),
                "hbm_roofline_evals_per_s": round(roof, 1),
                "hbm_roofline_evals_per_s_one_pass_per_mode": round(HBM_PEAK_GBS * 1e9 / (5 * 4 * 64 ** 5), 1),
                "five_mttkrps_ms_cross_mode_reuse": round(t_reuse, 3),
                "five_mttkrps_ms_one_pass_per_mode": round(t_per, 3),
                "cross_mode_reuse_speedup": round(t_per / t_reuse, 3)}
            if R5 == 32 and tag == "fp32":
                rooflines.append({"workload": "64^5 float32 R=32 cp_grad (two passes over X + leaves + Grams)",
                                  "bound": "hbm", "achieved": round(1e3 / ms, 2), "peak": round(roof, 1),
                                  "unit": "evals/s", "frac": round(1e3 / ms / roof, 4)})
            del ws5, wsa, wsm, outs5
        out["cp_grad_64p5_r%d_split_bf16_speedup_over_fp32" % R5] = round(res["fp32"] / res["bf16x2"], 3)
        if R5 == 32:
            # one CP-ALS sweep on 64^5 (Gauss-Seidel over the five modes with
            # the cross-mode reuse: two passes over X instead of five)
            Ua = [u.clone() for u in U5]
            wsa = torch.empty(_abi.cp_als_workspace_bytes(dims5, R5, _abi.CPM_F32), dtype=torch.uint8, device=dev)
            fitr = {}
            ms = timed(torch, stream, lambda: fitr.__setitem__("f", _abi.cp_als_step(
                X5, dims5, Ua, xnorm2=x5, want_fit=True, workspace=wsa)), 3, warm=2)
            one_pass = out["cp_grad_64p5_r32_fp32"]["five_mttkrps_ms_one_pass_per_mode"]
            out["cp_als_sweep_64p5_r32"] = {"ms": round(ms, 3), "fit": round(fitr["f"], 6),
                                            "five_mttkrps_ms_one_pass_per_mode": one_pass,
                                            "sweep_vs_five_single_mode_mttkrps": round(one_pass / ms, 3)}
            del Ua, wsa
        del U5, grads
    del X5, P5
    torch.cuda.empty_cache()


def sec_explicit(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """The straightforward MTTKRP (internal modes reordered into X_(n), the
    full Khatri-Rao product formed, one hipBLASLt GEMM) beside the fused
    kernels, per mode, on the 512^3 R=32, 256x256x512x32 R=64 and 64^5 R=32
    float32 workloads."""
    dev = X2.device
    cases = [("512cube_r32", dims2, 32, lambda: X2, lambda: U2),
             ("sym4d_r64", (256, 256, 512, 32), 64,
              lambda: inputs.symmetric_pair_tensor((256, 256, 512, 32), seed=6, device="cuda"),
              lambda: inputs.normal_factors((256, 256, 512, 32), 64, seed=7, device="cuda")),
             ("64p5_r32", (64,) * 5, 32,
              lambda: inputs.noisy_low_rank((64,) * 5, 32, seed_factors=9, seed_noise=10, eta=0.05,
                                            device="cuda")[0],
              lambda: inputs.normal_factors((64,) * 5, 32, seed=11, device="cuda"))]
    for tag, dims, R, mkX, mkU in cases:
        X = mkX()
        U = mkU()
        o = [torch.empty((d, R), device=dev) for d in dims]
        per_f, per_e = [], []
        for n in range(len(dims)):
            wsf = torch.empty(max(1, _abi.mttkrp_workspace_bytes(dims, R, n, _abi.CPM_F32)), dtype=torch.uint8,
                              device=dev)
            wse = torch.empty(_abi.explicit_workspace_bytes(dims, R, n, _abi.CPM_F32), dtype=torch.uint8,
                              device=dev)
            per_f.append(timed(torch, stream, lambda: _abi.mttkrp(X, dims, U, n, out=o[n], workspace=wsf), 3))
            per_e.append(timed(torch, stream, lambda: _abi.mttkrp_explicit(X, dims, U, n, out=o[n], workspace=wse),
                               3))
            del wsf, wse
        out["explicit_baseline_" + tag] = {
            "per_mode_ms_explicit": [round(t, 3) for t in per_e],
            "per_mode_ms_fused": [round(t, 3) for t in per_f],
            "per_mode_fused_speedup": [round(e / f, 3) for e, f in zip(per_e, per_f)],
            "all_modes_fused_speedup": round(sum(per_e) / sum(per_f), 3)}
        if tag != "512cube_r32":
            del X
        del U, o
        torch.cuda.empty_cache()


def sec_paper(torch, _abi, inputs, X2, dims2, U2, stream, out, rooflines):
    """Tensors shaped like the paper's workloads: equal-sided ~7.5e8-entry
    tensors at rank 25 (rank-25 model + 1% noise) and the fMRI shapes
    (entries uniform on [-1, 1), like correlations) at ranks 10, 20 and 30; every
    mode's time against its HBM roofline."""
    dev = X2.device
    rec = {}
    shapes = [("900^3", (900, 900, 900), (25,)), ("165^4", (165,) * 4, (25,)), ("60^5", (60,) * 5, (25,)),
              ("30^6", (30,) * 6, (25,)), ("fmri4d_225x59x200x200", (225, 59, 200, 200), (10, 20, 30)),
              ("fmri3d_225x59x19900", (225, 59, 19900), (10, 20, 30))]
    for tag, dims, ranks in shapes:
        if tag.startswith("fmri"):
            X = inputs.uniform_tensor(dims, seed=12, device="cuda", low=-1.0, high=1.0)
        else:
            X, _ = inputs.noisy_low_rank(dims, 25, seed_factors=13, seed_noise=14, eta=0.01, device="cuda")
        for R in ranks:
            U = inputs.normal_factors(dims, R, seed=15, device="cuda")
            o = [torch.empty((d, R), device=dev) for d in dims]
            ws = torch.empty(max(1, max(_abi.mttkrp_workspace_bytes(dims, R, n, _abi.CPM_F32)
                                        for n in range(len(dims)))), dtype=torch.uint8, device=dev)
            per = [timed(torch, stream, lambda: _abi.mttkrp(X, dims, U, n, out=o[n], workspace=ws), 5)
                   for n in range(len(dims))]
            rec["%s_r%d" % (tag, R)] = {
                "per_mode_us": [round(t * 1e3, 1) for t in per],
                "per_mode_hbm_frac": [round(algo_bytes(dims, R, n, 4) / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                      for n, t in enumerate(per)],
                "kernels": [_abi.describe(dims, R, n, _abi.CPM_F32, X).split(" ")[0] for n in range(len(dims))]}
            del U, o, ws
        del X
        torch.cuda.empty_cache()
    out["paper_shapes_fp32"] = rec


SECTIONS = {"als": sec_als, "residual": sec_residual, "sym4d": sec_sym4d, "sympair": sec_sympair,
            "grad": sec_grad, "explicit": sec_explicit, "paper": sec_paper}


if __name__ == "__main__":
    main()
