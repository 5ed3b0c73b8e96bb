#!/usr/bin/env python3
"""Throughput of the dimension-lifted FFT on one MI355X.

Workload: complex64 1-D transforms of n = 2^24 lifted to 4096 x 4096, inputs
iid standard normal (seeded), forward (sign -1) and inverse (sign +1).  The
same steps are also timed through the three-level lift 256 x 256 x 256 (the
library's default at this size), reported under "three_level".
One step = one forward transform of one buffer set plus one inverse transform
of the next buffer set, so every stage of the path (both passes, the
inter-pass weights, the redistribution and the natural-order store) runs in
both directions.  Buffer sets are rotated so that no transform reads an input
that is still resident in the 256 MB last-level cache from an earlier step.

Prints one JSON line (rank 0).  GFLOP/s uses the conventional 5 n log2 n flops
per transform; HBM GB/s uses the method's algorithmic traffic (each pass
reads and writes n elements: 32 n bytes per complex64 transform).

    python bench.py [--steps K] [--warmup W] [--log2n 24] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("GFLOP/s (5n·log2n) + HBM GB/s % peak, c64 n=2^24; fwd+bwd and batched "
          "vs plain")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c64_n2p24.txt")


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and blank lines removed, so
    that counter values stay attached to the code they were taken on (and
    only to it)."""
    import re
    h = hashlib.sha256()
    for f in ("liftfft.hip", "fft_engine.hpp"):
        with open(os.path.join(ROOT, "paper_0811_2535_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(text.encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, launches_bytes: float):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def _kernel_role(name: str) -> str | None:
    if "pass_kernel<float, 4096, 16, 1," in name:
        return "pass1"
    if "pass_kernel<float, 4096, 16, 2," in name:
        return "pass2"
    if "pass_kernel<float, 256, 16, 3," in name:
        return "axis"
    if "neg" in name:
        return "reference"
    return None


def summarize_counters(fetch_csv: str, write_csv: str, log2n: int, out_path: str) -> dict:
    """HBM traffic per launch of each pass from two rocprofv3 --pmc runs of this
    benchmark (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by
    what the same counter reads for the reference streaming kernel, which reads
    8n and writes 8n bytes."""
    import csv
    import statistics

    def per_role(path, counter):
        vals = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                role = _kernel_role(row["Kernel_Name"])
                if role:
                    vals.setdefault(role, []).append(float(row["Counter_Value"]) * 1024.0)
        return {k: statistics.mean(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}

    n = 1 << log2n
    known = 8.0 * n
    fetch, nf = per_role(fetch_csv, "FETCH_SIZE")
    write, nw = per_role(write_csv, "WRITE_SIZE")
    f_fac, w_fac = known / fetch["reference"], known / write["reference"]
    bargs = "--steps 2 --warmup 1 --sets 4 --copy-reps 3 --no-cpu-baseline --no-extras"
    rec = {"source_hash": kernel_source_hash(), "log2n": log2n,
           "commands": [
               "timeout -s KILL 60 rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch "
               "-o run -- python3 bench.py " + bargs,
               "timeout -s KILL 60 rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write "
               "-o run -- python3 bench.py " + bargs,
               "python3 bench.py --summarize-counters gpurun_out/pmc_fetch/run_counter_collection.csv "
               "gpurun_out/pmc_write/run_counter_collection.csv"],
           "reference": {"fetch_counter_bytes": fetch["reference"], "write_counter_bytes": write["reference"],
                         "fetch_scale": f_fac, "write_scale": w_fac, "bytes_each_way": known},
           "kernels": {}}
    for role in ("pass1", "pass2", "axis"):
        if role not in fetch or role not in write:
            continue
        fb, wb = fetch[role] * f_fac, write[role] * w_fac
        rec["kernels"][role] = {"fetch_bytes": fb, "write_bytes": wb, "hbm_bytes_per_launch": fb + wb,
                                "ratio_to_algorithmic": (fb + wb) / (2 * known),
                                "dispatches": [nf.get(role, 0), nw.get(role, 0)]}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def cpu_baseline(x0, x1, y0_gpu, y1_gpu):
    """The FP64 oracle (untuned, one thread) on one forward and one inverse
    transform of the benchmark's own inputs; also returns the parity of the
    GPU outputs of those two transforms."""
    import numpy as np

    import oracle
    n = x0.size
    t0 = time.perf_counter()
    r0 = oracle.fft(x0.astype(np.complex128), -1)
    r1 = oracle.fft(x1.astype(np.complex128), 1)
    dt = time.perf_counter() - t0
    flops = 2 * 5.0 * n * math.log2(n)
    base = {"value": round(flops / dt / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "one forward + one inverse c64 n=2^%d transform (FP64 recursive radix-2, "
                      "1 thread), %.2f s" % (int(math.log2(n)), dt),
            "seconds": round(dt, 3)}
    parity = {"rel_l2_forward": oracle.rel_l2(y0_gpu, r0), "rel_l2_inverse": oracle.rel_l2(y1_gpu, r1),
              "tolerance": 1e-6}
    return base, parity


def measure_fwd_bwd(torch, lf, datagen, reps: int = 5) -> dict:
    """Differentiation form on batch 8 x n = 2^22 complex64 (N(0,1) inputs,
    weights U[0,1], seed 5): loss = sum w |F x|^2 through the autograd
    Function, whose backward is the adjoint (sign +1) transform.  Reports the
    whole forward+backward step, the two transforms inside it (plan timing),
    and the same two transforms run as plain executes."""
    import numpy as np
    n, batch = 1 << 22, 8
    dev = torch.device("cuda:0")
    x = torch.from_numpy(datagen.signals(n, batch, np.complex64, "normal", 5)).to(dev).requires_grad_()
    w = torch.from_numpy(datagen.real_weights(n, batch, 5).astype(np.float32)).to(dev)
    plan = lf.cached_plan(n, batch, torch.complex64, dev)

    def step():
        y = lf.LiftFFT.apply(x, -1)
        loss = (w * (y.real * y.real + y.imag * y.imag)).sum()
        loss.backward()
        x.grad = None

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.read_timing(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / reps
    kms, kcnt = plan.read_timing(reset=True)
    fft_ms_ad = (kms[0] + kms[1]) / reps  # two transforms per step
    y = torch.empty_like(x.detach())
    g = torch.empty_like(y)
    xd = x.detach()
    for _ in range(reps):
        plan.execute(xd, y, -1)
        plan.execute(y, g, 1)
    kms, kcnt = plan.read_timing(reset=True)
    plan.set_timing(False)
    fft_ms_plain = (kms[0] + kms[1]) / reps
    flops = 2 * 5.0 * n * math.log2(n) * batch
    return {"workload": "c64 batch 8 x n=2^22, loss sum w|Fx|^2, forward + adjoint backward",
            "ms_step_total": round(ms_step, 4),
            "ms_two_ffts_in_autograd": round(fft_ms_ad, 4),
            "ms_two_plain_executes": round(fft_ms_plain, 4),
            "ratio_vs_plain": round(fft_ms_ad / fft_ms_plain, 4),
            "gflops_ffts": round(flops / (fft_ms_ad * 1e-3) / 1e9, 1),
            "hbm_gbps_ffts": round(2 * 32 * n * batch / (fft_ms_ad * 1e-3) / 1e9, 1)}


def measure_ragged(torch, lf, datagen, reps: int = 10) -> dict:
    """Batched uneven lengths: 4096 complex64 transforms with k ~ U{8..16}
    (seed 3), U[-1,1], packed back to back; the plan (direct launches, and
    replayed as a captured graph) against
    (a) one single-length batched plan per length class (each class gathered
    into its own contiguous buffer beforehand, not timed) and (b) one plain
    launch per transform."""
    import numpy as np
    ks = datagen.uneven_log2_lengths(4096, 8, 16, seed=3)
    lengths = [1 << int(k) for k in ks]
    total = sum(lengths)
    dev = torch.device("cuda:0")
    x_np = datagen.ragged_signals(lengths, np.complex64, "uniform", 3)
    sets = 3  # rotated so that no input is still in the last-level cache
    xs = [torch.from_numpy(x_np).to(dev) for _ in range(sets)]
    ys = [torch.empty_like(xs[0]) for _ in range(sets)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_mode = {}
    for graph in (False, True):
        plan = lf.Plan.uneven(lengths, torch.complex64, graph=graph)
        for i in range(sets):
            plan.execute(xs[i], ys[i], -1)
        torch.cuda.synchronize()
        e0.record()
        for i in range(reps):
            plan.execute(xs[i % sets], ys[i % sets], -1)
        e1.record()
        torch.cuda.synchronize()
        ms_mode[graph] = e0.elapsed_time(e1) / reps
        info = plan.info()
        plan.destroy()
    ms_direct, ms_graph = ms_mode[False], ms_mode[True]

    # (a) per-class batched plans on contiguous class buffers.
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    classes = {}
    for i, ln in enumerate(lengths):
        classes.setdefault(ln, []).append(i)
    cls_bufs = []
    for ln, idx in sorted(classes.items(), reverse=True):
        block = np.stack([x_np[offs[i]:offs[i] + ln] for i in idx])
        xb = [torch.from_numpy(block).to(dev) for _ in range(sets)]
        yb = [torch.empty_like(xb[0]) for _ in range(sets)]
        cls_bufs.append((lf.Plan(ln, len(idx), torch.complex64), xb, yb))
    for pl, xb, yb in cls_bufs:
        pl.execute(xb[0], yb[0], -1)
    torch.cuda.synchronize()
    e0.record()
    for i in range(reps):
        for pl, xb, yb in cls_bufs:
            pl.execute(xb[i % sets], yb[i % sets], -1)
    e1.record()
    torch.cuda.synchronize()
    ms_classes = e0.elapsed_time(e1) / reps
    for pl, _, _ in cls_bufs:
        pl.destroy()
    del cls_bufs

    # (b) one launch per transform (views into the packed buffers).
    plans = {ln: lf.Plan(ln, 1, torch.complex64) for ln in classes}
    views = [(plans[ln], int(o), ln) for o, ln in zip(offs, lengths)]
    torch.cuda.synchronize()
    e0.record()
    for pl, o, ln in views:
        pl.execute(xs[0][o:o + ln], ys[0][o:o + ln], -1)
    e1.record()
    torch.cuda.synchronize()
    ms_each = e0.elapsed_time(e1)
    for pl in plans.values():
        pl.destroy()
    flops = sum(5.0 * ln * math.log2(ln) for ln in lengths)
    alg_bytes = sum((16 if ln <= 16384 else 32) * ln for ln in lengths)  # one pass up to 2^14
    return {"workload": "4096 c64 transforms, n = 2^k with k ~ U{8..16} (seed 3), packed, forward",
            "elements": total, "length_classes": info["length_classes"],
            "ms": round(ms_direct, 4), "ms_graph_replay": round(ms_graph, 4),
            "gflops": round(flops / (ms_direct * 1e-3) / 1e9, 1),
            "hbm_gbps_algorithmic": round(alg_bytes / (ms_direct * 1e-3) / 1e9, 1),
            "ms_per_class_batched_plans": round(ms_classes, 4),
            "ms_one_launch_per_transform": round(ms_each, 4),
            "speedup_vs_per_class": round(ms_classes / ms_direct, 3),
            "speedup_vs_per_transform": round(ms_each / ms_direct, 3),
            "grid": [info["grid_pass1"], info["grid_pass2"]]}


def measure_precision(torch, lf, datagen, reps: int = 5):
    """Precision forms on 256 transforms of 2^20 complex64 (N(0,1), seed 4),
    lifted 4096 x 256 so every stage is radix 16: FP32 stages on the vector
    units against radix-16 stages on the matrix cores with FP16 / BF16 pairs.
    Reports each form's relative L2 difference from the FP32 path on all
    transforms; returns also transform 0's input and outputs, whose error
    against the FP64 oracle the CPU-baseline leg adds."""
    import numpy as np

    n, batch = 1 << 20, 256
    dev = torch.device("cuda:0")
    x_np = datagen.signals(n, batch, np.complex64, "normal", 4)
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    y32 = None
    firsts = {}
    plan = lf.Plan(n, batch, torch.complex64, log2_p=8)
    out = {"workload": "256 x 2^20 c64 forward, lift 4096 x 256 (all stages radix 16)"}
    flops = 5.0 * n * math.log2(n) * batch
    for mode in ("fp32", "f16x2", "bf16x2"):
        plan.set_precision(mode)
        plan.execute(x, y, -1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.execute(x, y, -1)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if y32 is None:
            y32 = y.clone()
        diff = float(torch.linalg.vector_norm((y - y32).to(torch.complex128)) /
                     torch.linalg.vector_norm(y32.to(torch.complex128)))
        firsts[mode] = y[0].cpu().numpy()
        out[mode] = {"ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                     "hbm_gbps_algorithmic": round(32 * n * batch / (ms * 1e-3) / 1e9, 1),
                     "rel_l2_vs_fp32_path": float("%.3g" % diff)}
    plan.destroy()
    del y32
    return out, (x_np[0], firsts)


def precision_oracle_errors(x0, firsts):
    """CPU-baseline leg: relative L2 of each precision form's transform 0
    against the FP64 oracle."""
    import numpy as np

    import oracle
    ref = oracle.fft(x0.astype(np.complex128), -1)
    return {mode: float("%.3g" % oracle.rel_l2(y, ref)) for mode, y in firsts.items()}


def measure_three_level(torch, lf, xs, S, steps, warmup, stream, n):
    """One forward + one inverse per step over the rotating sets, as for the
    headline, through the three-level lift; per-pass kernel averages from the
    plan's HIP events.  At 2^24 all three passes launch the same kernel
    (256-point lines, 16 per workgroup), so its average over the three passes
    is what a kernel trace reports for it."""
    plan = lf.Plan(n, 1, torch.complex64, flags=lf.binding.FFT_OPT_THREE_LEVEL)
    info = plan.info()
    ys = [torch.empty_like(x) for x in xs]  # outputs of its own

    def step(i):
        a, b = (2 * i) % S, (2 * i + 1) % S
        plan.execute(xs[a], ys[a], -1, stream)
        plan.execute(xs[b], ys[b], 1, stream)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.read_timing(reset=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(steps):
        step(warmup + i)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    kms, kcnt = plan.read_timing(reset=True)
    plan.set_timing(False)
    # forward of set 0 again, for agreement with the headline plan's output
    y3 = torch.empty_like(xs[0])
    plan.execute(xs[0], y3, -1, stream)
    torch.cuda.synchronize()
    plan.destroy()
    del ys
    esize = 8
    avg = [kms[k] / kcnt[k] for k in range(3)]
    mean_avg = sum(avg) / 3
    bytes_per_launch = 2 * n * esize
    achieved = bytes_per_launch / (mean_avg * 1e-3) / 1e9
    flops_step = 2 * 5.0 * n * math.log2(n)
    l1, l2, l3 = info["log2_n1"], info["log2_n2"], info["log2_n3"]
    return {
        "workload": "same steps and buffers, lifted %dx%dx%d (three axis passes)" % (1 << l3, 1 << l2, 1 << l1),
        "value": round(flops_step / (ms_step * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "ms_per_step": round(ms_step, 5),
        "lines_per_block": [info["lines_per_block_pass1"], info["lines_per_block_pass2"],
                            info["lines_per_block_pass3"]],
        "alg_bytes_per_step": 2 * 3 * bytes_per_launch,
        "roofline": {
            "bound": "hbm",
            "kernel": "axis",
            "kernels_avg_us": {"passA": round(avg[0] * 1e3, 2), "passB": round(avg[1] * 1e3, 2),
                               "passC": round(avg[2] * 1e3, 2)},
            "kernel_avg_us": round(mean_avg * 1e3, 2),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": load_traffic("axis", bytes_per_launch),
            "alg_bytes_per_launch": bytes_per_launch,
        },
        "_y_forward_set0": y3,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--sets", type=int, default=4, help="buffer sets rotated between transforms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the differentiation-form, uneven-batch, precision-form and "
                         "autotuner measurements")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this benchmark and exit")
    ap.add_argument("--copy-reps", type=int, default=10,
                    help="device-to-device copies of one pass's bytes, timed for context and "
                         "used as the known-size reference kernel for HBM counters")
    args = ap.parse_args()

    if args.summarize_counters:
        rec = summarize_counters(args.summarize_counters[0], args.summarize_counters[1], args.log2n,
                                 TRAFFIC_FILE)
        print(json.dumps(rec))
        return 0

    if args.gpus != 1:
        print("bench.py: measures one GPU only; --gpus %d is not supported "
              "(transforms shard across GPUs without exchange for batches, and with one "
              "all-to-all for a single large transform; neither is built here)" % args.gpus,
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import datagen
    import paper_0811_2535_amd as lf

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    lf.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 1 << args.log2n
    S = max(2, args.sets)

    print("[bench] generating %d input sets of n=2^%d c64" % (S, args.log2n), file=sys.stderr,
          flush=True)
    host_inputs = [datagen.signals(n, 1, np.complex64, "normal", 2 + 1000 * s)[0]
                   for s in range(S)]
    xs = [torch.from_numpy(h).to(dev) for h in host_inputs]
    ys = [torch.empty_like(x) for x in xs]
    # The configuration the headline is quoted on: the 4096 x 4096 two-level
    # lift (the library's own default at this size is the three-level lift,
    # measured separately below).
    plan = lf.Plan(n, 1, torch.complex64, flags=lf.binding.FFT_OPT_TWO_LEVEL)
    info = plan.info()
    stream = torch.cuda.current_stream(dev)

    def step(i):
        a, b = (2 * i) % S, (2 * i + 1) % S
        plan.execute(xs[a], ys[a], -1, stream)
        plan.execute(xs[b], ys[b], 1, stream)

    print("[bench] warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    print("[bench] timing %d steps" % args.steps, file=sys.stderr, flush=True)
    plan.set_timing(True)
    plan.read_timing(reset=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = ev0.elapsed_time(ev1)
    kms, kcnt = plan.read_timing(reset=True)
    plan.set_timing(False)

    ms_step = ms_total / args.steps
    flops_step = 2 * 5.0 * n * math.log2(n)
    esize = 8
    alg_bytes_step = 2 * (32 if info["passes"] == 2 else 16) * n * esize // 8
    gflops = flops_step / (ms_step * 1e-3) / 1e9
    gbs = alg_bytes_step / (ms_step * 1e-3) / 1e9

    # Dominant kernel: the pass with the larger average launch duration.
    names = ["pass1", "pass2"] if info["passes"] == 2 else ["single"]
    avg = [kms[k] / kcnt[k] if kcnt[k] else 0.0 for k in range(len(names))]
    kd = max(range(len(names)), key=lambda k: avg[k])
    bytes_per_launch = 2 * n * esize  # one read + one write of n elements
    achieved = bytes_per_launch / (avg[kd] * 1e-3) / 1e9
    traffic = load_traffic(names[kd], bytes_per_launch)

    # Output parity of the transforms timed (step 0 sets: forward of set 0,
    # inverse of set 1), from the same buffers.
    y0 = ys[0].cpu().numpy()
    y1 = ys[1].cpu().numpy()

    # The same steps through the three-level lift (n = n1 n2 n3, three axis
    # passes of one kernel shape at 2^24).
    three = None
    if args.log2n >= 15:
        print("[bench] three-level lift, %d steps" % args.steps, file=sys.stderr, flush=True)
        three = measure_three_level(torch, lf, xs, S, args.steps, args.warmup, stream, n)

    # Reference: a plain streaming kernel over n complex64 elements (reads 8n,
    # writes 8n bytes, the same algorithmic traffic as one pass), rotated over
    # the sets.  torch.neg is used rather than copy_ so the reference is an
    # ordinary elementwise kernel with a name of its own in profiles.
    copy_gbs = None
    if args.copy_reps > 0:
        dst = [torch.empty_like(x) for x in xs]
        for i in range(2):
            torch.neg(xs[(i + 1) % S], out=dst[i % S])
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        c0.record(stream)
        for i in range(args.copy_reps):
            torch.neg(xs[(i + 1) % S], out=dst[i % S])
        c1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 2 * n * esize * args.copy_reps / (c0.elapsed_time(c1) * 1e-3) / 1e9
        del dst

    if three is not None:
        y3 = three.pop("_y_forward_set0").cpu().numpy()
        three["max_abs_diff_vs_two_level"] = float("%.3g" % (np.abs(y3.astype(np.complex128) - y0).max() /
                                                            np.abs(y0).max()))
        del y3
    result = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "c64 1-D FFT n=2^%d lifted %dx%d, one forward + one inverse per step, "
                        "N(0,1) inputs seeds 2+1000s, %d rotating buffer sets"
                        % (args.log2n, 1 << info["log2_p"], 1 << info["log2_q"], S),
            "n": n, "batch": 1, "passes": info["passes"], "log2_p": info["log2_p"],
            "log2_q": info["log2_q"], "radix": info["radix"],
            "lines_per_block": [info["lines_per_block_pass1"], info["lines_per_block_pass2"]],
            "kernel_variants": [info["variant_pass1"], info["variant_pass2"]],
        },
        "hbm": {
            "alg_bytes_per_step": alg_bytes_step,
            "gbps": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "effective_gbps_16n": round(gbs / 2, 1),
            "copy_gbps_same_gpu": round(copy_gbs, 1) if copy_gbs else None,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": names[kd],
            "kernel_avg_us": round(avg[kd] * 1e3, 2),
            "kernels_avg_us": {names[k]: round(avg[k] * 1e3, 2) for k in range(len(names))},
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": bytes_per_launch,
        },
        "wall_s": round(wall, 4),
        "three_level": three,
    }
    precision_firsts = None
    if not args.no_extras:
        print("[bench] forward + adjoint backward, batch 8 x 2^22", file=sys.stderr, flush=True)
        del xs, ys
        result["fwd_bwd"] = measure_fwd_bwd(torch, lf, datagen)
        lf.clear_plan_cache()
        print("[bench] batched uneven lengths, 4096 transforms", file=sys.stderr, flush=True)
        result["ragged"] = measure_ragged(torch, lf, datagen)
        print("[bench] precision forms, 256 x 2^20", file=sys.stderr, flush=True)
        result["precision"], precision_firsts = measure_precision(torch, lf, datagen)
        print("[bench] autotuner on the headline shape", file=sys.stderr, flush=True)
        tplan, tres = lf.Plan.tuned(n, 1, torch.complex64, max_candidates=48)
        tplan.destroy()
        result["autotune"] = {"workload": "c64 n=2^%d forward, tuner's own timing" % args.log2n,
                              "candidates": tres["candidates"], "rejected": tres["rejected"],
                              "ms_default": round(tres["ms_default"], 4), "ms_tuned": round(tres["ms"], 4),
                              "chosen": tres["opts"]}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (FP64 oracle, 1 thread)", file=sys.stderr, flush=True)
        base, parity = cpu_baseline(host_inputs[0], host_inputs[1], y0, y1)
        result["cpu_baseline"] = base
        result["parity"] = parity
        if precision_firsts is not None:
            errs = precision_oracle_errors(*precision_firsts)
            for mode, e in errs.items():
                result["precision"][mode]["rel_l2_transform0_vs_oracle"] = e
    plan.destroy()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
