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
# The paper's own timing at this length, as context (another algorithm form on
# other hardware, so no ratio is formed): Table 7.1, the sequential
# "monolithic" FFT-UA at n = 2^24 on the SGI/Cray Origin2000 (R10000 at
# 195 MHz), 7.550 s; GFLOP/s derived here as 5 n log2 n / t.
PAPER_CONTEXT = {"source": "Table 7.1, FFT-UA (sequential), n = 2^24",
                 "hardware": "SGI/Cray Origin2000, R10000 195 MHz", "seconds": 7.550,
                 "gflops_derived": round(5.0 * (1 << 24) * 24 / 7.550 / 1e9, 3)}
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


def kernel_label(name: str) -> str:
    """Short description of a kernel in a rocprofv3 trace of this benchmark."""
    import re
    m = re.search(r"pass_kernel<(float|double), (\d+), (\d+), (\d), (\d+), (\w+), (\w+), (\w+), (\d)>", name)
    if m:
        real, N, rmax, kind, emax, split, persist, dense, prec = m.groups()
        kinds = {"0": "single pass", "1": "pass 1", "2": "pass 2", "3": "axis pass", "4": "axis pass (64-bit)"}
        parts = ["%s, %s-point lines" % (kinds[kind], N), "c64" if real == "float" else "c128"]
        if rmax != "16":
            parts.append("radix %s" % rmax)
        if emax != "16":
            parts.append("%s values/thread" % emax)
        if split == "true":
            parts.append("split exchange")
        if persist == "true":
            parts.append("persistent")
        if dense == "true":
            parts.append("64-VGPR cap")
        if prec != "0":
            parts.append({"1": "FP16 pairs on MFMA", "2": "BF16 pairs on MFMA"}[prec])
        return ", ".join(parts)
    for key, label in (("axis_shuffle_kernel", "axis pass, 256-point lines, shuffle exchange"),
                       ("pass1_rows_kernel<8>", "pass 1, 4096-point lines, c64, rows per thread, radix 8"),
                       ("pass1_rows_kernel<16>", "pass 1, 4096-point lines, c64, rows per thread, radix 16"),
                       ("pass1_dma_kernel", "pass 1, 4096-point lines, c64, staged in LDS by direct loads"),
                       ("ragged_kernel", "uneven batch, persistent lifted passes"),
                       ("block_phase", "paper's plan, block phase"), ("cyclic_phase", "paper's plan, cyclic phase"),
                       ("twiddle_table_kernel", "FP64 weight tables"), ("dft_operand_table", "MFMA operand table"),
                       ("neg_kernel", "streaming reference (torch.neg)"), ("copyBuffer", "host/device copies"),
                       ("fill_pattern", "tuner input"), ("compare_kernel", "tuner check")):
        if key in name:
            return label
    return name[:60]


def summarize_trace(stats_csv: str) -> str:
    """Markdown table of a rocprofv3 --stats kernel summary of this benchmark:
    calls, average and min/max duration per kernel, largest total first."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | min us | max us | total % |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append("| %s | %s | %.1f | %.1f | %.1f | %.2f |" % (
            kernel_label(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def host_facts() -> dict:
    """CPU model and core counts of the host the oracle legs run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "affinity": affinity}


def oracle_threads() -> int:
    """Threads for the batched oracle legs: this process's CPU share
    (OMP_NUM_THREADS when set, else the affinity mask), at most 16."""
    try:
        t = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        t = 0
    return max(1, min(16, t or host_facts()["affinity"]))


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
    base.update(host_facts())
    parity = {"rel_l2_forward": oracle.rel_l2(y0_gpu, r0), "rel_l2_inverse": oracle.rel_l2(y1_gpu, r1),
              "tolerance": 1e-6}
    return base, parity


def measure_config1(torch, lf, datagen, reps: int = 100):
    """Config 1: one n = 2^10 complex128 transform (U[-1,1], seed 1, sign -1)
    lifted 32 x 32 with radix-2 stages in both passes; latency-bound, so
    microseconds per transform over back-to-back executes."""
    import numpy as np
    x_np = datagen.signals(1024, 1, np.complex128, "uniform", 1)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    plan = lf.Plan(1024, 1, torch.complex128, log2_p=5, radix=2)
    for _ in range(5):
        plan.execute(x, y, -1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.execute(x, y, -1)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    plan.destroy()
    keep = (x_np[0], y.cpu().numpy()[0])
    # The same transform 4096 times in one batched execute: the device's rate
    # for this shape, without the per-call host work that bounds the above.
    nb = 4096
    xb = x.repeat(nb, 1)
    yb = torch.empty_like(xb)
    plan = lf.Plan(1024, nb, torch.complex128, log2_p=5, radix=2)
    for _ in range(3):
        plan.execute(xb, yb, -1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        plan.execute(xb, yb, -1)
    e1.record()
    torch.cuda.synchronize()
    us_b = e0.elapsed_time(e1) / 10 * 1e3 / nb
    same = bool(torch.equal(yb[nb - 1], y[0]))
    plan.destroy()
    out = {"workload": "c128 n=2^10, U[-1,1] seed 1, forward, lift 32 x 32, radix-2 stages",
           "us_per_transform": round(us, 2), "gflops": round(5.0 * 1024 * 10 / (us * 1e-6) / 1e9, 3),
           "us_per_transform_note": "one execute at a time from Python: bound by the host call and two launches",
           "us_per_transform_batched_4096": round(us_b, 4),
           "gflops_batched_4096": round(5.0 * 1024 * 10 / (us_b * 1e-6) / 1e9, 1),
           "batched_equals_single": same}
    return out, keep


def oracle_leg_config1(keep, reps: int = 200) -> dict:
    import numpy as np

    import oracle
    x0, y0 = keep
    xb = x0.astype(np.complex128)
    t0 = time.perf_counter()
    for _ in range(reps):
        ref = oracle.fft(xb, -1)
    dt = (time.perf_counter() - t0) / reps
    return {"sample": "the config-1 transform, %d repetitions" % reps, "threads": 1,
            "us_per_transform": round(dt * 1e6, 2), "rel_l2_gpu_vs_oracle": float("%.3g" % oracle.rel_l2(y0, ref)),
            "tolerance": 1e-12}


def oracle_leg_config3(keep, threads: int) -> dict:
    """All 4096 transforms of config 3 through the oracle, one batched call
    per length class on `threads` threads; the packed GPU output's largest
    per-transform relative L2 and the global one."""
    import numpy as np

    import oracle
    x_np, y_np, lengths = keep
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    classes = {}
    for i, ln in enumerate(lengths):
        classes.setdefault(ln, []).append(i)
    worst, num, den, secs = 0.0, 0.0, 0.0, 0.0
    for ln, idx in classes.items():
        X = np.stack([x_np[offs[i]:offs[i] + ln] for i in idx]).astype(np.complex128)
        t0 = time.perf_counter()
        R = oracle.fft_batch(X, -1, threads=threads)
        secs += time.perf_counter() - t0
        for r, i in zip(R, idx):
            g = y_np[offs[i]:offs[i] + ln].astype(np.complex128)
            d = float(np.sum(np.abs(g - r) ** 2))
            e = float(np.sum(np.abs(r) ** 2))
            worst = max(worst, math.sqrt(d / e))
            num += d
            den += e
    flops = sum(5.0 * ln * math.log2(ln) for ln in lengths)
    return {"sample": "all 4096 transforms", "threads": threads, "seconds": round(secs, 3),
            "gflops": round(flops / secs / 1e9, 3), "max_rel_l2": float("%.3g" % worst),
            "global_rel_l2": float("%.3g" % math.sqrt(num / den)), "tolerance": 1e-6}


def oracle_leg_config5(keep, threads: int, coords: int = 64, h: float = 1e-3) -> dict:
    """Config 5 in FP64 on the host: the reference gradient 2 F^H(w . F x) of
    L = sum w |F x|^2 through the oracle (`threads` threads), against the GPU
    autograd gradient; and central differences with step h at `coords`
    seeded coordinates, each from two full evaluations of L (L is quadratic,
    so the central difference has no truncation error)."""
    import numpy as np

    import oracle
    x, w, g_gpu = keep
    batch, n = x.shape
    xb = x.astype(np.complex128)
    t0 = time.perf_counter()
    y = oracle.fft_batch(xb, -1, threads=threads)
    gref = 2.0 * oracle.fft_batch(w * y, 1, threads=threads)
    secs = time.perf_counter() - t0
    grad_err = max(oracle.rel_l2(g_gpu[b], gref[b]) for b in range(batch))
    rng = np.random.default_rng(np.random.SeedSequence([5, 0xFD]))
    picks = [(int(rng.integers(batch)), int(rng.integers(n))) for _ in range(coords)]
    k = np.arange(n, dtype=np.int64)
    fd_err_gpu, fd_err_ref = 0.0, 0.0
    scale = float(np.abs(gref).max())
    t1 = time.perf_counter()
    for b, j in picks:
        c = np.exp(-2j * np.pi * ((j * k) % n) / n)  # column j of F (sign -1)
        def loss(delta):
            return float(np.sum(w[b] * np.abs(y[b] + delta * c) ** 2))
        d_re = (loss(h) - loss(-h)) / (2 * h)
        d_im = (loss(1j * h) - loss(-1j * h)) / (2 * h)
        fd = d_re + 1j * d_im  # conjugate Wirtinger gradient, PyTorch's convention
        fd_err_gpu = max(fd_err_gpu, abs(fd - complex(g_gpu[b, j])) / scale)
        fd_err_ref = max(fd_err_ref, abs(fd - gref[b, j]) / scale)
    fd_secs = time.perf_counter() - t1
    flops = 2 * 5.0 * n * math.log2(n) * batch
    return {"sample": "all 8 signals; %d coordinates for central differences" % coords, "threads": threads,
            "seconds_reference_gradient": round(secs, 3), "gflops": round(flops / secs / 1e9, 3),
            "seconds_central_differences": round(fd_secs, 3),
            "grad_rel_l2_gpu_vs_oracle": float("%.3g" % grad_err),
            "fd_max_err_gpu": float("%.3g" % fd_err_gpu), "fd_max_err_oracle": float("%.3g" % fd_err_ref),
            "fd_err_unit": "largest |difference| over the coordinates / largest |reference gradient|"}


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
    # one more step, keeping its gradient for the oracle leg
    y = lf.LiftFFT.apply(x, -1)
    (w * (y.real * y.real + y.imag * y.imag)).sum().backward()
    torch.cuda.synchronize()
    keep = (x.detach().cpu().numpy(), w.cpu().numpy().astype(np.float64), x.grad.cpu().numpy())
    x.grad = None
    return {"workload": "c64 batch 8 x n=2^22, loss sum w|Fx|^2, forward + adjoint backward",
            "ms_step_total": round(ms_step, 4),
            "ms_two_ffts_in_autograd": round(fft_ms_ad, 4),
            "ms_two_plain_executes": round(fft_ms_plain, 4),
            "ratio_vs_plain": round(fft_ms_ad / fft_ms_plain, 4),
            "gflops_ffts": round(flops / (fft_ms_ad * 1e-3) / 1e9, 1),
            "hbm_gbps_ffts": round(2 * 32 * n * batch / (fft_ms_ad * 1e-3) / 1e9, 1)}, keep


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
    # class plans on forked streams (the default), the persistent-launch
    # form, each launched directly and replayed as a captured graph, and the
    # class form with every class autotuned
    forms = {}
    for key, kw in ((("classes", False), {}), (("classes", True), {"graph": True}),
                    (("persistent", False), {"persistent": True}),
                    (("persistent", True), {"persistent": True, "graph": True}),
                    (("tuned", False), {"autotune": True})):
        forms[key] = lf.Plan.uneven(lengths, torch.complex64, **kw)
    info = forms[("classes", False)].info()

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

    def run_form(key, i):
        if key == "per_class":
            for pl, xb, yb in cls_bufs:
                pl.execute(xb[i % sets], yb[i % sets], -1)
        else:
            forms[key].execute(xs[i % sets], ys[i % sets], -1)

    # Every form warmed up, then timed in turn over three rounds (median).
    keys = list(forms) + ["per_class"]
    for key in keys:
        for i in range(sets):
            run_form(key, i)
    torch.cuda.synchronize()
    times = {k: [] for k in keys}
    for _ in range(3):
        for key in keys:
            e0.record()
            for i in range(reps):
                run_form(key, i)
            e1.record()
            torch.cuda.synchronize()
            times[key].append(e0.elapsed_time(e1) / reps)
    ms_mode = {k: sorted(v)[len(v) // 2] for k, v in times.items()}
    for plan in forms.values():
        plan.destroy()
    for pl, _, _ in cls_bufs:
        pl.destroy()
    del cls_bufs
    ms_direct, ms_graph, ms_classes = ms_mode[("classes", False)], ms_mode[("classes", True)], ms_mode["per_class"]
    plan = lf.Plan.uneven(lengths, torch.complex64)
    plan.execute(xs[0], ys[0], -1)
    torch.cuda.synchronize()
    plan.destroy()
    keep = (x_np, ys[0].cpu().numpy(), lengths)

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
            "elements": total, "length_classes": info["length_classes"], "streams": info["streams"],
            "ms": round(ms_direct, 4), "ms_graph_replay": round(ms_graph, 4),
            "ms_persistent_form": round(ms_mode[("persistent", False)], 4),
            "ms_persistent_form_graph_replay": round(ms_mode[("persistent", True)], 4),
            "ms_autotuned_classes": round(ms_mode[("tuned", False)], 4),
            "gflops": round(flops / (ms_direct * 1e-3) / 1e9, 1),
            "hbm_gbps_algorithmic": round(alg_bytes / (ms_direct * 1e-3) / 1e9, 1),
            "ms_per_class_batched_plans": round(ms_classes, 4),
            "ms_one_launch_per_transform": round(ms_each, 4),
            "speedup_vs_per_class": round(ms_classes / ms_direct, 3),
            "speedup_vs_per_transform": round(ms_each / ms_direct, 3)}, keep


def measure_precision(torch, lf, datagen, reps: int = 5, rounds: int = 3):
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
    modes = ("fp32", "f16x2", "bf16x2")
    # Steady state for every form: each is warmed up, then the forms are timed
    # in turn over `rounds` rounds and each keeps its median round (the first
    # executes after the buffers are allocated run measurably slower, which a
    # single round would charge to whichever form comes first).
    for mode in modes:
        plan.set_precision(mode)
        for _ in range(3):
            plan.execute(x, y, -1)
    torch.cuda.synchronize()
    times = {m: [] for m in modes}
    for _ in range(rounds):
        for mode in modes:
            plan.set_precision(mode)
            plan.execute(x, y, -1)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                plan.execute(x, y, -1)
            e1.record()
            torch.cuda.synchronize()
            times[mode].append(e0.elapsed_time(e1) / reps)
    for mode in modes:
        plan.set_precision(mode)
        plan.execute(x, y, -1)
        torch.cuda.synchronize()
        ms = sorted(times[mode])[len(times[mode]) // 2]
        if y32 is None:
            y32 = y.clone()
        diff = float(torch.linalg.vector_norm((y - y32).to(torch.complex128)) /
                     torch.linalg.vector_norm(y32.to(torch.complex128)))
        firsts[mode] = y[:PRECISION_SUBSET].cpu().numpy()
        out[mode] = {"ms": round(ms, 4), "ms_rounds": [round(v, 4) for v in times[mode]],
                     "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                     "hbm_gbps_algorithmic": round(32 * n * batch / (ms * 1e-3) / 1e9, 1),
                     "rel_l2_vs_fp32_path": float("%.3g" % diff)}
    plan.destroy()
    del y32
    return out, (x_np[:PRECISION_SUBSET], firsts)


PRECISION_SUBSET = 16  # transforms of config 4 checked against the oracle


def precision_oracle_errors(x_sub, firsts, threads):
    """CPU leg of config 4: the oracle on the first PRECISION_SUBSET
    transforms (nproc threads); each precision form's largest relative L2
    over them."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    ref = oracle.fft_batch(x_sub.astype(np.complex128), -1, threads=threads)
    dt = time.perf_counter() - t0
    n = x_sub.shape[1]
    errs = {mode: float("%.3g" % max(oracle.rel_l2(y[b], ref[b]) for b in range(len(ref))))
            for mode, y in firsts.items()}
    flops = 5.0 * n * math.log2(n) * len(ref)
    leg = {"sample": "%d of the 256 transforms of 2^20 (the first, seed 4)" % len(ref), "threads": threads,
           "seconds": round(dt, 3), "gflops": round(flops / dt / 1e9, 3),
           "max_rel_l2_vs_oracle": errs}
    return errs, leg


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
        "tile_order": "%#08x" % info["tile_order"],
        "alg_bytes_per_step": 2 * 3 * bytes_per_launch,
        # the transform against the two-pass method's 32 n bytes (the
        # roofline below counts each of the three passes' own 16 n bytes)
        "per_transform": {"us": round(ms_step / 2 * 1e3, 2),
                          "gbps_on_32n_bytes": round(4 * n * esize / (ms_step / 2 * 1e-3) / 1e9, 1),
                          "frac_of_peak_on_32n_bytes": round(4 * n * esize / (ms_step / 2 * 1e-3) / 1e9
                                                             / HBM_PEAK_GBS, 4)},
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


def run_sweep(torch, lf, log2n: int, sets: int = 4, reps: int = 12) -> int:
    """Per-pass kernel times of the plan configurations at one length (c64,
    N(0,1) inputs over rotating buffer sets, forward and inverse alternating,
    per-kernel HIP events), with streaming references over the same bytes:
    the numbers behind the tile-width, kernel-variant and lift comparisons.
    One JSON object per line."""
    from paper_0811_2535_amd import binding as B
    n = 1 << log2n
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(2)
    xs = [torch.randn(n, dtype=torch.complex64, device=dev, generator=gen) for _ in range(sets)]
    ys = [torch.empty_like(x) for x in xs]
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timeit(fn):
        for i in range(3):
            fn(i)
        torch.cuda.synchronize()
        e0.record(st)
        for i in range(reps):
            fn(i)
        e1.record(st)
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) / reps * 1e3, 1)

    def emit(rec):
        print(json.dumps(rec), flush=True)

    emit({"reference": "torch.neg, rotating buffers (8n bytes read + 8n written)",
          "us": timeit(lambda i: torch.neg(xs[(i + 1) % sets], out=ys[i % sets]))})
    emit({"reference": "torch copy_, rotating buffers", "us": timeit(lambda i: ys[i % sets].copy_(xs[(i + 1) % sets]))})
    emit({"reference": "torch.neg, same buffers every time (last-level cache warm)",
          "us": timeit(lambda i: torch.neg(xs[0], out=ys[0]))})
    tmp = torch.empty_like(xs[0])

    def chain(i):
        torch.neg(xs[(i + 1) % sets], out=ys[i % sets])
        torch.neg(ys[i % sets], out=tmp)
    emit({"reference": "two torch.neg in a chain, the second reading what the first wrote", "us": timeit(chain)})
    if log2n % 2 == 0:
        # Each pass's permutation of the elements without its arithmetic, as
        # torch copies (the kernel torch picks traverses the output in order).
        P = Q = 1 << (log2n // 2)
        emit({"reference": "pass 1's element movement x[j1 + p k2] -> S[j1/2][k2][j1%%2] (16-byte pairs "
                           "transposed, p = q = %d), torch copy_" % P,
              "us": timeit(lambda i: ys[i % sets].view(P // 2, Q, 2).copy_(
                  xs[(i + 1) % sets].view(Q, P // 2, 2).transpose(0, 1)))})
        emit({"reference": "pass 2's element movement S[k1/2][k2][k1%2] -> X[k2 + q k1], torch copy_",
              "us": timeit(lambda i: ys[i % sets].view(P // 2, 2, Q).copy_(
                  xs[(i + 1) % sets].view(P // 2, Q, 2).permute(0, 2, 1)))})

    def plan_times(label, **kw):
        try:
            p = lf.Plan(n, 1, torch.complex64, **kw)
        except B.FFTError as ex:
            emit({"config": label, "unsupported": ex.name})
            return
        info = p.info()
        for i in range(3):
            p.execute(xs[i % sets], ys[i % sets], -1, st)
        torch.cuda.synchronize()
        p.set_timing(True)
        p.read_timing(reset=True)
        for i in range(reps):
            p.execute(xs[i % sets], ys[i % sets], -1 if i % 2 == 0 else 1, st)
        ms, cnt = p.read_timing(reset=True)
        p.set_timing(False)
        p.destroy()
        per = [round(ms[k] / cnt[k] * 1e3, 1) for k in range(3) if cnt[k]]
        emit({"config": label, "us_per_pass": per, "us_total": round(sum(per), 1),
              "lines_per_block": [info["lines_per_block_pass1"], info["lines_per_block_pass2"]],
              "threads": [info["threads_pass1"], info["threads_pass2"]],
              "lds": [info["lds_bytes_pass1"], info["lds_bytes_pass2"]],
              "variants": [info["variant_pass1"], info["variant_pass2"]],
              "tile_order": "%#08x" % info["tile_order"]})

    TWO, THREE = B.FFT_OPT_TWO_LEVEL, B.FFT_OPT_THREE_LEVEL
    SPLIT, FULL = B.FFT_OPT_SPLIT_EXCHANGE, B.FFT_OPT_FULL_EXCHANGE
    plan_times("two-level default", flags=TWO)
    plan_times("two-level, pass 1 staged in LDS by direct loads", flags=TWO | B.FFT_OPT_LDS_PREFETCH)
    plan_times("three-level default", flags=THREE)
    plan_times("three-level shuffle exchange", flags=THREE | B.FFT_OPT_SHUFFLE_EXCHANGE)
    plan_times("three-level split exchange", flags=THREE | SPLIT)
    plan_times("three-level 32 lines", flags=THREE, lines_per_block=32)
    for T1 in (1, 2, 4, 8):
        for vpt in (16, 32):
            for fl, fn in ((SPLIT, "split"), (FULL, "complex")):
                plan_times("pass 1 T=%d, %d values/thread, %s exchange" % (T1, vpt, fn), flags=TWO | fl,
                           lines_per_block=T1, lines_per_block2=4, values_per_thread=vpt, values_per_thread2=16)
    for T2 in (2, 4, 8):
        for vpt in (16, 32):
            for fl, fn in ((SPLIT, "split"), (FULL, "complex")):
                plan_times("pass 2 T=%d, %d values/thread, %s exchange" % (T2, vpt, fn), flags=TWO | fl,
                           lines_per_block=2, lines_per_block2=T2, values_per_thread=16, values_per_thread2=vpt)
    for W in (1, 4, 8):
        plan_times("two-level, scratch slabs %d wide" % W, flags=TWO | SPLIT, lines_per_block=2,
                   lines_per_block2=4, scratch_width=W)
    plan_times("two-level, scratch slabs 8 wide, pass 2 32 values/thread", flags=TWO | SPLIT, lines_per_block=2,
               lines_per_block2=4, scratch_width=8, values_per_thread2=32)
    for flags, fn in ((B.FFT_OPT_PERSISTENT, "persistent"), (B.FFT_OPT_DENSE | SPLIT, "dense split")):
        plan_times("two-level %s" % fn, flags=TWO | flags)
    for lp in (10, 11, 13, 14):
        plan_times("two-level split p = 2^%d" % lp, flags=TWO, log2_p=lp)
    plan_times("two-level, hardware workgroup order", flags=TWO | B.FFT_OPT_NO_XCD_REMAP)
    plan_times("three-level, hardware workgroup order", flags=THREE | B.FFT_OPT_NO_XCD_REMAP)
    # Tile orders (byte k: pass k's (log2 g << 4) | log2 s; 0x80 hardware order)
    ORD = B.FFT_OPT_TILE_ORDER
    plan_times("two-level, XCD-contiguous order without spread (0x0000)", flags=TWO | ORD, tile_order=0)
    for ls in range(1, 6):
        plan_times("two-level, pass 1 order g 1, s %d (0x04%02x)" % (1 << ls, ls), flags=TWO | ORD,
                   tile_order=0x0400 | ls)
    for lg in (1, 2, 3):
        plan_times("two-level, pass 1 order g %d, s 4 (0x04%02x)" % (1 << lg, (lg << 4) | 2), flags=TWO | ORD,
                   tile_order=0x0400 | (lg << 4) | 2)
    for ls in range(1, 6):
        plan_times("two-level, pass 2 order g 1, s %d (0x%02x12)" % (1 << ls, ls), flags=TWO | ORD,
                   tile_order=(ls << 8) | 0x12)
    ROWS = B.FFT_OPT_ROW_LANES
    for vpt in (16, 32):  # pass 1 with whole rows per thread (8 rows radix 8, 16 rows radix 16)
        for o in (0x0400, 0x0401, 0x0412, 0x0421):
            plan_times("pass 1 with rows per thread, %d values/thread, order %#06x" % (vpt, o), flags=TWO | ROWS | ORD,
                       values_per_thread=vpt, tile_order=o)
    for o in (0x02, 0x03, 0x13):  # the wider pass-1 tiles in spread orders
        for vpt, fl, fn in ((32, SPLIT, "split"), (16, FULL, "complex")):
            plan_times("pass 1 T=4, %d values/thread, %s exchange, order 0x04%02x" % (vpt, fn, o),
                       flags=TWO | fl | ORD, lines_per_block=4, lines_per_block2=4, values_per_thread=vpt,
                       values_per_thread2=16, tile_order=0x0400 | o)
    plan_times("three-level, orders without spread, B and C hardware (0x808000)", flags=THREE | ORD,
               tile_order=0x808000)
    for ls in range(1, 7):
        plan_times("three-level, pass A order g 1, s %d (0x8003%02x)" % (1 << ls, ls), flags=THREE | ORD,
                   tile_order=0x800300 | ls)
    for ls in range(1, 7):
        plan_times("three-level, pass B order g 1, s %d (0x80%02x05)" % (1 << ls, ls), flags=THREE | ORD,
                   tile_order=0x800005 | (ls << 8))
    plan_times("three-level, pass C XCD-contiguous (0x000305)", flags=THREE | ORD, tile_order=0x000305)
    return 0


def run_lift_sweep(torch, lf, sizes, sets: int = 4, reps: int = 10) -> int:
    """Two-level against three-level lift per length (c64, one transform,
    rotating buffer sets, per-pass HIP events): where the library's default
    switches lifts.  One JSON object per line."""
    from paper_0811_2535_amd import binding as B
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    for t in sizes:
        n = 1 << t
        nsets = sets if t <= 26 else 2
        gen = torch.Generator(device=dev)
        gen.manual_seed(2)
        xs = [torch.randn(n, dtype=torch.complex64, device=dev, generator=gen) for _ in range(nsets)]
        ys = [torch.empty_like(x) for x in xs]
        rec = {"log2n": t}
        for flags, name in ((B.FFT_OPT_TWO_LEVEL, "two_level_us"), (B.FFT_OPT_THREE_LEVEL, "three_level_us")):
            try:
                p = lf.Plan(n, 1, torch.complex64, flags=flags)
            except B.FFTError as ex:
                rec[name] = ex.name
                continue
            for i in range(2):
                p.execute(xs[i % nsets], ys[i % nsets], -1, st)
            torch.cuda.synchronize()
            p.set_timing(True)
            p.read_timing(reset=True)
            for i in range(reps):
                p.execute(xs[i % nsets], ys[i % nsets], -1 if i % 2 == 0 else 1, st)
            ms, cnt = p.read_timing(reset=True)
            p.set_timing(False)
            p.destroy()
            rec[name] = [round(ms[k] / cnt[k] * 1e3, 1) for k in range(3) if cnt[k]]
        print(json.dumps(rec), flush=True)
        del xs, ys
        torch.cuda.empty_cache()
    return 0


def run_order_sweep(torch, lf, shapes, rounds: int = 3) -> int:
    """Tile orders per pass of the library's default plan (complex64), one
    shape at a time, "LOG2N" or "LOG2NxBATCH": starting from the XCD-contiguous
    order without spread, each pass in turn is timed in the hardware order
    and in spread orders (g 1, s 2..32; g 2, s 4 and 8) with the other passes
    at their best so far, and keeps the fastest.  Times are medians over
    `rounds` rounds of 20 executes (forward and inverse alternating, four
    rotating buffer sets, per-pass HIP events).  One JSON object per
    candidate; the last line of each shape holds the chosen orders and the
    library's own default orders, both timed again."""
    from paper_0811_2535_amd import binding as B
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    for shape in shapes:
        t, batch = (int(v) for v in shape.split("x")) if "x" in shape else (int(shape), 1)
        n = 1 << t
        nsets = 4 if n * batch <= 1 << 26 else 2
        gen = torch.Generator(device=dev)
        gen.manual_seed(2)
        xs = [torch.randn(batch, n, dtype=torch.complex64, device=dev, generator=gen) for _ in range(nsets)]
        ys = [torch.empty_like(x) for x in xs]

        def timed(**kw):
            try:
                p = lf.Plan(n, batch, torch.complex64, **kw)
            except B.FFTError as ex:
                return None, ex.name
            info = p.info()
            for i in range(2 * nsets):
                p.execute(xs[i % nsets], ys[i % nsets], -1 if i % 2 == 0 else 1, st)
            torch.cuda.synchronize()
            p.set_timing(True)
            p.read_timing(reset=True)
            per_round = []
            for _ in range(rounds):
                for i in range(20):
                    p.execute(xs[i % nsets], ys[i % nsets], -1 if i % 2 == 0 else 1, st)
                ms, cnt = p.read_timing(reset=True)
                per_round.append([ms[k] / cnt[k] * 1e3 for k in range(3) if cnt[k]])
            p.set_timing(False)
            p.destroy()
            per = [round(sorted(r[k] for r in per_round)[rounds // 2], 1) for k in range(len(per_round[0]))]
            return per, info

        per0, info0 = timed()
        if per0 is None:
            print(json.dumps({"shape": shape, "unsupported": info0}), flush=True)
            continue
        levels = info0["levels"]
        order = 0
        per_best, _ = timed(flags=B.FFT_OPT_TILE_ORDER, tile_order=order)
        print(json.dumps({"shape": shape, "order": "%#08x" % order, "us": per_best}), flush=True)
        for k in range(levels):
            for b in (0x80, 0x01, 0x02, 0x03, 0x04, 0x05, 0x12, 0x13):
                cand = (order & ~(0xff << (8 * k))) | (b << (8 * k))
                per, info = timed(flags=B.FFT_OPT_TILE_ORDER, tile_order=cand)
                if per is None:
                    print(json.dumps({"shape": shape, "order": "%#08x" % cand, "unsupported": info}), flush=True)
                    continue
                print(json.dumps({"shape": shape, "order": "%#08x" % cand, "us": per}), flush=True)
                if sum(per) < sum(per_best):
                    order, per_best = cand, per
        chosen, _ = timed(flags=B.FFT_OPT_TILE_ORDER, tile_order=order)
        plain, _ = timed(flags=B.FFT_OPT_TILE_ORDER, tile_order=0)
        default, info = timed()
        print(json.dumps({"shape": shape, "levels": levels, "chosen": "%#08x" % order, "chosen_us": chosen,
                          "plain_us": plain, "default": "%#08x" % info["tile_order"], "default_us": default,
                          "gain_chosen_vs_plain": round(sum(plain) / sum(chosen), 3)}), flush=True)
        del xs, ys
        torch.cuda.empty_cache()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--sets", type=int, default=4, help="buffer sets rotated between transforms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the differentiation-form, uneven-batch, precision-form and "
                         "autotuner measurements")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this benchmark and exit")
    ap.add_argument("--only", choices=["config1", "fwd_bwd", "ragged", "precision"],
                    help="run one of the extra measurements alone (for a kernel trace of it) and print "
                         "its JSON object")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="print a markdown table of a rocprofv3 --kernel-trace --stats summary of this "
                         "benchmark (run_kernel_stats.csv) and exit")
    ap.add_argument("--traversal-probe", action="store_true",
                    help="run the traversal probe (plain copies with each pass's tile traversal at n = 2^24, "
                         "built by __graft_entry__.build) and print its JSON lines")
    ap.add_argument("--sweep", action="store_true",
                    help="print per-pass kernel times of the plan configurations (tile widths, "
                         "kernel variants, lifts) with streaming references, one JSON object per "
                         "line, and exit")
    ap.add_argument("--sweep-lifts", metavar="LOG2N,...",
                    help="print two-level against three-level per-pass times at the given lengths "
                         "(e.g. 20,22,23,24,25,26,28) and exit")
    ap.add_argument("--sweep-orders", metavar="SHAPE,...",
                    help="search each pass's tile order for the default plans of the given shapes "
                         "(LOG2N or LOG2NxBATCH, complex64, e.g. 22,24,20x16) and exit")
    ap.add_argument("--copy-reps", type=int, default=10,
                    help="device-to-device copies of one pass's bytes, timed for context and "
                         "used as the known-size reference kernel for HBM counters")
    args = ap.parse_args()

    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return 0

    if args.traversal_probe:
        # a child process of its own; this process does not touch the GPU
        import subprocess
        probe = os.path.join(ROOT, "paper_0811_2535_amd", "traversal_probe")
        if not os.path.exists(probe):
            print("bench.py: %s is not built (run __graft_entry__.build())" % probe, file=sys.stderr)
            return 1
        return subprocess.run([probe]).returncode

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
    if args.only:
        fn = {"config1": measure_config1, "fwd_bwd": measure_fwd_bwd, "ragged": measure_ragged,
              "precision": measure_precision}[args.only]
        res, _ = fn(torch, lf, datagen)
        print(json.dumps({args.only: res}), flush=True)
        return 0
    if args.sweep:
        return run_sweep(torch, lf, args.log2n)
    if args.sweep_lifts:
        return run_lift_sweep(torch, lf, [int(v) for v in args.sweep_lifts.split(",")])
    if args.sweep_orders:
        return run_order_sweep(torch, lf, args.sweep_orders.split(","))
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
        "paper_context": PAPER_CONTEXT,
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
            "tile_order": "%#06x" % info["tile_order"],
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
    precision_firsts = keep1 = keep3 = keep5 = None
    if not args.no_extras:
        print("[bench] config 1: n=2^10 complex128", file=sys.stderr, flush=True)
        result["config1"], keep1 = measure_config1(torch, lf, datagen)
        print("[bench] forward + adjoint backward, batch 8 x 2^22", file=sys.stderr, flush=True)
        del xs, ys
        result["fwd_bwd"], keep5 = measure_fwd_bwd(torch, lf, datagen)
        lf.clear_plan_cache()
        print("[bench] batched uneven lengths, 4096 transforms", file=sys.stderr, flush=True)
        result["ragged"], keep3 = measure_ragged(torch, lf, datagen)
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
        threads = oracle_threads()
        legs = {}
        if keep1 is not None:
            legs["config1"] = oracle_leg_config1(keep1)
        if keep3 is not None:
            print("[bench] oracle leg, config 3 (%d threads)" % threads, file=sys.stderr, flush=True)
            legs["config3"] = oracle_leg_config3(keep3, threads)
            result["ragged"]["max_rel_l2_vs_oracle"] = legs["config3"]["max_rel_l2"]
        if precision_firsts is not None:
            print("[bench] oracle leg, config 4 (%d threads)" % threads, file=sys.stderr, flush=True)
            errs, legs["config4"] = precision_oracle_errors(*precision_firsts, threads)
            for mode, e in errs.items():
                result["precision"][mode]["max_rel_l2_vs_oracle_subset"] = e
        if keep5 is not None:
            print("[bench] oracle leg, config 5 (%d threads)" % threads, file=sys.stderr, flush=True)
            legs["config5"] = oracle_leg_config5(keep5, threads)
            result["fwd_bwd"]["grad_rel_l2_vs_oracle"] = legs["config5"]["grad_rel_l2_gpu_vs_oracle"]
        if legs:
            result["cpu_oracle_legs"] = legs
    plan.destroy()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
