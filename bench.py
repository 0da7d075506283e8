"""Throughput of the fused HLBM stream-collide sweep on one MI355X.

Workload: D3Q19 homogenized lattice BGK on a 512^3 fully periodic box, porosity
control d from a regular 16^3 array of spheres (cell edge 32, radius 10)
smoothed by a periodic Gaussian (sigma = 2), tau = 0.6, body force 1e-6 along x,
from rest.  A "step" is one fused pull-stream + collide sweep over all cells.

The headline form stores populations in FP32 (FP32 arithmetic).  The FP16- and
BF16-shifted storage forms (FP32 arithmetic) run on the same workload and are
reported beside it with their speed-up and their relative L2 error against the
FP64 oracle.  Forms suffixed "-aa" run the in-place (AA) pattern: one population
buffer instead of two, the same bytes per cell and bit-identical results.  The error is exact to evaluate at full size: the workload is
32-periodic, so every 32^3 tile equals a 32^3 run of one obstacle cell, which
the oracle computes (as part of the timed CPU-baseline sample).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
N_EDGE = 512
TAU = 0.6
FORCE = (1e-6, 0.0, 0.0)
SCALE_16 = 2.0 ** 24
ALG_BYTES = {"f32": 19 * 4 * 2 + 4, "f16s": 19 * 2 * 2 + 2, "bf16s": 19 * 2 * 2 + 2}
TENSOR_BYTES = 19 * 4 * 2 + 6 * 4
COUNTERS = os.path.join(ROOT, "profiles", "sweep_d3q19_f32_512_counters.json")
# sources the FP32 sweep kernel is compiled from (counters are valid for them only)
SWEEP_SRCS = [os.path.join(ROOT, "paper_2310_14746_amd", "csrc", f)
              for f in ("sweep.hip", "cell.hpp", "lattice.hpp", "storage.hpp", "hlbm_internal.hpp")]
METRIC = "MLUPS and % HBM roofline, D3Q19 HLBM 512^3; FP16-storage vs FP32 at stated L2 error"


def storage_of(form):
    """Storage name of a bench form ("f32", "f16s-aa", ...)."""
    return form.split("-")[0]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_l2_drho(dr, dr_ref, u_ref):
    floor = np.linalg.norm((u_ref ** 2).sum(axis=0) * 3.0)
    return float(np.linalg.norm(dr - dr_ref) / max(np.linalg.norm(dr_ref), floor))


# the 512^3 workload runs 500 steps: every form's error against the FP64 oracle
# is taken at that time level, whatever the number of timed steps
ERROR_STEPS = 500
# stated relative L2 tolerances against the FP64 oracle (u and drho); BF16 storage
# is reported against the FP16 figure, which it is not expected to meet
STATED_TOLERANCE = {"f32": 1e-5, "f16s": 2e-3, "bf16s": 2e-3}

TIMING_PARTS = {}   # (storage, pattern, porosity, edge) -> ms per step in five parts of the timed region


def time_form(hlbm, storage, d_tile, steps, warmup, block_x=0, porosity="scalar", edge=N_EDGE,
              pattern="ab", row_pad=None, error_steps=ERROR_STEPS):
    """row_pad None: the tuned population row pad for this shape (0 if none).
    The returned moments are those of time level error_steps (None: where the
    timing ended)."""
    import torch
    from paper_2310_14746_amd import tune
    if row_pad is None:
        row_pad = tune.lookup_row_pad(hlbm.D3Q19, storage, (edge,) * 3, pattern)
    reps = edge // 32
    dt = np.float32 if storage == "f32" else np.float16
    if porosity == "tensor":   # d_tile: (6, 32^3) rows of D
        d = np.stack([np.tile(r.reshape(32, 32, 32).astype(dt), (reps, reps, reps)).ravel()
                      for r in d_tile])
    else:
        d = np.tile(d_tile.astype(dt), (reps, reps, reps))
    sim = hlbm.HLBM(hlbm.D3Q19, storage, (edge,) * 3, tau=TAU, force=FORCE,
                    store_scale=SCALE_16 if storage != "f32" else 1.0, block_x=block_x,
                    porosity=porosity, pattern=pattern, row_pad=row_pad)
    try:
        sim.set_porosity(d)
        del d
        log(f"{storage}: warmup {warmup}")
        sim.step(warmup)
        sim.sync()
        torch.cuda.synchronize()
        # one timed region of `steps` sweeps; events recorded between five
        # equal parts of it (no synchronization inside) give the spread
        parts = [steps // 5 + (1 if k < steps % 5 else 0) for k in range(5)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(sim.stream)
        for k, n in enumerate(parts):
            sim.step(n)
            ev[k + 1].record(sim.stream)
        ev[5].synchronize()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[5])
        per_step = [ev[k].elapsed_time(ev[k + 1]) / n for k, n in enumerate(parts) if n]
        log(f"{storage}: {steps} steps in {ms:.1f} ms; per step in five parts: "
            + ", ".join(f"{v:.4f}" for v in per_step) + " ms")
        TIMING_PARTS[(storage, pattern, porosity, edge)] = per_step
        # errors are stated at the workload's own step count: continue the same
        # run (untimed) to it, or start it again from rest if the timing went past it
        done = warmup + steps
        if error_steps is not None and done != error_steps:
            if done > error_steps:
                sim.reset()
                done = 0
            log(f"{storage}: {error_steps - done} untimed steps to time level {error_steps} for the error")
            sim.step(error_steps - done)
            sim.sync()
        drho, u, tot = sim.moments("f64", totals=True)
        dr_t = drho[:32, :32, :32].cpu().numpy().ravel()
        u_t = u[:, :32, :32, :32].cpu().numpy().reshape(3, -1)
        # every 32^3 tile identical (exact periodicity of the workload)
        r = edge // 32
        v = drho.reshape(r, 32, r, 32, r, 32)
        tiles_equal = bool((v == v[:1, :, :1, :, :1, :]).all().item())
        del drho, u, v
        torch.cuda.empty_cache()
        return ms, dr_t, u_t, tot, tiles_equal
    finally:
        sim.close()


def copy_reference(gib=4.0, reps=10):
    """Device-to-device copy bandwidth, counted as bytes read + bytes written:
    what HBM sustains for streaming.  Two plain copies of 4 GiB: torch's
    copy_ (the runtime's blit kernel, which the counter calibration uses) and a
    vectorized elementwise kernel (b = a * 1); `GBs` is the faster."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    out = {"bytes_per_copy": 2 * 4 * n}
    for name, fn in (("blit", lambda: b.copy_(a)), ("elementwise", lambda: torch.mul(a, 1.0, out=b))):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_ms"] = round(ms, 4)
        out[name + "_GBs"] = round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)
    out["GBs"] = max(out["blit_GBs"], out["elementwise_GBs"])
    del a, b
    torch.cuda.empty_cache()
    return out


def pattern_reference(hlbm, block_x, row_pad, edge=N_EDGE, steps=50):
    """The sweep's own loads and stores with the collision left out
    (hlbm_ref_stream_pattern: pull streaming of the 19 FP32 rows with the
    sweep's gather, row pitch, block width and stores, plus the porosity read)
    at the headline's shape, block width and row pad; counted with the sweep's
    algorithmic 156 bytes per cell."""
    import ctypes
    import torch
    lib = hlbm.load()
    n = edge ** 3
    P = n + row_pad // 4
    a = torch.zeros(19 * P, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    d = torch.zeros(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(src, dst):
        rc = lib.hlbm_ref_stream_pattern(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                         ctypes.c_void_p(d.data_ptr()), edge, edge, edge, row_pad, block_x,
                                         ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"hlbm_ref_stream_pattern failed ({rc})")
    for k in range(4):
        run(a, b) if k % 2 == 0 else run(b, a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        run(a, b) if k % 2 == 0 else run(b, a)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del a, b, d
    torch.cuda.empty_cache()
    return {"ms": round(ms, 4), "GBs": round(156 * n / (ms * 1e-3) / 1e9, 1), "block_x": block_x,
            "row_pad_bytes": row_pad}


def summarize_profile(path):
    """Per-kernel duration summary of a rocprofv3 --kernel-trace output
    (SQLite results database or kernel_stats CSV) under `path`."""
    import glob
    import sqlite3
    dbs = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
    rows = []
    if dbs:
        con = sqlite3.connect(dbs[0])
        rows = con.execute("select name, count(*), avg(end-start), min(end-start), max(end-start), "
                           "sum(end-start) from kernels group by name order by sum(end-start) desc").fetchall()
    else:
        import csv
        for f in glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]),
                             float(r["MaxNs"]), float(r["TotalDurationNs"])))
    out = ["| kernel | calls | avg us | min us | max us | total ms |", "|---|---|---|---|---|---|"]
    for name, calls, avg, mn, mx, tot in rows:
        out.append(f"| `{name.split('(')[0]}` | {calls} | {avg / 1e3:.1f} | {mn / 1e3:.1f} | "
                   f"{mx / 1e3:.1f} | {tot / 1e6:.2f} |")
    # the same kernels split by launch grid (threads per axis), from the
    # per-dispatch trace: one kernel runs several box sizes in one bench run
    import csv
    groups = {}
    for f in glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"].split("(")[0]
            if not name.startswith("void hlbm::"):
                continue
            grid = "x".join(r[k] for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"))
            groups.setdefault((name, grid), []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if groups:
        out += ["", "| library kernel | grid (threads) | launches | avg us |", "|---|---|---|---|"]
        for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            out.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / len(v) / 1e3:.1f} |")
    return "\n".join(out)


def summarize_backward(path, steps=500):
    """Timeline of the last replayed backward pass of the differentiation
    workload (128x64x64) in a rocprofv3 --kernel-trace CSV under `path`: the span from its
    first to its last reverse step, the reverse steps and replay sweeps inside
    it, how long the GPU had a kernel running, and how many reverse steps ran
    beside a replay sweep (the two streams overlapping)."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            grid = tuple(int(r[k]) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"))
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"].split("(")[0],
                         int(r["Queue_Id"]), grid))
    rows.sort()
    c4 = (128, 64, 64)
    rev = [r for r in rows if "adjoint_kernel<" in r[2] and r[4] == c4]
    if len(rev) < steps:
        return f"fewer than {steps} reverse steps on 128x64x64 in the trace"
    # backward passes: consecutive runs of `steps` reverse steps; the last one
    # with replay sweeps inside its span (a moment-record pass has none)
    recs = [r for r in rows if "sweep_record_kernel<" in r[2] and r[4] == c4]
    last = None
    for k in range(len(rev) // steps):
        chunk = rev[k * steps:(k + 1) * steps]
        a, b = chunk[0][0], max(r[1] for r in chunk)
        if any(r[0] >= a and r[1] <= b for r in recs):
            last = chunk
    if last is None:
        return "no replayed backward pass on 128x64x64 in the trace"
    t0, t1 = last[0][0], max(r[1] for r in last)
    inside = [r for r in rows if r[0] >= t0 and r[1] <= t1]
    rec = [r for r in inside if "sweep_record_kernel<" in r[2] and r[4] == c4]
    iv = sorted((r[0], r[1]) for r in inside)
    busy, (cs, ce) = 0, iv[0]
    for a, b in iv[1:]:
        if a > ce:
            busy, cs, ce = busy + ce - cs, a, b
        else:
            ce = max(ce, b)
    busy += ce - cs
    beside = sum(1 for a in last if any(r[0] < a[1] and r[1] > a[0] for r in rec))
    def mean_us(v):
        return sum(r[1] - r[0] for r in v) / max(1, len(v)) / 1e3
    out = ["| quantity | value |", "|---|---|",
           f"| span of the reverse steps (first start to last end) | {(t1 - t0) / 1e6:.2f} ms |",
           f"| reverse steps / mean duration | {len(last)} / {mean_us(last):.1f} us |",
           f"| replay sweeps inside the span / mean duration | {len(rec)} / {mean_us(rec):.1f} us |",
           f"| sum of those kernels' durations | {(sum(r[1] - r[0] for r in last) + sum(r[1] - r[0] for r in rec)) / 1e6:.2f} ms |",
           f"| time with a kernel running | {busy / 1e6:.2f} ms |",
           f"| reverse steps that ran beside a replay sweep | {beside} of {len(last)} |",
           f"| queues of the reverse steps / replay sweeps | {sorted(set(r[3] for r in last))} / "
           f"{sorted(set(r[3] for r in rec))} |"]
    return "\n".join(out)


def _code_only(text):
    """Source text without comments and with whitespace collapsed: an edit of
    a comment does not change the kernel the counters were taken on."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def sweep_sources_sha256(texts=None):
    """Hash of the sweep's sources (comments stripped): the committed counter
    record carries it, and bench reports `traffic` only while it matches."""
    h = hashlib.sha256()
    for t in (texts if texts is not None else [open(f).read() for f in SWEEP_SRCS]):
        h.update(_code_only(t).encode())
    return h.hexdigest()


def counters_traffic(n_cells):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current sweep sources."""
    if not os.path.exists(COUNTERS):
        return None
    info = json.load(open(COUNTERS))
    if info.get("sweep_sources_sha256") != sweep_sources_sha256() or info.get("cells") != n_cells:
        return None
    return info.get("hbm_bytes_per_launch")


SWEEP_F32 = "hlbm::sweep_kernel<hlbm::D3Q19, hlbm::StoreF32, 0, 0>"  # periodic, scalar control
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def summarize_counters(fetch_dir, write_dir, n_cells=N_EDGE ** 3):
    """HBM traffic of the FP32 512^3 sweep from two rocprofv3 --pmc runs of
    bench.py (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Each counter is
    scaled by what it reads for the 4 GiB device copy that the same run makes
    (copy_reference: 4 GiB read, 4 GiB written).  Writes the JSON record bench
    reads and returns a markdown summary."""
    import csv
    import glob

    def per_dispatch(path, counter):
        rows = []
        for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == counter]
        # the calibration copy is the runtime's blit of 4 GiB: the blit
        # dispatches that read the most (smaller blits, such as tape
        # checkpoints, run on the same grid)
        big = max(float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith(COPY_KERNEL))
        vals = {}
        for r in rows:
            name = r["Kernel_Name"]
            key = ("sweep" if name.startswith("void " + SWEEP_F32) and int(r["Grid_Size"]) == n_cells else
                   "copy" if name.startswith(COPY_KERNEL) and float(r["Counter_Value"]) >= 0.5 * big else None)
            if key:
                vals.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}

    fetch, nf = per_dispatch(fetch_dir, "FETCH_SIZE")
    write, nw = per_dispatch(write_dir, "WRITE_SIZE")
    copy_bytes = 4.0 * 2 ** 30
    f_scale = copy_bytes / (fetch["copy"] * 1024)
    w_scale = copy_bytes / (write["copy"] * 1024)
    rd = fetch["sweep"] * 1024 * f_scale
    wr = write["sweep"] * 1024 * w_scale
    alg_rd, alg_wr = n_cells * (19 * 4 + 4), n_cells * 19 * 4
    info = {
        "kernel": SWEEP_F32, "cells": n_cells, "sweep_sources_sha256": sweep_sources_sha256(),
        "fetch_kib_per_dispatch": round(fetch["sweep"], 1), "write_kib_per_dispatch": round(write["sweep"], 1),
        "fetch_scale_from_copy": round(f_scale, 5), "write_scale_from_copy": round(w_scale, 5),
        "hbm_read_bytes_per_launch": round(rd), "hbm_write_bytes_per_launch": round(wr),
        "hbm_bytes_per_launch": round(rd + wr),
        "algorithmic_bytes_per_launch": alg_rd + alg_wr,
        "dispatches": {"fetch": nf, "write": nw},
    }
    json.dump(info, open(COUNTERS, "w"), indent=1)
    return "\n".join([
        "| quantity | read | write | total |", "|---|---|---|---|",
        f"| counter, KiB per dispatch | {fetch['sweep']:.1f} (FETCH_SIZE) | {write['sweep']:.1f} (WRITE_SIZE) | |",
        f"| copy calibration (4 GiB copy) | x{f_scale:.4f} | x{w_scale:.4f} | |",
        f"| HBM bytes per launch | {rd / 1e9:.3f} GB | {wr / 1e9:.3f} GB | {(rd + wr) / 1e9:.3f} GB |",
        f"| algorithmic bytes per launch | {alg_rd / 1e9:.3f} GB | {alg_wr / 1e9:.3f} GB | "
        f"{(alg_rd + alg_wr) / 1e9:.3f} GB |",
        f"| HBM / algorithmic | {rd / alg_rd:.4f} | {wr / alg_wr:.4f} | {(rd + wr) / (alg_rd + alg_wr):.4f} |",
    ])


def _timed_batch(hlbm, items, fields, steps, modes, sched, masks=None, rounds=2):
    """Timed hlbm_step calls of `steps` over one batch (one allocation), from
    rest, in each of `modes`, alternating over `rounds`; each mode's first call
    with this step count runs untimed first (a graph is built on the first
    call with a given step count and starting buffer).  Returns
    ({mode: min ms}, cells, {mode: totals after the last timed call}, schedule)."""
    import torch
    b = hlbm.HLBMBatch(items, "f32", mode=modes[0], **sched)
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
            if masks is not None:
                b.set_solid_mask(k, masks[k])
        ms, tot = {}, {}
        for r in range(rounds):
            for mode in modes:
                b.set_mode(mode)
                if r == 0:
                    b.step(steps if mode.startswith("graph") else 2)
                    b.sync()
                b.reset()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(b.stream)
                b.step(steps)
                e1.record(b.stream)
                b.sync()
                t = e0.elapsed_time(e1)
                ms[mode] = min(ms.get(mode, t), t)
                tot[mode] = b.totals()
        _, cells = b.info()
        return ms, cells, tot, b.schedule()
    finally:
        b.close()


# Algorithmic bytes per dispatch of the kernels the counter summary covers,
# by kernel name (up to its argument list) and total threads of the grid.
def _alg_bytes_per_dispatch(name, grid_threads, batched_steps):
    c512, cbatch, c4 = N_EDGE ** 3, 98254848, 128 * 64 * 64
    table = {
        ("void hlbm::sweep_kernel<hlbm::D3Q19, hlbm::StoreF32, 0, 0>", c512): 156 * c512,
        ("void hlbm::sweep_pair_kernel<hlbm::StoreF16S>", c512 // 2): 78 * c512,
        ("void hlbm::sweep_aa_kernel<hlbm::D3Q19, hlbm::StoreF32, 3, 0>", c512): 156 * c512,
        ("void hlbm::sweep_aa_kernel<hlbm::D3Q19, hlbm::StoreF32, 4, 0>", c512): 156 * c512,
        ("hlbm::stream_pattern_kernel", c512): 156 * c512,
        ("void hlbm::batch_step_kernel<hlbm::StoreF32, false>", None): 156 * cbatch,
        ("void hlbm::batch_persistent_kernel<hlbm::StoreF32, false>", None): 156 * cbatch * batched_steps,
        ("void hlbm::adjoint_kernel<hlbm::D3Q19, hlbm::StoreF32, 1, 0>", c4): ADJ_BYTES_REC * c4,
        ("void hlbm::sweep_kernel<hlbm::D3Q19, hlbm::StoreF32, 1, 0>", c4): 156 * c4,
        ("void hlbm::sweep_record_kernel<hlbm::D3Q19, hlbm::StoreF32, 1, 0>", c4): REC_SWEEP_BYTES * c4,
    }
    for (n, g), v in table.items():
        if name == n and (g is None or g == grid_threads):
            return v
    return None


def summarize_counters_all(fetch_dir, write_dir, batched_steps):
    """HBM traffic per dispatch of every kernel in the table above, from two
    rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE), each counter scaled by what
    it reads for the same run's 4 GiB blit copy; against the algorithmic bytes."""
    import csv
    import glob

    def per_kernel(path, counter):
        rows = []
        for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == counter]
        # the 4 GiB copy: the blit dispatches that read the most (smaller
        # blits, such as tape checkpoints, run on the same grid)
        big = max(float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith(COPY_KERNEL))
        vals = {}
        for r in rows:
            name = r["Kernel_Name"].split("(")[0]
            g = int(r["Grid_Size"])
            if name.startswith(COPY_KERNEL):
                if float(r["Counter_Value"]) >= 0.5 * big:
                    vals.setdefault("copy", []).append(float(r["Counter_Value"]))
                continue
            vals.setdefault((name, g), []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}

    fetch, nf = per_kernel(fetch_dir, "FETCH_SIZE")
    write, nw = per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = 4.0 * 2 ** 30
    f_scale = copy_bytes / (fetch["copy"] * 1024)
    w_scale = copy_bytes / (write["copy"] * 1024)
    out = [f"Calibration (the same runs' 4 GiB blit copy): FETCH_SIZE x{f_scale:.4f}, WRITE_SIZE x{w_scale:.4f}.",
           "", "| kernel | grid threads | dispatches | HBM read | HBM write | "
               "HBM total | algorithmic | total / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    for key in sorted(k for k in fetch if k != "copy"):
        name, g = key
        alg = _alg_bytes_per_dispatch(name, g, batched_steps)
        if alg is None or key not in write:
            continue
        rd = fetch[key] * 1024 * f_scale
        wr = write[key] * 1024 * w_scale
        out.append(f"| `{name.replace('void hlbm::', '')}` | {g} | {nf[key]} | {rd / 1e9:.4f} GB | "
                   f"{wr / 1e9:.4f} GB | {(rd + wr) / 1e9:.4f} GB | {alg / 1e9:.4f} GB | {(rd + wr) / alg:.4f} |")
    return "\n".join(out)


def time_batched(hlbm, steps=2000, seed=0):
    """256 homogenized periodic unit cells (edges 32..96), 2000 steps:
    * "graph": one HIP graph launch holding one per-step kernel node per step
      (the default batch mode);
    * "graph_persistent": one graph launch of the persistent kernel, which
      runs all steps with a grid barrier between them;
    * "per_step": one kernel launch per step.
    The modes alternate on one allocation (two rounds, the faster of each is
    reported).  Algorithmic bytes as for the FP32 sweep.  The same cells with
    the sphere resolved (solid mask, bounce-back links, d = 0) run as one graph
    too, and the permeabilities of both are reported."""
    from paper_2310_14746_amd import inputs, permeability, tune
    spec = inputs.batch_items(256, seed=seed)
    items = [dict(shape=(e, e, e), tau=t, force=(1e-6, 0, 0)) for e, _, t in spec]
    log("batched: building 256 unit-cell fields")
    fields = {}
    for e, phi, _ in spec:
        if (e, phi) not in fields:
            fields[(e, phi)] = inputs.round_to(inputs.batch_item_field(e, phi), "f32").astype(np.float32).ravel()
    item_fields = [fields[(e, phi)] for e, phi, _ in spec]
    sched = tune.lookup_batch(items, "f32") or {}
    out = {"workload": "256 periodic D3Q19 unit cells, edges {32,48,64,80,96}, phi U[0.1,0.9], "
                       f"tau U[0.55,1.0], F=1e-6, FP32, seed {seed}", "steps": steps}
    cells_k = np.array([e ** 3 for e, _, _ in spec], dtype=float)
    nu = (np.array([t for _, _, t in spec]) - 0.5) / 3.0
    modes = ("graph", "graph_persistent", "per_step")
    ms, cells, tot, sc = _timed_batch(hlbm, items, item_fields, steps, modes, sched)
    out["cells"] = cells
    out["schedule"] = dict(sc, tuned=bool(sched))
    for mode in modes:
        log(f"batched {mode}: {steps} steps in {ms[mode]:.0f} ms")
        out[mode] = {"ms": round(ms[mode], 1), "mlups": round(cells * steps / (ms[mode] * 1e-3) / 1e6, 1),
                     "alg_GBs": round(156 * cells * steps / (ms[mode] * 1e-3) / 1e9, 1)}
    # every mode gives the same bits (the totals of its last run)
    out["modes_bitwise_equal"] = bool(all(np.array_equal(tot[m], tot["per_step"]) for m in modes))
    k_hom = nu * (tot["graph"][:, 1] / cells_k) / 1e-6
    out["permeability"] = {"min": float(k_hom.min()), "median": float(np.median(k_hom)),
                           "max": float(k_hom.max()),
                           "all_finite_positive": bool((k_hom > 0).all() and np.isfinite(k_hom).all())}
    # resolved spheres: the geometry of the unit-cell Stokes problem
    log("batched: resolved spheres (solid masks)")
    r_items, r_fields, r_masks, _ = permeability.resolved_cells(256, seed=seed)
    ms_r, cells_r, tot_r, _ = _timed_batch(hlbm, r_items, r_fields, steps, ("graph",), sched, masks=r_masks,
                                           rounds=1)
    log(f"batched resolved graph: {steps} steps in {ms_r['graph']:.0f} ms")
    k_res = nu * (tot_r["graph"][:, 1] / cells_k) / 1e-6
    ratio = k_hom / k_res
    # a fluid cell moves 156 B + its 4-byte link mask; a solid cell loads only
    # its link mask and control (8 B) and stores 19 zeros (76 B)
    solid = sum(int(np.count_nonzero(m)) for m in r_masks) / cells_r
    bytes_r = 160 * (1 - solid) + 84 * solid
    out["resolved"] = {
        "workload": "the same 256 cells with the sphere resolved: solid mask, bounce-back links, d = 0",
        "ms": round(ms_r["graph"], 1), "mlups": round(cells_r * steps / (ms_r["graph"] * 1e-3) / 1e6, 1),
        "solid_fraction": round(solid, 4),
        "alg_bytes_per_cell": round(bytes_r, 1),
        "alg_GBs": round(bytes_r * cells_r * steps / (ms_r["graph"] * 1e-3) / 1e9, 1),
        "permeability": {"min": float(k_res.min()), "median": float(np.median(k_res)), "max": float(k_res.max())},
        "homogenized_over_resolved": {"min": float(ratio.min()), "median": float(np.median(ratio)),
                                      "max": float(ratio.max())},
    }
    return out


def time_permeability_tensor(hlbm, steps=2000, seed=0):
    """All nine components of the transient permeability of the 256 homogenized
    cells: each cell forced along x, y and z (768 items, one batch), k_ij(t) =
    nu <rho u_i>/F_j at five times; the centred spheres' tensors should be
    isotropic."""
    from paper_2310_14746_amd import inputs, permeability
    items, fields, spec = permeability.unit_cells(256, seed=seed)
    times = [steps // 8, steps // 4, steps // 2, 3 * steps // 4, steps]
    import time as _t
    t0 = _t.perf_counter()
    k = permeability.transient_permeability_tensor(hlbm, items, fields, times, mode="graph")
    secs = _t.perf_counter() - t0
    log(f"permeability tensor: 768 items x {steps} steps in {secs:.1f} s")
    kT = k[-1]
    diag = np.stack([kT[:, a, a] for a in range(3)], axis=1)
    off = np.abs(kT - np.einsum("ni,ij->nij", diag, np.eye(3))).max(axis=(1, 2))
    rate = permeability.transient_rate(times, k[:, :, 0, 0])
    return {
        "workload": "256 homogenized unit cells, each forced along x, y and z (768 items), FP32, "
                    f"{steps} steps; k_ij(t) = nu <rho u_i>/F_j",
        "times": times, "seconds": round(secs, 2),
        "k_xx_median": [float(np.median(k[n, :, 0, 0])) for n in range(len(times))],
        "transient_rate_xx_median": [float(np.median(r)) for r in rate],
        "max_rel_diag_spread": float((np.ptp(diag, axis=1) / diag.max(axis=1)).max()),
        "max_rel_offdiag": float((off / diag.max(axis=1)).max()),
    }


REC_BYTES = 4 * 4                          # moment record of one cell and step: 4 FP32 values
ADJ_BYTES_REC = 19 * 4 * 2 + REC_BYTES + 4 + 16  # the reverse step as built: lam in/out, moment record, d, dJ/dd r+w
REC_SWEEP_BYTES = 156 + REC_BYTES          # forward sweep that also writes the moment record
ADJT_BYTES_REC = 19 * 4 * 2 + REC_BYTES + 6 * 4 + 6 * 16  # tensor control: six rows of D and of dJ/dD


def time_gradient(hlbm, steps=500, every=50, seed=0, reps=4, kind="replay"):
    """Differentiation workload: D3Q19 128x64x64 channel, inlet u = 0.02,
    outlet rho = 1, walls in y and z, d ~ U[0,1), FP32 forward and reverse steps / FP64 gradient accumulation,
    500 steps with a checkpoint every 50; gradient of the channel objective
    through torch.autograd (forward with tape, objective, backward).
    kind "replay": the reverse sweep replays each segment from its checkpoint;
    "moments": the forward also records each cell's moments per step, and the
    reverse sweep replays nothing (same gradient bit for bit)."""
    import torch
    from paper_2310_14746_amd import inputs
    from paper_2310_14746_amd.autograd import channel_objective, moments_of_porosity
    shape = (128, 64, 64)
    nx, ny, nz = shape
    cells = nx * ny * nz
    kw = dict(tau=0.6, bc_lo=(2, 1, 1), bc_hi=(3, 1, 1), inlet_u=(0.02, 0, 0), outlet_rho=1.0)
    sim = hlbm.HLBM(19, "f32", shape, **kw)
    try:
        sim.set_tape_kind(kind)
        d = torch.tensor(inputs.uniform_noise((nz, ny, nx), seed), dtype=torch.float64,
                         device=sim.device, requires_grad=True)
        times = []
        for rep in range(max(2, reps)):
            d.grad = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            drho, u = moments_of_porosity(d, sim, steps, every)
            J = channel_objective(drho, u, d, kw["tau"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            J.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if rep:
                times.append((t1 - t0, t2 - t1))
        fwd = float(np.median([a for a, _ in times]))
        bwd = float(np.median([b for _, b in times]))
        grad = d.grad.detach().cpu().numpy()
        # a reverse step reads the 16-byte moment record of its forward step;
        # the replayed tape recomputes the steps below the top two segments
        # from the checkpoints with the recording sweep (156 + 16 bytes per
        # cell), and the forward steps of the top two segments wrote their
        # records themselves
        adj = ADJ_BYTES_REC
        replays = max(0, (steps - 1) // every - 1) * every if kind == "replay" else 0
        moved = cells * (steps * adj + replays * REC_SWEEP_BYTES)
        tape = sim.tape_info()["device_bytes"]
    finally:
        sim.close()
    log(f"gradient ({kind}): forward {fwd * 1e3:.1f} ms, backward {bwd * 1e3:.1f} ms")
    out = {"workload": "D3Q19 128x64x64 channel, inlet u=0.02, outlet rho=1, walls y/z, d~U[0,1) seed 0, "
                       "tau=0.6, 500 steps, checkpoint every 50, FP32 forward and reverse steps / FP64 gradient accumulation, "
                       "J = pressure drop + 0.1 dissipation",
           "tape": kind,
           "forward_ms": round(fwd * 1e3, 2), "backward_ms": round(bwd * 1e3, 2),
           "backward_alg_GBs": round(moved / bwd / 1e9, 1),
           "adjoint_bytes_per_cell_step": adj, "replay_steps": replays,
           "tape_MiB": round(tape / 2 ** 20, 1)}
    return out, grad


def time_tensor(hlbm, steps, warmup, block_x):
    """Anisotropic control at 512^3, FP32: the same sphere array with a fibre
    tensor D = d [0.2 I + 0.8 n n^T], n = (2, 1, 1)/sqrt(6); 19*4*2 + 6*4 = 176
    algorithmic bytes per cell.  Checked against the oracle's 32^3 tile."""
    import oracle
    from paper_2310_14746_amd import inputs
    tile = inputs.round_to(inputs.fiber_tensor_field(inputs.sphere_array_tile()), "f32")
    ms, dr, u, tot, teq = time_form(hlbm, "f32", tile, steps, warmup, block_x=block_x, porosity="tensor")
    cfg = oracle.OracleConfig(q=19, nx=32, ny=32, nz=32, tau=TAU, force=FORCE)
    nt = max(1, min(16, os.cpu_count() or 1))
    g = oracle.run_tensor(cfg, tile, ERROR_STEPS, nthreads=nt)
    dr_o, u_o = oracle.observe(cfg, g, nthreads=nt)
    n_cells = N_EDGE ** 3
    return {"workload": "D3Q19 512^3, sphere array with fibre tensor D = d (0.2 I + 0.8 n n^T), "
                        "n = (2,1,1)/sqrt(6), FP32",
            "mlups": round(n_cells * steps / (ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms / steps, 4),
            "alg_bytes_per_cell": TENSOR_BYTES,
            "alg_GBs": round(TENSOR_BYTES * n_cells * steps / (ms * 1e-3) / 1e9, 1),
            "tiles_identical": teq,
            "error_at_step": ERROR_STEPS,
            "rel_l2_u_vs_fp64": float("%.3e" % rel_l2(u, u_o)),
            "rel_l2_drho_vs_fp64": float("%.3e" % rel_l2_drho(dr, dr_o, u_o))}


def time_adjoint_large(hlbm, edge=256, steps=40, every=10, porosity="scalar", row_pad=None):
    """Reverse sweep on a large periodic box (the sphere array, FP32 forward,
    FP32 adjoint populations, FP64 gradient): time of hlbm_adjoint_step over
    `steps` steps, which also replays the forward inside each checkpoint
    segment.  Shows the adjoint kernel away from the small-domain limits of the
    128x64x64 workload.  porosity="tensor": the fibre tensor of the same array
    (six gradient rows).  row_pad: bytes after each population and adjoint
    row (None: the tuned pad of the FP32 sweep at this shape)."""
    import torch
    from paper_2310_14746_amd import inputs, tune
    if row_pad is None:
        row_pad = tune.lookup_row_pad(hlbm.D3Q19, "f32", (edge,) * 3)
    reps = edge // 32
    tensor = porosity == "tensor"
    if tensor:
        tile = inputs.fiber_tensor_field(inputs.sphere_array_tile()).reshape(6, 32, 32, 32)
        field = np.tile(tile, (1, reps, reps, reps))
    else:
        field = np.tile(inputs.sphere_array_tile(), (reps, reps, reps))
    field = inputs.round_to(field, "f32").astype(np.float32)
    sim = hlbm.HLBM(hlbm.D3Q19, "f32", (edge,) * 3, tau=TAU, force=FORCE, porosity=porosity,
                    row_pad=row_pad)
    try:
        sim.set_porosity(field)
        sim.set_tape(every, steps)
        sim.step(steps)
        n = edge ** 3
        g_r = torch.zeros(n, dtype=torch.float64, device=sim.device)
        g_u = torch.zeros(3 * n, dtype=torch.float64, device=sim.device)
        g_u[:n] = 1.0 / n                               # J = mean u_x
        sim.adjoint(steps, g_r, g_u)                    # warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.adjoint(steps, g_r, g_u)
        e1.record(sim.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
    finally:
        sim.close()
    # every reverse step reads its forward step's 16-byte moment record, which
    # the replay recomputes from the checkpoints with the recording sweep
    replays = steps
    adj, fwd = (ADJT_BYTES_REC, TENSOR_BYTES + REC_BYTES) if tensor else (ADJ_BYTES_REC, REC_SWEEP_BYTES)
    moved = edge ** 3 * (steps * adj + replays * fwd)
    what = "periodic sphere array with the fibre tensor" if tensor else "periodic sphere array"
    return {"workload": f"D3Q19 {edge}^3 {what}, {steps} reverse steps, checkpoint every {every}",
            "ms": round(ms, 2), "ms_per_reverse_step": round(ms / steps, 4),
            "alg_GBs": round(moved / (ms * 1e-3) / 1e9, 1), "replay_steps": replays,
            "row_pad_bytes": row_pad}


def time_c1(hlbm, block_x):
    """The same FP32 sweep on the 256^3 box (8^3 sphere cells), 1000 steps."""
    from paper_2310_14746_amd import inputs
    steps = 1000
    tile = inputs.round_to(inputs.sphere_array_tile(), "f32")
    ms, _, _, _, teq = time_form(hlbm, "f32", tile, steps, 20, block_x=block_x, edge=256, error_steps=None)
    n_cells = 256 ** 3
    return {"workload": "D3Q19 256^3 periodic, 8^3 sphere array, tau=0.6, F=1e-6 x, FP32, 1000 steps",
            "mlups": round(n_cells * steps / (ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms / steps, 4),
            "alg_GBs": round(156 * n_cells * steps / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round(156 * n_cells * steps / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "tiles_identical": teq}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo; None where that is absent)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(steps_total=ERROR_STEPS):
    """Oracle on a 128^3 crop (4^3 obstacle cells; exact by periodicity) -> MLUPS.
    About 1.05e9 cell updates at 500 steps: 10-30 s on the host's cores.  Its
    final moments are the FP64 reference of the 512^3 forms at that step."""
    import oracle
    from paper_2310_14746_amd import inputs
    nt = max(1, min(16, os.cpu_count() or 1))
    n = 128
    d = inputs.round_to(inputs.sphere_array(n), "f32").ravel()
    cfg = oracle.OracleConfig(q=19, nx=n, ny=n, nz=n, tau=TAU, force=FORCE)
    log(f"oracle: {n}^3 x {steps_total} steps on {nt} threads")
    t0 = time.perf_counter()
    g = oracle.run(cfg, d, steps_total, nthreads=nt)
    secs = time.perf_counter() - t0
    dr, u = oracle.observe(cfg, g, nthreads=nt)
    dr = dr.reshape(n, n, n)[:32, :32, :32].ravel()
    u = u.reshape(3, n, n, n)[:, :32, :32, :32].reshape(3, -1)
    # one host thread, on the 32^3 cell (exact by periodicity)
    cfg1 = oracle.OracleConfig(q=19, nx=32, ny=32, nz=32, tau=TAU, force=FORCE)
    d1 = d.reshape(n, n, n)[:32, :32, :32].ravel().copy()
    steps1 = 400
    t1 = time.perf_counter()
    oracle.run(cfg1, d1, steps1, nthreads=1)
    secs1 = time.perf_counter() - t1
    return {
        "value": n ** 3 * steps_total / secs / 1e6,
        "unit": "MLUPS",
        "cores": nt,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"FP64 oracle, {n}^3 periodic crop of the same workload ({n // 32}^3 obstacle cells, "
                  f"exact by 32-periodicity), {steps_total} steps, {secs:.1f} s",
        "single_thread": {"value": round(32 ** 3 * steps1 / secs1 / 1e6, 2), "unit": "MLUPS", "cores": 1,
                          "sample": f"32^3 cell, {steps1} steps, {secs1:.1f} s"},
    }, dr, u


def oracle_tile(d_tile, steps):
    """FP64 oracle on one 32^3 obstacle cell (untimed reference for an input rounding)."""
    import oracle
    nt = max(1, min(16, os.cpu_count() or 1))
    cfg = oracle.OracleConfig(q=19, nx=32, ny=32, nz=32, tau=TAU, force=FORCE)
    g = oracle.run(cfg, d_tile.ravel(), steps, nthreads=nt)
    return oracle.observe(cfg, g, nthreads=nt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="f32,f16s,bf16s,f32-aa,f16s-aa")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-reference", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--no-tensor", action="store_true")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--no-adjoint-large", action="store_true")
    ap.add_argument("--no-permeability-tensor", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000,
                    help="steps of the batched workload (2000 is the workload; fewer for profiling runs)")
    ap.add_argument("--gradient-reps", type=int, default=4,
                    help="forward+backward repetitions of the gradient workload (the first is untimed)")
    ap.add_argument("--block-x", type=int, default=-1,
                    help="threads per block along x (-1: tuned value, 0: library default)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the sweep's HBM traffic record from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-counters-all", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="per-kernel HBM traffic against algorithmic bytes from two rocprofv3 --pmc runs "
                         "(the batched step count of those runs: --batched-steps)")
    ap.add_argument("--summarize-backward", metavar="DIR",
                    help="timeline of the last replayed backward pass in a rocprofv3 kernel trace, then exit")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print a per-kernel summary of a rocprofv3 kernel trace and exit")
    args = ap.parse_args()
    if args.summarize_profile:
        print(summarize_profile(args.summarize_profile))
        return
    if args.summarize_backward:
        print(summarize_backward(args.summarize_backward))
        return
    if args.summarize_counters:
        print(summarize_counters(*args.summarize_counters))
        return
    if args.summarize_counters_all:
        print(summarize_counters_all(*args.summarize_counters_all, args.batched_steps))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_14746_amd import hlbm, inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    hlbm.load()
    d_tile = inputs.sphere_array_tile()
    n_cells = N_EDGE ** 3
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    from paper_2310_14746_amd import tune
    for f in forms:
        st, pattern = storage_of(f), ("aa" if f.endswith("-aa") else "ab")
        tile = inputs.round_to(d_tile, "f32" if st == "f32" else "f16")
        bx = args.block_x if args.block_x >= 0 else tune.lookup(hlbm.D3Q19, st, (N_EDGE,) * 3, pattern)
        rp = tune.lookup_row_pad(hlbm.D3Q19, st, (N_EDGE,) * 3, pattern)
        ms, dr, u, tot, teq = time_form(hlbm, st, tile, args.steps, args.warmup, block_x=bx, pattern=pattern,
                                        row_pad=rp)
        results[f] = dict(ms=ms, dr=dr, u=u, tot=tot, tiles_equal=teq, block_x=bx, row_pad=rp)
    copy_ref = None if args.no_copy_reference else copy_reference()
    pattern = None
    if not args.no_copy_reference and storage_of(forms[0]) == "f32":
        pattern = pattern_reference(hlbm, results[forms[0]]["block_x"] or 256, results[forms[0]]["row_pad"])
        log(f"pattern reference: {pattern['ms']:.4f} ms, {pattern['GBs']:.0f} GB/s")
    batched = None if args.no_batched else time_batched(hlbm, steps=args.batched_steps)
    if batched is not None and not args.no_permeability_tensor:
        batched["permeability_tensor"] = time_permeability_tensor(hlbm, steps=args.batched_steps)
    gradient = None
    if not args.no_gradient:
        gradient, g_replay = time_gradient(hlbm, reps=args.gradient_reps)
        rec, g_rec = time_gradient(hlbm, reps=args.gradient_reps, kind="moments")
        rec["gradient_equals_replay_bitwise"] = bool(np.array_equal(g_rec, g_replay))
        gradient["moment_record"] = rec
    if gradient is not None and not args.no_adjoint_large:
        gradient["large_periodic"] = time_adjoint_large(hlbm)
        gradient["large_periodic_tensor"] = time_adjoint_large(hlbm, porosity="tensor")
    c1 = None if args.no_c1 else time_c1(hlbm, tune.lookup(hlbm.D3Q19, "f32", (256,) * 3))
    tensor = None if args.no_tensor else time_tensor(
        hlbm, args.steps, args.warmup, args.block_x if args.block_x >= 0 else tune.lookup(hlbm.D3Q19, "f32", (N_EDGE,) * 3))

    cpu, refs = None, {}
    if not args.no_cpu_baseline:
        cpu, dr_o, u_o = cpu_baseline(ERROR_STEPS)
        refs["f32"] = (dr_o, u_o)
        if any(storage_of(f) != "f32" for f in forms):
            refs["f16"] = oracle_tile(inputs.round_to(d_tile, "f16"), ERROR_STEPS)

    head = forms[0]
    if head.endswith("-aa"):
        raise SystemExit("the first form is the headline and must be a two-buffer form")
    ms_step = results[head]["ms"] / args.steps
    mlups = n_cells * args.steps / (results[head]["ms"] * 1e-3) / 1e6
    achieved = ALG_BYTES[head] * n_cells / (ms_step * 1e-3) / 1e9
    traffic = counters_traffic(n_cells) if head == "f32" else None
    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D3Q19 HLBM {N_EDGE}^3 periodic, 16^3 sphere array (r=10, edge 32, "
                        f"sigma=2), tau={TAU}, F=1e-6 x, {head} storage, A/B buffers",
            "cells": n_cells,
            "storage": head,
            "block_x": results[head]["block_x"],
            "row_pad_bytes": results[head]["row_pad"],
            "parallelism": "1 GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_cell": ALG_BYTES[head],
            "copy_reference_GBs": copy_ref["GBs"] if copy_ref else None,
            "copy_reference": copy_ref,
            "frac_of_copy": round(achieved / copy_ref["GBs"], 4) if copy_ref else None,
            "pattern_reference": pattern,
            "frac_of_pattern": round(achieved / pattern["GBs"], 4) if pattern else None,
        },
        "cpu_baseline": cpu,
        "forms": {},
        "batched": batched,
        "gradient": gradient,
        "tensor_control": tensor,
        "c1_256": c1,
    }
    for f in forms:
        r = results[f]
        ent = {
            "mlups": round(n_cells * args.steps / (r["ms"] * 1e-3) / 1e6, 1),
            "ms_per_step": round(r["ms"] / args.steps, 4),
            "alg_GBs": round(ALG_BYTES[storage_of(f)] * n_cells * args.steps / (r["ms"] * 1e-3) / 1e9, 1),
            "speedup_vs_" + head: round(results[head]["ms"] / r["ms"], 3),
            "tiles_identical": r["tiles_equal"],
            "block_x": r["block_x"],
            "row_pad_bytes": r["row_pad"],
            "ms_per_step_parts": [round(v, 4) for v in
                                  TIMING_PARTS.get((storage_of(f), "aa" if f.endswith("-aa") else "ab", "scalar",
                                                    N_EDGE), [])],
            "mass_excess_total": float(r["tot"][0]),
        }
        if f.endswith("-aa") and storage_of(f) in results:
            twin = results[storage_of(f)]
            ent["pattern"] = "in-place (AA), one population buffer"
            # per-cell moments; the FP64 totals sum per-block partials, so they
            # are compared only at the same block width
            same = np.array_equal(r["u"], twin["u"]) and np.array_equal(r["dr"], twin["dr"])
            if r["block_x"] == twin["block_x"]:
                same = same and np.array_equal(r["tot"], twin["tot"])
            ent["equals_two_buffer_bitwise"] = bool(same)
        ref = refs.get("f32" if storage_of(f) == "f32" else "f16")
        if ref is not None:
            eu, er = rel_l2(r["u"], ref[1]), rel_l2_drho(r["dr"], ref[0], ref[1])
            tol = STATED_TOLERANCE[storage_of(f)]
            ent["error_at_step"] = ERROR_STEPS
            ent["rel_l2_u_vs_fp64"] = float("%.3e" % eu)
            ent["rel_l2_drho_vs_fp64"] = float("%.3e" % er)
            ent["stated_tolerance"] = tol
            ent["meets_stated_tolerance"] = {"u": bool(eu <= tol), "drho": bool(er <= tol)}
        line["forms"][f] = ent
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
