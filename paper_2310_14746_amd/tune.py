"""Block-shape and row-pad autotuner for the sweep.

For a lattice, storage form and box shape, every candidate number of threads
per block along x (multiples of 64 up to 1024) is timed through the C-ABI with
HIP events on the sweep's own stream; the fastest is stored in
``tuning.json`` beside this file, keyed by GPU architecture, lattice, storage
(suffixed "-aa" for the in-place pattern, whose kernels take at most 256
threads per block) and shape.  :func:`lookup` returns the stored value
(0 = library default).

The padding after each population row (hlbm_config.row_pad_bytes) decides
how the 19 read and 19 write streams of the sweep fall on the HBM channels.
Its effect depends on where the allocator places the buffers, so each
candidate pad is timed over several fresh allocations, interleaved with the
other candidates, and the lowest mean wins (``--row-pad``);
:func:`lookup_row_pad` returns it (0 = dense rows).

For a batch of periodic boxes it times the persistent kernel's schedule in
graph mode -- tile size (cells per tile = threads per block), resident blocks
per CU and tiles per draw -- over every combination that fits, and stores the
fastest under a key naming the storage and the batch's item shapes;
:func:`lookup_batch` returns it (None = library defaults).

Run on the target GPU:  python -m paper_2310_14746_amd.tune --shape 512 512 512
                        python -m paper_2310_14746_amd.tune --shape 512 512 512 --row-pad
                        python -m paper_2310_14746_amd.tune --batch 256
"""
from __future__ import annotations

import argparse
import json
import os

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
ARCH = "gfx950"
CANDIDATES = (64, 128, 192, 256, 320, 384, 512, 768, 1024)


def _key(lattice: int, storage: str, shape, pattern: str = "ab") -> str:
    lat = "D3Q19" if lattice == 19 else "D2Q9"
    form = storage + ("-aa" if pattern == "aa" else "")
    return f"{ARCH}/{lat}/{form}/" + "x".join(str(int(v)) for v in shape)


ROW_PADS = (0, 4352, 8448, 16640, 65792)   # bytes, multiples of 256
BATCH_TILES = (128, 256, 512)
BATCH_CHUNKS = (1, 2, 4)


def _batch_key(storage: str, items) -> str:
    import hashlib
    shapes = [[int(v) for v in it["shape"]] for it in items]
    cells = sum(a * b * c for a, b, c in shapes)
    sig = hashlib.sha1(json.dumps(shapes).encode()).hexdigest()[:12]
    return f"{ARCH}/batch/D3Q19/{storage}/{len(items)}items-{cells}cells-{sig}"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(lattice: int, storage: str, shape, pattern: str = "ab") -> int:
    """Tuned threads per block along x for this case, or 0 (library default)."""
    ent = load_cache().get(_key(lattice, storage, shape, pattern))
    return int(ent["block_x"]) if ent else 0


def lookup_row_pad(lattice: int, storage: str, shape, pattern: str = "ab") -> int:
    """Tuned padding in bytes after each population row for this case, or 0."""
    ent = load_cache().get(_key(lattice, storage, shape, pattern))
    return int(ent.get("row_pad", 0)) if ent else 0


def lookup_batch(items, storage: str = "f32"):
    """Tuned {tile, blocks_per_cu, chunk} for this batch, or None (library defaults)."""
    ent = load_cache().get(_batch_key(storage, items))
    if not ent:
        return None
    return {k: int(ent[k]) for k in ("tile", "blocks_per_cu", "chunk")}


def _time_graph(b, steps):
    import torch
    b.step(2)
    b.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    b.sync()
    return e0.elapsed_time(e1) / steps


def tune_batch(items, storage="f32", steps=40, tiles=BATCH_TILES, chunks=BATCH_CHUNKS, write=True, out=CACHE):
    """Time every (tile, blocks_per_cu, chunk) of the persistent kernel, launched
    from a graph, on this batch (porosity 0.1 everywhere: the sweep does the
    same work whatever the values) and store the fastest.  The tile is also the
    block of the per-step kernel."""
    import numpy as np
    from . import hlbm
    hlbm.load()
    scale = 2.0 ** 24 if storage in ("f16s", "bf16s") else 1.0
    dt = {"f64": np.float64, "f32": np.float32}.get(storage, np.float16)
    times = {}
    for tile in tiles:
        b = hlbm.HLBMBatch(items, storage, store_scale=scale, mode="graph_persistent", tile=tile)
        try:
            for k, it in enumerate(items):
                nx, ny, nz = it["shape"]
                b.set_porosity(k, np.full(nx * ny * nz, 0.1, dtype=dt))
            mx = b.schedule()["max_blocks_per_cu"]
            for bpc in range(1, mx + 1):
                for ch in chunks:
                    b.set_schedule(bpc, ch)
                    times[(tile, bpc, ch)] = _time_graph(b, steps)
                    print(f"[tune] batch {storage} tile={tile} blocks_per_cu={bpc} chunk={ch}: "
                          f"{times[(tile, bpc, ch)]:.4f} ms/step", flush=True)
        finally:
            b.close()
    best = min(times, key=times.get)
    ent = {"tile": best[0], "blocks_per_cu": best[1], "chunk": best[2], "ms_per_step": round(times[best], 4),
           "candidates": {f"{t}/{b}/{c}": round(v, 4) for (t, b, c), v in times.items()}}
    if write:
        cache = load_cache()
        if out != CACHE and os.path.exists(out):
            with open(out) as f:
                cache.update(json.load(f))
        cache[_batch_key(storage, items)] = ent
        with open(out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return ent


def time_block(hlbm, lattice, storage, shape, block_x, steps, warmup, pattern="ab", row_pad=0):
    import numpy as np
    import torch
    sim = hlbm.HLBM(lattice, storage, shape, tau=0.6, force=(1e-6, 0, 0),
                    store_scale=2.0 ** 24 if storage in ("f16s", "bf16s") else 1.0,
                    block_x=block_x, pattern=pattern, row_pad=row_pad)
    try:
        n = shape[0] * shape[1] * shape[2]
        dt = {"f64": np.float64, "f32": np.float32}.get(storage, np.float16)
        sim.set_porosity(np.full(n, 0.1, dtype=dt))
        sim.step(warmup)
        sim.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps
    finally:
        sim.close()


def tune(lattice, storage, shape, steps=20, warmup=5, write=True, out=CACHE, pattern="ab", reps=1):
    """Time every block width at the stored row pad, over `reps` fresh
    allocations (the widths interleaved within each repetition); keep the
    lowest mean."""
    import statistics
    from . import hlbm
    hlbm.load()
    nx = shape[0]
    cap = 256 if pattern == "aa" else 1024
    cands = [b for b in CANDIDATES if b <= min(cap, max(64, ((nx + 63) // 64) * 64))]
    pad = lookup_row_pad(lattice, storage, shape, pattern)
    runs = {b: [] for b in cands}
    for r in range(reps):
        for b in cands:
            t = time_block(hlbm, lattice, storage, shape, b, steps, warmup, pattern, row_pad=pad)
            runs[b].append(t)
            print(f"[tune] {storage} {shape} row_pad={pad} block_x={b} rep {r}: {t:.4f} ms/step", flush=True)
    times = {b: statistics.mean(v) for b, v in runs.items()}
    best = min(times, key=times.get)
    ent = {"block_x": best, "ms_per_step": round(times[best], 4),
           "candidates": {str(k): round(v, 4) for k, v in times.items()}}
    if write:
        cache = load_cache()
        if out != CACHE and os.path.exists(out):
            with open(out) as f:
                cache.update(json.load(f))
        old = cache.get(_key(lattice, storage, shape, pattern), {})
        ent.update({k: v for k, v in old.items() if k.startswith("row_pad")})
        cache[_key(lattice, storage, shape, pattern)] = ent
        with open(out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return ent


def tune_row_pad(lattice, storage, shape, pattern="ab", reps=6, steps=20, warmup=5, pads=ROW_PADS,
                 write=True, out=CACHE):
    """Mean time per step of each candidate pad over `reps` fresh allocations
    (the candidates interleaved within each repetition), at the tuned block
    width; the lowest mean is stored beside the block width."""
    import statistics
    import torch
    from . import hlbm
    hlbm.load()
    key = _key(lattice, storage, shape, pattern)
    bx = lookup(lattice, storage, shape, pattern)
    times = {pad: [] for pad in pads}
    for r in range(reps):
        # a differently sized allocation shifts where the buffers land
        shift = torch.empty((r * 37 + 1) << 20, dtype=torch.uint8, device="cuda")
        for pad in pads:
            t = time_block(hlbm, lattice, storage, shape, bx, steps, warmup, pattern, row_pad=pad)
            times[pad].append(t)
            print(f"[tune] {storage} {shape} {pattern} block_x={bx} row_pad={pad} rep {r}: {t:.4f} ms/step",
                  flush=True)
        del shift
        torch.cuda.empty_cache()
    means = {pad: statistics.mean(v) for pad, v in times.items()}
    best = min(means, key=means.get)
    res = {"row_pad": best, "row_pad_ms_per_step": round(means[best], 4),
           "row_pad_candidates": {str(k): round(v, 4) for k, v in means.items()}}
    if write:
        cache = load_cache()
        if out != CACHE and os.path.exists(out):
            with open(out) as f:
                cache.update(json.load(f))
        ent = cache.get(key, {"block_x": bx})
        ent.update(res)
        cache[key] = ent
        with open(out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", type=int, nargs=3, default=(512, 512, 512))
    ap.add_argument("--storage", default="f32,f16s,bf16s")
    ap.add_argument("--lattice", type=int, default=19)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--pattern", default="ab", choices=("ab", "aa"))
    ap.add_argument("--batch", type=int, default=0,
                    help="tune the batched kernel on this many homogenized unit cells instead")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--row-pad", action="store_true",
                    help="tune the population row pad at the stored block width instead")
    ap.add_argument("--reps", type=int, default=None,
                    help="fresh allocations per candidate (default: 6 for --row-pad, 1 for block widths)")
    ap.add_argument("--out", default=CACHE, help="cache file to write (default: the package's)")
    a = ap.parse_args()
    if a.batch:
        from . import inputs
        spec = inputs.batch_items(a.batch, seed=a.seed)
        items = [dict(shape=(e, e, e), tau=t, force=(1e-6, 0.0, 0.0)) for e, _, t in spec]
        for st in a.storage.split(","):
            ent = tune_batch(items, st, steps=a.steps, out=a.out)
            print(json.dumps({"batch": a.batch, "storage": st, **{k: ent[k] for k in ("tile", "blocks_per_cu",
                                                                                     "chunk", "ms_per_step")}}),
                  flush=True)
        return
    for st in a.storage.split(","):
        if a.row_pad:
            ent = tune_row_pad(a.lattice, st, tuple(a.shape), a.pattern, reps=a.reps or 6, steps=a.steps, out=a.out)
        else:
            ent = tune(a.lattice, st, tuple(a.shape), steps=a.steps, out=a.out, pattern=a.pattern, reps=a.reps or 1)
        print(json.dumps({"storage": st, "pattern": a.pattern, **ent}), flush=True)


if __name__ == "__main__":
    main()
