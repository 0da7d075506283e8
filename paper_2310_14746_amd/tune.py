"""Block-shape autotuner for the sweep.

For a lattice, storage form and box shape, every candidate number of threads
per block along x (multiples of 64 up to 1024) is timed through the C-ABI with
HIP events on the sweep's own stream; the fastest is stored in
``tuning.json`` beside this file, keyed by GPU architecture, lattice, storage
and shape.  :func:`lookup` returns the stored value (0 = library default).

Run on the target GPU:  python -m paper_2310_14746_amd.tune --shape 512 512 512
"""
from __future__ import annotations

import argparse
import json
import os

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
ARCH = "gfx950"
CANDIDATES = (64, 128, 192, 256, 320, 384, 512, 768, 1024)


def _key(lattice: int, storage: str, shape) -> str:
    lat = "D3Q19" if lattice == 19 else "D2Q9"
    return f"{ARCH}/{lat}/{storage}/" + "x".join(str(int(v)) for v in shape)


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(lattice: int, storage: str, shape) -> int:
    """Tuned threads per block along x for this case, or 0 (library default)."""
    ent = load_cache().get(_key(lattice, storage, shape))
    return int(ent["block_x"]) if ent else 0


def time_block(hlbm, lattice, storage, shape, block_x, steps, warmup):
    import numpy as np
    import torch
    sim = hlbm.HLBM(lattice, storage, shape, tau=0.6, force=(1e-6, 0, 0),
                    store_scale=2.0 ** 24 if storage in ("f16s", "bf16s") else 1.0,
                    block_x=block_x)
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


def tune(lattice, storage, shape, steps=20, warmup=5, write=True, out=CACHE):
    from . import hlbm
    hlbm.load()
    nx = shape[0]
    cands = [b for b in CANDIDATES if b <= max(64, ((nx + 63) // 64) * 64)]
    times = {}
    for b in cands:
        times[b] = time_block(hlbm, lattice, storage, shape, b, steps, warmup)
        print(f"[tune] {storage} {shape} block_x={b}: {times[b]:.4f} ms/step", flush=True)
    best = min(times, key=times.get)
    ent = {"block_x": best, "ms_per_step": round(times[best], 4),
           "candidates": {str(k): round(v, 4) for k, v in times.items()}}
    if write:
        cache = load_cache()
        if out != CACHE and os.path.exists(out):
            with open(out) as f:
                cache.update(json.load(f))
        cache[_key(lattice, storage, shape)] = ent
        with open(out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return ent


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", type=int, nargs=3, default=(512, 512, 512))
    ap.add_argument("--storage", default="f32,f16s,bf16s")
    ap.add_argument("--lattice", type=int, default=19)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--out", default=CACHE, help="cache file to write (default: the package's)")
    a = ap.parse_args()
    for st in a.storage.split(","):
        ent = tune(a.lattice, st, tuple(a.shape), steps=a.steps, out=a.out)
        print(json.dumps({"storage": st, **ent}), flush=True)


if __name__ == "__main__":
    main()
