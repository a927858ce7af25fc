"""Autotuner for the per-orbital-count launch shape (kubo_tile).

For each orbital count n it times the per-k kernel on a representative model
and keeps the fastest of:
  * threads: 64 (one wavefront per k-point, n <= 32 only) or 256 (one workgroup),
  * k_block: the number of consecutive k-points of a pencil one work item holds.
The sample is a plan of several copies of the model on its full grid (eight
32^3 grids by default, as in a batched plan), so every candidate launches many
times more work items than the GPU holds at once and the timing is the steady
state rather than how well a small sample fills the GPU.  Timing uses the
library's own event records (KUBO_F_TIMING) around the per-k kernel launches.
Results go to a JSON cache keyed by device name and n, which Plan consults when
no tiles are given.

    python -m paper_2309_06675_amd.autotune --ns 8,12,16,...,64 --n-R 125 --nf 16
"""

from __future__ import annotations

import argparse
import json
import os
import time
from typing import Dict, Iterable, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned_tiles.json")


def _device_key() -> str:
    import torch

    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load_cache(path: str = CACHE) -> Dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(ns: Iterable[int], path: str = CACHE, device: Optional[str] = None) -> List[Tuple]:
    """Cached (n, threads, k_block) tiles for the given orbital counts (missing n skipped)."""
    cache = load_cache(path)
    if not cache:
        return []
    if device is None:
        try:
            device = _device_key()
        except Exception:
            return []
    table = cache.get(device, {})
    out = []
    for n in sorted(set(int(x) for x in ns)):
        e = table.get(str(n))
        if e:
            out.append((n, int(e["threads"]), int(e["k_block"])))
    return out


def tune_one(n: int, L: int = 2, lam: float = 1.0, grid=(32, 32, 32), nf: int = 16,
             eta: float = 1e-3, kT: float = 0.0, copies: int = 8,
             k_blocks=(8, 16, 32), reps: int = 3, seed: int = 777) -> Dict:
    """Time every candidate shape for orbital count n; returns the best and all timings."""
    import torch

    from . import kubo, synth

    m = synth.random_model(n, L, lam, seed + n)
    models = [m] * copies
    t = kubo.to_device_t(models)
    ef = torch.linspace(-3.0, 3.0, nf, dtype=torch.float64, device="cuda").reshape(1, nf)
    ef = ef.repeat(copies, 1).contiguous()
    threads = (64, 256) if n <= 32 else (256,)
    results = []
    for th in threads:
        for kb in k_blocks:
            kb = min(kb, grid[0])
            plan = kubo.Plan(models, grid=grid, n_fermi=nf,
                             flags=kubo.KUBO_F_TIMING | kubo.KUBO_F_FORWARD_ONLY,
                             tiles=[(n, th, kb)])
            plan.forward(t, ef, eta, kT)  # warm-up (also uploads the tables)
            torch.cuda.synchronize()
            plan.kernel_time(0, reset=True)
            for _ in range(reps):
                plan.forward(t, ef, eta, kT)
            ms, launches, kpts = plan.kernel_time(0)
            results.append({"threads": th, "k_block": kb, "ms": ms / reps,
                            "k_points_per_s": kpts / (ms / 1e3), "items_k_points": kpts // reps})
            del plan
    best = min(results, key=lambda r: r["ms"])
    return {"threads": best["threads"], "k_block": best["k_block"],
            "k_points_per_s": best["k_points_per_s"], "candidates": results}


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune kubo_tile per orbital count")
    ap.add_argument("--ns", default="8,12,16,20,24,28,32,36,40,44,48,52,56,60,64")
    ap.add_argument("--L", type=int, default=2)
    ap.add_argument("--nf", type=int, default=16)
    ap.add_argument("--kT", type=float, default=0.0)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args(argv)
    dev = _device_key()
    cache = load_cache(args.out)
    table = cache.setdefault(dev, {})
    for n in [int(x) for x in args.ns.split(",")]:
        t0 = time.time()
        res = tune_one(n, L=args.L, nf=args.nf, kT=args.kT)
        table[str(n)] = res
        print(f"n={n}: threads={res['threads']} k_block={res['k_block']} "
              f"{res['k_points_per_s']:.3e} k/s ({time.time() - t0:.1f} s)", flush=True)
    with open(args.out, "w") as f:
        json.dump(cache, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
