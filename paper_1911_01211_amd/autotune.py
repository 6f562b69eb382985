"""Autotuner of the history-sum term chunks (cntr_set_tiles).

For each tunable orbital count (d = 1: the batched one-block-per-lane path,
d = 8: the MFMA path) and each band of slices, the candidates are timed on
the device: one time step at the band's representative slice of a batch
with the shape of the workload that uses that path (zero-filled histories:
the kernels' speed does not depend on the values), best of several
launches, HIP events on the launch stream. The winners form a table of
bands, applied through cntr_set_tiles and kept in tune_cache.json beside
this file, which apply_cache() loads.

    python -m paper_1911_01211_amd.autotune --write     # on an MI355X
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")

# candidates per d and the workload each path serves: (count, ntau, slices)
SPACE = {
    1: dict(candidates=[64, 128, 256], count=512, ntau=500, slices=[256, 1024, 2000]),
    8: dict(candidates=[16, 32, 64], count=1, ntau=400, slices=[256, 1024, 1500]),
}


def set_tiles(d: int, n_hi: list, tj: list):
    from . import _abi
    nb = len(tj)
    a = (C.c_int32 * max(nb, 1))(*n_hi) if nb else None
    b = (C.c_int32 * max(nb, 1))(*tj) if nb else None
    _abi.check(_abi.lib().cntr_set_tiles(int(d), nb, a, b))


def bands_from(slices: list, best: list):
    """Band edges halfway between the measured slices; the last band is open."""
    n_hi = [(slices[i] + slices[i + 1]) // 2 for i in range(len(slices) - 1)] + [1 << 30]
    # merge neighbours with the same chunk
    e, t = [], []
    for h, c in zip(n_hi, best):
        if t and t[-1] == c:
            e[-1] = h
        else:
            e.append(h)
            t.append(c)
    return e, t


def _batch(d: int, count: int, ntau: int, n: int):
    """`count` zero-filled problems of one grid with slice n last (one shared Sigma)."""
    import torch

    from . import contour as K
    from .workloads import GridSpec
    g = GridSpec(nt=n, ntau=ntau, d=d, sig=-1, k=5, beta=10.0, h=0.02, mu=0.0)
    G = [K.Contour(g, "cuda") for _ in range(count)]
    S = K.Contour(g, "cuda")
    e = torch.zeros((n + 2, d, d), dtype=torch.complex128, device="cuda")
    return K.Batch(G, [S] * count, [e] * count)


def time_step(B, n: int, reps: int = 5) -> float:
    """ms of one time step at slice n of the batch B, best of reps."""
    import torch
    B.step(n)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B.step(n)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def tune(d: int, log=print) -> dict:
    import torch
    sp = SPACE[d]
    best, times = [], {}
    for n in sp["slices"]:
        B = _batch(d, sp["count"], sp["ntau"], n)
        row = {}
        for tj in sp["candidates"]:
            set_tiles(d, [1 << 30], [tj])
            row[tj] = time_step(B, n)
            log(f"# tune d={d} n={n} chunk={tj}: {row[tj]:.3f} ms")
        del B
        torch.cuda.empty_cache()
        times[n] = row
        best.append(min(row, key=row.get))
    n_hi, tj = bands_from(sp["slices"], best)
    set_tiles(d, n_hi, tj)
    return {"n_hi": n_hi, "tj": tj, "times_ms": {str(n): {str(c): v for c, v in r.items()} for n, r in times.items()},
            "workload": {"count": sp["count"], "ntau": sp["ntau"]}}


def apply_cache(path: str = CACHE) -> dict | None:
    """Load the cached table (if any) into the library; returns it."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    for d, ent in cache.get("entries", {}).items():
        set_tiles(int(d), ent["n_hi"], ent["tj"])
    return cache


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true", help="write tune_cache.json")
    ap.add_argument("--out", default=CACHE, help="where --write puts the table")
    ap.add_argument("--d", type=int, nargs="*", default=sorted(SPACE))
    args = ap.parse_args()
    import torch
    entries = {}
    for d in args.d:
        entries[str(d)] = tune(d, log=lambda s: print(s, file=sys.stderr, flush=True))
    cache = {"device": torch.cuda.get_device_name(0), "entries": entries}
    print(json.dumps(cache), flush=True)
    if args.write:
        with open(args.out, "w") as f:
            json.dump(cache, f, indent=1)


if __name__ == "__main__":
    main()
