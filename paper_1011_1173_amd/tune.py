"""Autotuner of the batched launch plans.

A batch runs under one of two schedules (one persistent launch taking owner
items from a counter, or one launch per block step), and the persistent
launch has a shape: how many workgroups, in which order they take the items
(block-major or factor-major) and how long owners far from the chain sleep
between polls.  The best choice depends on the sizes in the batch, so the
library looks the plan up in a table indexed by the batch's dominant
(storage type, n bucket, k bucket) (include/cholmod_mi355x.h,
cholmod_set_plan).

This module fills that table by measurement: for every bucket it builds a
synthetic batch of factors whose sizes lie in the bucket (the SPD generator
of inputs.py), times every candidate plan on the GPU (an update by V and the
matching downdate per timed pair, HIP events on one stream, median of
`reps` pairs), checks that every candidate leaves each factor bit for bit
where the default plan leaves it, and writes the fastest plan of each bucket
to a JSON plan cache.  ``load_plans`` reads such a cache into the library;
the package does so once, before its first batched call, from the cache
shipped for the device's architecture (plans/<arch>.json) when it exists.

Usage on a GPU:  python -m paper_1011_1173_amd.tune --out paper_1011_1173_amd/plans/gfx950.json
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import random
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
PLAN_DIR = os.path.join(HERE, "plans")

# sizes of the synthetic batch of each n bucket: (n range, factors)
N_BUCKET_RANGES = {0: ((64, 256), 192), 1: ((257, 1024), 96), 2: ((1025, 4096), 32),
                   3: ((4097, 16384), 6)}
K_BUCKET_RANGES = {0: (1, 16), 1: (17, 32), 2: (33, 64)}


def candidates(cus: int):
    """The plans tried in every bucket (as dicts of cholmod_plan fields): the
    queued schedule with block maps, the library's default first, with other
    grids, item orders and poll levels.  All of them give every factor the
    single-factor default's result bit for bit (checked), so the table's
    choice never changes a result; the stepped schedule and plans without
    maps, which give the rotation-by-rotation result, are not candidates."""
    out = [{"schedule": 0, "grid": 0, "order": 0, "poll": 2, "maps": 1}]
    for grid in sorted({0, max(1, (3 * cus) // 4), max(1, cus // 2)}):
        for order in (0, 1):
            for poll in (0, 2):
                c = {"schedule": 0, "grid": grid, "order": order, "poll": poll, "maps": 1}
                if c != out[0]:
                    out.append(c)
    return out


def _plan(d):
    from . import _native
    return _native.Plan(int(d["schedule"]), int(d["grid"]), int(d["order"]), int(d["poll"]),
                        int(d.get("maps", 1)))


def arch_name() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # no GPU, or a torch without the attribute
        return "gfx950"


def default_cache() -> str:
    return os.path.join(PLAN_DIR, arch_name() + ".json")


def load_plans(path: str | None = None) -> int:
    """Set the library's plan table from a plan cache; returns the number of
    entries set (0 if the file does not exist)."""
    from . import _native
    path = path or default_cache()
    if not os.path.exists(path):
        return 0
    data = json.load(open(path))
    lib = _native.load()
    nset = 0
    for e in data.get("entries", []):
        p = _plan(e["plan"])
        st = lib.cholmod_set_plan(int(e["dtype"]), int(e["n_bucket"]), int(e["k_bucket"]),
                                  ctypes.byref(p))
        if st != _native.OK:
            raise ValueError("plan cache entry rejected by the library: %r" % (e,))
        nset += 1
    return nset


def _batch(nb: int, kb: int, f32: bool, seed: int):
    import torch
    from . import inputs
    (lo, hi), count = N_BUCKET_RANGES[nb]
    klo, khi = K_BUCKET_RANGES[kb]
    rng = random.Random(seed)
    dt = torch.float32 if f32 else torch.float64
    Ls, Vs = [], []
    for f in range(count):
        n = rng.randint(lo, hi)
        k = rng.randint(klo, khi)
        Ls.append(inputs.spd_factor(n, seed * 1000 + f, device="cuda").to(dt))
        Vs.append(inputs.update_vectors(n, k, seed * 1000 + f, device="cuda").to(dt))
    torch.cuda.synchronize()
    return Ls, Vs


def time_plan(Ls, Vs, plan, reps: int = 3, warmup: int = 1):
    """Median ms per batch of `plan` (update then matching downdate per pair)."""
    import torch
    import paper_1011_1173_amd as chm
    stream = torch.cuda.Stream()
    n = len(Ls)
    times = []
    with torch.cuda.stream(stream):
        for r in range(warmup + reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            p1 = chm.update_batched_async(Ls, Vs, [1] * n, stream=stream, plan=plan)
            p2 = chm.update_batched_async(Ls, Vs, [-1] * n, stream=stream, plan=plan)
            e1.record(stream)
            for pb in (p1, p2):
                st = pb.statuses()
                if any(x[0] != 0 for x in st):
                    raise RuntimeError("plan %r: a factor failed: %r" % (plan, st))
            if r >= warmup:
                times.append(e0.elapsed_time(e1) / 2.0)
    times.sort()
    return times[len(times) // 2]


def tune(out: str | None = None, dtypes=("f64", "f32s"), n_buckets=(0, 1, 2, 3),
         k_buckets=(0, 1, 2), reps: int = 3, log=sys.stderr):
    import torch
    import paper_1011_1173_amd as chm
    from . import _native
    lib = _native.load()
    cus = int(lib.cholmod_compute_units()) or 256
    cands = candidates(cus)
    entries = []
    t_start = time.time()
    for dt in dtypes:
        f32 = dt == "f32s"
        for nb in n_buckets:
            for kb in k_buckets:
                Ls, Vs = _batch(nb, kb, f32, seed=31 + 7 * nb + kb)
                # the timing runs modify Ls in place (an update and a downdate
                # do not restore a factor bit for bit), so every candidate's
                # result is checked from a copy of the original factors
                orig = [L.clone() for L in Ls]
                # the default plan's results, to check every candidate against
                ref = [L.clone() for L in orig]
                st = chm.update_batched(ref, Vs, [1] * len(ref), plan=cands[0])
                assert all(x[0] == 0 for x in st), st
                res = []
                for c in cands:
                    probe = [L.clone() for L in orig]
                    chm.update_batched(probe, Vs, [1] * len(probe), plan=c)
                    if not all(torch.equal(a, b) for a, b in zip(probe, ref)):
                        raise RuntimeError("plan %r gives a different result" % (c,))
                    del probe
                    ms = time_plan(Ls, Vs, c, reps=reps)
                    res.append((ms, c))
                res.sort(key=lambda x: x[0])
                best = res[0]
                entries.append({"dtype": 1 if f32 else 0, "n_bucket": nb, "k_bucket": kb,
                                "plan": best[1], "ms": best[0],
                                "default_ms": [m for m, c in res if c == cands[0]][0],
                                "candidates": [{"plan": c, "ms": m} for m, c in res]})
                print("tune: %s n-bucket %d k-bucket %d: best %.3f ms (default %.3f) %r"
                      % (dt, nb, kb, best[0], entries[-1]["default_ms"], best[1]),
                      file=log, flush=True)
                del Ls, Vs, ref, orig
                torch.cuda.empty_cache()
    data = {"arch": arch_name(), "compute_units": cus,
            "device": torch.cuda.get_device_name(0),
            "generated_s": round(time.time() - t_start, 1),
            "n_bucket_ranges": {str(k): v[0] for k, v in N_BUCKET_RANGES.items()},
            "k_bucket_ranges": {str(k): v for k, v in K_BUCKET_RANGES.items()},
            "entries": entries}
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
    return data


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=None, help="plan cache to write (default: plans/<arch>.json)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="FP64 and n buckets 1-2 only")
    a = ap.parse_args(argv)
    out = a.out or default_cache()
    if a.quick:
        tune(out, dtypes=("f64",), n_buckets=(1, 2), k_buckets=(0, 1), reps=a.reps)
    else:
        tune(out, reps=a.reps)
    print(out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
