"""Autotuner of the library's launch shapes, with a cache.

Three choices are measured on the GPU and kept:
- the NTT tile width (16, 8 or 4 columns or rows per workgroup, 512, 256 or
  128 threads) of every N = 2^16 NTT grid launch, per direction and number of
  limbs in the launch (the paper's limb-batch knob, Sec. III-F.1: how much of
  a transform one block takes);
- the persistent grid (workgroups per CU) of each step of a batch of key
  switches, per batch (ckks_batch_tune);
- the fusion depth of a batch (ckks_batch_set_schedule): one persistent
  launch per step, or the whole batch in one launch with its key switches
  pipelined in windows of 1 to n items, at one or two workgroups per CU.

Each candidate is timed as the median of several bursts of launches on
rotating buffers larger than the last-level cache.  Results are kept in a JSON
cache keyed by (logN, limbs, K, op, arch): op is "ntt_fwd" / "ntt_inv" or a
batch signature; limbs is the launch's number of limbs.  A later process with
the same parameter set and GPU architecture loads the cache instead of
measuring again.  The tuner only chooses among launch shapes that give the
same result bit for bit.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Optional

import torch

from . import ckks

CACHE_ENV = "CKKS_TUNE_CACHE"
TILES = (16, 8, 4)
# inverse launches also have tile code 2: 8 rows (columns) per workgroup with 4 elements per thread
INV_TILES = TILES + (2,)


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "paper_2507_04775_amd",
                                                      "tune.json")


def arch() -> str:
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _key(logn: int, limbs: int, K: int, op: str, arch_name: str) -> str:
    return "logN=%d|limbs=%d|K=%d|op=%s|arch=%s" % (logn, limbs, K, op, arch_name)


def load_cache(path: Optional[str] = None) -> dict:
    try:
        with open(path or cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: Optional[str] = None) -> None:
    p = path or cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _burst_ms(fn, stream, n: int) -> float:
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def tune_ntt_tiles(ctx: ckks.Context, limb_counts=None, samples: int = 5, burst: int = 8, cache: Optional[dict] = None,
                   use_cache: bool = True) -> dict:
    """Chooses the NTT tile width per direction and launch size at N = 2^16
    (launch sizes up to the number of primes of the context, taken over the
    context's own primes q_0.. then p_0..), applies it (ckks_ntt_tile_set) and
    records it in `cache`.  Returns {op: {limbs: {"tile", "us": {tile: us}}}}."""
    if ctx.logn != 16:
        return {}
    nmax = ctx.nq + ctx.np
    limb_counts = sorted(set(limb_counts or range(1, nmax + 1)))
    cache = {} if cache is None else cache
    an = arch()
    stream = torch.cuda.current_stream()
    mods = list(ctx.q) + list(ctx.p)
    # rotating polynomials, together larger than the 256 MB last-level cache
    ring = [torch.randint(0, int(min(mods)), (nmax, ctx.N), dtype=torch.int64, device="cuda").view(torch.uint64)
            for _ in range(12)]
    turn = [0]
    out = {}
    for inverse in (False, True):
        op = "ntt_inv" if inverse else "ntt_fwd"
        out[op] = {}
        for n in limb_counts:
            if n > nmax:
                continue
            key = _key(ctx.logn, n, ctx.np, op, an)
            if use_cache and key in cache:
                ckks.ntt_tile_set(inverse, n, int(cache[key]["tile"]))
                out[op][n] = cache[key]
                continue
            times = {}
            for tile in (INV_TILES if inverse else TILES):
                ckks.ntt_tile_set(inverse, n, tile)

                def launch():
                    p = ring[turn[0] % len(ring)][:n]
                    turn[0] += 1
                    (ctx.ckks_intt if inverse else ctx.ckks_ntt)(p, 0, n, stream)

                launch()
                xs = [_burst_ms(launch, stream, burst) for _ in range(samples)]
                times[tile] = statistics.median(xs) * 1e3
            best = min(times, key=times.get)
            ckks.ntt_tile_set(inverse, n, best)
            rec = {"tile": best, "us": {str(t): round(v, 2) for t, v in times.items()}}
            cache[key] = rec
            out[op][n] = rec
    return out


def op_launch_sizes(ctx: ckks.Context, level: int) -> dict:
    """Limb counts of the NTT launches inside HMult+relin and Rescale at
    `level` that exceed the context's primes (and so cannot be timed through
    ckks_ntt alone): ModUp's forward NTT (beta (l+1+K) - (l+1) rows), ModDown's
    (2 (l+1)) and Rescale's (2 l)."""
    n, K = level + 1, ctx.np
    beta = ctx.beta(level)
    return {"ntt_fwd": sorted({beta * (n + K) - n, 2 * n, 2 * level} - {0})}


def tune_op_launches(ctx: ckks.Context, level: int, samples: int = 5, burst: int = 4, cache: Optional[dict] = None,
                     use_cache: bool = True) -> dict:
    """Tile width of the launches op_launch_sizes names, chosen by timing the
    operation that contains each (HMult+relin for ModUp's and ModDown's,
    Rescale for its own) with every candidate width on that launch size."""
    if ctx.logn != 16:
        return {}
    cache = {} if cache is None else cache
    an = arch()
    stream = torch.cuda.current_stream()
    mods = list(ctx.q[: level + 1])

    def rnd(rows):
        return torch.randint(0, int(min(mods)), (rows, ctx.N), dtype=torch.int64, device="cuda").view(torch.uint64)

    allm = list(ctx.q) + list(ctx.p)
    kd = torch.randint(0, int(min(allm)), (ctx.dnum, 2, len(allm), ctx.N), dtype=torch.int64,
                       device="cuda").view(torch.uint64)
    rlk = ctx.key(kd, 0)
    cts = [ckks.Ciphertext(rnd(level + 1), rnd(level + 1), level) for _ in range(4)]
    out = ctx.empty_ct(level)
    low = ctx.empty_ct(level - 1)
    ws = ctx.workspace(ckks.OP_HMULT, level)
    turn = [0]

    def hmult():
        a, b = cts[turn[0] % 4], cts[(turn[0] + 1) % 4]
        turn[0] += 1
        ctx.ckks_hmult_relin(a, b, rlk, out, ws, stream)

    def rescale():
        a = cts[turn[0] % 4]
        turn[0] += 1
        ctx.ckks_rescale(a, low, ws, stream)

    n, K = level + 1, ctx.np
    sizes = {ctx.beta(level) * (n + K) - n: hmult, 2 * n: hmult, 2 * level: rescale}
    res = {}
    for size, fn in sorted(sizes.items()):
        if size <= 0 or size > 128:
            continue
        key = _key(ctx.logn, size, ctx.np, "ntt_fwd", an)
        if use_cache and key in cache:
            ckks.ntt_tile_set(False, size, int(cache[key]["tile"]))
            res[size] = cache[key]
            continue
        times = {}
        for tile in TILES:
            ckks.ntt_tile_set(False, size, tile)
            fn()
            times[tile] = statistics.median([_burst_ms(fn, stream, burst) for _ in range(samples)]) * 1e3
        best = min(times, key=times.get)
        ckks.ntt_tile_set(False, size, best)
        rec = {"tile": best, "op_us": {str(t): round(v, 2) for t, v in times.items()},
               "timed_through": fn.__name__}
        cache[key] = rec
        res[size] = rec
    return {"ntt_fwd": res}


def batch_signature(plan_items) -> str:
    """A cache op name for a batch: its item kinds and levels."""
    parts = ["%s@%d" % (k, l) for k, l in plan_items]
    return "batch[" + ",".join(parts) + "]"


def tune_batch(batch: ckks.Batch, ctx: ckks.Context, signature: str, stream, cache: Optional[dict] = None,
               use_cache: bool = True) -> list:
    """Persistent grid per batch step: from the cache when the same batch
    (signature) was tuned on this parameter set and architecture, else
    measured by ckks_batch_tune (median of five runs per candidate) and
    recorded.  Returns the grid per step."""
    cache = {} if cache is None else cache
    key = _key(ctx.logn, ctx.nq, ctx.np, signature, arch())
    if use_cache and key in cache:
        for step, g in enumerate(cache[key]["grid"]):
            batch.set_grid(step, int(g))
        return list(cache[key]["grid"])
    batch.tune(stream)
    grid = [batch.grid(i) for i in range(ckks.Batch.steps())]
    cache[key] = {"grid": grid}
    return grid


def schedule_candidates(n_items: int, logn: int):
    """(window, workgroups per CU) pairs tried by tune_batch_schedule: per-step
    launches (window 0), then one launch at windows of 1, 2, 4, ... items up to
    the whole batch, at two workgroups per CU, and the best-guess window at one."""
    if logn != 16:
        return [(0, 2)]
    ws, w = [], 1
    while w < n_items:
        ws.append(w)
        w *= 2
    ws.append(n_items)
    return [(0, 2)] + [(w, 2) for w in ws] + [(8 if n_items > 8 else n_items, 1)]


def tune_batch_schedule(batch: ckks.Batch, ctx: ckks.Context, signature: str, n_items: int, stream,
                        cache: Optional[dict] = None, use_cache: bool = True, samples: int = 3) -> dict:
    """Schedule of a batch (after tune_batch has set the per-step grids): each
    candidate of schedule_candidates runs the batch once to warm up, then
    `samples` times; the one with the smallest median time is applied and
    recorded.  Returns {"window", "wg", "ms": {candidate: median ms}}."""
    cache = {} if cache is None else cache
    key = _key(ctx.logn, ctx.nq, ctx.np, "schedule:" + signature, arch())
    if use_cache and key in cache:
        rec = cache[key]
        batch.set_schedule(int(rec["window"]), int(rec["wg"]))
        return rec
    times = {}
    for window, wg in schedule_candidates(n_items, ctx.logn):
        batch.set_schedule(window, wg)
        batch.run(stream)
        batch.faults(stream)
        xs = [_burst_ms(lambda: batch.run(stream), stream, 1) for _ in range(samples)]
        batch.faults(stream)
        times[(window, wg)] = statistics.median(xs)
    best = min(times, key=times.get)
    batch.set_schedule(*best)
    rec = {"window": best[0], "wg": best[1], "ms": {"%d/%d" % k: round(v, 3) for k, v in times.items()}}
    cache[key] = rec
    return rec
