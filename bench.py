"""Benchmark of the CKKS key-switching hot path on one MI355X.

Workload (N = 2^16, 31 ciphertext limbs (one 60-bit, thirty 50-bit primes),
dnum = 3, four 60-bit special primes, top level l = 30): one step is one
HMult+relinearisation, one Rescale of its result and one HRotate by a seeded
slot index, on seeded uniform ciphertexts and keys (timing does not depend on
the values).  Every step holds two key switches; `value` is key switches per
second over the timed steps.

Prints one JSON line.  Also reported: per-operation latencies (p50 / p99), a
cold-pool rate (each step on a different ciphertext pair and key set, cycling
through more than 1 GiB), the dominant kernel's roofline figures measured live
with HIP events on the library's stream, and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# a bootstrap whose decrypted slot error (log2 of the largest slot difference) exceeds this gets no rate
BOOT_PRECISION_BITS = -8.0
# one wave64 VALU instruction per CU per cycle (four SIMDs of 16 lanes, four cycles each): 256 CUs at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 2.4e9
# bytes of one limb at N = 2^16 (u64 residues)
LIMB = 65536 * 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-probe", action="store_true", help="skip the multiply-add rate probe")
    ap.add_argument("--cold-sets", type=int, default=6)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-items", type=int, default=128)
    ap.add_argument("--batch-reps", type=int, default=20)
    ap.add_argument("--no-boot", action="store_true")
    ap.add_argument("--no-uniform-boot", action="store_true", help="skip the uniform-secret bootstrap variant")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (the reference kernel for HBM counter scaling)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-w32", action="store_true", help="skip the 32-bit word path")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-loads", type=str, default="0.25,0.5,0.75,0.9,1.0,1.1")
    ap.add_argument("--serve-boot-handles", type=int, default=2)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-mem-gib", type=int, default=16)
    ap.add_argument("--boot-reps", type=int, default=10)
    return ap.parse_args()


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


NTT_SOURCES = ("ntt.hip", "unit_map.h", "internal.h", "modarith.h", "coef_units.h")


def ntt_sources_sha256():
    """SHA-256 over the NTT kernel sources in NTT_SOURCES order, with comments
    and runs of white space removed, so that only a change of code invalidates
    the counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in NTT_SOURCES:
        t = open(os.path.join(ROOT, "paper_2507_04775_amd", "csrc", f)).read()
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(re.sub(r"\s+", " ", t).strip().encode())
    return h.hexdigest()


_SLEEP_CYCLES_PER_US = [None]


def preload(stream, us: float):
    """Holds `stream` for about `us` microseconds with a one-thread spin kernel,
    so that the host enqueues the launches that follow before the GPU reaches
    them: per-launch event pairs then time the GPU, not host submission gaps."""
    import torch
    if _SLEEP_CYCLES_PER_US[0] is None:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            torch.cuda._sleep(1000)
            e0.record(stream)
            torch.cuda._sleep(2_000_000)
            e1.record(stream)
        stream.synchronize()
        _SLEEP_CYCLES_PER_US[0] = 2_000_000 / max(1e-3, e0.elapsed_time(e1) * 1e3)
    with torch.cuda.stream(stream):
        torch.cuda._sleep(int(us * _SLEEP_CYCLES_PER_US[0]))


def timed_launches(fn, reps: int, stream, host_us: float = 200.0):
    """GPU time of each of `reps` back-to-back calls of fn() on `stream` (ms),
    the stream held first long enough for all of them to be enqueued."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    preload(stream, 2000.0 + reps * host_us)
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]


def stats_ms(xs):
    return {"p50_ms": round(percentile(xs, 50), 4), "p99_ms": round(percentile(xs, 99), 4),
            "mean_ms": round(sum(xs) / len(xs), 4), "n": len(xs)}


KERNEL_SOURCES = ("kernels.hip", "ntt.hip", "unit_map.h", "internal.h", "modarith.h", "coef_units.h", "ks_args.cpp", "api.cpp")


def kernel_sources_sha256():
    """The same digest over every source the key-switching kernels and their
    launch sequence come from (validity of the VALU and inner-product counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        t = open(os.path.join(ROOT, "paper_2507_04775_amd", "csrc", f)).read()
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(re.sub(r"\s+", " ", t).strip().encode())
    return h.hexdigest()


def measured_ip_traffic():
    """HBM bytes per launch of k_inner_product from its committed counter
    summary, while the kernel sources are the profiled ones (else None)."""
    prof = os.path.join(ROOT, "profiles", "inner_product_logn16_l30_hbm_counters.md")
    try:
        fields = dict(l.split(":", 1) for l in open(prof)
                      if l.startswith(("traffic_bytes_per_launch:", "kernel_sources_sha256:")))
        if kernel_sources_sha256() != fields["kernel_sources_sha256"].strip():
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def step_inner_products():
    """The timed step's inner products (the fused forms of k_inner_product that
    HMult+relin and HRotate launch) from the committed counter and trace
    summaries, while the kernel sources are the profiled ones (else None): their
    algorithmic bytes, measured HBM bytes and profiled duration per launch."""
    prof = os.path.join(ROOT, "profiles", "inner_product_logn16_l30_hbm_counters.md")
    try:
        lines = open(prof).read().splitlines()
    except OSError:
        return None
    sha = next((l.split(":", 1)[1].strip() for l in lines if l.startswith("kernel_sources_sha256:")), None)
    if sha != kernel_sources_sha256():
        return None
    out = []
    for l in lines:
        if not l.startswith("step_kernel:"):
            continue
        name, grid, *kv = l.split(":", 1)[1].split()
        f = dict(x.split("=") for x in kv)
        alg, us = int(f["algorithmic_bytes"]), float(f["avg_us"])
        gbs = alg / (us / 1e6) / 1e9
        out.append({"kernel": name, "grid": grid, "algorithmic_bytes_per_launch": alg,
                    "traffic": int(f["traffic_bytes"]), "profiled_us": us, "achieved": round(gbs, 1),
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "source": os.path.relpath(prof, ROOT)})
    return out or None


def measured_traffic():
    """HBM bytes per launch of the roofline kernel, from the committed counter
    summary, valid only while the NTT sources (the kernel file and the headers
    it builds on) are the ones the counters were taken on (else None)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "ntt_fwd_logn16_35limbs_hbm_counters.md")
    try:
        fields = dict(l.split(":", 1) for l in open(prof) if l.startswith(("traffic_bytes_per_launch:", "ntt_sources_sha256:")))
        if ntt_sources_sha256() != fields["ntt_sources_sha256"].strip():
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def inner_product_roofline(ctx, ps, seed, stream):
    """Algorithmic HBM bytes of ckks_inner_product at the top level over its
    measured launch time (k_inner_product is its only kernel)."""
    import torch

    from paper_2507_04775_amd import inputs
    level = ps.L
    rows, beta = level + 1 + ps.K, ctx.beta(level)
    allm = list(ps.q) + list(ps.p)
    rowm = list(ps.q[: level + 1]) + list(ps.p)
    sets = []
    for i in range(2):
        ext = inputs.device_residues(seed + 800 + i, rowm * beta, ps.N).reshape(beta, rows, ps.N).contiguous()
        kd = inputs.device_residues(seed + 810 + i, allm * (2 * ps.dnum), ps.N).reshape(ps.dnum, 2, len(allm), ps.N)
        kd = kd.contiguous()
        sets.append((ext, ctx.key(kd, 0), torch.empty((2, rows, ps.N), dtype=torch.uint64, device="cuda"), kd))
    turn = [0]

    def launch():
        ext, key, acc, _ = sets[turn[0] % 2]
        turn[0] += 1
        ctx.ckks_inner_product(ext, level, key, 1, acc, stream)

    for _ in range(4):
        launch()
    n = 40
    torch.cuda.synchronize()
    preload(stream, 2000.0 + 100.0 * n)
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    for _ in range(n):
        launch()
    b1.record(stream)
    torch.cuda.synchronize()
    us = b0.elapsed_time(b1) / n * 1e3
    nbytes = (3 * beta + 2) * rows * LIMB
    gbs = nbytes / (us / 1e6) / 1e9
    return {"bound": "hbm", "kernel": "k_inner_product (key inner product, l = 30: 3 digits x 35 rows)",
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_ip_traffic(), "algorithmic_bytes_per_launch": nbytes, "launch_us": round(us, 2),
            "step_kernels": step_inner_products()}


def run_probe(stream):
    """Rate of the 32x32->64 multiply-add (v_mad_u64_u32) on the whole chip."""
    import torch

    from paper_2507_04775_amd import ckks
    blocks, iters = 256 * 8, 2048
    out = torch.empty(blocks * 256, dtype=torch.uint64, device="cuda")
    for _ in range(3):
        ckks.probe_mad64(out, blocks, iters, stream)
    xs = []
    n = 0
    for _ in range(7):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        n = ckks.probe_mad64(out, blocks, iters, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        xs.append(e0.elapsed_time(e1))
    ms = percentile(xs, 50)
    wave = n / 64 / (ms / 1e3)
    return {"workgroups": blocks, "threads": 256, "iters": iters, "chains": 8, "lane_mads_per_launch": n,
            "launch_ms": round(ms, 4), "lane_mads_per_s": round(n / (ms / 1e3), 1),
            "wave_instr_per_s": round(wave, 1), "frac_of_issue_peak": round(wave / VALU_ISSUE_PEAK, 4)}


def valu_fractions(probe):
    """VALU issue fractions of the key-switching kernels from the committed SQ
    counter profile, valid while the kernel sources are the ones profiled (else
    None): instructions per launch over the profiled duration, against the issue
    peak and against the measured multiply-add rate."""
    prof = os.path.join(ROOT, "profiles", "keyswitch_step_logn16_valu_counters.md")
    try:
        text = open(prof).read()
    except OSError:
        return None
    sha = None
    for line in text.splitlines():
        if line.startswith("kernel_sources_sha256:"):
            sha = line.split(":", 1)[1].strip()
    if sha != kernel_sources_sha256():
        return None
    rows = {}
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 7 and cells[0].startswith("k_") and cells[2].isdigit():
            name = "%s %s" % (cells[0], cells[1])
            if name in rows:
                continue
            waves, per, us = int(cells[2]), int(cells[3]), float(cells[4])
            rate = waves * per / (us / 1e6)
            rows[name] = {"wave_instr_per_launch": waves * per, "avg_us": us,
                          "frac_of_issue_peak": round(rate / VALU_ISSUE_PEAK, 3)}
    keep = ["k_fwd_col_bconv 8192x62x1", "k_inner_product 65536x35x1", "k_inner_product_tensor_rowpass 65536x35x1",
            "k_inner_product_rowpass 65536x35x1", "k_bconv 65536x3x5", "k_fwd_row_moddown 8192x62x1",
            "k_fwd_col_plain 8192x74x1", "k_fwd_row_plain 8192x74x1"]
    # the NTT passes appear under the tile width the autotuner chose (suffix _w8 or _w4 for 8 or 4)
    kernels = {}
    for k in keep:
        name, grid = k.split(" ")
        for v in (name, name + "_w8", name + "_w4"):
            if "%s %s" % (v, grid) in rows:
                kernels["%s %s" % (v, grid)] = rows["%s %s" % (v, grid)]
                break
    out = {"peak_wave_instr_per_s": VALU_ISSUE_PEAK, "source": os.path.relpath(prof, ROOT), "kernels": kernels}
    if probe:
        out["mad64_wave_instr_per_s_measured"] = probe["wave_instr_per_s"]
    return out


def cpu_baseline(ps, seed, level, g_rot, ks_per_step, runs):
    """The oracle on the host: one step (HMult+relin, Rescale, HRotate at the top
    level) per run on one thread, several steps per run on all cores; medians."""
    import oracle
    from paper_2507_04775_amd import inputs
    P = oracle.Params(ps.logn, ps.q, ps.p, ps.dnum)
    a = inputs.random_ct(seed, ps, level)
    b = inputs.random_ct(seed + 1, ps, level)
    rlk = inputs.random_key(seed + 2, ps)
    rk = inputs.random_key(seed + 3, ps)
    all_threads = oracle.max_threads()

    def step():
        mm = oracle.hmult_relin(P, a, b, rlk, level)
        oracle.rescale(P, mm, level)
        oracle.apply_galois(P, a, g_rot, rk, level)

    def measure(threads, steps):
        oracle.set_threads(threads)
        step()  # warm
        rates = []
        for _ in range(runs):
            t1 = time.perf_counter()
            for _ in range(steps):
                step()
            rates.append(ks_per_step * steps / (time.perf_counter() - t1))
        return rates

    one = measure(1, 1)
    many = measure(all_threads, 4)
    oracle.set_threads(all_threads)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(percentile(many, 50), 3), "unit": "key-switches/s", "cores": all_threads,
            "kind": "oracle", "cpu_model": model, "runs": runs,
            "sample": "HMult+relin, Rescale, HRotate at l=30, N=2^16: %d runs of 4 steps on %d threads, "
                      "%d runs of 1 step on 1 thread; medians" % (runs, all_threads, runs),
            "all_cores_runs": [round(x, 3) for x in many],
            "single_thread": {"value": round(percentile(one, 50), 4), "unit": "key-switches/s", "cores": 1,
                              "runs": [round(x, 4) for x in one]}}


def run_batch(ctx, ps, seed, args, tcache):
    """C3-style batch: one graph replay of the persistent stage kernels vs the same
    items issued as plain per-operation calls on one stream."""
    import torch

    from paper_2507_04775_amd import ckks, inputs, tune

    plan = inputs.batch_plan(seed + 500, args.batch_items, ps.logn, ps.L)
    allm = list(ps.q) + list(ps.p)

    def dev_key(s):
        k = torch.empty((ps.dnum, 2, len(allm), ps.N), dtype=torch.uint64, device="cuda")
        for j in range(ps.dnum):
            for t in range(2):
                k[j, t] = inputs.device_residues(s + 7 * j + t, allm, ps.N)
        return k

    rlk = ctx.key(dev_key(seed + 600), 0)
    rkeys = {}
    for k in inputs.batch_rotation_set(ps.logn):
        rkeys[k] = ctx.key(dev_key(seed + 700 + k), pow(5, k, 2 * ps.N))

    def dev_ct(s, level):
        return ckks.Ciphertext(inputs.device_residues(s, ps.q[: level + 1], ps.N),
                               inputs.device_residues(s + 1, ps.q[: level + 1], ps.N), level)

    items = []
    for i, (kind, level, ks) in enumerate(plan):
        a = dev_ct(seed + 1000 + 4 * i, level)
        if kind == "hmult":
            items.append((kind, a, dev_ct(seed + 1002 + 4 * i, level), ctx.empty_ct(level)))
        else:
            items.append((kind, a, ks, [ctx.empty_ct(level) for _ in ks]))
    batch = ckks.Batch(ctx)
    for kind, a, x, out in items:
        if kind == "hmult":
            batch.hmult(a, x, rlk, out)
        else:
            batch.hoisted(a, x, [rkeys[k] for k in x], out)
    batch.build()
    st = torch.cuda.Stream()
    n_ks = batch.keyswitches
    sig = tune.batch_signature([(k, l) for k, l, _ in plan])
    with torch.cuda.stream(st):
        t0 = time.perf_counter()
        tune.tune_batch(batch, ctx, sig, st, tcache)
        sched = tune.tune_batch_schedule(batch, ctx, sig, len(plan), st, tcache)
        t_tune = time.perf_counter() - t0

        def replays(window, wg):
            batch.set_schedule(window, wg)
            batch.capture(st)
            batch.replay(st)
            batch.faults(st)
            xs = timed_launches(lambda: batch.replay(st), max(20, args.batch_reps), st, host_us=100.0)
            batch.faults(st)
            return xs

        # both schedules as graph replays: per-step launches, and one launch at the best window the
        # tuner measured for it
        one = min(((w, g) for w, g in tune.schedule_candidates(len(plan), ps.logn) if w),
                  key=lambda c: sched["ms"].get("%d/%d" % c, 1e30), default=None)
        per_step = replays(0, 2)
        one_launch = replays(*one) if one else None
        reps = replays(sched["window"], sched["wg"])
        ws_h = ctx.workspace(ckks.OP_HMULT, ps.L)
        ws_o = ctx.workspace(ckks.OP_HOISTED, ps.L)

        def plain():
            for kind, a, x, out in items:
                if kind == "hmult":
                    ctx.ckks_hmult_relin(a, x, rlk, out, ws_h, st)
                else:
                    ctx.ckks_hrotate_hoisted(a, x, [rkeys[k] for k in x], out, ws_o, st)

        plain()
        st.synchronize()
        t0 = time.perf_counter()
        plain()
        host_ms = (time.perf_counter() - t0) * 1e3
        st.synchronize()
        preps = timed_launches(plain, max(20, args.batch_reps), st, host_us=1.5e3 * host_ms)
    bt, pt = percentile(reps, 50), percentile(preps, 50)
    res = {"workload": "%d ciphertexts, levels 4..%d, half HMult+relin, half hoisted 8-way rotations" % (
               len(plan), ps.L),
           "key_switches": n_ks, "batched_ms": round(bt, 3), "plain_ms": round(pt, 3),
           "batched": stats_ms(reps), "plain": stats_ms(preps),
           "batched_key_switches_per_s": round(n_ks / (bt / 1e3), 1),
           "plain_key_switches_per_s": round(n_ks / (pt / 1e3), 1),
           "batched_key_switches_per_s_at_p99": round(n_ks / (percentile(reps, 99) / 1e3), 1),
           "plain_key_switches_per_s_at_p99": round(n_ks / (percentile(preps, 99) / 1e3), 1),
           "speedup": round(pt / bt, 3), "workspace_bytes": int(batch.ws.numel() * 8),
           "tune_s": round(t_tune, 2), "tuned_grid_wg_per_cu": [batch.grid(i) for i in range(12)],
           "schedule": {"chosen_window": sched["window"], "chosen_wg_per_cu": sched["wg"],
                        "tuning_median_ms": sched["ms"],
                        "per_step_launches": stats_ms(per_step),
                        "one_launch": dict(stats_ms(one_launch), window=one[0], wg_per_cu=one[1]) if one else None}}
    batch.close()
    return res


def run_bootstrap(seed, args, sparse=True):
    """Full-slot bootstrap at N = 2^16 (L = 30, dnum = 3, ten special primes so
    that key switching keeps the message): keys and plaintexts made by the
    client helpers, one eager bootstrap per step and the captured HIP graph
    replayed; the decrypted error against the input slots is reported.  With
    `sparse`, the input is encapsulated under a sparse secret around ModRaise
    (degree 31, 3 double angles); without, EvalMod covers the uniform secret's
    range (degree 119, 6 double angles)."""
    import numpy as np
    import torch

    from paper_2507_04775_amd import bootplan, ckks, inputs
    from paper_2507_04775_amd.client import Client

    ps = inputs.params("large-nv")
    ctx = ckks.Context(ps.logn, ps.q, ps.p, ps.dnum, device=0)
    scale = 2.0 ** ps.log_scale
    cfg = bootplan.default_config(ps.logn, scale, sparse=sparse)
    t0 = time.perf_counter()
    pl = bootplan.plan(ps.q, cfg)
    t_plan = time.perf_counter() - t0
    cl = Client(ctx, ps, seed)
    t0 = time.perf_counter()
    rot = {k: cl.rotation_key(k) for k in pl.rotations}
    relin, conj = cl.relin_key(), cl.conjugation_key()
    sp = cl.sparse_keys(bootplan.SPARSE_H) if sparse else None
    torch.cuda.synchronize()
    t_keys = time.perf_counter() - t0
    z = inputs.complex_slots(inputs.rng(seed + 5), ps.N // 2)
    ct = cl.encrypt(z, 0, scale)
    reps = max(3, args.boot_reps)

    def measure(hoist):
        boot = ckks.Boot(ctx, cfg.cts_radix_logs, cfg.stc_radix_logs, pl.cts, pl.stc, pl.cheb, cfg.double_angles,
                         cfg.top_scale, relin, conj, rot, sparse=sp, hoist_moddown=hoist, input_gain=cfg.input_gain)
        out = ctx.empty_ct(boot.output_level)
        stream = torch.cuda.current_stream()
        boot.ckks_bootstrap(ct, out)
        torch.cuda.synchronize()
        err = float(np.log2(np.max(np.abs(cl.decrypt(out) - z))))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for i in range(reps):
            boot.ckks_bootstrap(ct, out)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        eager = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
        gs = torch.cuda.Stream()
        out_g = ctx.empty_ct(boot.output_level)
        boot.capture(ct, out_g, gs)
        boot.replay(gs)
        gs.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(gs)
        for i in range(reps):
            boot.replay(gs)
            ev[i + 1].record(gs)
        gs.synchronize()
        graph = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
        same = bool(torch.equal(out_g.c0, out.c0) and torch.equal(out_g.c1, out.c1))
        return boot, err, eager, graph, same

    # the plain schedule (one ModDown per rotation, as in the paper) for comparison
    plain, perr, _, pgraph, _ = measure(False)
    plain.close()
    boot, err, eager, graph, same = measure(cfg.hoist_moddown)
    g50 = percentile(graph, 50)
    usable = err <= BOOT_PRECISION_BITS
    res = {"bootstraps_per_s": round(1e3 / g50, 2) if usable else None,
           "precision_threshold_bits": BOOT_PRECISION_BITS, "meets_precision_threshold": usable,
           "graph_p50_ms": round(g50, 3),
           "graph_p99_ms": round(percentile(graph, 99), 3), "eager_p50_ms": round(percentile(eager, 50), 3),
           "eager_p99_ms": round(percentile(eager, 99), 3), "reps": reps, "graph_equals_eager": same,
           "key_switches": boot.keyswitches, "levels_left": boot.output_level, "slots": ps.N // 2,
           "decrypted_error_bits": round(err, 2), "device_bytes": boot.device_bytes,
           "rotation_keys": len(rot), "plan_s": round(t_plan, 2), "keygen_s": round(t_keys, 2),
           "plain_schedule": {"graph_p50_ms": round(percentile(pgraph, 50), 3),
                              "decrypted_error_bits": round(perr, 2)},
           "config": {"logN": ps.logn, "limbs": ps.L + 1, "special_primes": ps.K, "dnum": ps.dnum,
                      "cts_groups": cfg.cts_radix_logs, "stc_groups": cfg.stc_radix_logs,
                      "cheb_degree": cfg.cheb_degree, "cheb_baby": cfg.baby, "double_angles": cfg.double_angles,
                      "k_range": cfg.k_range, "sparse_secret_encapsulation": sparse,
                      "sparse_h": bootplan.SPARSE_H if sparse else None, "scale_log2": ps.log_scale,
                      "hoist_moddown": cfg.hoist_moddown}}
    boot.close()
    del rot, relin, conj, sp
    ctx.close()
    return res


def run_w32(seed, args):
    """The 32-bit word path at N = 2^16 on 52 + 8 primes of 30 bits (dnum 4; the
    64-bit "large" set's 1560-bit Q and 240-bit P): the same step (HMult+relin,
    Rescale, rotation at the top level) and its NTTs, with per-operation
    latencies."""
    import torch

    from paper_2507_04775_amd import ckks, inputs
    ps = inputs.params32("w32-large")
    ctx = ckks.Context32(ps.logn, ps.q, ps.p, ps.dnum)
    level = ps.L
    stream = torch.cuda.current_stream()
    dev = lambda a: ckks.to_device32(a)
    a = [dev(x) for x in inputs.random_ct(seed, ps, level)]
    b = [dev(x) for x in inputs.random_ct(seed + 1, ps, level)]
    key = inputs.random_key(seed + 2, ps)
    rlk = dev(key.reshape(-1, ps.N)).reshape(key.shape)
    key = inputs.random_key(seed + 3, ps)
    rk = dev(key.reshape(-1, ps.N)).reshape(key.shape)
    g = pow(5, inputs.rotation_index(seed, ps.logn), 2 * ps.N)
    m0, m1, r0, r1, o0, o1 = [ctx.empty(level + 1) for _ in range(6)]
    ws_h, ws_r, ws_g = (ctx.workspace(op, level) for op in (ckks.OP_HMULT, ckks.OP_RESCALE, ckks.OP_ROTATE))

    def hmult():
        ctx.hmult_relin(a[0], a[1], b[0], b[1], level, rlk, m0, m1, ws_h)

    def rescale():
        ctx.rescale(m0, m1, level, r0[:level], r1[:level], ws_r)

    def rotate():
        ctx.apply_galois(a[0], a[1], level, g, rk, o0, o1, ws_g)

    def step():
        hmult()
        rescale()
        rotate()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n = max(20, args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    nmods = ps.L + 1 + ps.K
    ring = [ctx.empty(nmods) for _ in range(8)]  # 8 x 15.7 MB
    for t in ring:
        t.copy_(dev(inputs.uniform_residues(inputs.rng(seed + 9), list(ps.q) + list(ps.p), ps.N)))
    turn = [0]

    def ntt_next(inverse):
        t = ring[turn[0] % len(ring)]
        turn[0] += 1
        (ctx.intt if inverse else ctx.ntt)(t, 0, nmods, stream)

    def stats(fn, reps):
        xs = timed_launches(fn, reps, stream)
        return {"p50_us": round(percentile(xs, 50) * 1e3, 2), "p99_us": round(percentile(xs, 99) * 1e3, 2)}

    ops = {"hmult_relin": stats(hmult, n), "rescale": stats(rescale, n), "rotate": stats(rotate, n),
           "ntt_%d_limbs" % nmods: stats(lambda: ntt_next(False), n),
           "intt_%d_limbs" % nmods: stats(lambda: ntt_next(True), n)}
    nb = (ps.L + 1) * ps.N * 4
    res = {"workload": "HMult+relin + Rescale + rotation at level %d, 32-bit words" % level,
           "logN": ps.logn, "limbs": ps.L + 1, "special_primes": ps.K, "dnum": ps.dnum, "prime_bits": 30,
           "ms_per_step": round(ms, 4), "key_switches_per_s": round(2 / (ms / 1e3), 1),
           "ciphertext_bytes": 2 * nb, "ops": ops}
    ctx.close()
    return res


def run_serving(ctx, ps, seed, args):
    """Served requests (op chains at levels 10..30, 10 % ending in a bootstrap)
    through the continuous-batching server: saturation throughput with every
    request queued at t = 0, the same requests run one at a time (plain), and
    Poisson arrivals at fractions of saturation with p50 / p99 latency."""
    import torch

    from paper_2507_04775_amd import bootplan, ckks, inputs
    from paper_2507_04775_amd.serve import Server

    def rkey(sd, g):
        mods = (list(ps.q) + list(ps.p)) * (2 * ps.dnum)
        d = inputs.device_residues(sd, mods, ps.N).reshape(ps.dnum, 2, -1, ps.N).contiguous()
        return ctx.key(d, g)

    rs = inputs.batch_rotation_set(ps.logn)
    rot = {k: rkey(seed + 100 + k, pow(5, k, 2 * ps.N)) for k in rs}
    relin = rkey(seed + 1, 0)
    pts = [inputs.device_residues(seed + 7 + i, ps.q, ps.N) for i in range(4)]
    cfg = bootplan.default_config(ps.logn, 2.0 ** ps.log_scale)
    pl = bootplan.plan(ps.q, cfg)
    bkeys = {k: rkey(seed + 5000 + k, pow(5, k, 2 * ps.N)) for k in pl.rotations}
    boot_conj, boot_sparse = rkey(seed + 2, 2 * ps.N - 1), (rkey(seed + 3, 0), rkey(seed + 4, 0))
    boot = ckks.Boot(ctx, cfg.cts_radix_logs, cfg.stc_radix_logs, pl.cts, pl.stc, pl.cheb, cfg.double_angles,
                     cfg.top_scale, relin, boot_conj, bkeys, sparse=boot_sparse, hoist_moddown=cfg.hoist_moddown, input_gain=cfg.input_gain)
    boots = [boot] + [ckks.Boot(ctx, cfg.cts_radix_logs, cfg.stc_radix_logs, pl.cts, pl.stc, pl.cheb,
                                cfg.double_angles, cfg.top_scale, relin, boot_conj, bkeys, sparse=boot_sparse,
                                hoist_moddown=cfg.hoist_moddown, input_gain=cfg.input_gain) for _ in range(args.serve_boot_handles - 1)]
    srv = Server(ctx, relin, rot, pts, boots, slots=args.serve_slots, mem_budget=args.serve_mem_gib << 30)
    n = args.serve_requests
    gen = lambda rate, sd, m=n: inputs.serving_requests(sd, m, ps.logn, rate)
    srv.run(gen(None, seed + 900, max(8, n // 16)))  # warm-up

    def summarise(done, reqs):
        ok = [d for d in done if not d.refused]
        lat = [d.latency * 1e3 for d in ok]
        span = max(d.finish for d in ok) - min(r.arrival for r in reqs)
        ks = sum(d.keyswitches for d in ok)
        return {"requests_per_s": round(len(ok) / span, 2), "key_switches_per_s": round(ks / span, 1),
                "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
                "makespan_s": round(span, 4), "completed": len(ok), "refused": len(done) - len(ok)}

    reqs = gen(None, seed + 901)
    sat = summarise(srv.run(reqs), reqs)
    print("bench: serving saturation %.1f requests/s" % sat["requests_per_s"], file=sys.stderr, flush=True)
    plain = summarise(srv.run(reqs, concurrent=False), reqs)
    sweep = []
    for f in [float(x) for x in args.serve_loads.split(",") if x]:
        rate = f * sat["requests_per_s"]
        rq = gen(rate, seed + 902 + int(f * 100))
        r = summarise(srv.run(rq), rq)
        r.update({"load": f, "offered_rps": round(rate, 2)})
        sweep.append(r)
        print("bench: serving load %.2f done" % f, file=sys.stderr, flush=True)
    for b in boots:
        b.close()
    return {"requests": n, "slots": args.serve_slots, "mem_budget_gib": args.serve_mem_gib,
            "boot_handles": len(boots), "boot_fraction": 0.1, "saturation": sat, "plain_sequential": plain,
            "poisson": sweep, "served_vs_plain": round(sat["requests_per_s"] / plain["requests_per_s"], 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library runs the key-switching path on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_04775_amd import ckks, inputs

    torch.cuda.set_device(0)
    ps = inputs.params("large")
    level = ps.L
    ctx = ckks.Context(ps.logn, ps.q, ps.p, ps.dnum, device=0)
    seed = inputs.BASE_SEED + 1
    k_rot = inputs.rotation_index(seed, ps.logn)
    g_rot = pow(5, k_rot, 2 * ps.N)

    def make_set(s):
        a = inputs.random_ct(s, ps, level)
        b = inputs.random_ct(s + 1, ps, level)
        ta = ckks.Ciphertext(ckks.to_device(a[0]), ckks.to_device(a[1]), level, 2.0 ** ps.log_scale)
        tb = ckks.Ciphertext(ckks.to_device(b[0]), ckks.to_device(b[1]), level, 2.0 ** ps.log_scale)
        rlk = ctx.key(ckks.to_device(inputs.random_key(s + 2, ps)), 0)
        rk = ctx.key(ckks.to_device(inputs.random_key(s + 3, ps)), g_rot)
        return ta, tb, rlk, rk

    # ---- autotuner: NTT tile width per direction and launch size (cached by logN, limbs, K, op, arch)
    from paper_2507_04775_amd import tune
    tcache = tune.load_cache()
    t0 = time.perf_counter()
    tiles = tune.tune_ntt_tiles(ctx, cache=tcache)
    big = tune.tune_op_launches(ctx, level, cache=tcache)
    t_tune = time.perf_counter() - t0
    tune.save_cache(tcache)
    step_launches = {"ntt_inv": [31, 8, 2, 35], "ntt_fwd": [35, 31, 8, 2]}
    autotune = {"ntt_tiles_s": round(t_tune, 2), "cache": tune.cache_path(),
                "ntt_tiles": {op: {str(n): tiles[op][n] for n in ns if n in tiles.get(op, {})}
                              for op, ns in step_launches.items()},
                "ntt_tiles_in_ops": {str(k): v for k, v in big.get("ntt_fwd", {}).items()}}

    sets = [make_set(seed + 10 * i) for i in range(max(1, args.cold_sets))]
    m = ctx.empty_ct(level)
    r = ctx.empty_ct(level - 1)
    rot = ctx.empty_ct(level)
    ws_h = ctx.workspace(ckks.OP_HMULT, level)
    ws_r = ctx.workspace(ckks.OP_RESCALE, level)
    ws_k = ctx.workspace(ckks.OP_ROTATE, level)
    stream = torch.cuda.current_stream()

    def hmult(s):
        ta, tb, rlk, _ = s
        ctx.ckks_hmult_relin(ta, tb, rlk, m, ws_h)

    def rescale(s):
        ctx.ckks_rescale(m, r, ws_r)

    def hrotate(s):
        ta, _, _, rk = s
        ctx.ckks_hrotate(ta, k_rot, rk, rot, ws_k)

    def step(s):
        hmult(s)
        rescale(s)
        hrotate(s)

    # ---- warm-up, then the timed region (same buffers every step: warm)
    for _ in range(args.warmup):
        step(sets[0])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step(sets[0])
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    total_ms = ev[0].elapsed_time(ev[-1])
    ms_per_step = total_ms / args.steps
    ks_per_step = 2
    value = ks_per_step * args.steps / (total_ms / 1e3)

    # ---- cold pool: every step on another ciphertext pair and key set
    cold = None
    if len(sets) > 1:
        for s in sets:
            step(s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n_cold = max(len(sets), args.steps)
        e0.record(stream)
        for i in range(n_cold):
            step(sets[i % len(sets)])
        e1.record(stream)
        torch.cuda.synchronize()
        cold_ms = e0.elapsed_time(e1) / n_cold
        pool_bytes = len(sets) * (4 * (level + 1) + 2 * ps.dnum * 2 * (ps.L + 1 + ps.K)) * ps.N * 8
        cold = {"ms_per_step": round(cold_ms, 4), "key_switches_per_s": round(ks_per_step / (cold_ms / 1e3), 1),
                "pool_bytes": pool_bytes, "sets": len(sets)}

    # ---- per-operation latencies: GPU time of back-to-back calls, the stream held until all are enqueued
    def op_stats(fn, reps):
        xs = timed_launches(lambda: fn(sets[0]), reps, stream)
        return {"p50_us": round(percentile(xs, 50) * 1e3, 2), "p99_us": round(percentile(xs, 99) * 1e3, 2),
                "mean_us": round(sum(xs) / len(xs) * 1e3, 2)}

    reps = max(20, args.steps)
    ops = {"hmult_relin": op_stats(hmult, reps), "rescale": op_stats(rescale, reps), "hrotate": op_stats(hrotate, reps)}
    ntt_poly = ctx.empty_poly(ps.L + ps.K)
    ntt_poly.copy_(ckks.to_device(inputs.uniform_residues(inputs.rng(seed + 99), list(ps.q) + list(ps.p), ps.N)))
    # the roofline kernel runs on inputs in HBM: 16 polynomials of 35 limbs (294 MB, more than the
    # 256 MB last-level cache) in turn, so no launch finds its data in a cache left by an earlier one
    ntt_ring = [ntt_poly] + [ntt_poly.clone() for _ in range(15)]
    turn = [0]

    def ntt_next(inverse):
        p = ntt_ring[turn[0] % len(ntt_ring)]
        turn[0] += 1
        (ctx.ckks_intt if inverse else ctx.ckks_ntt)(p)

    ops["ntt_35_limbs"] = op_stats(lambda s: ntt_next(False), reps)
    ops["intt_35_limbs"] = op_stats(lambda s: ntt_next(True), reps)

    # the roofline launch time: one event pair around a burst of back-to-back launches, so no event
    # and no host-side delay between calls falls inside the average (per-call events add both)
    def burst_us(inverse, n):
        for _ in range(4):
            ntt_next(inverse)
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b0.record(stream)
        for _ in range(n):
            ntt_next(inverse)
        b1.record(stream)
        torch.cuda.synchronize()
        return b0.elapsed_time(b1) / n * 1e3

    ntt_burst_us = burst_us(False, 4 * reps)

    # ---- the rest of Table I at level L: HSquare, then the support operations on whole ciphertexts
    # (memory-bound: HAdd reads 4 and writes 2 polynomials of L+1 limbs)
    pt = ctx.empty_poly(level)
    pt.copy_(ckks.to_device(inputs.random_poly(seed + 98, ps, level)))
    scal = [int(q) - 7 for q in ps.q[: level + 1]]
    sup = ctx.empty_ct(level)
    ops["hsquare"] = op_stats(lambda s: ctx.ckks_hsquare(s[0], s[2], m, ws_h), reps)
    ops["hadd"] = op_stats(lambda s: ctx.ckks_hadd(s[0], s[1], sup), reps)
    ops["ptadd"] = op_stats(lambda s: ctx.ckks_ptadd(s[0], pt, sup), reps)
    ops["ptmult"] = op_stats(lambda s: ctx.ckks_ptmult(s[0], pt, 2.0 ** ps.log_scale, sup), reps)
    ops["scalar_add"] = op_stats(lambda s: ctx.ckks_scalar_add(s[0], scal, sup), reps)
    ops["scalar_mult"] = op_stats(lambda s: ctx.ckks_scalar_mult(s[0], scal, 1.0, sup), reps)

    # ---- NTT / INTT over the 31 ciphertext limbs alone
    def ntt31_next(inverse):
        p = ntt_ring[turn[0] % len(ntt_ring)][: ps.L + 1]
        turn[0] += 1
        (ctx.ckks_intt if inverse else ctx.ckks_ntt)(p, 0, ps.L + 1)

    ops["ntt_31_limbs"] = op_stats(lambda s: ntt31_next(False), reps)
    ops["intt_31_limbs"] = op_stats(lambda s: ntt31_next(True), reps)

    # ---- HMult+relin (one key switch) against the level (the paper's Fig. 6 workload), mean us
    hmult_by_level = {}
    for lv in (30, 25, 20, 15, 10, 5, 1, 0):
        xa = ckks.Ciphertext(sets[0][0].c0[: lv + 1], sets[0][0].c1[: lv + 1], lv, 1.0)
        xb = ckks.Ciphertext(sets[0][1].c0[: lv + 1], sets[0][1].c1[: lv + 1], lv, 1.0)
        xo, wlv = ctx.empty_ct(lv), ctx.workspace(ckks.OP_HMULT, lv)
        hmult_by_level[str(lv)] = op_stats(
            lambda s, xa=xa, xb=xb, xo=xo, wlv=wlv: ctx.ckks_hmult_relin(xa, xb, s[2], xo, wlv), reps)["mean_us"]

    # ---- PtMult + Rescale against the level (the paper's Fig. 5 workload), mean us per pair
    ptmult_rescale = {}
    for lv in (30, 25, 20, 15, 10, 5, 1):
        src = ckks.Ciphertext(sets[0][0].c0[: lv + 1], sets[0][0].c1[: lv + 1], lv, 2.0 ** ps.log_scale)
        prod, low = ctx.empty_ct(lv), ctx.empty_ct(lv - 1)
        ws_lv = ctx.workspace(ckks.OP_RESCALE, lv)

        def pair(s, src=src, prod=prod, low=low, ws_lv=ws_lv, lv=lv):
            ctx.ckks_ptmult(src, pt[: lv + 1], 2.0 ** ps.log_scale, prod)
            ctx.ckks_rescale(prod, low, ws_lv)

        ptmult_rescale[str(lv)] = op_stats(pair, reps)["mean_us"]

    if args.copy_calibration:
        # 1 GiB copied once; a 512 MiB fill in between evicts the source from the 256 MiB last-level
        # cache, so the copy's counters see the full read and write
        src = torch.empty(128 << 20, dtype=torch.int64, device="cuda").fill_(1)
        flush = torch.empty(64 << 20, dtype=torch.int64, device="cuda").fill_(2)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush

    # ---- the NTT over all 35 limbs (two passes, 16 x 35 workgroups each), timed on the library's stream
    # with inputs in HBM (rotating buffers, above) as the mean over a burst of launches; algorithmic
    # bytes = read + write of every limb once.
    ntt_ms = ntt_burst_us / 1e3
    ntt_bytes = (ps.L + 1 + ps.K) * ps.N * 8 * 2
    ntt_gbs = ntt_bytes / (ntt_ms / 1e3) / 1e9
    ntt_roof = {"bound": "hbm", "kernel": "ntt16_fwd (column + row pass) over 35 limbs",
                "achieved": round(ntt_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ntt_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "algorithmic_bytes_per_launch": ntt_bytes, "launch_us": round(ntt_ms * 1e3, 2)}

    # ---- the dominant kernel of the step: the key inner product (one launch per key switch, the largest
    # single-kernel share of the step with ModDown's conversion pass), at l = 30 on inputs in HBM: two
    # operand sets (ext, key, acc: 385 limbs, 202 MB each) in turn, so no launch finds its operands in the
    # 256 MB last-level cache; mean over a burst of launches between two events on the library's stream.
    roofline = inner_product_roofline(ctx, ps, seed, stream)

    # ---- the step and one key switch against HBM in algorithmic bytes: per coefficient-limb, HMult+relin
    # reads a, b (4n) and the key (2 beta (n+K)) and writes 2n; Rescale reads 2n and writes 2(n-1);
    # HRotate reads 2n + key and writes 2n; a key switch reads d (n) and the key and writes 2n
    n_l, beta = level + 1, ctx.beta(level)
    key_limbs = 2 * beta * (n_l + ps.K)
    step_limbs = (6 * n_l + key_limbs) + (4 * n_l - 2) + (4 * n_l + key_limbs)
    step_bytes = step_limbs * LIMB
    ks_bytes = (3 * n_l + key_limbs) * LIMB
    ks_o0, ks_o1 = ctx.empty_poly(level), ctx.empty_poly(level)
    ws_ks = ctx.workspace(ckks.OP_KEYSWITCH, level)
    ks_ms = timed_launches(lambda: ctx.ckks_keyswitch(sets[0][1].c1, level, sets[0][2], ks_o0, ks_o1, ws_ks, stream),
                           reps, stream)
    ks50 = percentile(ks_ms, 50)
    hbm = {"step": {"algorithmic_bytes": step_bytes, "ms": round(ms_per_step, 4),
                    "achieved_GBs": round(step_bytes / (ms_per_step / 1e3) / 1e9, 1),
                    "frac": round(step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
           "keyswitch": {"algorithmic_bytes": ks_bytes, "p50_ms": round(ks50, 4),
                         "p99_ms": round(percentile(ks_ms, 99), 4),
                         "achieved_GBs": round(ks_bytes / (ks50 / 1e3) / 1e9, 1),
                         "frac": round(ks_bytes / (ks50 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}
    probe = None if args.no_probe else run_probe(stream)
    valu = valu_fractions(probe)

    # ---- batched: 128 ciphertexts at levels 4..30, half HMult+relin, half hoisted 8-way rotations
    batched = None
    if not args.no_batch:
        batched = run_batch(ctx, ps, seed, args, tcache)
        tune.save_cache(tcache)

    # ---- full-slot bootstrapping (its own context: ten special primes)
    boot = boot_dense = None
    if not args.no_boot:
        boot = run_bootstrap(seed + 500, args, sparse=True)
        if not args.no_uniform_boot:
            boot_dense = run_bootstrap(seed + 600, args, sparse=False)

    # ---- the 32-bit word path on the same modulus budget
    w32 = None if args.no_w32 else run_w32(seed + 800, args)

    # ---- served request chains with continuous batching
    serving = None
    if not args.no_serve:
        serving = run_serving(ctx, ps, seed + 700, args)

    # ---- CPU oracle on a bounded sample of the same step: medians over runs on one thread and on all cores
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ps, seed, level, g_rot, ks_per_step, max(3, args.cpu_runs))

    out = {
        "metric": "key-switches/s and bootstraps/s at logN=16 (1 GPU), batched vs plain; p99 latency",
        "value": round(value, 1),
        "unit": "key-switches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded uniform residues; timing is value-independent)",
        "config": {"workload": "HMult+relin + Rescale + HRotate at level 30", "logN": ps.logn,
                   "limbs": ps.L + 1, "special_primes": ps.K, "dnum": ps.dnum, "key_switches_per_step": ks_per_step,
                   "parallelism": "single GPU"},
        "step_p50_ms": round(percentile(step_ms, 50), 4),
        "step_p99_ms": round(percentile(step_ms, 99), 4),
        "wall_s": round(wall, 3),
        "cold": cold,
        "batched": batched,
        "bootstrap": boot,
        "bootstrap_uniform_secret": boot_dense,
        "serving": serving,
        "words32": w32,
        "ops": ops,
        "ptmult_rescale_us_by_level": ptmult_rescale,
        "hmult_relin_us_by_level": hmult_by_level,
        "autotune": autotune,
        "roofline": roofline,
        "roofline_ntt_35_limbs": ntt_roof,
        "hbm_fraction": hbm,
        "valu": valu,
        "mad64_probe": probe,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
