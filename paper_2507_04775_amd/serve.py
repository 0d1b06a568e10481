"""A continuous-batching server for homomorphic op chains on one GPU.

Requests (``inputs.Request``) arrive over time, each an op chain (HMult+relin
then Rescale, plaintext multiply-add then Rescale, HRotate) on two fresh
ciphertexts, some ending in a bootstrap.  Evaluation keys, the plaintext pool
and the bootstrap handles stay resident in HBM.

Admission (``Admission``): a request is refused at once when its buffers
alone exceed the memory budget; otherwise it is admitted as soon as it has
arrived, a slot (a HIP stream with its own workspace) is free and its buffers
fit beside those of the requests in flight.  Admitted requests run
concurrently, each on its own stream, so requests that arrive while others
are on the GPU overlap with them.  A request's buffers are released when its
completion event has fired, so device memory follows the requests in flight.

Bootstraps: a bootstrap handle owns its buffers, so calls on one handle run
one after another on that handle's stream; the server takes a list of
handles (built from the same keys and plaintexts) and gives each bootstrap
to the handle whose queue frees first, so bootstraps of different requests
overlap on the GPU.  A bootstrap waits for its request's chain through an
event.

Every operation is a call of the library's C ABI: the host only schedules.
Results do not depend on the mix: every kernel is deterministic, a request's
buffers are its own, and every bootstrap handle runs the same schedule.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import ckks, inputs


@dataclass
class Done:
    rid: int
    arrival: float
    admitted: float
    finish: float
    keyswitches: int
    output: Optional[tuple] = None
    refused: bool = False

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Admission:
    """Memory- and slot-based admission (host logic only).  `budget` bytes are
    shared by the requests in flight; `slots` requests run at once."""

    def __init__(self, slots: int, budget: int):
        self.free = list(range(slots))
        self.budget = budget
        self.used = 0

    def refuses(self, need: int) -> bool:
        """A request whose own buffers exceed the whole budget can never run."""
        return need > self.budget

    def admit(self, need: int) -> Optional[int]:
        """A free slot for a request of `need` bytes, or None to wait."""
        if not self.free or self.used + need > self.budget:
            return None
        self.used += need
        return self.free.pop(0)

    def release(self, slot: int, need: int):
        self.used -= need
        self.free.append(slot)


@dataclass
class _Active:
    req: inputs.Request
    slot: int
    bytes: int
    admitted: float
    done: torch.cuda.Event
    bufs: list = field(default_factory=list)
    out: Optional[ckks.Ciphertext] = None
    keyswitches: int = 0


class Server:
    def __init__(self, ctx: ckks.Context, relin: ckks.Key, rot_keys: dict, pts: list,
                 boot=None, slots: int = 8, mem_budget: int = 8 << 30):
        self.ctx, self.relin, self.rot_keys, self.pts = ctx, relin, rot_keys, pts
        self.boots = [] if boot is None else (list(boot) if isinstance(boot, (list, tuple)) else [boot])
        self.N, self.L = ctx.N, ctx.nq - 1
        words = max(ctx.workspace_bytes(op, self.L) for op in (ckks.OP_HMULT, ckks.OP_ROTATE, ckks.OP_RESCALE))
        self.slots = slots
        self.streams = [torch.cuda.Stream(device=ctx.device) for _ in range(slots)]
        self.ws = [torch.empty((words + 7) // 8, dtype=torch.uint64, device=ctx.device) for _ in range(slots)]
        self.boot_streams = [torch.cuda.Stream(device=ctx.device) for _ in self.boots]
        self.mem_budget = mem_budget
        self.mem_samples: list = []  # (requests in flight, their budgeted bytes, bytes allocated) per completion

    # ---------------------------------------------------------------- helpers
    def _ct_bytes(self, level: int) -> int:
        return 2 * (level + 1) * self.N * 8

    def footprint(self, r: inputs.Request) -> int:
        b = 3 * self._ct_bytes(r.level)
        if r.boot and self.boots:
            b += self._ct_bytes(self.boots[0].output_level)
        return b

    def _new_ct(self, level: int) -> ckks.Ciphertext:
        t = torch.empty((2, level + 1, self.N), dtype=torch.uint64, device=self.ctx.device)
        return ckks.Ciphertext(t[0], t[1], level)

    @staticmethod
    def _view(c: ckks.Ciphertext, level: int) -> ckks.Ciphertext:
        return ckks.Ciphertext(c.c0[: level + 1], c.c1[: level + 1], level, c.scale)

    def _pick_boot(self) -> int:
        """The handle whose queued bootstraps finish first (by count of unfinished ones)."""
        best, best_n = 0, None
        for h, q in enumerate(self._boot_queue):
            q[:] = [e for e in q if not e.query()]
            if best_n is None or len(q) < best_n:
                best, best_n = h, len(q)
        return best

    def _enqueue(self, r: inputs.Request, slot: int, a: _Active):
        ctx, st, ws = self.ctx, self.streams[slot], self.ws[slot]
        mods = ctx.q[: r.level + 1]
        with torch.cuda.stream(st):
            A, B, T = self._new_ct(r.level), self._new_ct(r.level), self._new_ct(r.level)
            for i, c in enumerate((A.c0, A.c1, B.c0, B.c1)):
                c.copy_(inputs.device_residues(r.seed * 4 + i, mods, self.N, device=ctx.device))
        a.bufs = [A, B, T]
        ks = 0
        for op in r.ops:
            l = A.level
            if op[0] == "hmult":
                T.level = l
                ctx.ckks_hmult_relin(A, self._view(B, l), self.relin, self._view(T, l), ws, st)
                out = self._view(A, l - 1)
                ctx.ckks_rescale(self._view(T, l), out, ws, st)
                A = ckks.Ciphertext(A.c0, A.c1, l - 1)
                ks += 1
            elif op[0] == "ptmuladd":
                pt = self.pts[r.rid % len(self.pts)][: l + 1]
                Bl = self._view(B, l)
                ctx.ckks_poly_mul_add(A.c0[: l + 1], pt, Bl.c0, T.c0[: l + 1], l, st)
                ctx.ckks_poly_mul_add(A.c1[: l + 1], pt, Bl.c1, T.c1[: l + 1], l, st)
                ctx.ckks_rescale(self._view(T, l), self._view(A, l - 1), ws, st)
                A = ckks.Ciphertext(A.c0, A.c1, l - 1)
            else:
                k = op[1]
                ctx.ckks_hrotate(self._view(A, l), k, self.rot_keys[k], self._view(T, l), ws, st)
                A, T = ckks.Ciphertext(T.c0, T.c1, l), ckks.Ciphertext(A.c0, A.c1, l)
                ks += 1
        if r.boot and self.boots:
            h = self._pick_boot()
            bst, boot = self.boot_streams[h], self.boots[h]
            ev = torch.cuda.Event()
            ev.record(st)
            bst.wait_event(ev)
            with torch.cuda.stream(bst):  # the output's memory belongs to the stream that writes it
                out = self._new_ct(boot.output_level)
            a.bufs.append(out)
            boot.ckks_bootstrap(self._view(A, 0), out, bst)
            a.done.record(bst)
            self._boot_queue[h].append(a.done)
            a.out = out
            ks += boot.keyswitches
        else:
            a.done.record(st)
            a.out = A
        a.keyswitches = ks

    # ---------------------------------------------------------------- serving
    def run(self, requests, keep_outputs: bool = False, concurrent: bool = True):
        """Serve `requests` (arrival times in seconds from the start).  With
        concurrent=False each request runs alone, after the previous one has
        finished, ignoring arrival times.  Requests larger than the memory
        budget come back refused (no output, no latency)."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        adm = Admission(self.slots if concurrent else 1, self.mem_budget)
        self._boot_queue = [[] for _ in self.boots]
        self.mem_samples = []
        active: list = []
        done: list = []
        refused: list = []
        torch.cuda.synchronize()
        origin = torch.cuda.Event(enable_timing=True)
        origin.record(self.streams[0])
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            progressed = False
            while pending and (not concurrent or pending[0].arrival <= now):
                r = pending[0]
                need = self.footprint(r)
                if adm.refuses(need):
                    pending.pop(0)
                    refused.append(Done(rid=r.rid, arrival=r.arrival if concurrent else 0.0,
                                        admitted=now, finish=now, keyswitches=0, refused=True))
                    progressed = True
                    continue
                if not concurrent and active:
                    break
                slot = adm.admit(need)
                if slot is None:
                    break
                pending.pop(0)
                a = _Active(req=r, slot=slot, bytes=need, admitted=time.perf_counter() - t0,
                            done=torch.cuda.Event(enable_timing=True))
                self._enqueue(r, slot, a)
                active.append(a)
                progressed = True
            still = []
            for a in active:
                if a.done.query():
                    out = None
                    if keep_outputs:
                        o = a.out
                        out = (o.c0[: o.level + 1].cpu().numpy(), o.c1[: o.level + 1].cpu().numpy(), o.level)
                    a.bufs, a.out = [], None  # the work on them has finished: back to the allocator
                    done.append((a, out))
                    adm.release(a.slot, a.bytes)
                    progressed = True
                else:
                    still.append(a)
            if len(still) != len(active):
                self.mem_samples.append((len(still), adm.used, torch.cuda.memory_allocated(self.ctx.device)))
            active = still
            if not progressed:
                if not active and pending and concurrent:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
                else:
                    time.sleep(0.0001)
        torch.cuda.synchronize()
        res = list(refused)
        for a, out in done:
            finish = origin.elapsed_time(a.done) / 1e3
            res.append(Done(rid=a.req.rid, arrival=a.req.arrival if concurrent else 0.0, admitted=a.admitted,
                            finish=finish, keyswitches=a.keyswitches, output=out))
        return sorted(res, key=lambda d: d.rid)
