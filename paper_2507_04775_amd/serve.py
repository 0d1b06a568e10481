"""A continuous-batching server for homomorphic op chains on one GPU.

Requests (``inputs.Request``) arrive over time, each an op chain (HMult+relin
then Rescale, plaintext multiply-add then Rescale, HRotate) on two fresh
ciphertexts, some ending in a bootstrap.  Evaluation keys, the plaintext pool
and the bootstrap handle stay resident in HBM.  The server admits a request
as soon as it has arrived, a slot (a HIP stream with its own workspace) is
free and its buffers fit the memory budget; admitted requests run
concurrently, each on its own stream, so requests that arrive while others
are on the GPU overlap with them.  Bootstraps share one handle and therefore
run on one stream of their own, ordered after their request's chain by an
event.  Every operation is a call of the library's C ABI: the host only
schedules.  Results do not depend on the mix: every kernel is deterministic
and a request's buffers are its own.
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

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


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
                 boot: Optional[ckks.Boot] = None, slots: int = 8, mem_budget: int = 8 << 30):
        self.ctx, self.relin, self.rot_keys, self.pts, self.boot = ctx, relin, rot_keys, pts, boot
        self.N, self.L = ctx.N, ctx.nq - 1
        words = max(ctx.workspace_bytes(op, self.L) for op in (ckks.OP_HMULT, ckks.OP_ROTATE, ckks.OP_RESCALE))
        self.streams = [torch.cuda.Stream(device=ctx.device) for _ in range(slots)]
        self.ws = [torch.empty((words + 7) // 8, dtype=torch.uint64, device=ctx.device) for _ in range(slots)]
        self.boot_stream = torch.cuda.Stream(device=ctx.device)
        self.mem_budget = mem_budget

    # ---------------------------------------------------------------- helpers
    def _ct_bytes(self, level: int) -> int:
        return 2 * (level + 1) * self.N * 8

    def footprint(self, r: inputs.Request) -> int:
        b = 3 * self._ct_bytes(r.level)
        if r.boot and self.boot is not None:
            b += self._ct_bytes(self.boot.output_level)
        return b

    def _new_ct(self, level: int) -> ckks.Ciphertext:
        t = torch.empty((2, level + 1, self.N), dtype=torch.uint64, device=self.ctx.device)
        return ckks.Ciphertext(t[0], t[1], level)

    @staticmethod
    def _view(c: ckks.Ciphertext, level: int) -> ckks.Ciphertext:
        return ckks.Ciphertext(c.c0[: level + 1], c.c1[: level + 1], level, c.scale)

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
        if r.boot and self.boot is not None:
            out = self._new_ct(self.boot.output_level)
            a.bufs.append(out)
            ev = torch.cuda.Event()
            ev.record(st)
            self.boot_stream.wait_event(ev)
            self.boot.ckks_bootstrap(self._view(A, 0), out, self.boot_stream)
            a.done.record(self.boot_stream)
            a.out = out
            ks += self.boot.keyswitches
        else:
            a.done.record(st)
            a.out = A
        a.keyswitches = ks

    # ---------------------------------------------------------------- serving
    def run(self, requests, keep_outputs: bool = False, concurrent: bool = True):
        """Serve `requests` (arrival times in seconds from the start).  With
        concurrent=False each request runs alone, after the previous one has
        finished, ignoring arrival times."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        nslots = len(self.streams) if concurrent else 1
        free = list(range(nslots))
        used = 0
        active: list = []
        done: list = []
        torch.cuda.synchronize()
        origin = torch.cuda.Event(enable_timing=True)
        origin.record(self.streams[0])
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            progressed = False
            while pending and free and (not concurrent or pending[0].arrival <= now):
                r = pending[0]
                need = self.footprint(r)
                if active and used + need > self.mem_budget:
                    break
                pending.pop(0)
                slot = free.pop(0)
                a = _Active(req=r, slot=slot, bytes=need, admitted=time.perf_counter() - t0,
                            done=torch.cuda.Event(enable_timing=True))
                self._enqueue(r, slot, a)
                used += need
                active.append(a)
                progressed = True
                if not concurrent:
                    break
            still = []
            for a in active:
                if a.done.query():
                    out = None
                    if keep_outputs:
                        o = a.out
                        out = (o.c0[: o.level + 1].cpu().numpy(), o.c1[: o.level + 1].cpu().numpy(), o.level)
                    done.append((a, out))
                    free.append(a.slot)
                    used -= a.bytes
                    progressed = True
                else:
                    still.append(a)
            active = still
            if not progressed:
                if not active and pending and concurrent:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
                else:
                    time.sleep(0.0001)
        torch.cuda.synchronize()
        res = []
        for a, out in done:
            finish = origin.elapsed_time(a.done) / 1e3
            res.append(Done(rid=a.req.rid, arrival=a.req.arrival if concurrent else 0.0, admitted=a.admitted,
                            finish=finish, keyswitches=a.keyswitches, output=out))
        return sorted(res, key=lambda d: d.rid)
