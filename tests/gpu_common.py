"""Shared fixtures of the GPU parity tests: a library context and the oracle
parameters of the same parameter set, seeded inputs for both."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2507_04775_amd import inputs


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


class Setup:
    def __init__(self, name: str):
        from paper_2507_04775_amd import ckks
        self.ps = inputs.params(name)
        self.P = oracle.Params(self.ps.logn, self.ps.q, self.ps.p, self.ps.dnum)
        self.ctx = ckks.Context(self.ps.logn, self.ps.q, self.ps.p, self.ps.dnum)
        self.ckks = ckks
        self.N = self.ps.N

    def dev(self, a: np.ndarray):
        return self.ckks.to_device(a)

    def host(self, t) -> np.ndarray:
        import torch
        torch.cuda.synchronize()
        return self.ckks.to_host(t)

    def key(self, seed: int, galois: int):
        k = inputs.random_key(seed, self.ps)
        return k, self.ctx.key(self.dev(k), galois)

    def ct(self, seed: int, level: int):
        c0, c1 = inputs.random_ct(seed, self.ps, level)
        return (c0, c1), self.ckks.Ciphertext(self.dev(c0), self.dev(c1), level, 1.0)


def assert_equal(got: np.ndarray, want: np.ndarray, what: str):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d mismatches, first at %s (got %d want %d)" % (
        what, len(bad), tuple(bad[0]), int(got[tuple(bad[0])]), int(want[tuple(bad[0])]))
