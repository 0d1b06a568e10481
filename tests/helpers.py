"""Shared helpers for the tests: parameter objects for the oracle and seeded
client material (keys, encryptions) built only from the oracle's client."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import client
from paper_2507_04775_amd import inputs


def oracle_params(ps: inputs.ParamSet) -> oracle.Params:
    return oracle.Params(ps.logn, ps.q, ps.p, ps.dnum)


def br(i: int, bits: int) -> int:
    return int(format(i, "0%db" % bits)[::-1], 2) if bits else 0


class ClientSetup:
    """A secret key plus relinearisation / Galois keys drawn from a fixed seed."""

    def __init__(self, ps: inputs.ParamSet, seed: int):
        self.ps = ps
        self.P = oracle_params(ps)
        self.g = inputs.rng(seed)
        self.sk = client.SecretKey(self.P, inputs.ternary(self.g, ps.N))
        self._keys = {}

    def _masks_errors(self):
        allm = list(self.ps.q) + list(self.ps.p)
        masks = [inputs.uniform_residues(self.g, allm, self.ps.N) for _ in range(self.ps.dnum)]
        errors = [inputs.gaussian(self.g, self.ps.N, self.ps.sigma) for _ in range(self.ps.dnum)]
        return masks, errors

    def relin_key(self):
        if "relin" not in self._keys:
            self._keys["relin"] = client.gen_relin_key(self.P, self.sk, *self._masks_errors())
        return self._keys["relin"]

    def galois_key(self, g: int):
        if g not in self._keys:
            self._keys[g] = client.gen_galois_key(self.P, self.sk, g, *self._masks_errors())
        return self._keys[g]

    def sparse_keys(self, h: int):
        """Switching keys s -> s' and s' -> s for a sparse secret s' with h nonzero coefficients."""
        if ("sparse", h) not in self._keys:
            sp = client.SecretKey(self.P, inputs.sparse_ternary(self.g, self.ps.N, h))
            to_sp = client.gen_switch_key(self.P, sp, self.sk.eval_all, *self._masks_errors())
            from_sp = client.gen_switch_key(self.P, self.sk, sp.eval_all, *self._masks_errors())
            self._keys[("sparse", h)] = (to_sp, from_sp)
        return self._keys[("sparse", h)]

    def encrypt(self, z, level: int, scale: float | None = None):
        scale = float(2 ** self.ps.log_scale) if scale is None else scale
        pt = client.encode(self.P, z, level, scale)
        mask = inputs.uniform_residues(self.g, self.ps.q[: level + 1], self.ps.N)
        err = inputs.gaussian(self.g, self.ps.N, self.ps.sigma)
        return client.encrypt(self.P, self.sk, pt, level, mask, err)

    def decrypt(self, ct, level: int, scale: float):
        return client.decode(self.P, client.decrypt(self.P, self.sk, ct, level), level, scale)


def max_err_bits(a, b) -> float:
    d = np.max(np.abs(np.asarray(a) - np.asarray(b)))
    return float(np.log2(d)) if d > 0 else -np.inf
