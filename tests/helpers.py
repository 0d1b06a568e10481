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


def prod(xs) -> int:
    r = 1
    for x in xs:
        r *= int(x)
    return r


def crt(res, mods) -> int:
    """The integer in [0, prod(mods)) with the given residues (Python big ints)."""
    M = prod(mods)
    x = 0
    for r, m in zip(res, mods):
        Mi = M // int(m)
        x += int(r) * Mi * pow(Mi, -1, int(m))
    return x % M


def scaled_inputs(y: np.ndarray, mods) -> np.ndarray:
    """Coefficient rows a_i = [y_i (B/b_i)]_{b_i} over the basis B = mods, so that
    the scaled inputs of a fast base conversion from B, y_i = [a_i (B/b_i)^-1]_{b_i},
    are exactly the given y (canonical residues, shape [len(mods)][N])."""
    B = prod(mods)
    out = np.empty_like(y)
    for i, m in enumerate(mods):
        h = (B // int(m)) % int(m)
        out[i] = np.array([(int(v) * h) % int(m) for v in y[i]], dtype=np.uint64)
    return out


def edge_values(m: int) -> list:
    """Residues at the edges of the modular arithmetic for modulus m: 0, 1, the
    centring threshold (m-1)/2 and (m+1)/2, m-2, m-1, and the 32-bit word
    boundaries 2^32 - 1, 2^32, 2^32 + 1 (below m)."""
    vals = [0, 1, (m - 1) // 2, (m + 1) // 2, m - 2, m - 1, (1 << 31), (1 << 32) - 1, 1 << 32, (1 << 32) + 1]
    return [v for v in vals if v < m]


def edge_rows(seed: int, mods, N: int, shift: int = 0) -> np.ndarray:
    """Rows over `mods` whose first coefficients cycle through edge_values (row i
    shifted by i + shift, so the rows of one coefficient mix different edges);
    every fourth block of the rest is uniform, the others keep cycling."""
    g = inputs.rng(seed)
    out = np.empty((len(mods), N), dtype=np.uint64)
    for i, m in enumerate(mods):
        ev = edge_values(int(m))
        idx = (np.arange(N) + i + shift) % len(ev)
        row = np.array(ev, dtype=np.uint64)[idx]
        rnd = g.integers(0, int(m), size=N, dtype=np.uint64)
        blk = (np.arange(N) // 64) % 4 == 3
        row[blk] = rnd[blk]
        out[i] = row
    return out
