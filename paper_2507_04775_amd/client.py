"""Client-side CKKS on top of the library: encoding, secret-key encryption,
decryption and evaluation-key generation.

The paper leaves these operations to the client library (Sec. III-A); they
are provided here so that the benchmark, the serving loop and users of the
library can work on real encryptions.  Every operation on residues runs in
the GPU library through its C ABI (NTT, limb-wise products, automorphisms);
the host only draws random numbers (from the seeded generators in
``inputs``) and does the floating-point FFT of encoding and decoding.

Conventions (those of the library's documentation): slot j of a plaintext
m(X) is m(zeta^(5^j mod 2N)) / scale with zeta = exp(i pi / N); encryption is
c1 = a, c0 = -a s + m + e; the key for s' has, for digit j (alpha consecutive
q limbs), k_j1 = a_j and k_j0 = -a_j s + e_j plus [P]_(q_i) s' on the rows q_i
of digit j, P the product of the special primes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ckks, inputs


def slots_to_coeffs(z: np.ndarray, logn: int) -> np.ndarray:
    """Real coefficients m with m(zeta^(5^j)) = z_j: m_k = (2/N) Re sum_j z_j zeta^(-5^j k)."""
    N = 1 << logn
    W = np.zeros(2 * N, complex)
    W[[pow(5, j, 2 * N) for j in range(N // 2)]] = z
    return (2.0 / N) * np.real(np.fft.fft(W)[:N])


def coeffs_to_slots(m: np.ndarray, logn: int) -> np.ndarray:
    """z_j = sum_k m_k zeta^(5^j k) for real m."""
    N = 1 << logn
    F = np.fft.fft(np.concatenate([m, np.zeros(N)]))
    return np.conj(F[[pow(5, j, 2 * N) for j in range(N // 2)]])


def _round(v: np.ndarray) -> np.ndarray:
    return np.where(v < 0, -np.floor(-v + 0.5), np.floor(v + 0.5))


class Client:
    def __init__(self, ctx: ckks.Context, ps: inputs.ParamSet, seed: int):
        self.ctx, self.ps = ctx, ps
        self.N, self.logn = ps.N, ps.logn
        self.mods = [int(m) for m in list(ps.q) + list(ps.p)]
        self.rows = len(self.mods)
        self.g = inputs.rng(seed)
        self.seed = seed
        self._draws = 0
        self.s_coeffs = inputs.ternary(self.g, self.N)
        self.s = self._small(self.s_coeffs, self.rows)
        P = 1
        for p in ps.p:
            P *= int(p)
        self.P_mod_q = [P % int(q) for q in ps.q]

    # -- residues on the device
    def _small(self, v: np.ndarray, nrows: int) -> torch.Tensor:
        """Signed int64 coefficients -> evaluation-domain rows 0..nrows-1 on the device."""
        r = np.empty((nrows, self.N), dtype=np.uint64)
        for i in range(nrows):
            r[i] = np.mod(v, self.mods[i]).astype(np.uint64)
        t = ckks.to_device(r, self.ctx.device)
        self.ctx.ckks_ntt(t, 0, nrows)
        return t

    def _uniform(self, nrows: int) -> torch.Tensor:
        self._draws += 1
        return inputs.device_residues(self.seed * 1000003 + self._draws, self.mods[:nrows], self.N,
                                      device=self.ctx.device)

    def _error(self, nrows: int) -> torch.Tensor:
        return self._small(inputs.gaussian(self.g, self.N, self.ps.sigma), nrows)

    # -- encoding
    def encode(self, z: np.ndarray, level: int, scale: float) -> torch.Tensor:
        m = _round(slots_to_coeffs(np.asarray(z, complex), self.logn) * scale)
        if np.max(np.abs(m)) >= 2.0 ** 62:
            raise ValueError("scale too large for the message")
        return self._small(m.astype(np.int64), level + 1)

    def decode(self, pt: torch.Tensor, level: int, scale: float) -> np.ndarray:
        """Decode from the two lowest limbs (exact while |m| < q_0 q_1 / 2)."""
        c = pt[:2].clone() if level >= 1 else pt[:1].clone()
        self.ctx.ckks_intt(c, 0, c.shape[0])
        x = ckks.to_host(c)
        q0 = self.mods[0]
        if level == 0:
            v = np.array([int(a) - q0 if int(a) > q0 // 2 else int(a) for a in x[0]], dtype=float)
        else:
            q1 = self.mods[1]
            inv = pow(q0, -1, q1)
            Q = q0 * q1
            vals = []
            for a, b in zip(x[0].tolist(), x[1].tolist()):
                t = a + q0 * (((b - a) * inv) % q1)
                vals.append(float(t - Q if t > Q // 2 else t))
            v = np.array(vals)
        return coeffs_to_slots(v / scale, self.logn)

    # -- encryption
    def encrypt(self, z: np.ndarray, level: int, scale: float) -> ckks.Ciphertext:
        m = self.encode(z, level, scale)
        a = self._uniform(level + 1)
        e = self._error(level + 1)
        c0 = torch.empty_like(a)
        self.ctx.ckks_poly_mul(a, self.s, c0, level)
        self.ctx.ckks_poly_sub(e, c0, c0, level)
        self.ctx.ckks_poly_add(c0, m, c0, level)
        return ckks.Ciphertext(c0, a, level, scale)

    def decrypt(self, ct: ckks.Ciphertext) -> np.ndarray:
        l = ct.level
        m = torch.empty_like(ct.c0[: l + 1])
        self.ctx.ckks_poly_mul(ct.c1[: l + 1].contiguous(), self.s, m, l)
        self.ctx.ckks_poly_add(ct.c0[: l + 1].contiguous(), m, m, l)
        return self.decode(m, l, ct.scale)

    # -- evaluation keys
    def switch_key(self, s_prime: torch.Tensor, galois: int, target: torch.Tensor | None = None) -> ckks.Key:
        """Key switching s' to `target` (the secret key by default)."""
        ps, R, N = self.ps, self.rows, self.N
        target = self.s if target is None else target
        nq = len(ps.q)
        alpha = -(-nq // ps.dnum)
        key = torch.empty((ps.dnum, 2, R, N), dtype=torch.uint64, device=self.ctx.device)
        t = torch.empty((R, N), dtype=torch.uint64, device=self.ctx.device)
        for j in range(ps.dnum):
            a = self._uniform(R)
            b = self._error(R)
            self.ctx.ckks_poly_mul(a, target, t, R - 1)
            self.ctx.ckks_poly_sub(b, t, b, R - 1)
            sc = [self.P_mod_q[i] if j * alpha <= i < min((j + 1) * alpha, nq) else 0 for i in range(R)]
            self.ctx.ckks_poly_scalar_mul(s_prime, sc, t, R - 1)
            self.ctx.ckks_poly_add(b, t, b, R - 1)
            key[j, 0].copy_(b)
            key[j, 1].copy_(a)
        return self.ctx.key(key, galois)

    def relin_key(self) -> ckks.Key:
        s2 = torch.empty_like(self.s)
        self.ctx.ckks_poly_mul(self.s, self.s, s2, self.rows - 1)
        return self.switch_key(s2, 0)

    def galois_key(self, g: int) -> ckks.Key:
        sg = torch.empty_like(self.s)
        self.ctx.ckks_automorph(self.s, g, sg, self.rows)
        return self.switch_key(sg, g)

    def rotation_key(self, k: int) -> ckks.Key:
        return self.galois_key(pow(5, k % (self.N // 2), 2 * self.N))

    def conjugation_key(self) -> ckks.Key:
        return self.galois_key(2 * self.N - 1)

    def sparse_keys(self, h: int) -> tuple:
        """Switching keys s -> s' and s' -> s for a fresh sparse secret s' with h
        nonzero coefficients (the encapsulation used by bootstrapping)."""
        sp = self._small(inputs.sparse_ternary(self.g, self.N, h), self.rows)
        return self.switch_key(self.s, 0, target=sp), self.switch_key(sp, 0)
