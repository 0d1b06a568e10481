"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no CKKS arithmetic: it chooses NTT-friendly primes (a
parameter choice, by a fixed scan and a Miller-Rabin test), and it draws
uniform residues, ternary secrets, rounded Gaussian errors and complex slot
vectors from numpy's PCG64 with fixed seeds.  The GPU library and the oracle
both consume these arrays; neither is imported here.

Parameter sets (sizes from the paper's evaluation, Sec. IV, and the workloads
this library is measured on):

* ``small``    : N = 2^12, q = 1 x 60-bit + 3 x 40-bit, dnum = 2, K = 1 special prime.
* ``small-nv`` : as ``small`` with K = 2 (the smallest K whose P exceeds the
                 largest digit, so decryptions after key switching are meaningful).
* ``large``    : N = 2^16, q = 1 x 60-bit + 30 x 50-bit, dnum = 3, K = 4.
* ``large-nv`` : as ``large`` with K = 10.
* ``large-fp`` : N = 2^16, q = 7 x 50-bit, K = 3 special primes of 50 bits, dnum = 3:
                 every prime below 2^50, so every limb (the special ones
                 included) takes the FP64 arithmetic.
* ``boot-small``: N = 2^12, q = 1 x 60-bit + 20 x 50-bit, dnum = 3, K = 7: the
                 smallest set with room for a full-slot bootstrap (18 levels).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 250704775

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (covers every 64-bit word)."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for b in _MR_BASES:
        x = pow(b, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, count: int, logn: int, skip: int = 0) -> list[int]:
    """The primes q = 2^bits - t*2N + 1, t = 1, 2, ..., in descending order.

    Every such prime is 1 mod 2N, so a primitive 2N-th root of unity exists.
    ``skip`` drops that many primes from the front of the scan.
    """
    two_n = 2 << logn
    out: list[int] = []
    t = 1
    while len(out) < skip + count:
        q = (1 << bits) - t * two_n + 1
        if q < (1 << (bits - 1)):
            raise ValueError("ran out of %d-bit primes" % bits)
        if is_prime(q):
            out.append(q)
        t += 1
    return out[skip:]


@dataclass
class ParamSet:
    name: str
    logn: int
    q: list[int]
    p: list[int]
    dnum: int
    log_scale: int
    sigma: float = 3.2
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return 1 << self.logn

    @property
    def L(self) -> int:
        return len(self.q) - 1

    @property
    def K(self) -> int:
        return len(self.p)

    @property
    def alpha(self) -> int:
        return -(-len(self.q) // self.dnum)

    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)


def make_params(logn: int, small_bits: int, L: int, K: int, dnum: int, log_scale: int, name: str) -> ParamSet:
    """q_0 = first 60-bit prime, p_0..p_{K-1} = the next K 60-bit primes,
    q_1..q_L = the first L primes of ``small_bits`` bits."""
    big = ntt_primes(60, 1 + K, logn)
    small = ntt_primes(small_bits, L, logn)
    return ParamSet(name=name, logn=logn, q=[big[0]] + small, p=big[1:], dnum=dnum, log_scale=log_scale)


def params32(name: str) -> ParamSet:
    """Parameter sets of the 32-bit word path (N = 2^16, every prime a 30-bit
    NTT prime, q_0.. first, then p_0..): "w32-small" 10 + 3 primes, dnum 3
    (digits of 4, 4, 2); "w32-large" 52 + 8 primes, dnum 4 (digits of 13), a
    1560-bit Q and 240-bit P like the 64-bit "large" set."""
    if name == "w32-small":
        nq, K, dnum = 10, 3, 3
    elif name == "w32-large":
        nq, K, dnum = 52, 8, 4
    else:
        raise KeyError(name)
    pr = ntt_primes(30, nq + K, 16)
    return ParamSet(name=name, logn=16, q=pr[:nq], p=pr[nq:], dnum=dnum, log_scale=26)


def params(name: str) -> ParamSet:
    if name == "small":
        return make_params(12, 40, 3, 1, 2, 40, name)
    if name == "small-nv":
        return make_params(12, 40, 3, 2, 2, 40, name)
    if name == "large":
        return make_params(16, 50, 30, 4, 3, 50, name)
    if name == "large-nv":
        return make_params(16, 50, 30, 10, 3, 50, name)
    if name == "large-fp":
        pr = ntt_primes(50, 10, 16)
        return ParamSet(name=name, logn=16, q=pr[:7], p=pr[7:], dnum=3, log_scale=40)
    if name == "boot-small":
        return make_params(12, 50, 20, 7, 3, 50, name)
    if name == "tiny":  # N = 2^6, for brute-force pins
        return make_params(6, 30, 3, 2, 2, 20, name)
    raise KeyError(name)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_residues(g: np.random.Generator, moduli, N: int) -> np.ndarray:
    """Rows of uniform residues, row i in [0, moduli[i])."""
    out = np.empty((len(moduli), N), dtype=np.uint64)
    for i, m in enumerate(moduli):
        out[i] = g.integers(0, int(m), size=N, dtype=np.uint64)
    return out


def random_poly(seed: int, ps: ParamSet, level: int) -> np.ndarray:
    """A uniform eval-domain polynomial at ``level`` (rows q_0..q_level)."""
    return uniform_residues(rng(seed), ps.q[: level + 1], ps.N)


def random_ct(seed: int, ps: ParamSet, level: int):
    g = rng(seed)
    return (uniform_residues(g, ps.q[: level + 1], ps.N), uniform_residues(g, ps.q[: level + 1], ps.N))


def random_key(seed: int, ps: ParamSet) -> np.ndarray:
    """A uniform top-level key [dnum][2][L+1+K][N] (bit-level parity does not
    depend on whether the key is a valid encryption)."""
    g = rng(seed)
    mods = list(ps.q) + list(ps.p)
    key = np.empty((ps.dnum, 2, len(mods), ps.N), dtype=np.uint64)
    for j in range(ps.dnum):
        for t in range(2):
            key[j, t] = uniform_residues(g, mods, ps.N)
    return key


def device_residues(seed: int, moduli, N: int, device="cuda"):
    """Uniform residues generated directly in device memory (torch's Philox
    generator, seeded): rows of a [len(moduli)][N] uint64 tensor, row i in
    [0, moduli[i]).  Used where the inputs are too large to draw on the host
    quickly (batched and served workloads); run time does not depend on values."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty((len(moduli), N), dtype=torch.int64, device=device)
    for i, m in enumerate(moduli):
        out[i] = torch.randint(0, int(m), (N,), generator=gen, dtype=torch.int64, device=device)
    return out.view(torch.uint64)


def ternary(g: np.random.Generator, N: int) -> np.ndarray:
    """Secret coefficients iid uniform in {-1, 0, 1}."""
    return g.integers(-1, 2, size=N).astype(np.int64)


def sparse_ternary(g: np.random.Generator, N: int, h: int) -> np.ndarray:
    """h coefficients +-1 (uniform signs) at uniformly chosen positions, the rest 0."""
    out = np.zeros(N, dtype=np.int64)
    pos = g.choice(N, size=h, replace=False)
    out[pos] = 2 * g.integers(0, 2, size=h) - 1
    return out


def gaussian(g: np.random.Generator, N: int, sigma: float = 3.2) -> np.ndarray:
    """Rounded Gaussian errors, truncated at 6 sigma."""
    e = np.rint(g.normal(0.0, sigma, size=N))
    bound = np.floor(6 * sigma)
    return np.clip(e, -bound, bound).astype(np.int64)


def complex_slots(g: np.random.Generator, n: int) -> np.ndarray:
    """Slots with real and imaginary parts iid uniform on [-1, 1]."""
    return g.uniform(-1, 1, size=n) + 1j * g.uniform(-1, 1, size=n)


def rotation_index(seed: int, logn: int) -> int:
    return int(rng(seed).integers(1, 1 << (logn - 1)))


# Rotation indices of the batched workload: 1..16 and the powers of two up to N/4.
def batch_rotation_set(logn: int) -> list[int]:
    return list(range(1, 17)) + [1 << k for k in range(5, logn - 1)]


def batch_plan(seed: int, n_items: int, logn: int, max_level: int, min_level: int = 4, n_rot: int = 8):
    """The mixed batch: half HMult+relin items, half hoisted-rotation items,
    levels uniform in [min_level, max_level], n_rot distinct rotations each."""
    g = rng(seed)
    rs = batch_rotation_set(logn)
    plan = []
    for i in range(n_items):
        level = int(g.integers(min_level, max_level + 1))
        if i % 2 == 0:
            plan.append(("hmult", level, None))
        else:
            plan.append(("hoisted", level, [int(x) for x in g.choice(rs, size=n_rot, replace=False)]))
    return plan


@dataclass
class Request:
    """One served request: an op chain on two fresh ciphertexts (A, B) at
    `level`.  ops: ("hmult",) A <- rescale(A * B), ("ptmuladd",) A <-
    rescale(A * pt + B), ("rotate", k) A <- rot(A, k); with `boot`, A is then
    truncated to level 0 and bootstrapped."""
    rid: int
    arrival: float
    level: int
    ops: list
    boot: bool
    seed: int


def serving_requests(seed: int, n: int, logn: int, rate: float | None, min_level: int = 10, max_level: int = 30,
                     min_ops: int = 4, max_ops: int = 40, boot_frac: float = 0.1) -> list:
    """Poisson arrivals at `rate` requests/s (all at t = 0 when rate is None);
    start levels uniform in [min_level, max_level]; chains of uniform length
    mixing the three ops, never leaving level 1 before the last op."""
    g = rng(seed)
    rs = batch_rotation_set(logn)
    t, out = 0.0, []
    for i in range(n):
        if rate is not None:
            t += float(g.exponential(1.0 / rate))
        level = int(g.integers(min_level, max_level + 1))
        length = int(g.integers(min_ops, max_ops + 1))
        ops, lv = [], level
        for _ in range(length):
            kind = int(g.integers(0, 3))
            if kind < 2 and lv >= 2:
                ops.append(("hmult",) if kind == 0 else ("ptmuladd",))
                lv -= 1
            else:
                ops.append(("rotate", int(g.choice(rs))))
        out.append(Request(rid=i, arrival=t, level=level, ops=ops, boot=bool(g.random() < boot_frac),
                           seed=int(g.integers(1, 2 ** 31))))
    return out
