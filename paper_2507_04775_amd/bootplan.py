"""Client-side planning of a bootstrap (paper Sec. III-F.7): the plaintext
diagonals of the homomorphic DFT factors and the Chebyshev coefficients of
EvalMod, in the form ckks_boot_create takes them.

Like the paper's split between server and client (constants are encoded on
the host, the GPU only runs the schedule), this module computes constants and
nothing else; the library derives the schedule itself from the same few
parameters (group sizes, Chebyshev degree, double-angle steps).

The factors are the stages of the special FFT on n = N/2 slots: at half-size
h, slot x in the lower half of its block of 2h (j = x mod 2h < h) pairs with
x + h under the twiddle xi_j = exp(2 pi i (5^j mod 8h) / 8h); forward:
(u, w) -> (u + xi w, u - xi w); inverse: (u, w) -> ((u + w) / 2, (u - w) / (2 xi)).
CoeffToSlot runs the inverse stages from half-size n/2 down to 1, SlotToCoeff
the forward stages from 1 up to n/2; neither reverses bits.  A group of r
consecutive stages acts only on the r index bits of its half-sizes, so its
matrix entry M[x][y] is nonzero only where y differs from x in those bits:
the diagonals are read off by pushing R = 2^r probe vectors (the indicator of
each value of that bit field) through the stages.

Scales follow the library's discipline: Delta_L = top_scale, Delta_(l-1) =
(Delta_l * Delta_l) / q_l; a plaintext multiplied into a level-l ciphertext
before k rescales carries (Delta_(l-k) q_(l-k+1) .. q_l) / Delta_l.  The first
CoeffToSlot group is taken at k = 2 and carries Delta_L / (2 q_0 K) so that
EvalMod sees t / (q_0 K) for the raised coefficients t; the first SlotToCoeff
group carries q_0 / (2 pi Delta_in G), G the integer gain the level-0 input is
multiplied by before ModRaise (the message then fills more of q_0 while the
sine's argument stays small).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class BootConfig:
    logn: int
    cts_radix_logs: list
    stc_radix_logs: list
    cheb_degree: int
    double_angles: int
    k_range: float
    top_scale: float
    in_scale: float
    cheb_baby: int = 0   # baby-step size of the Chebyshev evaluation (0: smallest power of two b with b^2 > d)
    hoist_moddown: bool = True  # giant steps summed over Q u P with one ModDown per group
    input_gain: int = 1  # integer the level-0 input is multiplied by before ModRaise

    @property
    def n(self) -> int:
        return 1 << (self.logn - 1)

    @property
    def baby(self) -> int:
        if self.cheb_baby:
            return self.cheb_baby
        b = 2
        while b * b <= self.cheb_degree:
            b *= 2
        return b


# The schedule used for the full-slot workloads: three merged groups each way.
def default_config(logn: int, scale: float, sparse: bool = True) -> BootConfig:
    """Stages split as evenly as possible over three groups.  With sparse-secret
    encapsulation (h = 32, so |t_k / q_0| stays below K = 12) a degree-31
    interpolant with 3 double angles; for the uniform ternary secret itself a
    degree-119 interpolant over K = 512 with 6 double angles at N = 2^16, or
    degree 63 over K = 128 with 5 at smaller N.  The input gain multiplies the
    message before ModRaise: at scale 2^50 a full-slot message of slots in
    [-1, 1]^2 fills about 2^-16 of q_0, the gain brings it to 2^-9 (sparse) or
    2^-6 (uniform), where the sine's own error stays below the noise that
    EvalMod amplifies; measured at N = 2^16 (oracle, CPU) the error went from
    2^-9.1 to 2^-15.8 (sparse) and from 2^-0.8 to 2^-10.3 (uniform).  Smaller
    N has larger coefficients for the same slots (they scale as N^-1/2), so
    N = 2^12 takes 16."""
    s = logn - 1
    parts = [s // 3 + (1 if i < s % 3 else 0) for i in range(3)]
    if sparse:
        return BootConfig(logn, parts, parts[::-1], 31, 3, 12.0, scale, scale, input_gain=128 if logn >= 16 else 16)
    if logn >= 16:
        return BootConfig(logn, parts, parts[::-1], 119, 6, 512.0, scale, scale, input_gain=1024)
    return BootConfig(logn, parts, parts[::-1], 63, 5, 128.0, scale, scale, input_gain=16)


SPARSE_H = 32  # nonzero coefficients of the encapsulation secret


def _scales(q, top: float) -> list:
    L = len(q) - 1
    d = [0.0] * (L + 1)
    d[L] = float(top)
    for l in range(L, 0, -1):
        d[l - 1] = (d[l] * d[l]) / float(int(q[l]))
    return d


def _pt_scale(d, q, l: int, k: int) -> float:
    x = d[l - k]
    for j in range(l - k + 1, l + 1):
        x *= float(int(q[j]))
    return x / d[l]


def _halves(logn: int, radix_logs, forward: bool):
    order = [1 << i for i in range(logn - 1)]
    if not forward:
        order.reverse()
    out, at = [], 0
    for r in radix_logs:
        out.append(order[at:at + r])
        at += r
    if at != logn - 1:
        raise ValueError("the groups must cover all %d stages" % (logn - 1))
    return out


def _layout(n: int, halves):
    r, h0 = len(halves), min(halves)
    R = 1 << r
    m_lo, count = (0, R) if R * h0 == n else (1 - R, 2 * R - 1)
    baby = 1
    while baby * baby < count:
        baby <<= 1
    return m_lo, count, baby, -(-count // baby), h0


def _stage(v: np.ndarray, logn: int, h: int, inverse: bool) -> np.ndarray:
    """One butterfly stage on the last axis of v (probe vectors stacked in front)."""
    n = v.shape[-1]
    j = np.arange(h)
    e = np.array([pow(5, int(t), 8 * h) for t in j])
    xi = np.exp(2j * np.pi * e / (8 * h))
    b = v.reshape(v.shape[:-1] + (n // (2 * h), 2, h))
    u, w = b[..., 0, :], b[..., 1, :]
    if inverse:
        top, bot = (u + w) / 2, (u - w) / (2 * xi)
    else:
        top, bot = u + xi * w, u - xi * w
    return np.stack([top, bot], axis=-2).reshape(v.shape)


def group_diagonals(logn: int, halves, inverse: bool) -> dict:
    """{m: d_m} with the group map = sum_m d_m * rot(v, m h0), rot(v, a)[x] = v[x + a]."""
    n = 1 << (logn - 1)
    r, h0 = len(halves), min(halves)
    R = 1 << r
    x = np.arange(n)
    fld = (x // h0) % R                       # the r index bits the group acts on
    probes = (fld[None, :] == np.arange(R)[:, None]).astype(complex)
    for h in halves:
        probes = _stage(probes, logn, h, inverse)
    wrap = R * h0 == n
    diags = {}
    for v in range(R):                        # column field v, row field fld[x]: offset v - fld[x]
        m = v - fld
        if wrap:
            m = m % R
        for mm in np.unique(m):
            sel = m == mm
            d = diags.setdefault(int(mm), np.zeros(n, complex))
            d[sel] += probes[v][sel]
    return diags


def coeffs_of_slots(z: np.ndarray, logn: int) -> np.ndarray:
    """Real coefficients m with m(zeta^(5^j)) = z_j: m_k = (2/N) Re sum_j z_j zeta^(-5^j k)."""
    N = 1 << logn
    W = np.zeros(2 * N, complex)
    W[[pow(5, j, 2 * N) for j in range(N // 2)]] = z
    return (2.0 / N) * np.real(np.fft.fft(W)[:N])


def _round(v: np.ndarray) -> np.ndarray:
    a = np.abs(v)
    r = np.where(a >= 2.0 ** 52, a, np.floor(a + 0.5))
    return np.where(v < 0, -r, r)


def encode_group(cfg: BootConfig, halves, inverse: bool, factor: float, scale: float) -> np.ndarray:
    n = cfg.n
    m_lo, count, baby, giants, h0 = _layout(n, halves)
    diags = group_diagonals(cfg.logn, halves, inverse)
    out = np.empty((count, 1 << cfg.logn))
    for i in range(count):
        g = i // baby
        G = (g * baby + m_lo) * h0
        d = diags.get(i + m_lo, np.zeros(n, complex)) * factor
        out[i] = _round(coeffs_of_slots(np.roll(d, G), cfg.logn) * scale)   # rot(d, -G)
    return out


def chebyshev(cfg: BootConfig) -> np.ndarray:
    """Chebyshev interpolant of cos(2 pi (K y - 1/4) / 2^r) at the d + 1 Chebyshev-Gauss nodes."""
    d = cfg.cheb_degree
    theta = np.pi * (np.arange(d + 1) + 0.5) / (d + 1)
    f = np.cos(2 * np.pi * (cfg.k_range * np.cos(theta) - 0.25) / (1 << cfg.double_angles))
    c = (2.0 / (d + 1)) * np.cos(np.outer(np.arange(d + 1), theta)) @ f
    c[0] /= 2
    return c


def cheb_depth(d: int, b: int) -> int:
    """Levels of the baby-step/giant-step Chebyshev evaluation: babies T_k at
    depth 0 (k = 1), one more per product; giants T_2b, T_4b, .. by squaring;
    leaves one level below the deepest of T_1..T_(b-1); a split q T_G + r one
    below the deeper of q and T_G (of T_G alone for a constant q), and no
    higher than r."""
    dep = {1: 0}
    for k in range(2, min(b, d) + 1):
        dep[k] = 1 + (dep[k // 2] if k % 2 == 0 else max(dep[k // 2], dep[k // 2 + 1]))
    G = b
    while 2 * G <= d:
        dep[2 * G] = dep[G] + 1
        G *= 2
    leaf = 1 + max(dep[k] for k in range(1, min(b - 1, d) + 1))

    def node(D):
        if D < b:
            return leaf
        G = b
        while 2 * G <= D:
            G *= 2
        prod = dep[G] + 1 if D == G else max(node(D - G), dep[G]) + 1
        return max(prod, node(G - 1))
    return node(d)


def rotations(cfg: BootConfig) -> list:
    n, out = cfg.n, set()
    for radix, fwd in ((cfg.cts_radix_logs, False), (cfg.stc_radix_logs, True)):
        for halves in _halves(cfg.logn, radix, fwd):
            m_lo, count, baby, giants, h0 = _layout(n, halves)
            out.update((b * h0) % n for b in range(1, min(baby, count)))
            out.update(((g * baby + m_lo) * h0) % n for g in range(giants))
    out.discard(0)
    return sorted(out)


@dataclass
class BootPlan:
    cfg: BootConfig
    cts: list = field(default_factory=list)
    stc: list = field(default_factory=list)
    cheb: np.ndarray = None
    rotations: list = field(default_factory=list)
    output_level: int = 0


def plan(q, cfg: BootConfig) -> BootPlan:
    """Constants for a context whose ciphertext primes are q (q_0 first)."""
    q = [int(x) for x in q]
    L = len(q) - 1
    d = _scales(q, cfg.top_scale)
    p = BootPlan(cfg=cfg, cheb=chebyshev(cfg), rotations=rotations(cfg))
    lv = L
    for i, halves in enumerate(_halves(cfg.logn, cfg.cts_radix_logs, False)):
        k = 2 if i == 0 else 1
        f = d[L] / (2.0 * q[0] * cfg.k_range) if i == 0 else 1.0
        p.cts.append(encode_group(cfg, halves, True, f, _pt_scale(d, q, lv, k)))
        lv -= k
    lv -= cheb_depth(cfg.cheb_degree, cfg.baby) + cfg.double_angles
    for i, halves in enumerate(_halves(cfg.logn, cfg.stc_radix_logs, True)):
        f = q[0] / (2.0 * np.pi * cfg.in_scale * cfg.input_gain) if i == 0 else 1.0
        p.stc.append(encode_group(cfg, halves, False, f, _pt_scale(d, q, lv, 1)))
        lv -= 1
    if lv < 0:
        raise ValueError("not enough levels for this schedule")
    p.output_level = lv
    return p
