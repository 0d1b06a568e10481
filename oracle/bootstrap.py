"""CKKS bootstrapping for the oracle: a client-side planner and a plain
executor built from the oracle's primitives.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The pipeline follows the paper's description of bootstrapping (Sec. III-F.7):
ModRaise, CoeffToSlot as a homomorphic DFT split into sparse factors, each
evaluated with baby-step/giant-step over hoisted rotations, EvalMod as a
Chebyshev approximation of a scaled cosine followed by double-angle steps,
and SlotToCoeff.  The schedule is fixed by a handful of parameters; the GPU
library derives the same schedule independently and takes the same planned
constants, so the two results are compared bit for bit.

Schedule (n = N/2 slots, full packing):

1. ModRaise: the level-0 ciphertext's coefficients are lifted centred from
   q_0 to every prime of the top level L.  With sparse-secret encapsulation
   (optional), the ciphertext is first switched to a sparse secret s' (h
   nonzero coefficients), so that t = c0 + c1 s' stays within a small
   multiple K of q_0, and switched back to s right after ModRaise (the
   encapsulation of Bossuat, Troncoso-Pastoriza and Hubaux, ACNS 2022).
2. CoeffToSlot: the stages of the special FFT (the iterative transform whose
   butterfly at half-size h pairs slots x and x + h with the twiddle
   zeta^((5^j mod 8h) * 2N / 8h)) are merged into groups and inverted, the
   largest half-size first; no bit reversal is applied (SlotToCoeff expects the
   same order).  A group of r stages with smallest half-size h0 is the map
   sum_m d_m * rot(v, m h0) (layout in ``group_layout``), evaluated as
   sum_g rot(sum_b d'_(g,b) * rot(v, b h0), G_g) with the baby rotations
   b h0 taken in one hoisted call and the diagonals pre-rotated by -G_g.
   Every group ends with one rescale, except the first, whose plaintexts are
   encoded at the scale of two primes and which rescales twice: its input
   holds the raised coefficients t ~ q_0 I, so a plaintext rounded at the
   scale of one prime would leave an error of order |t| / q_l in every slot.
3. Split: ct_re = ct + conj(ct), ct_im = (ct - conj(ct)) * X^(3N/2); the 1/2
   factors and Delta_L / (q_0 K) are folded into the first CoeffToSlot
   group, so the slots of both hold t_k / (q_0 K) for the coefficients t_k of
   the raised plaintext (slot x of ct_re holds t at position br(x), of ct_im
   at br(x) + n).
4. EvalMod on each: p(y) = sum_k c_k T_k(y) by baby-step/giant-step.  The
   babies T_1..T_min(b,d) (b a power of two, by default the smallest with
   b^2 > d) come from
   T_2m = 2 T_m^2 - 1 and T_2m+1 = 2 T_m T_m+1 - T_1, the giants T_2b, T_4b, ..
   (up to d) by squaring.  A polynomial of degree D >= b is split at the
   largest giant G <= D as p = q T_G + r (Chebyshev division: q_0 = c_G,
   q_i = 2 c_(G+i), r_(G-i) = c_(G-i) - c_(G+i)), q and r evaluated the same
   way and combined by one multiplication; below degree b a leaf
   c_0 + sum_k c_k T_k is one integer combination of the babies at the level
   one above the lowest baby T_1..T_(b-1), rescaled once.  Then r double-angle
   steps y <- 2 y^2 - 1.  With p interpolating cos(2 pi (K y - 1/4) / 2^r) on
   [-1, 1] this yields sin(2 pi t_k / q_0).
5. Recombine: ct = ct_re + ct_im * X^(N/2).
6. SlotToCoeff: the forward special-FFT stages merged into groups, the
   smallest half-size first, with q_0 / (2 pi Delta_in) folded into the first.

Scale discipline: level L carries Delta_L (a parameter) and
Delta_{l-1} = (Delta_l * Delta_l) / q_l in double arithmetic, in that order.
A product of two level-l ciphertexts, rescaled, lands on Delta_{l-1}.
Taking a level-l ciphertext times a real constant c down to level t < l drops
its limbs above t + 1, multiplies by the integer round(c * X) with
X = (Delta_t * q_(t+1)) / Delta_l, and rescales once.  A constant added at
level l is round(c * Delta_l).  Rounding is half away from zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import apply_galois, automorph_eval, galois_conjugate, galois_for_rotation, hmult_relin, hoisted_rotate
from . import Params, inner_product, intt, keyswitch, moddown, modup, ntt, reduce_f64, rescale, vec
from .client import embed_inverse


@dataclass
class BootParams:
    logn: int
    cts_radix_logs: list          # log2 radix of each CoeffToSlot group, in application order
    stc_radix_logs: list          # same for SlotToCoeff
    cheb_degree: int
    double_angles: int
    k_range: float                # |t_k / q_0| is assumed below k_range
    top_scale: float              # Delta_L
    in_scale: float               # scale of the level-0 input
    cheb_baby: int = 0            # baby-step size of the Chebyshev evaluation (0: smallest b with b^2 > d)
    hoist_moddown: bool = False   # giant steps key-switched without ModDown, summed over Q u P, one ModDown per group
    input_gain: int = 1           # the level-0 input is multiplied by this integer before ModRaise

    @property
    def baby(self) -> int:
        return self.cheb_baby or baby_size(self.cheb_degree)

    @property
    def n(self) -> int:
        return 1 << (self.logn - 1)


def round_half_away(v: float) -> int:
    a = np.floor(abs(float(v)) + 0.5)
    return int(a) if v >= 0 else -int(a)


def level_scales(q, L: int, top: float) -> list:
    d = [0.0] * (L + 1)
    d[L] = float(top)
    for l in range(L, 0, -1):
        d[l - 1] = (d[l] * d[l]) / float(int(q[l]))
    return d


def const_factor(scales, q, l: int, t: int) -> float:
    """X with round(c X) the integer that takes a level-l ciphertext times c to level t."""
    return (scales[t] * float(int(q[t + 1]))) / scales[l]


def pt_scale(scales, q, l: int, k: int) -> float:
    """Scale of a plaintext multiplied into a level-l ciphertext before k rescales:
    (Delta_(l-k) q_(l-k+1) ... q_l) / Delta_l, multiplied left to right."""
    x = scales[l - k]
    for j in range(l - k + 1, l + 1):
        x *= float(int(q[j]))
    return x / scales[l]


def round_vec(v: np.ndarray) -> np.ndarray:
    """Round half away from zero in double; values from 2^52 up are integers already."""
    a = np.abs(v)
    r = np.where(a >= 2.0 ** 52, a, np.floor(a + 0.5))
    return np.where(v < 0, -r, r)


def stage_groups(logn: int, radix_logs, forward: bool):
    """Half-size lists of the merged groups in application order."""
    hs = [1 << i for i in range(logn - 1)]          # half-sizes 1, 2, .., n/2 (forward order)
    if not forward:
        hs = hs[::-1]
    groups, i = [], 0
    for r in radix_logs:
        groups.append(hs[i:i + r])
        i += r
    assert i == len(hs), "radix logs must cover every stage"
    return groups


def group_layout(n: int, halves):
    """BSGS layout of one merged group: (m_lo, count, baby, giants, h0).

    The group's map has diagonals at offsets m h0, m in [m_lo, m_lo + count).
    When R h0 = n (R = 2^len(halves); the group holds the stage of half-size
    n/2) offsets m and m - R coincide mod n, so only m = 0..R-1 exist;
    otherwise m = -(R-1)..R-1.  Diagonal index i = m - m_lo = g baby + b, with
    baby the smallest power of two whose square reaches count."""
    R, h0 = 1 << len(halves), min(halves)
    if R * h0 == n:
        m_lo, count = 0, R
    else:
        m_lo, count = -(R - 1), 2 * R - 1
    baby = 1
    while baby * baby < count:
        baby *= 2
    giants = -(-count // baby)
    return m_lo, count, baby, giants, h0


def giant_offsets(n: int, halves):
    m_lo, count, baby, giants, h0 = group_layout(n, halves)
    return [(g * baby + m_lo) * h0 for g in range(giants)]


def baby_offsets(n: int, halves):
    m_lo, count, baby, giants, h0 = group_layout(n, halves)
    return [b * h0 for b in range(1, min(baby, count))]


def baby_size(d: int) -> int:
    b = 2
    while b * b <= d:
        b *= 2
    return b


def cheb_split(c, G: int):
    """p = q T_G + r for Chebyshev coefficients c of degree D with G <= D < 2G."""
    D = len(c) - 1
    q = [0.0] * (D - G + 1)
    r = list(c[:G])
    q[0] = c[G]
    for i in range(1, D - G + 1):
        q[i] = 2.0 * c[G + i]
        r[G - i] = r[G - i] - c[G + i]
    return q, r


def cheb_schedule_depth(d: int, b: int) -> int:
    """Levels the baby-step/giant-step evaluation of degree d with baby size b
    consumes (a dry run of Executor.chebyshev on levels alone)."""
    lv = {1: 0}
    for k in range(2, min(b, d) + 1):
        lv[k] = lv[k // 2] - 1 if k % 2 == 0 else min(lv[k // 2], lv[k // 2 + 1]) - 1
    G = b
    while 2 * G <= d:
        lv[2 * G] = lv[G] - 1
        G *= 2
    t_leaf = min(lv[k] for k in range(1, min(b - 1, d) + 1)) - 1

    def poly(D):
        if D < b:
            return t_leaf
        G = b
        while 2 * G <= D:
            G *= 2
        r = poly(G - 1)
        p = lv[G] - 1 if D == G else min(poly(D - G), lv[G]) - 1
        return min(p, r)
    return -poly(d)


def levels_used(bp: BootParams) -> dict:
    """Levels consumed by each phase."""
    return {"cts": len(bp.cts_radix_logs) + 1,
            "evalmod": cheb_schedule_depth(bp.cheb_degree, bp.baby) + bp.double_angles,
            "stc": len(bp.stc_radix_logs)}


def output_level(P: Params, bp: BootParams) -> int:
    return (P.nq - 1) - sum(levels_used(bp).values())


# ------------------------------------------------------------------ planner

def ext_p(P: Params, x: np.ndarray, l: int, g: int = 1) -> np.ndarray:
    """The extended polynomial equal to P phi_g(x) for x at level l: rows
    q_0..q_l hold [P]_(q_i) phi_g(x), rows p_0..p_(K-1) are zero (P vanishes
    there)."""
    src = x if g == 1 else automorph_eval(P.logn, g, x)
    Pp = 1
    for m in P.p:
        Pp *= int(m)
    mods = P.q[: l + 1]
    consts = np.array([[Pp % int(m)] * P.N for m in mods], dtype=np.uint64)
    out = np.zeros((l + 1 + len(P.p), P.N), dtype=np.uint64)
    out[: l + 1] = vec(mods, src, consts, "mul", P.logn)
    return out


def special_fft_stage(n: int, logn: int, h: int, inverse: bool):
    """One butterfly stage of the special FFT (or its inverse) as {offset mod n: diagonal}."""
    M = 4 * n
    a = np.zeros(n, complex)
    up = np.zeros(n, complex)    # offset +h
    dn = np.zeros(n, complex)    # offset -h
    lenq = 8 * h
    for x in range(n):
        j = x % (2 * h)
        low = j < h
        e = pow(5, j if low else j - h, M)
        xi = np.exp(2j * np.pi * ((e % lenq) * (M // lenq)) / M)
        if low:
            a[x], up[x] = (1.0, xi) if not inverse else (0.5, 0.5)
        else:
            a[x], dn[x] = (-xi, 1.0) if not inverse else (-0.5 / xi, 0.5 / xi)
    out = {0: a}
    for o, d in ((h % n, up), ((-h) % n, dn)):   # +h and -h coincide when h = n/2
        out[o] = out.get(o, 0) + d
    return out


def compose(A: dict, B: dict, n: int) -> dict:
    """The map A(B(v)): (A o B)_(a+b) = sum A_a * rot(B_b, a), rot(u, a)[x] = u[x + a]."""
    out = {}
    for oa, da in A.items():
        for ob, db in B.items():
            o = (oa + ob) % n
            out[o] = out.get(o, 0) + da * np.roll(db, -oa)
    return out


def group_map(n: int, logn: int, halves, inverse: bool) -> dict:
    m = None
    for h in halves:
        s = special_fft_stage(n, logn, h, inverse)
        m = s if m is None else compose(s, m, n)
    return m


def group_diagonals(n: int, logn: int, halves, inverse: bool, factor: complex = 1.0) -> list:
    """The group's diagonals pre-rotated by their giant step, in index order
    i = g baby + b: entry i is rot(d_m, -G_g) for m = i + m_lo."""
    m_lo, count, baby, giants, h0 = group_layout(n, halves)
    mp = group_map(n, logn, halves, inverse)
    G = giant_offsets(n, halves)
    out = []
    for i in range(count):
        d = mp.get(((i + m_lo) * h0) % n, np.zeros(n, complex)) * factor
        out.append(np.roll(d, G[i // baby]))      # pd[x] = d[x - G_g]
    return out


def plan_group(bp: BootParams, halves, inverse: bool, factor: float, scale: float) -> np.ndarray:
    """Coefficient vectors [count][N] (integer-valued doubles) of the group's
    pre-rotated diagonals encoded at ``scale``."""
    pds = group_diagonals(bp.n, bp.logn, halves, inverse, factor)
    return np.stack([round_vec(embed_inverse(pd, bp.logn) * scale) for pd in pds])


def rotations_needed(bp: BootParams) -> list:
    """Slot rotations (mod n) of every group: baby steps and nonzero giant steps."""
    rots = set()
    for radix_logs, fwd in ((bp.cts_radix_logs, False), (bp.stc_radix_logs, True)):
        for halves in stage_groups(bp.logn, radix_logs, fwd):
            rots.update(k % bp.n for k in baby_offsets(bp.n, halves))
            rots.update(G % bp.n for G in giant_offsets(bp.n, halves) if G % bp.n)
    return sorted(rots)


def chebyshev_coeffs(bp: BootParams) -> np.ndarray:
    f = lambda y: np.cos(2 * np.pi * (bp.k_range * y - 0.25) / (1 << bp.double_angles))
    return np.polynomial.chebyshev.Chebyshev.interpolate(f, bp.cheb_degree).coef.astype(np.float64)


@dataclass
class BootPlan:
    params: BootParams
    cts: list = field(default_factory=list)     # per group: float64 [count][N], integer-valued
    stc: list = field(default_factory=list)
    cheb: np.ndarray = None


def plan(P: Params, bp: BootParams) -> BootPlan:
    """The constants of a bootstrap whose ModRaise lands on level L = nq - 1."""
    q, L = [int(x) for x in P.q], P.nq - 1
    sc = level_scales(q, L, bp.top_scale)
    pl = BootPlan(params=bp)
    lv = L
    for i, halves in enumerate(stage_groups(bp.logn, bp.cts_radix_logs, False)):
        factor = sc[L] / (2.0 * q[0] * bp.k_range) if i == 0 else 1.0
        k = 2 if i == 0 else 1
        pl.cts.append(plan_group(bp, halves, True, factor, pt_scale(sc, q, lv, k)))
        lv -= k
    lv -= levels_used(bp)["evalmod"]
    for i, halves in enumerate(stage_groups(bp.logn, bp.stc_radix_logs, True)):
        factor = q[0] / (2.0 * np.pi * bp.in_scale * bp.input_gain) if i == 0 else 1.0
        pl.stc.append(plan_group(bp, halves, False, factor, pt_scale(sc, q, lv, 1)))
        lv -= 1
    pl.cheb = chebyshev_coeffs(bp)
    return pl


# ------------------------------------------------------------------ executor

class Executor:
    """Runs the schedule with the oracle's primitives on ciphertexts (c0, c1, level)."""

    def __init__(self, P: Params, pl: BootPlan, relin_key, conj_key, rot_keys: dict, to_sparse=None,
                 from_sparse=None):
        self.P, self.bp, self.pl = P, pl.params, pl
        self.q = [int(x) for x in P.q]
        self.L = P.nq - 1
        self.sc = level_scales(self.q, self.L, self.bp.top_scale)
        self.rlk, self.ck, self.rk = relin_key, conj_key, rot_keys
        self.to_sparse, self.from_sparse = to_sparse, from_sparse

    # -- elementary steps
    def mods(self, l):
        return self.P.q[: l + 1]

    def _const(self, C: int, l: int) -> np.ndarray:
        col = np.array([[C % m] for m in self.q[: l + 1]], dtype=np.uint64)
        return np.ascontiguousarray(np.broadcast_to(col, (l + 1, self.P.N)))

    def scalar_mul_int(self, ct, C: int):
        c0, c1, l = ct
        s = self._const(C, l)
        return (vec(self.mods(l), c0, s, "mul", self.P.logn), vec(self.mods(l), c1, s, "mul", self.P.logn), l)

    def scalar_add(self, ct, c: float):
        c0, c1, l = ct
        s = self._const(round_half_away(c * self.sc[l]), l)
        return (vec(self.mods(l), c0, s, "add", self.P.logn), c1, l)

    def drop(self, ct, l: int):
        return (ct[0][: l + 1], ct[1][: l + 1], l)

    def rescale(self, ct):
        c0, c1, l = ct
        r0, r1 = rescale(self.P, (c0, c1), l)
        return (r0, r1, l - 1)

    def mult_const_to(self, ct, c: float, t: int):
        """ct times the real constant c, taken to level t < level(ct)."""
        l = ct[2]
        assert t < l
        C = round_half_away(c * const_factor(self.sc, self.q, l, t))
        return self.rescale(self.scalar_mul_int(self.drop(ct, t + 1), C))

    def level_down(self, ct, t: int):
        return ct if ct[2] == t else self.mult_const_to(ct, 1.0, t)

    def add(self, a, b, op="add"):
        assert a[2] == b[2]
        l = a[2]
        return (vec(self.mods(l), a[0], b[0], op, self.P.logn), vec(self.mods(l), a[1], b[1], op, self.P.logn), l)

    def mul(self, a, b):
        l = min(a[2], b[2])
        a, b = self.level_down(a, l), self.level_down(b, l)
        o0, o1 = hmult_relin(self.P, (a[0], a[1]), (b[0], b[1]), self.rlk, l)
        return self.rescale((o0, o1, l))

    def monomial(self, ct, k: int):
        """ct * X^k, 0 <= k < 2N (exact; scale unchanged)."""
        N = 1 << self.P.logn
        c0, c1, l = ct
        e = np.zeros((l + 1, N), dtype=np.uint64)
        for i, m in enumerate(self.q[: l + 1]):
            e[i, k % N] = 1 if k < N else m - 1
        E = ntt(self.mods(l), e, self.P.logn)
        return (vec(self.mods(l), c0, E, "mul", self.P.logn), vec(self.mods(l), c1, E, "mul", self.P.logn), l)

    def switch(self, ct, key):
        """Key switching of (c0, c1) with a switching key: (c0 + k0, k1)."""
        c0, c1, l = ct
        k0, k1 = keyswitch(self.P, c1, key, l)
        return (vec(self.mods(l), c0, k0, "add", self.P.logn), k1, l)

    def conj(self, ct):
        o0, o1 = apply_galois(self.P, (ct[0], ct[1]), galois_conjugate(self.P.logn), self.ck, ct[2])
        return (o0, o1, ct[2])

    def rotate(self, ct, k: int):
        k %= self.bp.n
        o0, o1 = apply_galois(self.P, (ct[0], ct[1]), galois_for_rotation(self.P.logn, k), self.rk[k], ct[2])
        return (o0, o1, ct[2])

    def plaintext(self, coeffs: np.ndarray, l: int) -> np.ndarray:
        return ntt(self.mods(l), reduce_f64(self.mods(l), coeffs), self.P.logn)

    # -- phases
    def modraise(self, ct):
        c0, c1, l = ct
        assert l == 0
        q0 = self.q[0]
        out = []
        for c in (c0, c1):
            v = [int(x) for x in intt(self.P.q[:1], c[:1], self.P.logn)[0]]
            v = [x - q0 if x > (q0 - 1) // 2 else x for x in v]
            lifted = np.empty((self.L + 1, len(v)), dtype=np.uint64)
            for i, m in enumerate(self.q):
                lifted[i] = np.array([x % m for x in v], dtype=np.uint64)
            out.append(ntt(self.P.q, lifted, self.P.logn))
        return (out[0], out[1], self.L)

    def linear_transform(self, ct, diags: np.ndarray, halves, rescales: int = 1):
        n = self.bp.n
        m_lo, count, baby, giants, h0 = group_layout(n, halves)
        assert diags.shape[0] == count
        l = ct[2]
        bk = baby_offsets(n, halves)
        if bk:
            gs = [galois_for_rotation(self.P.logn, k) for k in bk]
            r0, r1 = hoisted_rotate(self.P, (ct[0], ct[1]), gs, [self.rk[k % n] for k in bk], l)
            rots = [(ct[0], ct[1])] + [(r0[i], r1[i]) for i in range(len(bk))]
        else:
            rots = [(ct[0], ct[1])]
        mods = self.mods(l)
        G = giant_offsets(n, halves)
        if self.bp.hoist_moddown:
            return self._linear_transform_hoisted(rots, diags, count, baby, giants, G, l, rescales)
        total = None
        for g in range(giants):
            s0 = s1 = None
            for b in range(baby):
                i = g * baby + b
                if i >= count:
                    break
                pt = self.plaintext(diags[i], l)
                t0 = vec(mods, rots[b][0], pt, "mul", self.P.logn)
                t1 = vec(mods, rots[b][1], pt, "mul", self.P.logn)
                s0 = t0 if s0 is None else vec(mods, s0, t0, "add", self.P.logn)
                s1 = t1 if s1 is None else vec(mods, s1, t1, "add", self.P.logn)
            part = (s0, s1, l)
            if G[g] % n:
                part = self.rotate(part, G[g])
            total = part if total is None else self.add(total, part)
        for _ in range(rescales):
            total = self.rescale(total)
        return total

    def _linear_transform_hoisted(self, rots, diags, count, baby, giants, G, l, rescales):
        """Giant steps with the ModDown hoisted out of the loop.  Each giant's
        sum s = sum_b pt_b rot_b is rotated by G without its ModDown: the key
        switch of phi_G(s_1) stays in the extended basis Q u P and P phi_G(s_0)
        joins it there, so (k_0 + P phi_G(s_0), k_1) is P times the rotation
        of s before rounding.  A giant with G = 0 enters as P s.  The parts
        are summed over Q u P and divided by P with one ModDown per half;
        ModDown(P y + z) = y + ModDown(z) exactly, so each giant contributes as
        in the plain schedule except for the single rounding."""
        n, lg = self.bp.n, self.P.logn
        mods = self.mods(l)
        emods = list(mods) + [int(m) for m in self.P.p]
        tot = None
        for g in range(giants):
            s0 = s1 = None
            for b in range(baby):
                i = g * baby + b
                if i >= count:
                    break
                pt = self.plaintext(diags[i], l)
                t0 = vec(mods, rots[b][0], pt, "mul", lg)
                t1 = vec(mods, rots[b][1], pt, "mul", lg)
                s0 = t0 if s0 is None else vec(mods, s0, t0, "add", lg)
                s1 = t1 if s1 is None else vec(mods, s1, t1, "add", lg)
            k = G[g] % n
            if k:
                gal = galois_for_rotation(lg, k)
                acc = inner_product(self.P, modup(self.P, automorph_eval(lg, gal, s1), l), self.rk[k], l)
                part = (vec(emods, acc[0], ext_p(self.P, s0, l, gal), "add", lg), acc[1])
            else:
                part = (ext_p(self.P, s0, l), ext_p(self.P, s1, l))
            tot = part if tot is None else tuple(vec(emods, tot[t], part[t], "add", lg) for t in range(2))
        total = (moddown(self.P, tot[0], l), moddown(self.P, tot[1], l), l)
        for _ in range(rescales):
            total = self.rescale(total)
        return total

    def chebyshev(self, y):
        c = [float(x) for x in self.pl.cheb]
        d = len(c) - 1
        b = self.bp.baby
        T = {1: y}
        for k in range(2, min(b, d) + 1):
            if k % 2 == 0:
                p = self.scalar_mul_int(self.mul(T[k // 2], T[k // 2]), 2)
                T[k] = self.scalar_add(p, -1.0)
            else:
                p = self.scalar_mul_int(self.mul(T[k // 2], T[k // 2 + 1]), 2)
                T[k] = self.add(p, self.level_down(T[1], p[2]), "sub")
        G = b
        while 2 * G <= d:
            p = self.scalar_mul_int(self.mul(T[G], T[G]), 2)
            T[2 * G] = self.scalar_add(p, -1.0)
            G *= 2
        t_leaf = min(T[k][2] for k in range(1, min(b - 1, d) + 1)) - 1
        return self._poly(c, T, b, t_leaf)

    def _leaf(self, c, T, t: int):
        """c_0 + sum_k c_k T_k: the babies truncated to level t + 1, times
        round(c_k (Delta_t q_(t+1)) / Delta_level(T_k)), summed, rescaled once."""
        acc = None
        for k in range(1, len(c)):
            C = round_half_away(c[k] * const_factor(self.sc, self.q, T[k][2], t))
            u = self.scalar_mul_int(self.drop(T[k], t + 1), C)
            acc = u if acc is None else self.add(acc, u)
        return self.scalar_add(self.rescale(acc), c[0])

    def _poly(self, c, T, b: int, t_leaf: int):
        D = len(c) - 1
        if D < b:
            return self._leaf(c, T, t_leaf)
        G = b
        while 2 * G <= D:
            G *= 2
        q, r = cheb_split(c, G)
        R = self._poly(r, T, b, t_leaf)
        if len(q) == 1:
            P = self.mult_const_to(T[G], q[0], T[G][2] - 1)
        else:
            P = self.mul(self._poly(q, T, b, t_leaf), T[G])
        l = min(P[2], R[2])
        return self.add(self.level_down(P, l), self.level_down(R, l))

    def eval_mod(self, y):
        y = self.chebyshev(y)
        for _ in range(self.bp.double_angles):
            y = self.scalar_add(self.scalar_mul_int(self.mul(y, y), 2), -1.0)
        return y

    def coeff_to_slot(self, ct):
        groups = stage_groups(self.bp.logn, self.bp.cts_radix_logs, False)
        for i, (diags, halves) in enumerate(zip(self.pl.cts, groups)):
            ct = self.linear_transform(ct, diags, halves, 2 if i == 0 else 1)
        return ct

    def slot_to_coeff(self, ct):
        for diags, halves in zip(self.pl.stc, stage_groups(self.bp.logn, self.bp.stc_radix_logs, True)):
            ct = self.linear_transform(ct, diags, halves)
        return ct

    def bootstrap(self, ct):
        N = 1 << self.bp.logn
        if self.bp.input_gain != 1:  # m -> G m: the message uses more of q_0, the sine's input stays small
            ct = self.scalar_mul_int(ct, self.bp.input_gain)
        if self.to_sparse is not None:
            ct = self.switch(ct, self.to_sparse)
        ct = self.modraise(ct)
        if self.from_sparse is not None:
            ct = self.switch(ct, self.from_sparse)
        ct = self.coeff_to_slot(ct)
        cj = self.conj(ct)
        re = self.add(ct, cj)
        im = self.monomial(self.add(ct, cj, "sub"), 3 * N // 2)
        re, im = self.eval_mod(re), self.eval_mod(im)
        return self.slot_to_coeff(self.add(re, self.monomial(im, N // 2)))
