"""Client side of CKKS for the oracle's decryption checks.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper leaves key
generation, encryption, decryption and encoding to the client library
(Sec. III-A); these plain versions exist so that the oracle's server-side
results can be decrypted and compared with the plaintext computation.

Every random draw (secret, uniform masks, errors) is passed in by the caller.

Conventions: slot j of a plaintext m(X) is m(zeta^(5^j mod 2N)) / scale with
zeta = exp(i pi / N), j < N/2; encoding rounds half away from zero; the secret
is ternary; encryption is the secret-key form c1 = a, c0 = -a s + m + e.
Key for s' under digit j of the top-level partition (digits of alpha
consecutive q limbs): k_{j,1} = a_j, k_{j,0} = -a_j s + e_j + [P]_{q_i} s' on
the rows q_i of digit j, -a_j s + e_j on every other row.
"""
from __future__ import annotations

import numpy as np

from . import Params, automorph_eval, intt, ntt, vec


def _round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def slot_exponents(logn: int) -> np.ndarray:
    """e_j = 5^j mod 2N for the N/2 slots."""
    two_n = 2 << logn
    e = np.empty(1 << (logn - 1), dtype=np.int64)
    cur = 1
    for j in range(len(e)):
        e[j] = cur
        cur = cur * 5 % two_n
    return e


def embed_inverse(z: np.ndarray, logn: int) -> np.ndarray:
    """Real coefficients m_k (unscaled) with m(zeta^(5^j)) = z_j and m(zeta^(-5^j)) = conj(z_j)."""
    N = 1 << logn
    e = slot_exponents(logn)
    w = np.zeros(N, dtype=np.complex128)  # w[l] holds the value at exponent 2l+1
    w[(e - 1) // 2] = z
    w[((2 * N - e) - 1) // 2] = np.conj(z)
    k = np.arange(N)
    zeta_mk = np.exp(-1j * np.pi * k / N)
    return np.real(zeta_mk * np.fft.fft(w) / N)


def embed(m: np.ndarray, logn: int) -> np.ndarray:
    """Slots z_j = m(zeta^(5^j)) of real coefficients m."""
    N = 1 << logn
    k = np.arange(N)
    v = N * np.fft.ifft(m * np.exp(1j * np.pi * k / N))
    e = slot_exponents(logn)
    return v[(e - 1) // 2]


def encode_coeffs(z: np.ndarray, logn: int, scale: float) -> np.ndarray:
    """Integer coefficients round(scale * tau^-1(z)) (int64 when they fit, else object)."""
    m = _round_half_away(embed_inverse(np.asarray(z, dtype=np.complex128), logn) * scale)
    if np.max(np.abs(m)) < 2.0 ** 62:
        return m.astype(np.int64)
    return np.array([int(x) for x in m], dtype=object)


def to_rns(coeffs: np.ndarray, mods) -> np.ndarray:
    """Signed integer coefficients reduced into every modulus (coefficient domain)."""
    out = np.empty((len(mods), len(coeffs)), dtype=np.uint64)
    for i, m in enumerate(mods):
        m = int(m)
        if coeffs.dtype == object:
            out[i] = np.array([int(c) % m for c in coeffs], dtype=np.uint64)
        else:
            out[i] = np.mod(coeffs, m).astype(np.uint64)  # int64 % m, m < 2^61
    return out


def encode(P: Params, z: np.ndarray, level: int, scale: float) -> np.ndarray:
    """Eval-domain plaintext at ``level``."""
    mods = P.q[: level + 1]
    return ntt(mods, to_rns(encode_coeffs(z, P.logn, scale), mods), P.logn)


def crt_centred(x: np.ndarray, mods) -> list[int]:
    """Centred integers with the given residues (coefficient domain rows)."""
    mods = [int(m) for m in mods]
    Q = 1
    for m in mods:
        Q *= m
    acc = np.zeros(x.shape[1], dtype=object)
    for i, m in enumerate(mods):
        Mi = Q // m
        ci = Mi * pow(Mi % m, -1, m)
        acc = acc + x[i].astype(object) * ci
    acc = acc % Q
    half = Q // 2
    return [int(v) - Q if v > half else int(v) for v in acc]


def decode(P: Params, pt: np.ndarray, level: int, scale: float) -> np.ndarray:
    mods = P.q[: level + 1]
    coef = crt_centred(intt(mods, pt, P.logn), mods)
    m = np.array([float(c) for c in coef]) / scale
    return embed(m, P.logn)


class SecretKey:
    def __init__(self, P: Params, s_coeffs: np.ndarray):
        self.P = P
        self.coeffs = np.asarray(s_coeffs, dtype=np.int64)
        allm = list(P.q) + list(P.p)
        self.eval_all = ntt(allm, to_rns(self.coeffs, allm), P.logn)  # rows q_0..q_L, p_0..p_{K-1}

    def eval_q(self, level: int) -> np.ndarray:
        return self.eval_all[: level + 1]


def _mods_all(P: Params):
    return np.concatenate([P.q, P.p])


def gen_switch_key(P: Params, sk: SecretKey, s_prime_eval: np.ndarray, masks, errors) -> np.ndarray:
    """Key [dnum][2][nq+np][N] switching s' to s.  masks[j]: uniform eval rows
    (nq+np, N); errors[j]: signed error coefficients (N,)."""
    allm = _mods_all(P)
    rows = len(allm)
    key = np.zeros((P.dnum, 2, rows, P.N), dtype=np.uint64)
    Pmod = [1] * P.nq
    for i in range(P.nq):
        v = 1
        for pk in P.p:
            v = v * int(pk) % int(P.q[i])
        Pmod[i] = v
    for j in range(P.dnum):
        lo, hi = j * P.alpha, min((j + 1) * P.alpha, P.nq)
        a = np.asarray(masks[j], dtype=np.uint64)
        e = ntt(allm, to_rns(np.asarray(errors[j], dtype=np.int64), allm), P.logn)
        b = vec(allm, e, vec(allm, a, sk.eval_all, "mul", P.logn), "sub", P.logn)  # -a s + e
        for i in range(lo, hi):
            c = np.full(P.N, Pmod[i], dtype=np.uint64)
            term = vec([P.q[i]], c[None], s_prime_eval[i][None], "mul", P.logn)
            b[i] = vec([P.q[i]], b[i][None], term, "add", P.logn)[0]
        key[j, 0] = b
        key[j, 1] = a
    return key


def gen_relin_key(P: Params, sk: SecretKey, masks, errors) -> np.ndarray:
    allm = _mods_all(P)
    s2 = vec(allm, sk.eval_all, sk.eval_all, "mul", P.logn)
    return gen_switch_key(P, sk, s2, masks, errors)


def gen_galois_key(P: Params, sk: SecretKey, g: int, masks, errors) -> np.ndarray:
    sg = automorph_eval(P.logn, g, sk.eval_all)
    return gen_switch_key(P, sk, sg, masks, errors)


def encrypt(P: Params, sk: SecretKey, pt: np.ndarray, level: int, mask: np.ndarray, error: np.ndarray):
    """Secret-key encryption: c1 = a, c0 = -a s + m + e (eval domain)."""
    mods = P.q[: level + 1]
    a = np.asarray(mask, dtype=np.uint64)
    e = ntt(mods, to_rns(np.asarray(error, dtype=np.int64), mods), P.logn)
    c0 = vec(mods, vec(mods, pt, e, "add", P.logn), vec(mods, a, sk.eval_q(level), "mul", P.logn), "sub", P.logn)
    return c0, a


def decrypt(P: Params, sk: SecretKey, ct, level: int) -> np.ndarray:
    mods = P.q[: level + 1]
    return vec(mods, ct[0], vec(mods, ct[1], sk.eval_q(level), "mul", P.logn), "add", P.logn)
