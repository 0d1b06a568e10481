"""Plain CPU oracle for the RNS-CKKS key-switching hot path.

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or runs
anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library:
``ckks_oracle.c`` derives every constant (psi, twiddles, CRT constants) again
from the prime list, with textbook loops and exact 128-bit products reduced by
``%``.

Every function takes and returns numpy ``uint64`` arrays of canonical residues,
limb-major ``[limbs][N]``, evaluation domain unless stated otherwise.  Keys are
top-level keys laid out ``[dnum][2][nq+np][N]``.

Pins (tests/test_oracle_*.py) check these functions against what the paper and
the mathematics fix: the O(N^2) definition of the NTT and schoolbook negacyclic
products, exact big-integer CRT semantics of the base conversion, ModDown and
Rescale, automorphism laws, and decryption of HMult / HRotate results against
the plaintext computation.  The hoisted rotation is pinned by decryption only
(its bit pattern differs from the plain HRotate by design): beyond that it is
parity unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libckks_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP over independent limbs only)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.orc_psi.restype = u64
        L.orc_psi.argtypes = [u64, u32]
        L.orc_ntt.argtypes = [u64p, u32, u32, u64p, i32]
        L.orc_bconv.argtypes = [u64p, u32, u64p, u32, u32, u64p, u64p]
        L.orc_modup.argtypes = [u32, u64p, u32, u64p, u32, u32, u32, u64p, u64p]
        L.orc_inner_product.argtypes = [u32, u64p, u32, u64p, u32, u32, u32, u64p, u64p, u64, u64p]
        L.orc_moddown.argtypes = [u32, u64p, u32, u64p, u32, u32, u64p, u64p]
        L.orc_keyswitch.argtypes = [u32, u64p, u32, u64p, u32, u32, u32, u64p, u64p, u64p, u64p]
        L.orc_vec.argtypes = [u64p, u32, u32, u64p, u64p, u64p, i32]
        L.orc_hmult_relin.argtypes = [u32, u64p, u32, u64p, u32, u32, u32, u64p, u64p, u64p, u64p,
                                      u64p, u64p, u64p]
        L.orc_rescale.argtypes = [u32, u64p, u32, u64p, u64p]
        L.orc_automorph_eval.argtypes = [u32, u32, u64, u64p, u64p]
        L.orc_automorph_coef.argtypes = [u64p, u32, u32, u64, u64p, u64p]
        L.orc_apply_galois.argtypes = [u32, u64p, u32, u64p, u32, u32, u32, u64p, u64p, u64, u64p,
                                       u64p, u64p]
        L.orc_hoisted_rotate.argtypes = [u32, u64p, u32, u64p, u32, u32, u32, u64p, u64p, u32, u64p,
                                         ctypes.POINTER(u64p), u64p, u64p]
        L.orc_reduce_f64.argtypes = [u64p, u32, u32, ctypes.POINTER(ctypes.c_double), u64p]
        L.orc_set_threads.argtypes = [i32]
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], "oracle wants C-contiguous uint64"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


class Params:
    """Parameter set [N, L, dnum] with its primes q_0..q_L and p_0..p_{K-1}."""

    def __init__(self, logn: int, q, p, dnum: int):
        self.logn = int(logn)
        self.q = _u64(q)
        self.p = _u64(p)
        self.dnum = int(dnum)

    @property
    def N(self) -> int:
        return 1 << self.logn

    @property
    def nq(self) -> int:
        return len(self.q)

    @property
    def np_(self) -> int:
        return len(self.p)

    @property
    def alpha(self) -> int:
        return -(-self.nq // self.dnum)

    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def row_moduli(self, level: int) -> np.ndarray:
        """Moduli of the l+1+K rows of an extended polynomial at level l."""
        return _u64(list(self.q[: level + 1]) + list(self.p))

    def _args(self):
        return self.logn, _p(self.q), self.nq, _p(self.p), self.np_


def psi(q: int, logn: int) -> int:
    """Smallest primitive 2N-th root of unity mod q (0 if q != 1 mod 2N)."""
    return int(lib().orc_psi(int(q), int(logn)))


def ntt(mods, a: np.ndarray, logn: int) -> np.ndarray:
    a = _u64(a).copy()
    mods = _u64(mods)
    lib().orc_ntt(_p(mods), len(mods), logn, _p(a), 0)
    return a


def intt(mods, a: np.ndarray, logn: int) -> np.ndarray:
    a = _u64(a).copy()
    mods = _u64(mods)
    lib().orc_ntt(_p(mods), len(mods), logn, _p(a), 1)
    return a


def bconv(src, dst, x: np.ndarray, logn: int) -> np.ndarray:
    src, dst, x = _u64(src), _u64(dst), _u64(x)
    out = np.zeros((len(dst), 1 << logn), dtype=np.uint64)
    lib().orc_bconv(_p(src), len(src), _p(dst), len(dst), logn, _p(x), _p(out))
    return out


def modup(P: Params, d: np.ndarray, level: int) -> np.ndarray:
    d = _u64(d)
    assert d.shape == (level + 1, P.N)
    ext = np.zeros((P.beta(level), level + 1 + P.np_, P.N), dtype=np.uint64)
    lib().orc_modup(*P._args(), P.dnum, level, _p(d), _p(ext))
    return ext


def inner_product(P: Params, ext: np.ndarray, key: np.ndarray, level: int, g: int = 1) -> np.ndarray:
    ext, key = _u64(ext), _u64(key)
    assert key.shape == (P.dnum, 2, P.nq + P.np_, P.N)
    acc = np.zeros((2, level + 1 + P.np_, P.N), dtype=np.uint64)
    lib().orc_inner_product(*P._args(), P.dnum, level, _p(ext), _p(key), int(g), _p(acc))
    return acc


def moddown(P: Params, x: np.ndarray, level: int) -> np.ndarray:
    x = _u64(x)
    assert x.shape == (level + 1 + P.np_, P.N)
    out = np.zeros((level + 1, P.N), dtype=np.uint64)
    lib().orc_moddown(*P._args(), level, _p(x), _p(out))
    return out


def keyswitch(P: Params, d: np.ndarray, key: np.ndarray, level: int):
    d, key = _u64(d), _u64(key)
    assert d.shape == (level + 1, P.N) and key.shape == (P.dnum, 2, P.nq + P.np_, P.N)
    o0 = np.zeros((level + 1, P.N), dtype=np.uint64)
    o1 = np.zeros_like(o0)
    lib().orc_keyswitch(*P._args(), P.dnum, level, _p(d), _p(key), _p(o0), _p(o1))
    return o0, o1


def vec(mods, a, b, op: str, logn: int) -> np.ndarray:
    mods, a, b = _u64(mods), _u64(a), _u64(b)
    out = np.zeros_like(a)
    lib().orc_vec(_p(mods), len(mods), logn, _p(a), _p(b), _p(out), {"add": 0, "sub": 1, "mul": 2}[op])
    return out


def hmult_relin(P: Params, a, b, key, level: int):
    """a, b: (c0, c1) pairs at the same level. Returns (out0, out1), no rescale."""
    a0, a1 = _u64(a[0]), _u64(a[1])
    b0, b1 = _u64(b[0]), _u64(b[1])
    key = _u64(key)
    o0 = np.zeros((level + 1, P.N), dtype=np.uint64)
    o1 = np.zeros_like(o0)
    lib().orc_hmult_relin(*P._args(), P.dnum, level, _p(a0), _p(a1), _p(b0), _p(b1), _p(key), _p(o0), _p(o1))
    return o0, o1


def rescale_poly(P: Params, c: np.ndarray, level: int) -> np.ndarray:
    c = _u64(c)
    assert c.shape == (level + 1, P.N) and level >= 1
    out = np.zeros((level, P.N), dtype=np.uint64)
    lib().orc_rescale(P.logn, _p(P.q), level, _p(c), _p(out))
    return out


def rescale(P: Params, ct, level: int):
    return rescale_poly(P, ct[0], level), rescale_poly(P, ct[1], level)


def automorph_eval(logn: int, g: int, a: np.ndarray) -> np.ndarray:
    a = _u64(a)
    out = np.zeros_like(a)
    lib().orc_automorph_eval(logn, a.shape[0], int(g), _p(a), _p(out))
    return out


def automorph_coef(mods, logn: int, g: int, a: np.ndarray) -> np.ndarray:
    mods, a = _u64(mods), _u64(a)
    out = np.zeros_like(a)
    lib().orc_automorph_coef(_p(mods), len(mods), logn, int(g), _p(a), _p(out))
    return out


def apply_galois(P: Params, ct, g: int, key, level: int):
    c0, c1, key = _u64(ct[0]), _u64(ct[1]), _u64(key)
    o0 = np.zeros((level + 1, P.N), dtype=np.uint64)
    o1 = np.zeros_like(o0)
    lib().orc_apply_galois(*P._args(), P.dnum, level, _p(c0), _p(c1), int(g), _p(key), _p(o0), _p(o1))
    return o0, o1


def hoisted_rotate(P: Params, ct, gs, keys, level: int):
    c0, c1 = _u64(ct[0]), _u64(ct[1])
    keys = [_u64(k) for k in keys]
    n = len(gs)
    gs_a = _u64(gs)
    kp = (ctypes.POINTER(ctypes.c_uint64) * n)(*[_p(k) for k in keys])
    o0 = np.zeros((n, level + 1, P.N), dtype=np.uint64)
    o1 = np.zeros_like(o0)
    lib().orc_hoisted_rotate(*P._args(), P.dnum, level, _p(c0), _p(c1), n, _p(gs_a), kp, _p(o0), _p(o1))
    return o0, o1


def reduce_f64(mods, x: np.ndarray) -> np.ndarray:
    """Exact residues [len(mods)][len(x)] of integer-valued doubles."""
    mods = _u64(mods)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    assert np.all(np.floor(x) == x), "plaintext coefficients must be integers"
    out = np.zeros((len(mods), len(x)), dtype=np.uint64)
    lib().orc_reduce_f64(_p(mods), len(mods), len(x), x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _p(out))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def galois_for_rotation(logn: int, k: int) -> int:
    """g = 5^k mod 2N (left rotation by k slots; negative k through 5^-1)."""
    two_n = 2 << logn
    return pow(5, k % (1 << (logn - 1)), two_n)


def galois_conjugate(logn: int) -> int:
    return (2 << logn) - 1
