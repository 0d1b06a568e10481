"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2507_04775_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckks.h")
LIB = os.path.join(ROOT, "paper_2507_04775_amd", "libckks.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ckks_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2507_04775_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path_calls():
    syms = declared_symbols()
    for name in ["ckks_ntt", "ckks_intt", "ckks_modup", "ckks_moddown", "ckks_keyswitch", "ckks_hmult_relin",
                 "ckks_hrotate", "ckks_rescale", "ckks_inner_product", "ckks_hrotate_hoisted", "ckks_conjugate"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2507_04775_amd import ckks
    assert sorted(set(declared_symbols()) - set(ckks.EXPORTED)) == []


def _create(lib, logn, q, p, dnum):
    u64 = ctypes.c_uint64
    qa = (u64 * len(q))(*q)
    pa = (u64 * len(p))(*p)
    h = ctypes.c_void_p()
    lib.ckks_ctx_create.restype = ctypes.c_int
    return lib.ckks_ctx_create(ctypes.c_uint32(logn), qa, ctypes.c_uint32(len(q)), pa, ctypes.c_uint32(len(p)),
                               ctypes.c_uint32(dnum), 0, ctypes.byref(h)), h


def _err(lib):
    lib.ckks_last_error.restype = ctypes.c_char_p
    return lib.ckks_last_error().decode()


def test_ctx_create_rejects_bad_parameters_on_host(lib):
    ps = inputs.params("small")
    st, h = _create(lib, 13, ps.q, ps.p, 2)
    assert st == -6 and "log_n" in _err(lib)
    st, _ = _create(lib, 12, ps.q, ps.p, 0)
    assert st == -1
    st, _ = _create(lib, 12, ps.q, ps.p, 5)
    assert st == -1
    st, _ = _create(lib, 12, [ps.q[0] + 2] + ps.q[1:], ps.p, 2)   # not a prime congruent to 1 mod 2N
    assert st == -1 and "prime 0" in _err(lib)
    st, _ = _create(lib, 12, ps.q + [ps.q[1]], ps.p, 2)            # repeated prime
    assert st == -1 and "distinct" in _err(lib)
    big = inputs.ntt_primes(60, 20, 12)
    st, _ = _create(lib, 12, big[:17], big[17:18], 1)              # 17 primes in one digit
    assert st == -6


def test_null_context_is_rejected(lib):
    for name in ["ckks_ntt", "ckks_intt"]:
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        assert f(None, None, 0, 1, None) == -1
    lib.ckks_workspace_bytes.restype = ctypes.c_size_t
    assert lib.ckks_workspace_bytes(None, 3, 0) == 0


def test_w32_parameter_sets_are_valid():
    """The 32-bit word path's sets: distinct primes below 2^30, 1 mod 2N at
    N = 2^16, digits of at most 16 primes and at most 64 primes in all."""
    from paper_2507_04775_amd import inputs
    for name in ("w32-small", "w32-large"):
        ps = inputs.params32(name)
        allp = list(ps.q) + list(ps.p)
        assert len(set(allp)) == len(allp) <= 64
        assert all(p < 2 ** 30 and p % (2 << 16) == 1 and inputs.is_prime(p) for p in allp)
        assert ps.alpha <= 16 and ps.K <= 16 and ps.logn == 16
