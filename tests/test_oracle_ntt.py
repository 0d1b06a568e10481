"""Pins of the oracle's (i)NTT (Sec. III-F.4) against the definition of the
negacyclic transform and against schoolbook polynomial arithmetic."""
import numpy as np
import pytest

import oracle
from helpers import br
from paper_2507_04775_amd import inputs


@pytest.mark.parametrize("q,logn", [(97, 4), (193, 5), (257, 7), (7681, 8), (12289, 9)])
def test_psi_is_smallest_primitive_root_bruteforce(q, logn):
    N = 1 << logn
    # x^N = -1 (mod q) holds exactly for the primitive 2N-th roots (2N is a power of two)
    roots = [x for x in range(2, q) if pow(x, N, q) == q - 1]
    assert oracle.psi(q, logn) == min(roots)


@pytest.mark.parametrize("name", ["tiny", "small", "large"])
def test_psi_order_for_parameter_primes(name):
    ps = inputs.params(name)
    for m in list(ps.q) + list(ps.p):
        r = oracle.psi(m, ps.logn)
        assert pow(r, ps.N, m) == m - 1
        assert pow(r, 2 * ps.N, m) == 1


def _ntt_definition(a, q, psi, logn):
    N = 1 << logn
    return [sum(int(a[j]) * pow(psi, (2 * br(i, logn) + 1) * j, q) for j in range(N)) % q for i in range(N)]


@pytest.mark.parametrize("logn", [3, 4, 6])
def test_ntt_matches_quadratic_definition(logn):
    g = inputs.rng(11 + logn)
    ps = inputs.params("tiny")
    mods = [m for m in list(ps.q) + list(ps.p)]
    mods = [m for m in mods if (m - 1) % (2 << logn) == 0]
    for q in mods:
        a = g.integers(0, q, size=1 << logn, dtype=np.uint64)
        got = oracle.ntt([q], a[None], logn)[0]
        assert [int(v) for v in got] == _ntt_definition(a, q, oracle.psi(q, logn), logn)
        back = oracle.intt([q], got[None], logn)[0]
        assert np.array_equal(back, a)


def _negacyclic(a, b, q):
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            v = int(a[i]) * int(b[j])
            if k < N:
                c[k] += v
            else:
                c[k - N] -= v
    return [x % q for x in c]


@pytest.mark.parametrize("logn", [5, 8])
def test_pointwise_product_is_negacyclic_convolution(logn):
    g = inputs.rng(100 + logn)
    q = inputs.ntt_primes(60, 1, logn)[0]
    a = g.integers(0, q, size=1 << logn, dtype=np.uint64)
    b = g.integers(0, q, size=1 << logn, dtype=np.uint64)
    A = oracle.ntt([q], a[None], logn)
    B = oracle.ntt([q], b[None], logn)
    c = oracle.intt([q], oracle.vec([q], A, B, "mul", logn), logn)[0]
    assert [int(v) for v in c] == _negacyclic(a, b, q)


@pytest.mark.parametrize("name", ["small", "large"])
def test_ntt_intt_roundtrip_full_size(name):
    ps = inputs.params(name)
    mods = [ps.q[0], ps.q[-1], ps.p[-1]]
    a = inputs.uniform_residues(inputs.rng(5), mods, ps.N)
    A = oracle.ntt(mods, a, ps.logn)
    assert not np.array_equal(A, a)
    assert np.array_equal(oracle.intt(mods, A, ps.logn), a)
    assert np.array_equal(oracle.ntt(mods, oracle.intt(mods, a, ps.logn), ps.logn), a)
    assert (A < np.array(mods, dtype=np.uint64)[:, None]).all()


def test_ntt_of_monomial_full_size():
    # NTT(X)[i] = psi^(2 br(i) + 1): a closed form at N = 2^16
    ps = inputs.params("large")
    q = ps.q[5]
    a = np.zeros((1, ps.N), dtype=np.uint64)
    a[0, 1] = 1
    A = oracle.ntt([q], a, ps.logn)[0]
    psi = oracle.psi(q, ps.logn)
    for i in [0, 1, 2, 777, 4096, ps.N - 1]:
        assert int(A[i]) == pow(psi, 2 * br(i, ps.logn) + 1, q)
