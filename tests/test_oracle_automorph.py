"""Pins of the oracle's automorphism X -> X^g against evaluation at the 2N-th
roots and against the group laws of the Galois elements."""
import numpy as np
import pytest

import oracle
from helpers import br
from paper_2507_04775_amd import inputs


@pytest.mark.parametrize("g", [3, 5, 25, 127, 2 * 64 - 1])
def test_coef_automorphism_by_evaluation(g):
    logn, N = 6, 64
    q = inputs.ntt_primes(40, 1, logn)[0]
    psi = oracle.psi(q, logn)
    a = inputs.rng(g).integers(0, q, size=N, dtype=np.uint64)
    b = oracle.automorph_coef([q], logn, g, a[None])[0]
    for e in range(1, 2 * N, 2):   # b(psi^e) must equal a(psi^(e g))
        lhs = sum(int(b[j]) * pow(psi, e * j, q) for j in range(N)) % q
        rhs = sum(int(a[j]) * pow(psi, e * g * j, q) for j in range(N)) % q
        assert lhs == rhs


@pytest.mark.parametrize("name", ["tiny", "small"])
@pytest.mark.parametrize("g", [5, 25, 3, None])
def test_eval_automorphism_commutes_with_ntt(name, g):
    ps = inputs.params(name)
    g = g or 2 * ps.N - 1
    mods = ps.q
    a = inputs.uniform_residues(inputs.rng(3), mods, ps.N)
    lhs = oracle.ntt(mods, oracle.automorph_coef(mods, ps.logn, g, a), ps.logn)
    rhs = oracle.automorph_eval(ps.logn, g, oracle.ntt(mods, a, ps.logn))
    assert np.array_equal(lhs, rhs)


def test_eval_automorphism_is_the_stated_gather():
    logn, N, g = 5, 32, 7
    a = np.arange(N, dtype=np.uint64)[None]
    out = oracle.automorph_eval(logn, g, a)[0]
    for i in range(N):
        e = (2 * br(i, logn) + 1) * g % (2 * N)
        assert out[i] == br((e - 1) // 2, logn)


@pytest.mark.parametrize("name", ["small", "large"])
def test_galois_group_laws(name):
    ps = inputs.params(name)
    two_n = 2 * ps.N
    a = inputs.uniform_residues(inputs.rng(1), ps.q[:2], ps.N)
    g, h = pow(5, 3, two_n), pow(5, 1000, two_n)
    A = oracle.automorph_eval
    assert np.array_equal(A(ps.logn, h, A(ps.logn, g, a)), A(ps.logn, g * h % two_n, a))
    assert np.array_equal(A(ps.logn, pow(g, -1, two_n), A(ps.logn, g, a)), a)
    c = two_n - 1
    assert np.array_equal(A(ps.logn, c, A(ps.logn, c, a)), a)
    assert np.array_equal(A(ps.logn, 1, a), a)
