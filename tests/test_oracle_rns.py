"""Pins of the oracle's fast base conversion (Eq. (1)), ModUp, ModDown and
Rescale against exact big-integer CRT semantics."""
import numpy as np
import pytest

import oracle
from helpers import crt, edge_rows, oracle_params, prod, scaled_inputs
from paper_2507_04775_amd import inputs


def _prod(xs):
    r = 1
    for x in xs:
        r *= int(x)
    return r


def _crt(res, mods):
    """Integer in [0, prod(mods)) with the given residues (Python's own CRT)."""
    M = _prod(mods)
    x = 0
    for r, m in zip(res, mods):
        Mi = M // int(m)
        x += int(r) * Mi * pow(Mi, -1, int(m))
    return x % M


def _check_conversion(xs, outs, src, dst):
    """outs_c = X + u*B (mod c) for every target c with one u in [0, len(src))."""
    B = _prod(src)
    X = _crt(xs, src)
    hits = [u for u in range(len(src)) if all((X + u * B - int(o)) % int(c) == 0 for o, c in zip(outs, dst))]
    assert len(hits) == 1, (hits, X)


@pytest.mark.parametrize("ns,nd", [(1, 3), (3, 4), (4, 2), (11, 5)])
def test_bconv_exact_semantics(ns, nd):
    logn = 6
    pool = inputs.ntt_primes(60, 8, logn) + inputs.ntt_primes(50, 12, logn)
    src, dst = pool[:ns], pool[ns: ns + nd]
    x = inputs.uniform_residues(inputs.rng(ns * 10 + nd), src, 1 << logn)
    out = oracle.bconv(src, dst, x, logn)
    for n in range(1 << logn):
        _check_conversion(x[:, n], out[:, n], src, dst)


def test_bconv_edge_values():
    logn = 6
    src = inputs.ntt_primes(60, 3, logn)
    dst = inputs.ntt_primes(50, 3, logn)
    N = 1 << logn
    x = np.zeros((3, N), dtype=np.uint64)
    for i, m in enumerate(src):
        x[i, 1] = m - 1          # X = -1 mod B
        x[i, 2] = 1
        x[i, 3] = m - 1 if i == 0 else 0
    out = oracle.bconv(src, dst, x, logn)
    assert (out[:, 0] == 0).all()   # X = 0 converts to 0 exactly
    for n in range(N):
        _check_conversion(x[:, n], out[:, n], src, dst)


@pytest.mark.parametrize("name,level", [("tiny", 3), ("tiny", 2), ("tiny", 0), ("small", 3), ("small", 1)])
def test_modup_digit_semantics(name, level):
    ps = inputs.params(name)
    P = oracle_params(ps)
    d = inputs.random_poly(7 + level, ps, level)
    ext = oracle.modup(P, d, level)
    rows = P.row_moduli(level)
    assert ext.shape == (P.beta(level), len(rows), ps.N)
    dc = oracle.intt(ps.q[: level + 1], d, ps.logn)
    coeffs = range(ps.N) if ps.N <= 64 else [0, 1, 5, 100, ps.N - 1]
    for j in range(P.beta(level)):
        lo, hi = j * P.alpha, min((j + 1) * P.alpha, level + 1)
        assert np.array_equal(ext[j, lo:hi], d[lo:hi])    # the digit's own rows are copied
        other = [r for r in range(len(rows)) if not lo <= r < hi]
        ec = oracle.intt(rows[other], ext[j, other], ps.logn)
        for n in coeffs:
            _check_conversion(dc[lo:hi, n], ec[:, n], ps.q[lo:hi], rows[other])


def _moddown_case(ps, level, seed):
    P = oracle_params(ps)
    rows = P.row_moduli(level)
    x = inputs.uniform_residues(inputs.rng(seed), rows, ps.N)
    out = oracle.moddown(P, x, level)
    return P, rows, x, out


@pytest.mark.parametrize("name,level", [("tiny", 3), ("tiny", 0), ("small", 2), ("small-nv", 1)])
def test_moddown_is_centred_division(name, level):
    """out = (X - v) / P exactly, with v = X mod P and |v| < K P / 2 (X the
    integer the rows represent); for K = 1 that is X / P rounded."""
    ps = inputs.params(name)
    P, rows, x, out = _moddown_case(ps, level, 31 + level)
    xc = oracle.intt(rows, x, ps.logn)
    oc = oracle.intt(ps.q[: level + 1], out, ps.logn)
    Pp = _prod(ps.p)
    Ql = _prod(ps.q[: level + 1])
    coeffs = range(ps.N) if ps.N <= 64 else [0, 3, 99, ps.N - 1]
    for n in coeffs:
        A = _crt(xc[:, n], rows)
        o = _crt(oc[:, n], ps.q[: level + 1])
        v = (A - o * Pp) % (Ql * Pp)
        if v > Ql * Pp // 2:
            v -= Ql * Pp
        assert 2 * abs(v) < ps.K * Pp
        if ps.K == 1:
            assert 2 * abs(v) < Pp


def moddown_threshold_input(ps, level, seed):
    """An extended polynomial (evaluation domain, rows q_0..q_l, p_0..p_{K-1})
    whose special rows give scaled conversion inputs y_k (coefficient domain)
    cycling through 0, 1, (p_k-1)/2, (p_k+1)/2, p_k-2, p_k-1 and the 32-bit
    word boundaries, mixed across k; the q rows are uniform."""
    rows = list(ps.q[: level + 1]) + list(ps.p)
    g = inputs.rng(seed)
    qc = inputs.uniform_residues(g, ps.q[: level + 1], ps.N)
    pc = scaled_inputs(edge_rows(seed + 1, ps.p, ps.N), ps.p)
    return oracle.ntt(rows, np.concatenate([qc, pc]), ps.logn)


def centred_v(ps, pcoef) -> int:
    """v = sum_k y_k^ctr (P/p_k), y_k = [a_k (P/p_k)^-1]_{p_k} lifted to
    y_k - p_k above (p_k - 1)/2, for the special-row coefficients a_k."""
    Pp = prod(ps.p)
    v = 0
    for a, pk in zip(pcoef, ps.p):
        pk = int(pk)
        Pk = Pp // pk
        y = int(a) * pow(Pk, -1, pk) % pk
        v += (y - pk if y > (pk - 1) // 2 else y) * Pk
    return v


@pytest.mark.parametrize("name,level", [("tiny", 3), ("small", 2), ("small-nv", 3), ("small-nv", 0),
                                        ("large-nv", 30), ("large-nv", 0)])
def test_moddown_exact_centred_conversion(name, level):
    """Bit-determining for any K: out = (X - v) / P mod Q_l exactly, with v the
    centred conversion sum (ModDown reading of Eq. (1), III-F.3), on inputs that
    put y_k on both sides of the centring threshold (p_k-1)/2."""
    ps = inputs.params(name)
    P = oracle_params(ps)
    rows = P.row_moduli(level)
    x = moddown_threshold_input(ps, level, 40 + level)
    out = oracle.moddown(P, x, level)
    xc = oracle.intt(rows, x, ps.logn)
    oc = oracle.intt(ps.q[: level + 1], out, ps.logn)
    Pp, Ql = prod(ps.p), prod(ps.q[: level + 1])
    coeffs = range(ps.N) if ps.N <= 4096 else list(range(0, 64)) + list(range(ps.N - 64, ps.N, 3))
    nq = level + 1
    for n in coeffs:
        A = crt(xc[:, n], rows)
        v = centred_v(ps, xc[nq:, n])
        assert (A - v) % Pp == 0
        assert crt(oc[:, n], ps.q[: level + 1]) == ((A - v) // Pp) % Ql, n


@pytest.mark.parametrize("name", ["small", "small-nv"])
def test_moddown_error_has_zero_mean(name):
    """The rounding error v / P of ModDown averages to zero over a polynomial
    (a canonical conversion would average about -K/2)."""
    ps = inputs.params(name)
    level = 2
    P, rows, x, out = _moddown_case(ps, level, 77)
    xc = oracle.intt(rows, x, ps.logn)
    oc = oracle.intt(ps.q[: level + 1], out, ps.logn)
    Pp, Ql = _prod(ps.p), _prod(ps.q[: level + 1])
    errs = []
    for n in range(0, ps.N, 4):
        A = _crt(xc[:, n], rows)
        o = _crt(oc[:, n], ps.q[: level + 1])
        v = (A - o * Pp) % (Ql * Pp)
        if v > Ql * Pp // 2:
            v -= Ql * Pp
        errs.append(v / Pp)
    assert abs(np.mean(errs)) < 0.05 * ps.K


@pytest.mark.parametrize("name,level", [("tiny", 3), ("small", 3), ("small", 0)])
def test_moddown_of_multiple_of_P_is_exact(name, level):
    ps = inputs.params(name)
    P = oracle_params(ps)
    xq = inputs.random_poly(3, ps, level)
    Pmod = np.array([_prod(ps.p) % int(q) for q in ps.q[: level + 1]], dtype=np.uint64)
    scaled = oracle.vec(ps.q[: level + 1], xq, np.broadcast_to(Pmod[:, None], xq.shape).copy(), "mul", ps.logn)
    x = np.concatenate([scaled, np.zeros((ps.K, ps.N), dtype=np.uint64)])
    assert np.array_equal(oracle.moddown(P, x, level), xq)


@pytest.mark.parametrize("name,level", [("tiny", 3), ("tiny", 1), ("small", 3), ("small", 1)])
def test_rescale_is_rounded_division(name, level):
    ps = inputs.params(name)
    P = oracle_params(ps)
    c = inputs.random_poly(50 + level, ps, level)
    out = oracle.rescale_poly(P, c, level)
    cc = oracle.intt(ps.q[: level + 1], c, ps.logn)
    oc = oracle.intt(ps.q[:level], out, ps.logn)
    ql = int(ps.q[level])
    Qm = _prod(ps.q[:level])
    coeffs = range(ps.N) if ps.N <= 64 else [0, 1, 2, 1000, ps.N - 1]
    for n in coeffs:
        C = _crt(cc[:, n], ps.q[: level + 1])
        want = ((2 * C + ql) // (2 * ql)) % Qm     # nearest integer to C / q_l (q_l odd: no ties)
        assert _crt(oc[:, n], ps.q[:level]) == want


def test_rescale_of_exact_multiple():
    # c = q_l * m (coefficients) rescales to m exactly
    ps = inputs.params("small")
    P = oracle_params(ps)
    level = 3
    m = inputs.rng(9).integers(-1000, 1000, size=ps.N)
    ql = int(ps.q[level])
    mods = ps.q[: level + 1]
    coef = np.array([[(int(v) * ql) % int(q) for v in m] for q in mods], dtype=np.uint64)
    c = oracle.ntt(mods, coef, ps.logn)
    out = oracle.intt(ps.q[:level], oracle.rescale_poly(P, c, level), ps.logn)
    want = np.array([[int(v) % int(q) for v in m] for q in ps.q[:level]], dtype=np.uint64)
    assert np.array_equal(out, want)
