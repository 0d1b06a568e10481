"""GPU parity on inputs built to reach the edges of the arithmetic, through the
C ABI against the oracle, bit for bit:
- ModDown inputs whose scaled conversion inputs y_k sit on both sides of the
  centring threshold (p_k - 1)/2 (and at 0, 1, p_k - 2, p_k - 1 and the 32-bit
  word boundaries), with K = 2, 4 and 10 special primes;
- ModUp inputs whose scaled digit inputs take the same edge values, which
  drives the exact column sums of the conversion to their largest terms;
- inner products, HMult+relin and key switching on edge residues with keys
  whose every residue is q - 1."""
import numpy as np
import pytest

import oracle
from gpu_common import Setup, assert_equal, gpu_available
from helpers import edge_rows, scaled_inputs
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

_setups = {}


def setup(name):
    if name not in _setups:
        _setups[name] = Setup(name)
    return _setups[name]


def _say(msg):
    print(msg, flush=True)


def moddown_edge_input(s, level, seed):
    """Extended polynomial (evaluation domain) whose special rows carry edge
    scaled inputs y_k in the coefficient domain; q rows uniform."""
    ps = s.ps
    rows = list(ps.q[: level + 1]) + list(ps.p)
    qc = inputs.uniform_residues(inputs.rng(seed), ps.q[: level + 1], ps.N)
    pc = scaled_inputs(edge_rows(seed + 1, ps.p, ps.N), ps.p)
    return oracle.ntt(rows, np.concatenate([qc, pc]), ps.logn)


def modup_edge_input(s, level, seed):
    """Polynomial at `level` (evaluation domain) whose every digit's scaled
    conversion inputs take the edge values in the coefficient domain."""
    ps = s.ps
    a = np.empty((level + 1, ps.N), dtype=np.uint64)
    for j in range(s.P.beta(level)):
        lo, hi = j * s.P.alpha, min((j + 1) * s.P.alpha, level + 1)
        a[lo:hi] = scaled_inputs(edge_rows(seed + j, ps.q[lo:hi], ps.N, shift=j), ps.q[lo:hi])
    return oracle.ntt(ps.q[: level + 1], a, ps.logn)


def max_key(s):
    mods = list(s.ps.q) + list(s.ps.p)
    row = np.array([[m - 1] * s.N for m in mods], dtype=np.uint64)
    return np.ascontiguousarray(np.broadcast_to(row, (s.ps.dnum, 2) + row.shape))


@pytest.mark.parametrize("name,levels", [("small-nv", [3, 0]), ("large", [30, 12, 0]), ("large-nv", [30, 0])])
def test_moddown_centring_threshold(name, levels):
    s = setup(name)
    for level in levels:
        _say("moddown threshold %s level %d" % (name, level))
        x = moddown_edge_input(s, level, 500 + level)
        out = s.ctx.empty_poly(level)
        s.ctx.ckks_moddown(s.dev(x), level, out)
        assert_equal(s.host(out), oracle.moddown(s.P, x, level), "moddown edge %s level %d" % (name, level))


@pytest.mark.parametrize("name,levels", [("small", [3, 0]), ("large", [30, 21, 0]), ("large-nv", [30, 12])])
def test_modup_edge_digits(name, levels):
    s = setup(name)
    for level in levels:
        _say("modup edges %s level %d" % (name, level))
        d = modup_edge_input(s, level, 600 + level)
        ext = s.ctx.empty_poly(0).new_empty((s.ctx.beta(level), level + 1 + s.ps.K, s.N))
        s.ctx.ckks_modup(s.dev(d), level, ext)
        assert_equal(s.host(ext), oracle.modup(s.P, d, level), "modup edge %s level %d" % (name, level))


@pytest.mark.parametrize("name", ["small", "large"])
def test_inner_product_edge_residues_max_key(name):
    s = setup(name)
    key = max_key(s)
    kh = s.ctx.key(s.dev(key), 0)
    level = s.ps.L
    mods = s.P.row_moduli(level)
    ext = np.stack([edge_rows(700 + j, mods, s.N, shift=j) for j in range(s.ctx.beta(level))])
    te = s.dev(ext)
    for g in [1, 5]:
        _say("inner product edges %s g %d" % (name, g))
        acc = te.new_empty((2, len(mods), s.N))
        s.ctx.ckks_inner_product(te, level, kh, g, acc)
        assert_equal(s.host(acc), oracle.inner_product(s.P, ext, key, level, g), "ip edge g %d" % g)


@pytest.mark.parametrize("name", ["small", "large"])
def test_hmult_and_keyswitch_edge_residues_max_key(name):
    s = setup(name)
    key = max_key(s)
    kh = s.ctx.key(s.dev(key), 0)
    level = s.ps.L
    mods = s.ps.q[: level + 1]
    a = (edge_rows(800, mods, s.N), edge_rows(801, mods, s.N, shift=3))
    b = (edge_rows(802, mods, s.N, shift=5), modup_edge_input(s, level, 803))
    _say("hmult edges %s" % name)
    ta = s.ckks.Ciphertext(s.dev(a[0]), s.dev(a[1]), level, 1.0)
    tb = s.ckks.Ciphertext(s.dev(b[0]), s.dev(b[1]), level, 1.0)
    out = s.ctx.empty_ct(level)
    s.ctx.ckks_hmult_relin(ta, tb, kh, out)
    w0, w1 = oracle.hmult_relin(s.P, a, b, key, level)
    assert_equal(s.host(out.c0), w0, "hmult edge c0")
    assert_equal(s.host(out.c1), w1, "hmult edge c1")
    _say("keyswitch edges %s" % name)
    d = modup_edge_input(s, level, 804)
    o0, o1 = s.ctx.empty_poly(level), s.ctx.empty_poly(level)
    s.ctx.ckks_keyswitch(s.dev(d), level, kh, o0, o1)
    w0, w1 = oracle.keyswitch(s.P, d, key, level)
    assert_equal(s.host(o0), w0, "keyswitch edge 0")
    assert_equal(s.host(o1), w1, "keyswitch edge 1")
