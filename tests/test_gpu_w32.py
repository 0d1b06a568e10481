"""The 32-bit word path (ckks32_* through the C ABI) against the CPU oracle,
bit for bit on every limb: the oracle's definitions do not depend on the word
size, so each 32-bit result must equal the oracle on the same 30-bit primes.
N = 2^16; "w32-small" has 10 + 3 primes and dnum 3 (digits 4, 4, 2, so the
top level has a partial digit), "w32-large" 52 + 8 primes and dnum 4."""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import assert_equal, gpu_available
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

_ctx = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def setup(name):
    if name not in _ctx:
        from paper_2507_04775_amd import ckks
        ps = inputs.params32(name)
        _ctx[name] = (ps, oracle.Params(ps.logn, ps.q, ps.p, ps.dnum), ckks.Context32(ps.logn, ps.q, ps.p, ps.dnum))
    return _ctx[name]


def dev(a):
    from paper_2507_04775_amd import ckks
    return ckks.to_device32(a)


def host(t):
    import torch
    from paper_2507_04775_amd import ckks
    torch.cuda.synchronize()
    return ckks.to_host32(t)


LEVELS = {"w32-small": [9, 7, 4, 0], "w32-large": [51, 30, 12]}


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_ntt_intt_all_primes(name):
    ps, P, ctx = setup(name)
    mods = list(ps.q) + list(ps.p)
    a = inputs.uniform_residues(inputs.rng(1), mods, ps.N)
    t = dev(a)
    ctx.ntt(t, 0, len(mods))
    assert_equal(host(t), oracle.ntt(mods, a, ps.logn), "ntt32")
    ctx.intt(t, 0, len(mods))
    assert_equal(host(t), a, "intt32(ntt32)")
    b = inputs.uniform_residues(inputs.rng(2), mods, ps.N)
    tb = dev(b)
    ctx.intt(tb, 0, len(mods))
    assert_equal(host(tb), oracle.intt(mods, b, ps.logn), "intt32")


def test_ntt_edge_values():
    ps, P, ctx = setup("w32-small")
    mods = [ps.q[0], ps.q[-1], ps.p[-1]]
    a = np.zeros((3, ps.N), dtype=np.uint64)
    for i, m in enumerate(mods):
        a[i, ::2] = m - 1
        a[i, 1::4] = 1
    t = dev(a)
    ctx.ntt(t[:1], 0, 1)
    ctx.ntt(t[1:2], ps.L, 1)
    ctx.ntt(t[2:], ps.L + 1 + ps.K - 1, 1)
    assert_equal(host(t), oracle.ntt(mods, a, ps.logn), "ntt32 edge")
    ctx.intt(t[:1], 0, 1)
    ctx.intt(t[1:2], ps.L, 1)
    ctx.intt(t[2:], ps.L + 1 + ps.K - 1, 1)
    assert_equal(host(t), a, "intt32 edge")


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_modup(name):
    ps, P, ctx = setup(name)
    for level in LEVELS[name]:
        d = inputs.random_poly(10 + level, ps, level)
        ext = ctx.empty(ctx.beta(level), level + 1 + ps.K)
        ctx.modup(dev(d), level, ext)
        assert_equal(host(ext), oracle.modup(P, d, level), "modup32 level %d" % level)


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_moddown(name):
    ps, P, ctx = setup(name)
    for level in LEVELS[name]:
        x = np.stack([inputs.uniform_residues(inputs.rng(30 + level + t), P.row_moduli(level), ps.N) for t in range(2)])
        o0, o1 = ctx.empty(level + 1), ctx.empty(level + 1)
        ctx.moddown(dev(x), level, o0, o1)
        assert_equal(host(o0), oracle.moddown(P, x[0], level), "moddown32 0 level %d" % level)
        assert_equal(host(o1), oracle.moddown(P, x[1], level), "moddown32 1 level %d" % level)


def test_moddown_centring_threshold():
    """ModDown inputs whose special-prime residues after the inverse NTT sit at
    (p-1)/2 and (p+1)/2: the two sides of the centred conversion."""
    ps, P, ctx = setup("w32-small")
    level = ps.L
    rows = P.row_moduli(level)
    x = inputs.uniform_residues(inputs.rng(77), rows, ps.N)
    for k, p in enumerate(ps.p):
        coef = np.zeros(ps.N, dtype=np.uint64)
        coef[::2] = (p - 1) // 2
        coef[1::2] = (p + 1) // 2
        x[level + 1 + k] = oracle.ntt([p], coef[None, :], ps.logn)[0]
    xx = np.stack([x, x])
    o0, o1 = ctx.empty(level + 1), ctx.empty(level + 1)
    ctx.moddown(dev(xx), level, o0, o1)
    want = oracle.moddown(P, x, level)
    assert_equal(host(o0), want, "moddown32 centring 0")
    assert_equal(host(o1), want, "moddown32 centring 1")


def _key(ps, seed):
    return inputs.random_key(seed, ps)


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_keyswitch(name):
    ps, P, ctx = setup(name)
    key = _key(ps, 6)
    kd = dev(key.reshape(-1, ps.N)).reshape(key.shape)
    for level in LEVELS[name]:
        d = inputs.random_poly(40 + level, ps, level)
        o0, o1 = ctx.empty(level + 1), ctx.empty(level + 1)
        ctx.keyswitch(dev(d), level, kd, o0, o1)
        w0, w1 = oracle.keyswitch(P, d, key, level)
        assert_equal(host(o0), w0, "ks32 0 level %d" % level)
        assert_equal(host(o1), w1, "ks32 1 level %d" % level)


def test_keyswitch_max_residues():
    """Every input residue q - 1 and every key residue its prime minus one:
    the largest products and sums the 64-bit accumulations see."""
    ps, P, ctx = setup("w32-small")
    level = ps.L
    d = np.stack([np.full(ps.N, q - 1, dtype=np.uint64) for q in ps.q[: level + 1]])
    allm = list(ps.q) + list(ps.p)
    key = np.stack([np.stack([np.stack([np.full(ps.N, m - 1, dtype=np.uint64) for m in allm])] * 2)] * ps.dnum)
    o0, o1 = ctx.empty(level + 1), ctx.empty(level + 1)
    ctx.keyswitch(dev(d), level, dev(key.reshape(-1, ps.N)).reshape(key.shape), o0, o1)
    w0, w1 = oracle.keyswitch(P, d, key, level)
    assert_equal(host(o0), w0, "ks32 max 0")
    assert_equal(host(o1), w1, "ks32 max 1")


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_hmult_relin(name):
    ps, P, ctx = setup(name)
    key = _key(ps, 7)
    kd = dev(key.reshape(-1, ps.N)).reshape(key.shape)
    for level in LEVELS[name][:3]:
        a = inputs.random_ct(50 + level, ps, level)
        b = inputs.random_ct(60 + level, ps, level)
        o0, o1 = ctx.empty(level + 1), ctx.empty(level + 1)
        ctx.hmult_relin(dev(a[0]), dev(a[1]), dev(b[0]), dev(b[1]), level, kd, o0, o1)
        w0, w1 = oracle.hmult_relin(P, a, b, key, level)
        assert_equal(host(o0), w0, "hmult32 c0 level %d" % level)
        assert_equal(host(o1), w1, "hmult32 c1 level %d" % level)


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_rescale_out_of_place_and_in_place(name):
    ps, P, ctx = setup(name)
    for level in [l for l in LEVELS[name] if l > 0] + [1]:
        c = inputs.random_ct(70 + level, ps, level)
        w0, w1 = oracle.rescale(P, c, level)
        t0, t1 = dev(c[0]), dev(c[1])
        o0, o1 = ctx.empty(level), ctx.empty(level)
        ctx.rescale(t0, t1, level, o0, o1)
        assert_equal(host(o0), w0, "rescale32 c0 level %d" % level)
        assert_equal(host(o1), w1, "rescale32 c1 level %d" % level)
        ctx.rescale(t0, t1, level, t0[:level], t1[:level])
        assert_equal(host(t0[:level]), w0, "rescale32 in place c0 level %d" % level)
        assert_equal(host(t1[:level]), w1, "rescale32 in place c1 level %d" % level)


@pytest.mark.parametrize("name", ["w32-small", "w32-large"])
def test_rotation_and_conjugation(name):
    ps, P, ctx = setup(name)
    level = LEVELS[name][1]
    c = inputs.random_ct(80, ps, level)
    for g in [oracle.galois_for_rotation(ps.logn, 1), oracle.galois_for_rotation(ps.logn, inputs.rotation_index(3, 16)),
              2 * ps.N - 1]:
        key = _key(ps, 90 + g % 1000)
        o0, o1 = ctx.empty(level + 1), ctx.empty(level + 1)
        ctx.apply_galois(dev(c[0]), dev(c[1]), level, g, dev(key.reshape(-1, ps.N)).reshape(key.shape), o0, o1)
        w0, w1 = oracle.apply_galois(P, c, g, key, level)
        assert_equal(host(o0), w0, "galois32 %d c0" % g)
        assert_equal(host(o1), w1, "galois32 %d c1" % g)


def test_rejections():
    """Host-side refusals: primes at or above 2^30, log_n other than 16, a level out of range."""
    from paper_2507_04775_amd import ckks
    big = inputs.ntt_primes(31, 2, 16)
    with pytest.raises(ckks.CkksError, match="below 2\\^30"):
        ckks.Context32(16, big[:1], big[1:], 1)
    small = inputs.ntt_primes(30, 2, 12)
    with pytest.raises(ckks.CkksError, match="log_n"):
        ckks.Context32(12, small[:1], small[1:], 1)
    ps, P, ctx = setup("w32-small")
    d = ctx.empty(ps.L + 1)
    with pytest.raises(ckks.CkksError, match="out of range"):
        ctx.keyswitch(d, ps.L + 1, d, d, d)
