"""Bit-exact parity of every C-ABI call with the CPU oracle on seeded inputs,
at N = 2^12 (four limbs, dnum = 2) and N = 2^16 (31 limbs, dnum = 3, the
paper-scale shape), at several levels including partial last digits."""
import numpy as np
import pytest

import oracle
from gpu_common import Setup, assert_equal, gpu_available
from helpers import br
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

_setups = {}


def setup(name):
    if name not in _setups:
        _setups[name] = Setup(name)
    return _setups[name]


LEVELS = {"small": [3, 2, 1, 0], "large": [30, 21, 12, 0], "large-nv": [30, 12, 0]}


@pytest.mark.parametrize("name", ["small", "large"])
def test_twiddle_tables_match_oracle_roots(name):
    s = setup(name)
    for limb, m in enumerate(list(s.ps.q) + list(s.ps.p)):
        tw = s.ctx.twiddles(limb)
        psi = oracle.psi(m, s.ps.logn)
        for k in [0, 1, 2, 3, 100, s.N // 2, s.N - 1]:
            assert int(tw[k]) == pow(psi, br(k, s.ps.logn), m)


@pytest.mark.parametrize("name", ["small", "large"])
def test_ntt_intt_all_primes(name):
    s = setup(name)
    mods = list(s.ps.q) + list(s.ps.p)
    a = inputs.uniform_residues(inputs.rng(1), mods, s.N)
    t = s.dev(a)
    s.ctx.ckks_ntt(t, 0, len(mods))
    want = oracle.ntt(mods, a, s.ps.logn)
    assert_equal(s.host(t), want, "ntt")
    s.ctx.ckks_intt(t, 0, len(mods))
    assert_equal(s.host(t), a, "intt(ntt)")
    b = inputs.uniform_residues(inputs.rng(2), mods, s.N)
    tb = s.dev(b)
    s.ctx.ckks_intt(tb, 0, len(mods))
    assert_equal(s.host(tb), oracle.intt(mods, b, s.ps.logn), "intt")


@pytest.mark.parametrize("name", ["small", "large"])
def test_ntt_edge_values(name):
    s = setup(name)
    mods = list(s.ps.q[:2]) + list(s.ps.p[:1])
    a = np.zeros((3, s.N), dtype=np.uint64)
    for i, m in enumerate(mods):
        a[i, ::2] = m - 1          # maximal residues
        a[i, 1::4] = 1
    t = s.dev(a)
    s.ctx.ckks_ntt(t, 0, 2)
    s.ctx.ckks_ntt(t[2:], s.ps.L + 1, 1)
    assert_equal(s.host(t), oracle.ntt(mods, a, s.ps.logn), "ntt edge")


@pytest.mark.parametrize("name", ["small", "large", "large-nv"])
def test_modup(name):
    s = setup(name)
    for level in LEVELS[name]:
        d = inputs.random_poly(10 + level, s.ps, level)
        ext = s.ctx.empty_poly(0).new_empty((s.ctx.beta(level), level + 1 + s.ps.K, s.N))
        s.ctx.ckks_modup(s.dev(d), level, ext)
        assert_equal(s.host(ext), oracle.modup(s.P, d, level), "modup level %d" % level)


@pytest.mark.parametrize("name", ["small", "large", "large-nv"])
def test_inner_product(name):
    s = setup(name)
    key, kh = s.key(5, 0)
    for level in LEVELS[name][:2]:
        beta, rows = s.ctx.beta(level), level + 1 + s.ps.K
        mods = s.P.row_moduli(level)
        ext = np.stack([inputs.uniform_residues(inputs.rng(20 + j), mods, s.N) for j in range(beta)])
        te = s.dev(ext)
        for g in [1, 5, 2 * s.N - 1]:
            acc = te.new_empty((2, rows, s.N))
            s.ctx.ckks_inner_product(te, level, kh, g, acc)
            assert_equal(s.host(acc), oracle.inner_product(s.P, ext, key, level, g), "ip level %d g %d" % (level, g))


@pytest.mark.parametrize("name", ["small", "large", "large-nv"])
def test_moddown(name):
    s = setup(name)
    for level in LEVELS[name]:
        x = inputs.uniform_residues(inputs.rng(30 + level), s.P.row_moduli(level), s.N)
        out = s.ctx.empty_poly(level)
        s.ctx.ckks_moddown(s.dev(x), level, out)
        assert_equal(s.host(out), oracle.moddown(s.P, x, level), "moddown level %d" % level)


@pytest.mark.parametrize("name", ["small", "large", "large-nv"])
def test_keyswitch(name):
    s = setup(name)
    key, kh = s.key(6, 0)
    for level in LEVELS[name]:
        d = inputs.random_poly(40 + level, s.ps, level)
        o0, o1 = s.ctx.empty_poly(level), s.ctx.empty_poly(level)
        s.ctx.ckks_keyswitch(s.dev(d), level, kh, o0, o1)
        w0, w1 = oracle.keyswitch(s.P, d, key, level)
        assert_equal(s.host(o0), w0, "ks0 level %d" % level)
        assert_equal(s.host(o1), w1, "ks1 level %d" % level)


@pytest.mark.parametrize("name", ["small", "large"])
def test_hmult_relin(name):
    s = setup(name)
    key, kh = s.key(7, 0)
    for level in LEVELS[name][:3]:
        a, ta = s.ct(50 + level, level)
        b, tb = s.ct(60 + level, level)
        out = s.ctx.empty_ct(level)
        s.ctx.ckks_hmult_relin(ta, tb, kh, out)
        w0, w1 = oracle.hmult_relin(s.P, a, b, key, level)
        assert_equal(s.host(out.c0), w0, "hmult c0 level %d" % level)
        assert_equal(s.host(out.c1), w1, "hmult c1 level %d" % level)


@pytest.mark.parametrize("name", ["small", "large"])
def test_rescale_out_of_place_and_in_place(name):
    s = setup(name)
    for level in [l for l in LEVELS[name] if l > 0] + [1]:
        c, tc = s.ct(70 + level, level)
        w0, w1 = oracle.rescale(s.P, c, level)
        out = s.ctx.empty_ct(level - 1)
        s.ctx.ckks_rescale(tc, out)
        assert out.level == level - 1
        assert_equal(s.host(out.c0), w0, "rescale c0 level %d" % level)
        assert_equal(s.host(out.c1), w1, "rescale c1 level %d" % level)
        # in place: the output views the first `level` limbs of the input buffers
        inplace = s.ckks.Ciphertext(tc.c0[:level], tc.c1[:level], level - 1)
        s.ctx.ckks_rescale(tc, inplace)
        assert_equal(s.host(tc.c0[:level]), w0, "rescale in place c0")
        assert_equal(s.host(tc.c1[:level]), w1, "rescale in place c1")


@pytest.mark.parametrize("name", ["small", "large"])
def test_hrotate_and_conjugate(name):
    s = setup(name)
    level = LEVELS[name][0]
    c, tc = s.ct(80, level)
    for k in [1, inputs.rotation_index(3, s.ps.logn), -1]:
        g = oracle.galois_for_rotation(s.ps.logn, k)
        key, kh = s.key(90 + g % 1000, g)
        out = s.ctx.empty_ct(level)
        s.ctx.ckks_hrotate(tc, k, kh, out)
        w0, w1 = oracle.apply_galois(s.P, c, g, key, level)
        assert_equal(s.host(out.c0), w0, "rotate %d c0" % k)
        assert_equal(s.host(out.c1), w1, "rotate %d c1" % k)
    g = 2 * s.N - 1
    key, kh = s.key(99, g)
    out = s.ctx.empty_ct(level)
    s.ctx.ckks_conjugate(tc, kh, out)
    w0, w1 = oracle.apply_galois(s.P, c, g, key, level)
    assert_equal(s.host(out.c0), w0, "conjugate c0")
    assert_equal(s.host(out.c1), w1, "conjugate c1")


@pytest.mark.parametrize("name", ["small", "large"])
def test_hoisted_rotations(name):
    s = setup(name)
    level = LEVELS[name][1]
    c, tc = s.ct(81, level)
    ks = [1, 2, 16, 5]
    gs = [oracle.galois_for_rotation(s.ps.logn, k) for k in ks]
    keys = [s.key(200 + i, g) for i, g in enumerate(gs)]
    outs = [s.ctx.empty_ct(level) for _ in ks]
    s.ctx.ckks_hrotate_hoisted(tc, ks, [k[1] for k in keys], outs)
    w0, w1 = oracle.hoisted_rotate(s.P, c, gs, [k[0] for k in keys], level)
    for i in range(len(ks)):
        assert_equal(s.host(outs[i].c0), w0[i], "hoisted %d c0" % ks[i])
        assert_equal(s.host(outs[i].c1), w1[i], "hoisted %d c1" % ks[i])


def test_key_switching_with_every_prime_below_2_50():
    """N = 2^16 with every prime below 2^50 (seven ciphertext primes, three
    special ones): the special limbs take the FP64 arithmetic too, in the
    inner product's run of ModDown's first INTT pass and in ModDown's
    conversions, whose targets are all below 2^50 (split columns)."""
    s = setup("large-fp")
    assert all(q < 2 ** 50 for q in s.ps.q + s.ps.p) and len(set(s.ps.q + s.ps.p)) == 10
    key, kh = s.key(300, 0)
    g = oracle.galois_for_rotation(s.ps.logn, 3)
    rkey, rkh = s.key(301, g)
    for level in (6, 4, 0):
        d = inputs.random_poly(310 + level, s.ps, level)
        o0, o1 = s.ctx.empty_poly(level), s.ctx.empty_poly(level)
        s.ctx.ckks_keyswitch(s.dev(d), level, kh, o0, o1)
        w0, w1 = oracle.keyswitch(s.P, d, key, level)
        assert_equal(s.host(o0), w0, "ks0 level %d" % level)
        assert_equal(s.host(o1), w1, "ks1 level %d" % level)
        a, ta = s.ct(320 + level, level)
        b, tb = s.ct(330 + level, level)
        out = s.ctx.empty_ct(level)
        s.ctx.ckks_hmult_relin(ta, tb, kh, out)
        w0, w1 = oracle.hmult_relin(s.P, a, b, key, level)
        assert_equal(s.host(out.c0), w0, "hmult c0 level %d" % level)
        assert_equal(s.host(out.c1), w1, "hmult c1 level %d" % level)
        s.ctx.ckks_hrotate(ta, 3, rkh, out)
        w0, w1 = oracle.apply_galois(s.P, a, g, rkey, level)
        assert_equal(s.host(out.c0), w0, "rotate c0 level %d" % level)
        assert_equal(s.host(out.c1), w1, "rotate c1 level %d" % level)
        outs = [s.ctx.empty_ct(level)]
        s.ctx.ckks_hrotate_hoisted(ta, [3], [rkh], outs)
        w0, w1 = oracle.hoisted_rotate(s.P, a, [g], [rkey], level)
        assert_equal(s.host(outs[0].c0), w0[0], "hoisted c0 level %d" % level)
        assert_equal(s.host(outs[0].c1), w1[0], "hoisted c1 level %d" % level)


def test_hoisted_rotations_ten_special_primes_all_levels():
    """Hoisted rotations with K = 10 (ten-source ModDown conversions, 41-row
    extended polynomials) at l = 30, 12 and 0."""
    s = setup("large-nv")
    ks = [1, 3, 1024]
    gs = [oracle.galois_for_rotation(s.ps.logn, k) for k in ks]
    keys = [s.key(230 + i, g) for i, g in enumerate(gs)]
    for level in LEVELS["large-nv"]:
        c, tc = s.ct(82 + level, level)
        outs = [s.ctx.empty_ct(level) for _ in ks]
        s.ctx.ckks_hrotate_hoisted(tc, ks, [k[1] for k in keys], outs)
        w0, w1 = oracle.hoisted_rotate(s.P, c, gs, [k[0] for k in keys], level)
        for i in range(len(ks)):
            assert_equal(s.host(outs[i].c0), w0[i], "hoisted K=10 level %d rot %d c0" % (level, ks[i]))
            assert_equal(s.host(outs[i].c1), w1[i], "hoisted K=10 level %d rot %d c1" % (level, ks[i]))


@pytest.mark.parametrize("name", ["small", "large"])
def test_elementwise_ops(name):
    s = setup(name)
    level = LEVELS[name][1]
    mods = s.ps.q[: level + 1]
    a, b, c = (inputs.random_poly(300 + i, s.ps, level) for i in range(3))
    ta, tb, tc = s.dev(a), s.dev(b), s.dev(c)
    out = s.ctx.empty_poly(level)
    lg = s.ps.logn
    s.ctx.ckks_poly_add(ta, tb, out, level)
    assert_equal(s.host(out), oracle.vec(mods, a, b, "add", lg), "add")
    s.ctx.ckks_poly_sub(ta, tb, out, level)
    assert_equal(s.host(out), oracle.vec(mods, a, b, "sub", lg), "sub")
    s.ctx.ckks_poly_mul(ta, tb, out, level)
    assert_equal(s.host(out), oracle.vec(mods, a, b, "mul", lg), "mul")
    s.ctx.ckks_poly_mul_add(ta, tb, tc, out, level)
    assert_equal(s.host(out), oracle.vec(mods, oracle.vec(mods, a, b, "mul", lg), c, "add", lg), "mul_add")
    sc = [int(m) - 1 - i for i, m in enumerate(mods)]
    scal = np.array([[v] * s.N for v in sc], dtype=np.uint64)
    s.ctx.ckks_poly_scalar_mul(ta, sc, out, level)
    assert_equal(s.host(out), oracle.vec(mods, a, scal, "mul", lg), "scalar_mul")
    s.ctx.ckks_poly_scalar_add(ta, sc, out, level)
    assert_equal(s.host(out), oracle.vec(mods, a, scal, "add", lg), "scalar_add")
    g = oracle.galois_for_rotation(lg, 7)
    s.ctx.ckks_automorph(ta, g, out)
    assert_equal(s.host(out), oracle.automorph_eval(lg, g, a), "automorph")


@pytest.mark.parametrize("name", ["small", "large"])
def test_table_i_ciphertext_ops(name):
    """HAdd, PtAdd, PtMult, ScalarAdd, ScalarMult on whole ciphertexts (out of
    place and in place) and HSquare, each against the oracle applied per half."""
    s = setup(name)
    lg = s.ps.logn
    key, kh = s.key(9, 0)
    for level in (LEVELS[name][0], LEVELS[name][2], 0):
        mods = s.ps.q[: level + 1]
        (a0, a1), ta = s.ct(400 + level, level)
        (b0, b1), tb = s.ct(410 + level, level)
        pt = inputs.random_poly(420 + level, s.ps, level)
        tpt = s.dev(pt)
        sc = [int(m) - 2 - 3 * i for i, m in enumerate(mods)]
        scal = np.array([[v] * s.N for v in sc], dtype=np.uint64)
        add = lambda x, y: oracle.vec(mods, x, y, "add", lg)
        mul = lambda x, y: oracle.vec(mods, x, y, "mul", lg)
        cases = [
            ("hadd", lambda o: s.ctx.ckks_hadd(ta, tb, o), (add(a0, b0), add(a1, b1))),
            ("ptadd", lambda o: s.ctx.ckks_ptadd(ta, tpt, o), (add(a0, pt), a1)),
            ("ptmult", lambda o: s.ctx.ckks_ptmult(ta, tpt, 2.0 ** 40, o), (mul(a0, pt), mul(a1, pt))),
            ("scalar_add", lambda o: s.ctx.ckks_scalar_add(ta, sc, o), (add(a0, scal), a1)),
            ("scalar_mult", lambda o: s.ctx.ckks_scalar_mult(ta, sc, 3.0, o), (mul(a0, scal), mul(a1, scal))),
        ]
        for what, run, (w0, w1) in cases:
            out = s.ctx.empty_ct(level)
            run(out)
            assert out.level == level
            assert_equal(s.host(out.c0), w0, "%s c0 level %d" % (what, level))
            assert_equal(s.host(out.c1), w1, "%s c1 level %d" % (what, level))
        assert out.scale == 3.0 * ta.scale
        # in place: the output is the input's own buffers
        c0, c1 = ta.c0.clone(), ta.c1.clone()
        tin = s.ckks.Ciphertext(c0, c1, level, 1.0)
        s.ctx.ckks_ptadd(tin, tpt, tin)
        s.ctx.ckks_hadd(tin, tb, tin)
        s.ctx.ckks_scalar_mult(tin, sc, 1.0, tin)
        assert_equal(s.host(c0), mul(add(add(a0, pt), b0), scal), "in place c0 level %d" % level)
        assert_equal(s.host(c1), mul(add(a1, b1), scal), "in place c1 level %d" % level)
        if level > 0:
            out = s.ctx.empty_ct(level)
            s.ctx.ckks_hsquare(ta, kh, out)
            w0, w1 = oracle.hmult_relin(s.P, (a0, a1), (a0, a1), key, level)
            assert_equal(s.host(out.c0), w0, "hsquare c0 level %d" % level)
            assert_equal(s.host(out.c1), w1, "hsquare c1 level %d" % level)


@pytest.mark.parametrize("name", ["small"])
def test_table_i_ops_reject_bad_arguments(name):
    s = setup(name)
    (_, _), ta = s.ct(430, 2)
    (_, _), tb = s.ct(431, 1)
    out = s.ctx.empty_ct(2)
    with pytest.raises(s.ckks.CkksError, match="different levels"):
        s.ctx.ckks_hadd(ta, tb, out)
    with pytest.raises(s.ckks.CkksError, match="not reduced"):
        s.ctx.ckks_scalar_add(ta, [int(m) for m in s.ps.q[:3]], out)
    part = s.ckks.Ciphertext(ta.c0, out.c1, 2, 1.0)  # shares c0 with the input but not c1
    with pytest.raises(s.ckks.CkksError, match="overlaps"):
        s.ctx.ckks_ptadd(ta, s.dev(inputs.random_poly(432, s.ps, 2)), part)


def test_four_element_inverse_passes_are_bit_exact():
    """Tile code 2 on every inverse launch (8 rows or columns per workgroup, 4
    elements per thread; the default for plain inverse launches of at most 8
    limbs; the gathered and tensor row passes take 8-wide tiles, their column
    passes the 4-element form): INTT over 35, 8, 2 and 1 limbs, and HMult+relin,
    Rescale, HRotate at l = 30 and 12, against the oracle."""
    from paper_2507_04775_amd import ckks
    s = setup("large")
    try:
        for n in range(1, 129):
            ckks.ntt_tile_set(1, n, 2)
        assert ckks.ntt_tile_get(True, 35) == 2
        mods = list(s.ps.q) + list(s.ps.p)
        a = inputs.uniform_residues(inputs.rng(950), mods, s.N)
        for lo, n in [(0, len(mods)), (s.ps.L + 1, s.ps.K), (3, 2), (0, 8), (s.ps.L, 1)]:
            t = s.dev(a[lo: lo + n])
            s.ctx.ckks_intt(t, lo, n)
            assert_equal(s.host(t), oracle.intt(mods[lo: lo + n], a[lo: lo + n], s.ps.logn), "intt4 %d limbs" % n)
        key, kh = s.key(960, 0)
        g = oracle.galois_for_rotation(s.ps.logn, 3)
        rkey, rkh = s.key(961, g)
        for level in (30, 12):
            x, tx = s.ct(970 + level, level)
            y, ty = s.ct(980 + level, level)
            out = s.ctx.empty_ct(level)
            s.ctx.ckks_hmult_relin(tx, ty, kh, out)
            w0, w1 = oracle.hmult_relin(s.P, x, y, key, level)
            assert_equal(s.host(out.c0), w0, "hmult level %d" % level)
            assert_equal(s.host(out.c1), w1, "hmult level %d" % level)
            low = s.ctx.empty_ct(level - 1)
            s.ctx.ckks_rescale(tx, low)
            w0, w1 = oracle.rescale(s.P, x, level)
            assert_equal(s.host(low.c0), w0, "rescale level %d" % level)
            assert_equal(s.host(low.c1), w1, "rescale level %d" % level)
            s.ctx.ckks_hrotate(tx, 3, rkh, out)
            w0, w1 = oracle.apply_galois(s.P, x, g, rkey, level)
            assert_equal(s.host(out.c0), w0, "hrotate level %d" % level)
            assert_equal(s.host(out.c1), w1, "hrotate level %d" % level)
    finally:
        for n in range(1, 129):
            ckks.ntt_tile_set(1, n, 0)


@pytest.mark.parametrize("tile", [4, 8, 16])
def test_every_ntt_tile_width_is_bit_exact(tile):
    """The N = 2^16 passes with 4-, 8- and 16-wide tiles forced on every launch
    (the autotuner's design space): NTT / INTT over all 35 limbs and over 2 and
    8 limbs, HMult+relin, Rescale and HRotate at l = 30 and 12, each against
    the oracle."""
    from paper_2507_04775_amd import ckks
    s = setup("large")
    try:
        for inv in (0, 1):
            for n in range(1, 129):
                ckks.ntt_tile_set(inv, n, tile)
        assert ckks.ntt_tile_get(False, 35) == tile and ckks.ntt_tile_get(True, 2) == tile
        mods = list(s.ps.q) + list(s.ps.p)
        a = inputs.uniform_residues(inputs.rng(900 + tile), mods, s.N)
        for lo, n in [(0, len(mods)), (s.ps.L + 1, s.ps.K), (3, 2), (0, 8)]:
            t = s.dev(a[lo: lo + n])
            s.ctx.ckks_ntt(t, lo, n)
            assert_equal(s.host(t), oracle.ntt(mods[lo: lo + n], a[lo: lo + n], s.ps.logn), "ntt tile %d" % tile)
            s.ctx.ckks_intt(t, lo, n)
            assert_equal(s.host(t), a[lo: lo + n], "intt(ntt) tile %d" % tile)
        key, kh = s.key(910, 0)
        k = 5
        g = oracle.galois_for_rotation(s.ps.logn, k)
        rkey, rkh = s.key(911, g)
        for level in (30, 12):
            x, tx = s.ct(920 + level, level)
            y, ty = s.ct(930 + level, level)
            out = s.ctx.empty_ct(level)
            s.ctx.ckks_hmult_relin(tx, ty, kh, out)
            w0, w1 = oracle.hmult_relin(s.P, x, y, key, level)
            assert_equal(s.host(out.c0), w0, "hmult tile %d level %d" % (tile, level))
            assert_equal(s.host(out.c1), w1, "hmult tile %d level %d" % (tile, level))
            low = s.ctx.empty_ct(level - 1)
            s.ctx.ckks_rescale(tx, low)
            w0, w1 = oracle.rescale(s.P, x, level)
            assert_equal(s.host(low.c0), w0, "rescale tile %d level %d" % (tile, level))
            assert_equal(s.host(low.c1), w1, "rescale tile %d level %d" % (tile, level))
            s.ctx.ckks_hrotate(tx, k, rkh, out)
            w0, w1 = oracle.apply_galois(s.P, x, g, rkey, level)
            assert_equal(s.host(out.c0), w0, "hrotate tile %d level %d" % (tile, level))
            assert_equal(s.host(out.c1), w1, "hrotate tile %d level %d" % (tile, level))
    finally:
        for inv in (0, 1):
            for n in range(1, 129):
                ckks.ntt_tile_set(inv, n, 0)
