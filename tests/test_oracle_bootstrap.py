"""Pins of the oracle's bootstrapping (Sec. III-F.7): the homomorphic DFT
factors against the brute-force canonical embedding, the baby-step/giant-step
evaluation against the dense map, and each homomorphic phase (ModRaise,
CoeffToSlot, EvalMod, the whole bootstrap) through decryption against what it
must compute on the plaintext."""
import numpy as np
import pytest

import oracle
from oracle import bootstrap as B
from oracle import client
from helpers import ClientSetup, br, max_err_bits
from paper_2507_04775_amd import inputs


def _dense_embedding(logn):
    """U[j][k] = zeta^(5^j k), j, k < n: z = U (t_lo + i t_hi) for the slots z of t."""
    N, n = 1 << logn, 1 << (logn - 1)
    e = client.slot_exponents(logn)
    return np.exp(1j * np.pi * np.outer(e, np.arange(n)) / N)


def _apply(mp, v):
    return sum(d * np.roll(v, -o) for o, d in mp.items())


@pytest.mark.parametrize("logn", [5, 6, 7])
def test_stages_compose_to_the_embedding(logn):
    n = 1 << (logn - 1)
    w = inputs.complex_slots(inputs.rng(logn), n)
    perm = np.array([br(x, logn - 1) for x in range(n)])
    U = _dense_embedding(logn)
    v = w[perm]
    for h in [1 << i for i in range(logn - 1)]:
        v = _apply(B.special_fft_stage(n, logn, h, False), v)
    assert np.max(np.abs(v - U @ w)) < 1e-10
    v = U @ w
    for h in [1 << i for i in range(logn - 1)][::-1]:
        v = _apply(B.special_fft_stage(n, logn, h, True), v)
    assert np.max(np.abs(v - w[perm])) < 1e-12


@pytest.mark.parametrize("logn,radix", [(6, [2, 2, 1]), (6, [5]), (7, [3, 3]), (7, [1, 4, 1])])
def test_groups_by_bsgs_equal_the_dense_transform(logn, radix):
    """Merged groups evaluated as sum_g rot(sum_b d'_(g,b) rot(v, b h0), G_g)
    reproduce the inverse and forward special FFT."""
    n = 1 << (logn - 1)
    w = inputs.complex_slots(inputs.rng(10 + logn), n)
    perm = np.array([br(x, logn - 1) for x in range(n)])
    U = _dense_embedding(logn)

    def bsgs(v, halves, inverse):
        m_lo, count, baby, giants, h0 = B.group_layout(n, halves)
        pds = B.group_diagonals(n, logn, halves, inverse)
        G = B.giant_offsets(n, halves)
        babies = [np.roll(v, -b * h0) for b in range(baby)]
        out = 0
        for g in range(giants):
            part = sum(pds[i] * babies[i - g * baby] for i in range(g * baby, min(count, (g + 1) * baby)))
            out = out + np.roll(part, -G[g])
        return out

    v = U @ w
    for halves in B.stage_groups(logn, radix, False):
        v = bsgs(v, halves, True)
    assert np.max(np.abs(v - w[perm])) < 1e-12
    v = w[perm]
    for halves in B.stage_groups(logn, radix[::-1], True):
        v = bsgs(v, halves, False)
    assert np.max(np.abs(v - U @ w)) < 1e-10


def test_layout_counts_and_rotations():
    # 2^11 slots, CoeffToSlot groups of 4, 4, 3 stages
    n = 2048
    g0, g1, g2 = B.stage_groups(12, [4, 4, 3], False)
    assert g0 == [1024, 512, 256, 128] and g2 == [4, 2, 1]
    assert B.group_layout(n, g0) == (0, 16, 4, 4, 128)        # holds n/2: offsets wrap
    assert B.group_layout(n, g1) == (-15, 31, 8, 4, 8)
    assert B.giant_offsets(n, g1) == [-120, -56, 8, 72]
    assert B.baby_offsets(n, g2) == [1, 2, 3]


def test_layout_at_n_2_15_three_groups_each_way():
    """The N = 2^16 full-slot layout (n = 2^15 slots, groups [5, 5, 5]) against
    values derived by hand from the group definition: a group holding the stage
    of half-size n/2 has R = 32 diagonals at m h0, m in [0, 32); the others 63
    at m in [-31, 31]; baby 8 (the smallest power of two whose square reaches
    the count), giants G_g = (8 g + m_lo) h0; 38 distinct rotations in all."""
    n = 1 << 15
    cts = B.stage_groups(16, [5, 5, 5], False)
    stc = B.stage_groups(16, [5, 5, 5], True)
    assert cts == [[16384, 8192, 4096, 2048, 1024], [512, 256, 128, 64, 32], [16, 8, 4, 2, 1]]
    assert stc == [[1, 2, 4, 8, 16], [32, 64, 128, 256, 512], [1024, 2048, 4096, 8192, 16384]]
    assert B.group_layout(n, cts[0]) == (0, 32, 8, 4, 1024)
    assert B.group_layout(n, cts[1]) == (-31, 63, 8, 8, 32)
    assert B.group_layout(n, cts[2]) == (-31, 63, 8, 8, 1)
    assert B.group_layout(n, stc[2]) == (0, 32, 8, 4, 1024)
    assert B.giant_offsets(n, cts[0]) == [0, 8192, 16384, 24576]
    assert B.giant_offsets(n, cts[1]) == [-992, -736, -480, -224, 32, 288, 544, 800]
    assert B.giant_offsets(n, cts[2]) == [-31, -23, -15, -7, 1, 9, 17, 25]
    assert B.baby_offsets(n, cts[0]) == [1024 * b for b in range(1, 8)]
    assert B.baby_offsets(n, stc[0]) == list(range(1, 8))
    bp = B.BootParams(logn=16, cts_radix_logs=[5, 5, 5], stc_radix_logs=[5, 5, 5], cheb_degree=31,
                      double_angles=3, k_range=12.0, top_scale=2.0 ** 50, in_scale=2.0 ** 50)
    assert len(B.rotations_needed(bp)) == 38


@pytest.fixture(scope="module")
def stages_16():
    n = 1 << 15
    return {h: (B.special_fft_stage(n, 16, h, False), B.special_fft_stage(n, 16, h, True))
            for h in [1 << i for i in range(15)]}


@pytest.mark.parametrize("forward,gi", [(False, 0), (False, 1), (False, 2), (True, 0), (True, 1), (True, 2)])
def test_groups_by_bsgs_equal_their_stages_at_n_2_15(stages_16, forward, gi):
    """Each merged group of the N = 2^16 schedule, evaluated in the BSGS form
    the executors use (pre-rotated diagonals, hoisted babies, giant steps),
    equals its butterfly stages applied one by one to a vector of 2^15 slots."""
    n = 1 << 15
    halves = B.stage_groups(16, [5, 5, 5], forward)[gi]
    v = inputs.complex_slots(inputs.rng(40 + gi + 3 * forward), n)
    want = v
    for h in halves:
        want = _apply(stages_16[h][0 if forward else 1], want)
    m_lo, count, baby, giants, h0 = B.group_layout(n, halves)
    pds = B.group_diagonals(n, 16, halves, not forward)
    G = B.giant_offsets(n, halves)
    babies = [np.roll(v, -b * h0) for b in range(baby)]
    got = 0
    for g in range(giants):
        part = sum(pds[i] * babies[i - g * baby] for i in range(g * baby, min(count, (g + 1) * baby)))
        got = got + np.roll(part, -G[g])
    assert np.max(np.abs(got - want)) < 1e-9


def test_stages_compose_to_the_embedding_on_sampled_rows_at_n_2_15(stages_16):
    """The 15 forward stages applied to bit-reversed slots reproduce sampled
    rows of the canonical embedding z_j = sum_k zeta^(5^j k) w_k at N = 2^16."""
    logn, n, N = 16, 1 << 15, 1 << 16
    w = inputs.complex_slots(inputs.rng(77), n)
    perm = np.array([br(x, logn - 1) for x in range(n)])
    v = w[perm]
    for h in [1 << i for i in range(logn - 1)]:
        v = _apply(stages_16[h][0], v)
    e = client.slot_exponents(logn)
    for j in [0, 1, 2, 777, 12345, n // 2, n - 1]:
        zj = np.sum(np.exp(1j * np.pi * (int(e[j]) * np.arange(n) % (2 * N)) / N) * w)
        assert abs(v[j] - zj) < 1e-7 * np.sqrt(n)


def test_scale_chain():
    ps = inputs.params("boot-small")
    q = ps.q
    sc = B.level_scales(q, ps.L, 2.0 ** 50)
    for l in range(1, ps.L + 1):
        assert abs(sc[l] * sc[l] / q[l] / sc[l - 1] - 1) < 1e-15
        assert abs(B.pt_scale(sc, q, l, 1) * sc[l] / q[l] / sc[l - 1] - 1) < 1e-15
        assert B.pt_scale(sc, q, l, 1) == B.const_factor(sc, q, l, l - 1)
    assert abs(B.pt_scale(sc, q, 20, 2) * sc[20] / (q[20] * q[19]) / sc[18] - 1) < 1e-15
    assert B.round_half_away(2.5) == 3 and B.round_half_away(-2.5) == -3 and B.round_half_away(-0.4) == 0


def test_reduce_f64_is_exact():
    mods = inputs.params("boot-small").q[:3]
    x = np.array([0.0, -1.0, 2.0 ** 53 + 2, -(2.0 ** 77) - 2.0 ** 30, 123456789012345.0, 3.0 * 2 ** 61])
    r = oracle.reduce_f64(mods, x)
    for i, m in enumerate(mods):
        assert [int(v) for v in r[i]] == [int(v) % m for v in x]


BP_SMALL = dict(logn=12, cts_radix_logs=[4, 4, 3], stc_radix_logs=[3, 4, 4], cheb_degree=63,
                double_angles=5, k_range=128.0, top_scale=2.0 ** 50, in_scale=2.0 ** 50)


@pytest.fixture(scope="module")
def boot_small():
    ps = inputs.params("boot-small")
    cs = ClientSetup(ps, seed=31)
    bp = B.BootParams(**BP_SMALL)
    pl = B.plan(cs.P, bp)
    rk = {k: cs.galois_key(oracle.galois_for_rotation(ps.logn, k)) for k in B.rotations_needed(bp)}
    ex = B.Executor(cs.P, pl, cs.relin_key(), cs.galois_key(oracle.galois_conjugate(ps.logn)), rk)
    z = inputs.complex_slots(inputs.rng(32), ps.N // 2)
    c0, c1 = cs.encrypt(z, 0, bp.in_scale)
    return cs, ex, z, (c0, c1, 0)


def _raised_coefficients(cs, ct):
    P = cs.P
    pt = client.decrypt(P, cs.sk, (ct[0], ct[1]), ct[2])
    return np.array(client.crt_centred(oracle.intt(P.q[: ct[2] + 1], pt, P.logn), P.q[: ct[2] + 1]), dtype=object)


def test_modraise_keeps_the_message_mod_q0(boot_small):
    cs, ex, z, ct = boot_small
    r = ex.modraise(ct)
    assert r[2] == cs.ps.L
    t = _raised_coefficients(cs, r)
    q0 = cs.ps.q[0]
    m = _raised_coefficients(cs, ct)   # the level-0 plaintext, centred mod q0
    assert all((int(a) - int(b)) % q0 == 0 for a, b in zip(t, m))
    assert max(abs(int(a) - int(b)) // q0 for a, b in zip(t, m)) < ex.bp.k_range


def test_coeff_to_slot_moves_coefficients_into_slots(boot_small):
    cs, ex, z, ct = boot_small
    r = ex.modraise(ct)
    t = _raised_coefficients(cs, r)
    n, q0, K = cs.ps.N // 2, cs.ps.q[0], ex.bp.k_range
    c = ex.coeff_to_slot(r)
    assert c[2] == cs.ps.L - 4
    perm = np.array([br(x, cs.ps.logn - 1) for x in range(n)])
    want = (t[:n].astype(float) + 1j * t[n:].astype(float))[perm] / (2 * q0 * K)
    assert max_err_bits(cs.decrypt((c[0], c[1]), c[2], ex.sc[c[2]]), want) < -30


def test_eval_mod_computes_the_scaled_sine(boot_small):
    cs, ex, z, ct = boot_small
    n = cs.ps.N // 2
    y = inputs.rng(33).uniform(-0.5, 0.5, size=n)
    yc = cs.encrypt(y, ex.L - 4, ex.sc[ex.L - 4])
    out = ex.eval_mod((yc[0], yc[1], ex.L - 4))
    assert out[2] == ex.L - 4 - B.levels_used(ex.bp)["evalmod"]
    got = cs.decrypt((out[0], out[1]), out[2], ex.sc[out[2]])
    assert max_err_bits(got, np.sin(2 * np.pi * ex.bp.k_range * y)) < -18


def test_bootstrap_recovers_the_input(boot_small):
    """Baby-step/giant-step EvalMod (b = 8): about 2^-10 at N = 2^12."""
    cs, ex, z, ct = boot_small
    out = ex.bootstrap(ct)
    assert out[2] == B.output_level(cs.P, ex.bp) == 1
    err = max_err_bits(cs.decrypt((out[0], out[1]), out[2], ex.sc[out[2]]), z)
    assert err < -9.5, err


def test_bootstrap_with_one_leaf_is_more_precise(boot_small):
    """With b above the degree the series is a single leaf (every T_k from the
    product tree): fewer noisy giants, about 2^-12.9."""
    cs, ex0, z, ct = boot_small
    bp = B.BootParams(**dict(BP_SMALL, cheb_baby=64))
    ex = B.Executor(cs.P, ex0.pl, ex0.rlk, ex0.ck, ex0.rk)
    ex.bp = bp
    out = ex.bootstrap(ct)
    assert out[2] == B.output_level(cs.P, bp) == 1
    err = max_err_bits(cs.decrypt((out[0], out[1]), out[2], ex.sc[out[2]]), z)
    assert err < -12, err


def test_bootstrap_with_sparse_secret_encapsulation():
    """Switching to a sparse secret (h = 32) around ModRaise keeps |I| small, so
    K = 12 with a degree-31 interpolant and 3 double angles suffices: three
    more levels left and about 2^-15."""
    ps = inputs.params("boot-small")
    cs = ClientSetup(ps, seed=31)
    bp = B.BootParams(**dict(BP_SMALL, cheb_degree=31, double_angles=3, k_range=12.0))
    pl = B.plan(cs.P, bp)
    rk = {k: cs.galois_key(oracle.galois_for_rotation(ps.logn, k)) for k in B.rotations_needed(bp)}
    to_sp, from_sp = cs.sparse_keys(32)
    ex = B.Executor(cs.P, pl, cs.relin_key(), cs.galois_key(oracle.galois_conjugate(ps.logn)), rk, to_sp, from_sp)
    z = inputs.complex_slots(inputs.rng(34), ps.N // 2)
    c0, c1 = cs.encrypt(z, 0, bp.in_scale)
    r = ex.switch((c0, c1, 0), to_sp)
    t = _raised_coefficients(cs, ex.switch(ex.modraise(r), from_sp))
    q0 = ps.q[0]
    assert max(abs(round(int(v) / q0)) for v in t) < 12
    out = ex.bootstrap((c0, c1, 0))
    assert out[2] == B.output_level(cs.P, bp) == 4
    err = max_err_bits(cs.decrypt((out[0], out[1]), out[2], ex.sc[out[2]]), z)
    assert err < -14, err


def test_chebyshev_split_reconstructs_the_series():
    """q T_G + r equals the series on [-1, 1] (Chebyshev product identity)."""
    c = list(inputs.rng(9).normal(size=40))
    y = np.linspace(-1, 1, 101)
    for G in (32, 21):
        q, r = B.cheb_split(c, G)
        TG = np.cos(G * np.arccos(y))
        got = np.polynomial.chebyshev.chebval(y, q) * TG + np.polynomial.chebyshev.chebval(y, r)
        assert np.max(np.abs(got - np.polynomial.chebyshev.chebval(y, c))) < 1e-12


def test_moddown_passes_multiples_of_p_exactly():
    """ModDown(P y + z) = y + ModDown(z) on every limb: the identity that lets
    a hoisted schedule add P-scaled terms in the extended basis."""
    ps = inputs.params("boot-small")
    cs = ClientSetup(ps, seed=5)
    l = 3
    g = inputs.rng(77)
    y = inputs.uniform_residues(g, ps.q[: l + 1], ps.N)
    z = inputs.uniform_residues(g, list(ps.q[: l + 1]) + list(ps.p), ps.N)
    emods = list(ps.q[: l + 1]) + list(ps.p)
    lhs = oracle.moddown(cs.P, oracle.vec(emods, B.ext_p(cs.P, y, l), z, "add", ps.logn), l)
    rhs = oracle.vec(ps.q[: l + 1], y, oracle.moddown(cs.P, z, l), "add", ps.logn)
    assert np.array_equal(lhs, rhs)


def test_hoisted_giant_with_one_part_is_the_plain_rotation():
    """One giant of the hoisted schedule, ModDown applied to it alone, is
    bit-identical to the oracle's plain HRotate of the same ciphertext."""
    ps = inputs.params("boot-small")
    cs = ClientSetup(ps, seed=6)
    l, k = 3, 5
    gal = oracle.galois_for_rotation(ps.logn, k)
    key = cs.galois_key(gal)
    g = inputs.rng(78)
    s0, s1 = (inputs.uniform_residues(g, ps.q[: l + 1], ps.N) for _ in range(2))
    emods = list(ps.q[: l + 1]) + list(ps.p)
    acc = oracle.inner_product(cs.P, oracle.modup(cs.P, oracle.automorph_eval(ps.logn, gal, s1), l), key, l)
    got0 = oracle.moddown(cs.P, oracle.vec(emods, acc[0], B.ext_p(cs.P, s0, l, gal), "add", ps.logn), l)
    got1 = oracle.moddown(cs.P, acc[1], l)
    want0, want1 = oracle.apply_galois(cs.P, (s0, s1), gal, key, l)
    assert np.array_equal(got0, want0) and np.array_equal(got1, want1)


def test_hoisted_coeff_to_slot_and_bootstrap(boot_small):
    """ModDown hoisted out of every giant-step loop: CoeffToSlot still moves
    the coefficients into the slots, and the bootstrap recovers the input as
    precisely as the plain schedule."""
    cs, ex0, z, ct = boot_small
    ex = B.Executor(cs.P, ex0.pl, ex0.rlk, ex0.ck, ex0.rk)
    ex.bp = B.BootParams(**dict(BP_SMALL, hoist_moddown=True))
    r = ex.modraise(ct)
    t = _raised_coefficients(cs, r)
    n, q0, K = cs.ps.N // 2, cs.ps.q[0], ex.bp.k_range
    c = ex.coeff_to_slot(r)
    perm = np.array([br(x, cs.ps.logn - 1) for x in range(n)])
    want = (t[:n].astype(float) + 1j * t[n:].astype(float))[perm] / (2 * q0 * K)
    assert max_err_bits(cs.decrypt((c[0], c[1]), c[2], ex.sc[c[2]]), want) < -30
    out = ex.bootstrap(ct)
    err = max_err_bits(cs.decrypt((out[0], out[1]), out[2], ex.sc[out[2]]), z)
    assert out[2] == 1 and err < -9.5, err


def test_error_budget_phases_at_n_2_12():
    """The phase-by-phase error budget (oracle.error_budget) at N = 2^12 with
    encapsulation: |I| inside K, CoeffToSlot far below EvalMod, EvalMod below
    the final error, and the final error within the bootstrap test's bound."""
    import re

    from oracle import error_budget
    rows = dict(error_budget.run(logn=12, uniform=False, verbose=False))
    I, K = map(float, re.findall(r"= ([0-9.]+)", rows["ModRaise"]))
    assert I < K
    bits = {k: float(re.search(r"2\^(-[0-9.]+)", v).group(1)) for k, v in rows.items() if k != "ModRaise"}
    assert bits["CoeffToSlot"] < bits["EvalMod re"] - 5 and bits["CoeffToSlot"] < bits["EvalMod im"] - 5
    assert max(bits["EvalMod re"], bits["EvalMod im"]) < bits["SlotToCoeff"] < -14
