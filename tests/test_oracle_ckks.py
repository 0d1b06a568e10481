"""Pins of the oracle's CKKS operations through decryption: encoding against
the canonical embedding, key switching against its noise bound, and HMult,
Rescale, HRotate, Conjugate and hoisted rotations against the plaintext
computation on noise-valid parameters."""
import numpy as np
import pytest

import oracle
from oracle import client
from helpers import ClientSetup, max_err_bits
from paper_2507_04775_amd import inputs


def test_embedding_matches_bruteforce_evaluation():
    logn, N = 5, 32
    g = inputs.rng(2)
    z = inputs.complex_slots(g, N // 2)
    m = client.embed_inverse(z, logn)
    zeta = np.exp(1j * np.pi / N)
    e = client.slot_exponents(logn)
    for j in range(N // 2):   # m(zeta^(5^j)) = z_j, m(zeta^(-5^j)) = conj(z_j)
        assert abs(sum(m[k] * zeta ** (e[j] * k) for k in range(N)) - z[j]) < 1e-12
        assert abs(sum(m[k] * zeta ** (-e[j] * k) for k in range(N)) - np.conj(z[j])) < 1e-12
    assert np.allclose(client.embed(m, logn), z, atol=1e-12)


@pytest.mark.parametrize("name", ["small-nv", "large-nv"])
def test_encode_decode_roundtrip(name):
    ps = inputs.params(name)
    P = oracle.Params(ps.logn, ps.q, ps.p, ps.dnum)
    z = inputs.complex_slots(inputs.rng(4), ps.N // 2)
    pt = client.encode(P, z, 2, 2.0 ** ps.log_scale)
    assert max_err_bits(client.decode(P, pt, 2, 2.0 ** ps.log_scale), z) < -(ps.log_scale - ps.logn - 4)


@pytest.fixture(scope="module")
def small_nv():
    return ClientSetup(inputs.params("small-nv"), seed=1234)


def _ks_error_coeffs(cs, d, k0, k1, s_prime, level):
    P, mods = cs.P, cs.ps.q[: level + 1]
    lhs = oracle.vec(mods, k0, oracle.vec(mods, k1, cs.sk.eval_q(level), "mul", P.logn), "add", P.logn)
    rhs = oracle.vec(mods, d, s_prime[: level + 1], "mul", P.logn)
    diff = oracle.intt(mods, oracle.vec(mods, lhs, rhs, "sub", P.logn), P.logn)
    return np.array(client.crt_centred(diff, mods), dtype=object)


@pytest.mark.parametrize("level", [3, 2, 0])
def test_keyswitch_noise_bound(small_nv, level):
    cs = small_nv
    d = inputs.random_poly(77 + level, cs.ps, level)
    k0, k1 = oracle.keyswitch(cs.P, d, cs.relin_key(), level)
    s2 = oracle.vec(list(cs.ps.q), cs.sk.eval_all[: cs.ps.L + 1], cs.sk.eval_all[: cs.ps.L + 1], "mul", cs.ps.logn)
    err = _ks_error_coeffs(cs, d, k0, k1, s2, level)
    assert max(abs(int(v)) for v in err) < 2 ** 16


def test_keyswitch_literal_K_is_too_noisy():
    # with K = 1 the special modulus is smaller than a digit: the error is huge
    cs = ClientSetup(inputs.params("small"), seed=99)
    level = 3
    d = inputs.random_poly(5, cs.ps, level)
    k0, k1 = oracle.keyswitch(cs.P, d, cs.relin_key(), level)
    s2 = oracle.vec(list(cs.ps.q), cs.sk.eval_all[:4], cs.sk.eval_all[:4], "mul", cs.ps.logn)
    err = _ks_error_coeffs(cs, d, k0, k1, s2, level)
    assert max(abs(int(v)) for v in err) > 2 ** 30


def test_hmult_rescale_decrypts_to_product(small_nv):
    cs = small_nv
    ps, level = cs.ps, 3
    sc = 2.0 ** ps.log_scale
    za, zb = inputs.complex_slots(cs.g, ps.N // 2), inputs.complex_slots(cs.g, ps.N // 2)
    a, b = cs.encrypt(za, level), cs.encrypt(zb, level)
    assert max_err_bits(cs.decrypt(a, level, sc), za) < -20
    m = oracle.hmult_relin(cs.P, a, b, cs.relin_key(), level)
    assert max_err_bits(cs.decrypt(m, level, sc * sc), za * zb) < -20
    r = oracle.rescale(cs.P, m, level)
    assert max_err_bits(cs.decrypt(r, level - 1, sc * sc / int(ps.q[level])), za * zb) < -20


@pytest.mark.parametrize("k", [1, 7, -3])
def test_hrotate_decrypts_to_rolled_slots(small_nv, k):
    cs = small_nv
    ps, level = cs.ps, 2
    sc = 2.0 ** ps.log_scale
    z = inputs.complex_slots(cs.g, ps.N // 2)
    ct = cs.encrypt(z, level)
    g = oracle.galois_for_rotation(ps.logn, k)
    r = oracle.apply_galois(cs.P, ct, g, cs.galois_key(g), level)
    assert max_err_bits(cs.decrypt(r, level, sc), np.roll(z, -k)) < -20


def test_conjugate_decrypts_to_conjugate(small_nv):
    cs = small_nv
    ps, level = cs.ps, 3
    sc = 2.0 ** ps.log_scale
    z = inputs.complex_slots(cs.g, ps.N // 2)
    ct = cs.encrypt(z, level)
    g = oracle.galois_conjugate(ps.logn)
    r = oracle.apply_galois(cs.P, ct, g, cs.galois_key(g), level)
    assert max_err_bits(cs.decrypt(r, level, sc), np.conj(z)) < -20


def test_hoisted_rotations_decrypt_to_rolls(small_nv):
    cs = small_nv
    ps, level = cs.ps, 3
    sc = 2.0 ** ps.log_scale
    z = inputs.complex_slots(cs.g, ps.N // 2)
    ct = cs.encrypt(z, level)
    ks = [1, 2, 5, 16]
    gs = [oracle.galois_for_rotation(ps.logn, k) for k in ks]
    o0, o1 = oracle.hoisted_rotate(cs.P, ct, gs, [cs.galois_key(g) for g in gs], level)
    for i, k in enumerate(ks):
        assert max_err_bits(cs.decrypt((o0[i], o1[i]), level, sc), np.roll(z, -k)) < -20


def test_rotation_composition_decrypts(small_nv):
    cs = small_nv
    ps, level = cs.ps, 3
    sc = 2.0 ** ps.log_scale
    z = inputs.complex_slots(cs.g, ps.N // 2)
    ct = cs.encrypt(z, level)
    g1, g2 = oracle.galois_for_rotation(ps.logn, 3), oracle.galois_for_rotation(ps.logn, 4)
    r = oracle.apply_galois(cs.P, oracle.apply_galois(cs.P, ct, g1, cs.galois_key(g1), level),
                            g2, cs.galois_key(g2), level)
    assert max_err_bits(cs.decrypt(r, level, sc), np.roll(z, -7)) < -20


@pytest.mark.slow
def test_large_nv_hmult_and_rotate_decrypt():
    cs = ClientSetup(inputs.params("large-nv"), seed=4321)
    ps, level = cs.ps, 4
    sc = 2.0 ** ps.log_scale
    za, zb = inputs.complex_slots(cs.g, ps.N // 2), inputs.complex_slots(cs.g, ps.N // 2)
    a, b = cs.encrypt(za, level), cs.encrypt(zb, level)
    m = oracle.rescale(cs.P, oracle.hmult_relin(cs.P, a, b, cs.relin_key(), level), level)
    assert max_err_bits(cs.decrypt(m, level - 1, sc * sc / int(ps.q[level])), za * zb) < -20
    k = inputs.rotation_index(7, ps.logn)
    g = oracle.galois_for_rotation(ps.logn, k)
    r = oracle.apply_galois(cs.P, a, g, cs.galois_key(g), level)
    assert max_err_bits(cs.decrypt(r, level, sc), np.roll(za, -k)) < -20
