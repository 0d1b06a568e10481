"""The library's client helpers (encoding, encryption, key generation on the
device) against the oracle's client: encryptions and keys made here decrypt
correctly under the oracle, and HMult / HRotate with keys made here decrypt
to the plaintext computation."""
import numpy as np
import pytest

import oracle
from oracle import client as oc
from gpu_common import Setup, gpu_available
from helpers import max_err_bits
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("name", ["small-nv", "large-nv"])
def test_client_roundtrip_and_keys(name):
    from paper_2507_04775_amd.client import Client
    s = Setup(name)
    cl = Client(s.ctx, s.ps, seed=77)
    sk = oc.SecretKey(s.P, cl.s_coeffs)
    scale = 2.0 ** s.ps.log_scale
    lv = s.ps.L
    za = inputs.complex_slots(inputs.rng(1), s.N // 2)
    zb = inputs.complex_slots(inputs.rng(2), s.N // 2)
    a, b = cl.encrypt(za, lv, scale), cl.encrypt(zb, lv, scale)
    assert max_err_bits(cl.decrypt(a), za) < -(s.ps.log_scale - s.ps.logn - 8)
    got = oc.decode(s.P, oc.decrypt(s.P, sk, (s.host(a.c0), s.host(a.c1)), lv), lv, scale)
    assert max_err_bits(got, za) < -(s.ps.log_scale - s.ps.logn - 8)

    rlk = cl.relin_key()
    out = s.ctx.empty_ct(lv)
    s.ctx.ckks_hmult_relin(a, b, rlk, out)
    res = s.ctx.empty_ct(lv - 1)
    s.ctx.ckks_rescale(out, res)
    assert max_err_bits(cl.decrypt(res), za * zb) < -12

    k = 5
    rk = cl.rotation_key(k)
    rot = s.ctx.empty_ct(lv)
    s.ctx.ckks_hrotate(a, k, rk, rot)
    assert max_err_bits(cl.decrypt(rot), np.roll(za, -k)) < -12
    cj = s.ctx.empty_ct(lv)
    s.ctx.ckks_conjugate(a, cl.conjugation_key(), cj)
    assert max_err_bits(cl.decrypt(cj), np.conj(za)) < -12
