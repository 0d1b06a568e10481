"""Batched key switching through the persistent work-queue kernels: every item
of a mixed batch (HMult+relin, key switch, rotation, hoisted rotations, at
different levels) must equal, bit for bit, the single-operation call and the
oracle; HIP-graph replays and autotuned grids must not change a bit."""
import numpy as np
import pytest

import oracle
from gpu_common import Setup, assert_equal, gpu_available
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

_setups = {}


def setup(name):
    if name not in _setups:
        _setups[name] = Setup(name)
    return _setups[name]


PLANS = {
    "small": dict(hmult=[3, 1], ks=[2], rot=[(3, 1)], hoisted=[(2, [1, 3])]),
    "large": dict(hmult=[30, 4], ks=[17], rot=[(21, 5)], hoisted=[(12, [1, 2, 64])]),
    # items sharing keys, as in a serving batch: ten relinearisations (more than one group of
    # inner products per key) and rotations by the same amounts at different levels
    "small_shared": dict(params="small", shared_keys=True, hmult=[3, 1, 2, 3, 0, 1, 2, 3, 1, 2], ks=[2],
                         rot=[(3, 1), (0, 3)], hoisted=[(2, [1, 3]), (3, [1, 3]), (1, [3, 1]), (0, [1])]),
}


def params_of(name):
    return PLANS[name].get("params", name)


def build_batch(s, plan, seed):
    """Returns (batch, expected-result thunks, output list)."""
    ck = s.ckks
    ctx = s.ctx
    b = ck.Batch(ctx)
    checks = []
    rlk_np, rlk = s.key(seed, 0)
    cache = {}

    def rot_key(key_seed, g):
        """A rotation key; with shared keys, one key object per Galois element."""
        if not plan.get("shared_keys"):
            return s.key(key_seed, g)
        if g not in cache:
            cache[g] = s.key(seed + 50 + g, g)
        return cache[g]
    for i, lv in enumerate(plan["hmult"]):
        a_np, a = s.ct(seed + 10 + i, lv)
        b_np, bb = s.ct(seed + 20 + i, lv)
        out = ctx.empty_ct(lv)
        b.hmult(a, bb, rlk, out)
        checks.append(("hmult", lv, (a, bb, rlk), [out], (a_np, b_np, rlk_np)))
    for i, lv in enumerate(plan["ks"]):
        d_np = inputs.random_poly(seed + 30 + i, s.ps, lv)
        d = s.dev(d_np)
        o0, o1 = ctx.empty_poly(lv), ctx.empty_poly(lv)
        b.keyswitch(d, lv, rlk, o0, o1)
        checks.append(("ks", lv, (d, rlk), [ck.Ciphertext(o0, o1, lv)], (d_np, rlk_np)))
    for i, (lv, k) in enumerate(plan["rot"]):
        g = oracle.galois_for_rotation(s.ps.logn, k)
        key_np, key = rot_key(seed + 40 + i, g)
        c_np, c = s.ct(seed + 45 + i, lv)
        out = ctx.empty_ct(lv)
        b.rotate(c, g, key, out)
        checks.append(("rot", lv, (c, g, key), [out], (c_np, key_np)))
    for i, (lv, ks) in enumerate(plan["hoisted"]):
        gs = [oracle.galois_for_rotation(s.ps.logn, k) for k in ks]
        keys = [rot_key(seed + 50 + 5 * i + j, g) for j, g in enumerate(gs)]
        c_np, c = s.ct(seed + 60 + i, lv)
        outs = [ctx.empty_ct(lv) for _ in ks]
        b.hoisted(c, ks, [k[1] for k in keys], outs)
        checks.append(("hoisted", lv, (c, ks, [k[1] for k in keys]), outs, (c_np, gs, [k[0] for k in keys])))
    b.build()
    return b, checks


def single_op(s, kind, lv, args):
    ctx = s.ctx
    if kind == "hmult":
        out = ctx.empty_ct(lv)
        ctx.ckks_hmult_relin(*args, out)
        return [out]
    if kind == "ks":
        d, key = args
        o0, o1 = ctx.empty_poly(lv), ctx.empty_poly(lv)
        ctx.ckks_keyswitch(d, lv, key, o0, o1)
        return [s.ckks.Ciphertext(o0, o1, lv)]
    if kind == "rot":
        c, g, key = args
        out = ctx.empty_ct(lv)
        ctx.ckks_apply_galois(c, g, key, out)
        return [out]
    c, ks, keys = args
    outs = [ctx.empty_ct(lv) for _ in ks]
    ctx.ckks_hrotate_hoisted(c, ks, keys, outs)
    return outs


def compare_to_single(s, checks, tag):
    for kind, lv, args, outs, _ in checks:
        want = single_op(s, kind, lv, args)
        for o, w in zip(outs, want):
            assert_equal(s.host(o.c0), s.host(w.c0), "%s %s level %d c0" % (tag, kind, lv))
            assert_equal(s.host(o.c1), s.host(w.c1), "%s %s level %d c1" % (tag, kind, lv))


@pytest.mark.parametrize("name", ["small", "large", "small_shared"])
def test_batch_matches_single_ops_and_oracle(name):
    s = setup(params_of(name))
    b, checks = build_batch(s, PLANS[name], 700)
    assert b.keyswitches == sum(len(c[3]) for c in checks)
    b.run()
    compare_to_single(s, checks, "batch")
    for kind, lv, args, outs, np_args in checks:   # the oracle on a subset
        if kind == "hmult" and lv == min(PLANS[name]["hmult"]):
            w0, w1 = oracle.hmult_relin(s.P, np_args[0], np_args[1], np_args[2], lv)
            assert_equal(s.host(outs[0].c0), w0, "oracle hmult c0")
            assert_equal(s.host(outs[0].c1), w1, "oracle hmult c1")
        if kind == "hoisted":
            c_np, gs, keys_np = np_args
            w0, w1 = oracle.hoisted_rotate(s.P, c_np, gs, keys_np, lv)
            for i in range(len(gs)):
                assert_equal(s.host(outs[i].c0), w0[i], "oracle hoisted c0")
                assert_equal(s.host(outs[i].c1), w1[i], "oracle hoisted c1")
    b.close()


@pytest.mark.parametrize("name", ["small", "large", "small_shared"])
def test_batch_graph_replays_and_tuning_are_bit_stable(name):
    import torch
    s = setup(params_of(name))
    b, checks = build_batch(s, PLANS[name], 900)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.tune(st)
        b.capture(st)
    torch.cuda.synchronize()
    for rep in range(3):
        for _, _, _, outs, _ in checks:   # clear the outputs so a replay must rewrite them
            for o in outs:
                o.c0.zero_()
                o.c1.zero_()
        torch.cuda.synchronize()
        b.replay(st)
        st.synchronize()
        compare_to_single(s, checks, "replay %d" % rep)   # eager single-op work between replays
        torch.cuda.synchronize()
    b.close()
