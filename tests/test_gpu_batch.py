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
        checks.append(("rot", lv, (c, g, key), [out], (c_np, key_np, g)))
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
    # the oracle on every item of the N = 2^12 plans; at N = 2^16 on the lowest HMult and the hoisted items
    every = params_of(name) == "small"
    for kind, lv, args, outs, np_args in checks:
        if not every and not (kind == "hoisted" or (kind == "hmult" and lv == min(PLANS[name]["hmult"]))):
            continue
        for i, (w0, w1) in enumerate(oracle_of(s, kind, lv, np_args)):
            assert_equal(s.host(outs[i].c0), w0, "oracle %s level %d c0" % (kind, lv))
            assert_equal(s.host(outs[i].c1), w1, "oracle %s level %d c1" % (kind, lv))
    b.close()


def oracle_of(s, kind, lv, np_args):
    """The oracle's results [(c0, c1), ...] for one batch item."""
    if kind == "hmult":
        return [oracle.hmult_relin(s.P, np_args[0], np_args[1], np_args[2], lv)]
    if kind == "ks":
        return [oracle.keyswitch(s.P, np_args[0], np_args[1], lv)]
    if kind == "rot":
        c_np, key_np, g = np_args
        return [oracle.apply_galois(s.P, c_np, g, key_np, lv)]
    c_np, gs, keys_np = np_args
    w0, w1 = oracle.hoisted_rotate(s.P, c_np, gs, keys_np, lv)
    return [(w0[i], w1[i]) for i in range(len(gs))]


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


def build_plan_batch(s, plan, seed):
    """A batch of the bench's kind (inputs.batch_plan: HMult+relin items and
    hoisted 8-way rotations at mixed levels) with uniform keys."""
    b = s.ckks.Batch(s.ctx)
    rlk_np, rlk = s.key(seed, 0)
    keys = {}
    checks = []
    for i, (kind, lv, ks) in enumerate(plan):
        c_np, c = s.ct(seed + 10 + 3 * i, lv)
        if kind == "hmult":
            d_np, d = s.ct(seed + 11 + 3 * i, lv)
            out = s.ctx.empty_ct(lv)
            b.hmult(c, d, rlk, out)
            checks.append(("hmult", lv, (c, d, rlk), [out], (c_np, d_np, rlk_np)))
        else:
            gs = [oracle.galois_for_rotation(s.ps.logn, k) for k in ks]
            for k, g in zip(ks, gs):
                if k not in keys:
                    keys[k] = s.key(seed + 1000 + k, g)
            outs = [s.ctx.empty_ct(lv) for _ in ks]
            b.hoisted(c, ks, [keys[k][1] for k in ks], outs)
            checks.append(("hoisted", lv, (c, ks, [keys[k][1] for k in ks]), outs, (c_np, gs, [keys[k][0] for k in ks])))
    b.build()
    return b, checks


def test_bench_kind_plan_every_item_against_oracle():
    """The bench's batch shape at N = 2^12 (20 levels, 16 items, levels 4..20):
    every item against the oracle, and the persistent-kernel run against the
    single-operation calls."""
    s = setup("boot-small")
    plan = inputs.batch_plan(inputs.BASE_SEED + 77, 16, s.ps.logn, s.ps.L)
    b, checks = build_plan_batch(s, plan, 1300)
    b.run()
    compare_to_single(s, checks, "plan batch")
    for kind, lv, args, outs, np_args in checks:
        for i, (w0, w1) in enumerate(oracle_of(s, kind, lv, np_args)):
            assert_equal(s.host(outs[i].c0), w0, "oracle plan %s level %d c0" % (kind, lv))
            assert_equal(s.host(outs[i].c1), w1, "oracle plan %s level %d c1" % (kind, lv))
    b.close()


def test_bench_batch_128_items_equals_single_ops():
    """The bench's own 128-item batch at N = 2^16 (levels 4..30, 64 HMult+relin
    and 64 hoisted 8-way rotations): the graph replay equals the single-operation
    calls on every item, and the oracle on one item of each kind."""
    import torch
    s = setup("large")
    plan = inputs.batch_plan(inputs.BASE_SEED + 1 + 500, 128, s.ps.logn, s.ps.L)
    b, checks = build_plan_batch(s, plan, 1500)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.capture(st)
        b.replay(st)
    st.synchronize()
    compare_to_single(s, checks, "128-item batch")
    done = set()
    for kind, lv, args, outs, np_args in checks:
        if kind in done:
            continue
        done.add(kind)
        for i, (w0, w1) in enumerate(oracle_of(s, kind, lv, np_args)):
            assert_equal(s.host(outs[i].c0), w0, "oracle 128-item %s level %d c0" % (kind, lv))
            assert_equal(s.host(outs[i].c1), w1, "oracle 128-item %s level %d c1" % (kind, lv))
    b.close()
