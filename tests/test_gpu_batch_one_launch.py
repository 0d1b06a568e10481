"""The one-launch schedule of a batch (ckks_batch_set_schedule): every step of
every key switch in one persistent launch, ordered by dependency counters.
Every item must equal, bit for bit, the single-operation call (and the
oracle on a sample), for several pipeline windows and grid sizes, as an
eager run and as replays of a captured graph; no run may give up waiting."""
import sys

import pytest

from gpu_common import assert_equal, gpu_available
from paper_2507_04775_amd import inputs
from test_gpu_batch import PLANS, build_batch, build_plan_batch, oracle_of, setup, single_op

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _clear(checks):
    for _, _, _, outs, _ in checks:
        for o in outs:
            o.c0.fill_(3)
            o.c1.fill_(3)


def _equal_on_device(s, checks, tag):
    import torch
    for kind, lv, args, outs, _ in checks:
        want = single_op(s, kind, lv, args)
        for o, w in zip(outs, want):
            ok = torch.equal(o.c0, w.c0) and torch.equal(o.c1, w.c1)
            if not ok:  # name the first difference
                assert_equal(s.host(o.c0), s.host(w.c0), "%s %s level %d c0" % (tag, kind, lv))
                assert_equal(s.host(o.c1), s.host(w.c1), "%s %s level %d c1" % (tag, kind, lv))


@pytest.mark.parametrize("window,wg", [(1, 2), (2, 2), (64, 2), (1, 1)])
def test_one_launch_mixed_batch_equals_single_ops(window, wg):
    import torch
    s = setup("large")
    b, checks = build_batch(s, PLANS["large"], 700)
    b.set_schedule(window, wg)
    assert b.schedule == window
    _say("one launch: mixed batch, window %d, %d workgroups per CU" % (window, wg))
    _clear(checks)
    torch.cuda.synchronize()
    b.run()
    b.faults()
    _equal_on_device(s, checks, "one launch w%d" % window)
    for kind, lv, args, outs, np_args in checks:
        if kind not in ("hoisted", "hmult") or (kind == "hmult" and lv != min(PLANS["large"]["hmult"])):
            continue
        for i, (w0, w1) in enumerate(oracle_of(s, kind, lv, np_args)):
            assert_equal(s.host(outs[i].c0), w0, "oracle %s level %d c0" % (kind, lv))
            assert_equal(s.host(outs[i].c1), w1, "oracle %s level %d c1" % (kind, lv))
    # back to the per-step launches on the same batch
    b.set_schedule(0, 2)
    _clear(checks)
    b.run()
    b.faults()
    _equal_on_device(s, checks, "per-step launches after one launch")
    b.close()


def test_one_launch_128_items_graph_replays():
    """The bench's 128-item batch at N = 2^16 (levels 4..30, 64 HMult+relin and
    64 hoisted 8-way rotations, 576 key switches) in one launch, captured and
    replayed three times with eager work in between."""
    import torch
    s = setup("large")
    plan = inputs.batch_plan(inputs.BASE_SEED + 1 + 500, 128, s.ps.logn, s.ps.L)
    b, checks = build_plan_batch(s, plan, 1500)
    b.set_schedule(8, 2)
    st = torch.cuda.Stream()
    _say("one launch: 128 items, capture")
    with torch.cuda.stream(st):
        b.capture(st)
    for rep in range(3):
        _clear(checks)
        torch.cuda.synchronize()
        b.replay(st)
        b.faults(st)
        _say("one launch: 128 items, replay %d done" % rep)
        _equal_on_device(s, checks, "128-item one-launch replay %d" % rep)
        torch.cuda.synchronize()
    done = set()
    for kind, lv, args, outs, np_args in checks:
        if kind in done:
            continue
        done.add(kind)
        for i, (w0, w1) in enumerate(oracle_of(s, kind, lv, np_args)):
            assert_equal(s.host(outs[i].c0), w0, "oracle 128-item %s level %d c0" % (kind, lv))
            assert_equal(s.host(outs[i].c1), w1, "oracle 128-item %s level %d c1" % (kind, lv))
    b.close()


def test_one_launch_rejections():
    """Host-side refusals: N = 2^12, a grid above the kernel's occupancy, a
    replay after a schedule change dropped the captured graph."""
    import torch
    from paper_2507_04775_amd import ckks
    small = setup("small")
    b, _ = build_batch(small, PLANS["small"], 710)
    with pytest.raises(ckks.CkksError, match="N = 2\\^16"):
        b.set_schedule(4, 2)
    b.set_schedule(0, 2)  # per-step launches stay available
    b.close()
    s = setup("large")
    b, _ = build_batch(s, PLANS["large"], 720)
    with pytest.raises(ckks.CkksError, match="workgroups per CU"):
        b.set_schedule(4, 3)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.capture(st)
        b.set_schedule(4, 2)  # drops the graph of the per-step launches
        with pytest.raises(ckks.CkksError, match="nothing captured"):
            b.replay(st)
    b.close()
