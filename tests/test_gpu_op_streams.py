"""Key-switching operations in stream order, bit-exact against the oracle:
chains enqueued without a host synchronisation in between, several caller
streams at once, and graph capture replayed several times with eager calls
between the replays.  N = 2^16, the `large` set (31 limbs, K = 4, dnum = 3)."""
import pytest

import oracle
from gpu_common import Setup, assert_equal, gpu_available
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

_s = {}


def setup():
    if "large" not in _s:
        _s["large"] = Setup("large")
    return _s["large"]


def _check_ct(s, out, want, what):
    assert_equal(s.host(out.c0), want[0], what + " c0")
    assert_equal(s.host(out.c1), want[1], what + " c1")


def test_chain_without_host_sync():
    """HMult -> rotation -> HSquare -> key switch of c1, each reading the
    previous output, all enqueued before one synchronisation."""
    s = setup()
    level = 30
    rk, rkh = s.key(8, 0)
    g = oracle.galois_for_rotation(s.ps.logn, 5)
    gk, gkh = s.key(9, g)
    a, ta = s.ct(200, level)
    b, tb = s.ct(201, level)
    m = s.ctx.empty_ct(level)
    r = s.ctx.empty_ct(level)
    q = s.ctx.empty_ct(level)
    o0, o1 = s.ctx.empty_poly(level), s.ctx.empty_poly(level)
    s.ctx.ckks_hmult_relin(ta, tb, rkh, m)
    s.ctx.ckks_hrotate(m, 5, gkh, r)
    s.ctx.ckks_hsquare(r, rkh, q)
    s.ctx.ckks_keyswitch(q.c1, level, rkh, o0, o1)
    wm = oracle.hmult_relin(s.P, a, b, rk, level)
    wr = oracle.apply_galois(s.P, wm, g, gk, level)
    wq = oracle.hmult_relin(s.P, wr, wr, rk, level)
    wk = oracle.keyswitch(s.P, wq[1], rk, level)
    _check_ct(s, m, wm, "chain hmult")
    _check_ct(s, r, wr, "chain rotate")
    _check_ct(s, q, wq, "chain hsquare")
    assert_equal(s.host(o0), wk[0], "chain ks0")
    assert_equal(s.host(o1), wk[1], "chain ks1")


def test_two_caller_streams():
    """HMults on one stream and rotations on another, interleaved from one
    host thread, each stream with its own workspace."""
    import torch
    s = setup()
    level = 30
    rk, rkh = s.key(10, 0)
    g = oracle.galois_for_rotation(s.ps.logn, 1)
    gk, gkh = s.key(11, g)
    a, ta = s.ct(210, level)
    b, tb = s.ct(211, level)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ws1 = torch.empty(s.ctx.workspace_bytes(s.ckks.OP_HMULT, level) // 8 + 1, dtype=torch.uint64, device="cuda")
    ws2 = torch.empty(s.ctx.workspace_bytes(s.ckks.OP_ROTATE, level) // 8 + 1, dtype=torch.uint64, device="cuda")
    outs1 = [s.ctx.empty_ct(level) for _ in range(3)]
    outs2 = [s.ctx.empty_ct(level) for _ in range(3)]
    torch.cuda.synchronize()
    for i in range(3):
        s.ctx.ckks_hmult_relin(ta, tb, rkh, outs1[i], ws1, s1)
        s.ctx.ckks_hrotate(ta, 1, gkh, outs2[i], ws2, s2)
    torch.cuda.synchronize()
    wm = oracle.hmult_relin(s.P, a, b, rk, level)
    wr = oracle.apply_galois(s.P, a, g, gk, level)
    for i in range(3):
        _check_ct(s, outs1[i], wm, "stream 1 hmult %d" % i)
        _check_ct(s, outs2[i], wr, "stream 2 rotate %d" % i)


def test_graph_capture_replays():
    """An HMult captured into a graph and replayed three times, with eager
    HMults on the same inputs between the replays."""
    import torch
    s = setup()
    level = 12
    rk, rkh = s.key(12, 0)
    a, ta = s.ct(220, level)
    b, tb = s.ct(221, level)
    want = oracle.hmult_relin(s.P, a, b, rk, level)
    ws = torch.empty(s.ctx.workspace_bytes(s.ckks.OP_HMULT, level) // 8 + 1, dtype=torch.uint64, device="cuda")
    gout = s.ctx.empty_ct(level)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        s.ctx.ckks_hmult_relin(ta, tb, rkh, gout, ws, st)  # eager warm-up on the capture stream
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        s.ctx.ckks_hmult_relin(ta, tb, rkh, gout, ws, st)
    for rep in range(3):
        gout.c0.zero_()
        gout.c1.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _check_ct(s, gout, want, "graph replay %d" % rep)
        eager = s.ctx.empty_ct(level)
        s.ctx.ckks_hmult_relin(ta, tb, rkh, eager)
        _check_ct(s, eager, want, "eager between replays %d" % rep)
    del graph
