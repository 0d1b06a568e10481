"""ckks_keyswitch_noalloc (the key switch whose workspace is the library's
static device scratch) against ckks_keyswitch with a caller workspace, bit for
bit, on two calls in a row: N = 2^16 at the top level with ten special primes
(the largest workspace the scratch is sized for), then a smaller input at a
lower level, which must not see anything the first call left in the scratch.
The second context (four special primes) shares the same scratch on the GPU.
A level whose workspace exceeds the scratch is refused on the host."""
import sys

import numpy as np
import pytest

from gpu_common import Setup, assert_equal, gpu_available
from paper_2507_04775_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(s, seed, level, key):
    import torch
    d = s.dev(inputs.random_poly(seed, s.ps, level))
    want0, want1 = s.ctx.empty_poly(level), s.ctx.empty_poly(level)
    got0, got1 = s.ctx.empty_poly(level), s.ctx.empty_poly(level)
    got0.fill_(7)
    got1.fill_(7)
    s.ctx.ckks_keyswitch(d, level, key, want0, want1)
    s.ctx.ckks_keyswitch_noalloc(d, level, key, got0, got1)
    torch.cuda.synchronize()
    assert_equal(s.host(got0), s.host(want0), "noalloc out0 at level %d" % level)
    assert_equal(s.host(got1), s.host(want1), "noalloc out1 at level %d" % level)


@pytest.mark.parametrize("name,levels", [("large-nv", [30, 12]), ("large", [30, 4]), ("small", [3, 1])])
def test_keyswitch_noalloc_equals_keyswitch(name, levels):
    from paper_2507_04775_amd import ckks
    s = Setup(name)
    _say("noalloc %s: levels %s, scratch %d bytes" % (name, levels, ckks.noalloc_scratch_bytes()))
    for lv in levels:
        assert s.ctx.workspace_bytes(ckks.OP_KEYSWITCH, lv) <= ckks.noalloc_scratch_bytes()
    _, key = s.key(41, 0)
    for i, lv in enumerate(levels):
        _pair(s, 50 + i, lv, key)
        _say("noalloc %s: level %d bit-exact" % (name, lv))


def test_keyswitch_noalloc_refuses_a_workspace_above_the_scratch():
    """Forty ciphertext limbs at N = 2^16 with sixteen special primes need more
    than the scratch at the top level; the call is refused before any launch
    and a level that fits still runs."""
    import torch
    from paper_2507_04775_amd import ckks
    ps = inputs.make_params(16, 50, 39, 16, 3, 50, "forty-limbs")
    ctx = ckks.Context(ps.logn, ps.q, ps.p, ps.dnum)
    top = ps.L
    assert ctx.workspace_bytes(ckks.OP_KEYSWITCH, top) > ckks.noalloc_scratch_bytes()
    kd = torch.zeros((ps.dnum, 2, len(ps.q) + len(ps.p), ps.N), dtype=torch.uint64, device="cuda")
    key = ctx.key(kd, 0)
    d = torch.zeros((top + 1, 1 << 16), dtype=torch.uint64, device="cuda")
    o0, o1 = torch.empty_like(d), torch.empty_like(d)
    with pytest.raises(ckks.CkksError, match="static scratch"):
        ctx.ckks_keyswitch_noalloc(d, top, key, o0, o1)
    ctx.ckks_keyswitch_noalloc(d[:3], 2, key, o0[:3], o1[:3])
    torch.cuda.synchronize()
    assert int(o0[:3].count_nonzero()) == 0 and int(o1[:3].count_nonzero()) == 0
