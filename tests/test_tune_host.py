"""Host logic of the autotuner's cache: keys name (logN, limbs, K, op, arch),
the cache survives a save / load round trip, and a cached batch grid is
applied without measuring.  No GPU."""
import os

from paper_2507_04775_amd import tune


def test_cache_key_names_every_field():
    k = tune._key(16, 35, 4, "ntt_fwd", "gfx950")
    for part in ("logN=16", "limbs=35", "K=4", "op=ntt_fwd", "arch=gfx950"):
        assert part in k
    assert tune._key(16, 35, 4, "ntt_fwd", "gfx950") != tune._key(16, 35, 10, "ntt_fwd", "gfx950")


def test_cache_round_trip(tmp_path, monkeypatch):
    path = os.path.join(str(tmp_path), "sub", "tune.json")
    monkeypatch.setenv(tune.CACHE_ENV, path)
    assert tune.cache_path() == path
    assert tune.load_cache() == {}
    c = {tune._key(16, 8, 4, "ntt_inv", "gfx950"): {"tile": 4, "us": {"16": 9.1, "8": 6.0, "4": 5.2}}}
    tune.save_cache(c)
    assert tune.load_cache() == c


class _FakeBatch:
    def __init__(self):
        self.grids = {}
        self.tuned = False

    def set_grid(self, step, g):
        self.grids[step] = g

    def tune(self, stream):
        self.tuned = True


class _Ctx:
    logn, nq, np = 16, 31, 4


def test_cached_batch_grid_is_applied_without_measuring(monkeypatch):
    monkeypatch.setattr(tune, "arch", lambda: "gfx950")
    sig = tune.batch_signature([("hmult", 30), ("hoisted", 12)])
    cache = {tune._key(16, 31, 4, sig, "gfx950"): {"grid": [3, 2, 4]}}
    b = _FakeBatch()
    assert tune.tune_batch(b, _Ctx(), sig, None, cache) == [3, 2, 4]
    assert b.grids == {0: 3, 1: 2, 2: 4} and not b.tuned


class _FakeSchedBatch:
    def __init__(self):
        self.set = None

    def set_schedule(self, window, wg):
        self.set = (window, wg)

    def run(self, stream=None):
        raise AssertionError("a cached schedule must not be measured")


def test_schedule_candidates_cover_steps_and_windows():
    c = tune.schedule_candidates(128, 16)
    assert c[0] == (0, 2) and (1, 2) in c and (128, 2) in c and (8, 1) in c
    windows = [w for w, g in c if g == 2 and w]
    assert windows == sorted(windows) and all(w & (w - 1) == 0 for w in windows[:-1])
    assert tune.schedule_candidates(16, 12) == [(0, 2)]  # one launch is N = 2^16 only


def test_cached_schedule_is_applied_without_measuring(monkeypatch):
    monkeypatch.setattr(tune, "arch", lambda: "gfx950")
    sig = tune.batch_signature([("hmult", 30), ("hoisted", 12)])
    cache = {tune._key(16, 31, 4, "schedule:" + sig, "gfx950"): {"window": 8, "wg": 2, "ms": {}}}
    b = _FakeSchedBatch()
    assert tune.tune_batch_schedule(b, _Ctx(), sig, 2, None, cache)["window"] == 8
    assert b.set == (8, 2)
