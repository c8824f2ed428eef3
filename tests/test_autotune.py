"""The autotuners' selection and cache logic on the host, with a stand-in
context whose timings are fixed (no device): the fastest candidate wins, it
is set on the context, it is cached under the workload's key, and a second
call takes it from the cache without timing anything."""
import numpy as np
import pytest

from paper_1811_10270_amd import autotune
from paper_1811_10270_amd import ehdbim as E


class FakeCtx:
    device = 0
    ntargets = 1000

    def __init__(self, self_ms, far_ms):
        self.self_ms, self.far_ms = self_ms, far_ms
        self.self_set, self.far_set, self.timed = {}, None, 0

    def time_self(self, cls, pf, f, sg, reps):
        self.timed += 1
        return self.self_ms[(cls, pf)]

    def set_self_config(self, cls, pf):
        self.self_set[cls] = pf

    def time_far(self, prec, tpt, nch, reps, kinds=31):
        self.timed += 1
        return self.far_ms[(tpt, nch)]

    def set_far_config(self, tpt, nch):
        self.far_set = (tpt, nch)


@pytest.fixture
def keys(monkeypatch):
    E.load()
    monkeypatch.setattr(autotune, "self_signature", lambda ctx, cls, pq, gm: f"self|{cls}|{sorted(set(pq))}|{gm}")
    monkeypatch.setattr(autotune, "signature",
                        lambda ctx, p, q, gm, prec, kinds: f"far|{list(p)}|{list(q)}|{gm}|{prec}|{kinds}")


def test_self_autotuner_picks_caches_and_reuses(keys, tmp_path):
    p = np.array([16, 32, 32, 16])            # classes 0 and 2 only
    q = 2 * p
    ms = {}
    for cls in range(4):
        for k, pf in enumerate(E.self_config_candidates(cls)):
            ms[(cls, pf)] = 10.0 + cls + (0.5 if k != 1 else 0.0)   # the second candidate is fastest
    ctx = FakeCtx(ms, {})
    cache = str(tmp_path / "tune.json")
    best, timings, cached = autotune.autotune_self(ctx, p, q, 0, None, None, reps=3, cache_path=cache)
    assert not cached
    assert sorted(best) == [16, 32]
    for cls, pm in ((0, 16), (2, 32)):
        want = E.self_config_candidates(cls)[1]
        assert best[pm] == want and ctx.self_set[cls] == want
        assert set(timings[pm]) == {str(v) for v in E.self_config_candidates(cls)}
    assert ctx.timed == 2 * 3 * 3                # two classes, three candidates, three timings each (short)
    ctx2 = FakeCtx({}, {})                      # any timing call would raise KeyError
    best2, _, cached2 = autotune.autotune_self(ctx2, p, q, 0, None, None, cache_path=cache)
    assert cached2 and best2 == best and ctx2.timed == 0
    assert ctx2.self_set == {0: best[16], 2: best[32]}


def test_far_autotuner_picks_caches_and_reuses(keys, tmp_path):
    far = {(t, c): 50.0 + t + c for t in autotune.TPT_CANDIDATES for c in autotune.CHUNK_CANDIDATES}
    far[(2, 4)] = 10.0
    ctx = FakeCtx({}, far)
    cache = str(tmp_path / "tune.json")
    tpt, nch, timings, cached = autotune.autotune_far(ctx, [32, 32], [64, 64], 0, 0, kinds=15, cache_path=cache)
    assert (tpt, nch) == (2, 4) and ctx.far_set == (2, 4) and not cached
    assert len(timings) == len(autotune.TPT_CANDIDATES) * len(autotune.CHUNK_CANDIDATES)
    ctx2 = FakeCtx({}, {})
    tpt2, nch2, _, cached2 = autotune.autotune_far(ctx2, [32, 32], [64, 64], 0, 0, kinds=15, cache_path=cache)
    assert cached2 and (tpt2, nch2) == (2, 4) and ctx2.timed == 0 and ctx2.far_set == (2, 4)
    # another kinds mask is another key: timed again
    ctx3 = FakeCtx({}, far)
    _, _, _, cached3 = autotune.autotune_far(ctx3, [32, 32], [64, 64], 0, 0, kinds=31, cache_path=cache)
    assert not cached3 and ctx3.timed > 0
