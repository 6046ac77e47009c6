"""Host logic of the tuning cache: bucketing, reuse and the JSON round trip
(a stand-in planner records the calls; no device)."""
import json

from paper_1904_01567_amd.tuning import TuningCache, family


class FakePlanner:
    def __init__(self, K, M, max_plans=1000):
        self.K, self.M, self.max_plans = K, M, max_plans
        self.calls = []
        self._t = {}

    def autotune(self, dtype=None, reps=5):
        self.calls.append(("autotune", dtype))
        self._t[dtype] = {"split": 24, "tuned": 1, "lp_shape": 1, "xcd_map": 0}
        return 24, 100.0

    def set_tuning(self, split, lp_shape=0, xcd_map=1, dtype=None):
        self.calls.append(("set", dtype, split, lp_shape, xcd_map))
        self._t[dtype] = {"split": split, "tuned": 1, "lp_shape": lp_shape, "xcd_map": xcd_map}

    def tuning(self, dtype=None):
        return dict(self._t[dtype])


def test_buckets_reuse_and_round_trip(tmp_path):
    path = str(tmp_path / "tuning.json")
    cache = TuningCache(path, point_bucket=4000)
    a = FakePlanner(360, 20000)
    b = FakePlanner(352, 21500)   # Kp 352 differs from 384: own bucket
    c = FakePlanner(370, 21000)   # Kp 384, 21,000 points -> the 20,000 bucket of a
    assert cache.key(a, "f32acc64") == "f32acc64:Kp384:M20000:Pp1024"
    assert cache.key(c, "f32acc64") == cache.key(a, "f32acc64")
    assert cache.key(b, "f32acc64") != cache.key(a, "f32acc64")
    assert cache.key(a, "bf16") == cache.key(a, "fp8")  # one kernel family
    assert family("f32chunk64") == family("f32") != family("f32acc64")
    cache.tune(a, "f32acc64")
    cache.tune(c, "f32acc64")
    assert a.calls == [("autotune", "f32acc64")]
    assert c.calls == [("set", "f32acc64", 24, 1, 0)]
    assert (cache.hits, cache.misses) == (1, 1)
    cache.save()
    with open(path) as fh:
        assert json.load(fh)["entries"]["f32acc64:Kp384:M20000:Pp1024"]["split"] == 24
    again = TuningCache(path, point_bucket=4000)
    d = FakePlanner(360, 19000)
    again.tune(d, "f32acc64")
    assert d.calls == [("set", "f32acc64", 24, 1, 0)]
    # another bucket width does not reuse the file's entries
    assert TuningCache(path, point_bucket=2000).entries == {}
