"""Autotuner logic on the CPU with a scripted runner: the fastest candidate
with identical output wins, candidates with different output or invalid
parameters are skipped, stages compose, and the cache round-trips."""
import json

from paper_1310_7556_amd import tune


class ScriptedRunner:
    """time = table[stage][frozen tuning of that stage's fields]; output
    differs for candidates listed in `wrong`; `bad` raise."""

    def __init__(self, times, wrong=(), bad=()):
        self.times, self.wrong, self.bad = times, wrong, bad
        self.calls = []

    def _key(self, stage, tuning):
        fields = {"vote": ("vote_algo", "vote_rows", "vote_threads", "vote_wgs_per_cu"),
                  "peaks": ("peak_rows",), "rz": ("rz_waves_per_cu", "rz_counter_bits")}[stage]
        return tuple((f, tuning[f]) for f in fields if f in tuning)

    def same_output(self, stage, tuning):
        k = self._key(stage, tuning)
        if k in self.bad:
            raise RuntimeError("invalid")
        return k not in self.wrong

    def time_stage(self, stage, tuning, reps):
        self.calls.append((stage, dict(tuning)))
        return self.times[stage].get(self._key(stage, tuning), 10.0)


def stages():
    return (("vote", lambda: [dict(vote_rows=8), dict(vote_rows=16), dict(vote_rows=32)]),
            ("peaks", lambda: [dict(peak_rows=4), dict(peak_rows=8)]),
            ("rz", lambda: [dict(rz_waves_per_cu=8)]))


def test_fastest_valid_candidate_wins_per_stage():
    times = {"vote": {(): 5.0, (("vote_rows", 8),): 4.0, (("vote_rows", 16),): 1.0, (("vote_rows", 32),): 0.5},
             "peaks": {(): 2.0, (("peak_rows", 4),): 3.0, (("peak_rows", 8),): 1.5},
             "rz": {(): 1.0, (("rz_waves_per_cu", 8),): 2.0}}
    r = ScriptedRunner(times, wrong={(("vote_rows", 32),)})
    tuning, report = tune.tune(r, stages=stages(), reps=1)
    assert tuning == dict(vote_rows=16, peak_rows=8)          # 32 is faster but wrong; rz default kept
    assert report["vote"]["rejected"] == [dict(vote_rows=32)]
    assert report["vote"]["best_ms"] == 1.0 and report["rz"]["best"] == {}


def test_later_stages_run_with_earlier_winners():
    times = {"vote": {(("vote_rows", 16),): 1.0}, "peaks": {}, "rz": {}}
    r = ScriptedRunner(times)
    tune.tune(r, stages=stages(), reps=1)
    peak_calls = [t for s, t in r.calls if s == "peaks"]
    assert peak_calls and all(t.get("vote_rows") == 16 for t in peak_calls)


def test_invalid_candidates_are_skipped():
    times = {"vote": {(): 5.0}, "peaks": {}, "rz": {}}
    r = ScriptedRunner(times, bad={(("vote_rows", 8),), (("vote_rows", 16),), (("vote_rows", 32),)})
    tuning, report = tune.tune(r, stages=stages(), reps=1)
    assert "vote_rows" not in tuning and report["vote"]["invalid"] == 3


def test_cache_round_trip_and_key(tmp_path):
    path = str(tmp_path / "cache.json")
    spec = dict(n_phi=512, n_qpt=512, n_layers=10)
    k1 = tune.workload_key(spec, 4096, 4096 * 25000, "gpu")
    k2 = tune.workload_key(dict(reversed(list(spec.items()))), 4096, 4096 * 24000, "gpu")
    assert k1 == k2                                            # same spec, same size bucket
    assert tune.workload_key(spec, 4095, 4096 * 25000, "gpu") != k1
    assert tune.lookup(k1, path) is None
    tune.store(k1, dict(vote_rows=16), dict(note="x"), path)
    tune.store("other", dict(peak_rows=8), {}, path)
    assert tune.lookup(k1, path) == dict(vote_rows=16)
    assert json.load(open(path))["other"]["tuning"] == dict(peak_rows=8)


def test_search_spaces_hold_only_tuning_fields():
    from paper_1310_7556_amd.hough import Tuning
    names = {n for n, _ in Tuning._fields_}
    for _, space in tune.STAGES:
        for cand in space():
            assert set(cand) <= names
