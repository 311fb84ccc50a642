"""The batched autotuner's choice and its JSON cache (host logic, no GPU): the fastest
candidate wins, a repeated tuning problem is answered from the cache without timing,
and the key separates precisions, overlaps, candidate lists, instance-size mixes and
subdomain solvers."""
import json

import numpy as np

from paper_2007_04560_amd.batch import autotune, tune_key


def _fields(sizes):
    return [(np.zeros((n, n)), np.zeros((n, n))) for n in sizes]


class FakeTimer:
    def __init__(self, table):
        self.table = table
        self.calls = []

    def __call__(self, fields, params, box, steps, **common):
        self.calls.append((box, common.get("precision", "fp64"), common.get("overlap")))
        return self.table[(box, common.get("precision", "fp64"))]


TABLE = {(32, "fp64"): 0.30, (48, "fp64"): 0.20, (64, "fp64"): 0.25,
         (32, "mixed"): 0.21, (48, "mixed"): 0.24, (64, "mixed"): 0.22}


def test_fastest_candidate_is_kept_and_cached(tmp_path):
    cache = str(tmp_path / "tune.json")
    fields = _fields([96, 128, 128, 256])
    timer = FakeTimer(TABLE)
    best, t = autotune(fields, [{}] * 4, boxes=(32, 48, 64), cache=cache, timer=timer, overlap=2, precision="fp64")
    assert best == 48 and t == {32: 0.30, 48: 0.20, 64: 0.25}
    assert len(timer.calls) == 3
    # the same problem again: answered from the file, nothing timed
    best2, t2 = autotune(fields, [{}] * 4, boxes=(32, 48, 64), cache=cache, timer=timer, overlap=2,
                         precision="fp64")
    assert (best2, t2) == (best, t) and len(timer.calls) == 3
    # another precision is another problem
    best3, _ = autotune(fields, [{}] * 4, boxes=(32, 48, 64), cache=cache, timer=timer, overlap=2,
                        precision="mixed")
    assert best3 == 32 and len(timer.calls) == 6
    data = json.load(open(cache))
    assert len(data) == 2 and {v["box"] for v in data.values()} == {48, 32}


def test_key_depends_on_the_problem_only():
    base = tune_key([(128, 128), (96, 96), (128, 128)], "fp64", 2, (32, 48))
    assert base == tune_key([(96, 96), (128, 128), (128, 128)], "fp64", 2, (32, 48))   # order of instances
    for other in (tune_key([(128, 128), (96, 96)], "fp64", 2, (32, 48)),
                  tune_key([(128, 128), (96, 96), (128, 128)], "mixed", 2, (32, 48)),
                  tune_key([(128, 128), (96, 96), (128, 128)], "fp64", 1, (32, 48)),
                  tune_key([(128, 128), (96, 96), (128, 128)], "fp64", 2, (32, 48, 64)),
                  tune_key([(128, 128), (96, 96), (128, 128)], "fp64", 2, (32, 48), ("iluk_box", 0, 0.0)),
                  tune_key([(128, 128), (96, 96), (128, 128)], "fp64", 2, (32, 48), ("ilu0", 0, 0.02))):
        assert other != base


def test_subdomain_solver_is_another_problem(tmp_path):
    """A width tuned for the stencil-pattern ILU(0) is not reused for the box pattern."""
    cache = str(tmp_path / "tune.json")
    fields = _fields([96, 128])
    timer = FakeTimer(TABLE)
    autotune(fields, [{}] * 2, boxes=(32, 48), cache=cache, timer=timer, overlap=2, ilu_shift=0.02)
    autotune(fields, [{}] * 2, boxes=(32, 48), cache=cache, timer=timer, overlap=2, subsolver="iluk_box",
             fill_level=0, ilu_shift=0.0)
    assert len(timer.calls) == 4 and len(json.load(open(cache))) == 2


def test_unreadable_cache_is_retuned_and_rewritten(tmp_path):
    cache = tmp_path / "tune.json"
    cache.write_text("{not json")
    timer = FakeTimer(TABLE)
    best, _ = autotune(_fields([96]), [{}], boxes=(32, 64), cache=str(cache), timer=timer, overlap=2)
    assert best == 64 and len(timer.calls) == 2
    assert list(json.load(open(cache)).values())[0]["box"] == 64
