"""The autotuner's shape classes and its JSON cache (host logic, no device)."""
import json

import paper_1201_2222_amd as rt
from paper_1201_2222_amd import tuning


def test_shape_class_rounds_to_powers_of_two():
    a = tuning.shape_class(rt.make_desc((100, 120, 128), nf=3, n_mu=6, precision=rt.RT_F32))
    b = tuning.shape_class(rt.make_desc((128, 65, 97), nf=4, n_mu=6, precision=rt.RT_F32))
    assert a == b == "p1-o0-R6-nf4-128x128x128"
    assert tuning.shape_class(rt.make_desc((128, 128, 128), n_mu=8)) != a


def test_cache_round_trip_and_lookup(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tuning.load_cache(path) == {}
    tuning.store("k1", {"waves": 3, "ms": {"3": 1.5}}, path)
    tuning.store("k2", {"waves": 6, "ms": {}}, path)
    data = json.load(open(path))
    assert data["k1"]["waves"] == 3 and data["k2"]["waves"] == 6

    class Fake:
        desc = rt.make_desc((32, 32, 32), n_mu=4)

        def __init__(self):
            self.waves = None

        def set_waves(self, w):
            self.waves = w

        def tune(self, S, reps=3, stream=None):
            return 2, {1: 3.0, 2: 1.0, 3: 2.0}

    p = Fake()
    e = tuning.autotune(p, None, path)             # tuned, then recorded
    assert e["waves"] == 2 and p.waves is None
    q = Fake()
    e2 = tuning.autotune(q, None, path)            # looked up
    assert e2["waves"] == 2 and q.waves == 2
    assert tuning.shape_class(Fake.desc) in json.load(open(path))


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tuning.load_cache(str(path)) == {}
