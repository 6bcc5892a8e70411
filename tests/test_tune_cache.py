"""Host logic of the autotuner's cache lookup (no GPU)."""
import json

from paper_0809_2811_amd import tune


def test_best_reads_winner_and_per_skin_lanes(tmp_path, monkeypatch):
    cache = {"gfx950/n12_rho1.00": {
        "best": {"lanes_per_atom": 32, "skin": 1.0, "persistent": 0, "graph_steps": 50},
        "by_skin": {"0.50": {"lanes_per_atom": 16, "s_per_step": 1e-5},
                    "1.00": {"lanes_per_atom": 32, "s_per_step": 9e-6}},
        "s_per_step": 9e-6}}
    path = tmp_path / "cache.json"
    path.write_text(json.dumps(cache))
    monkeypatch.setattr(tune, "CACHE", path)
    free = tune.best(4096, 1.0, None)
    assert free["lanes_per_atom"] == 32 and free["skin"] == 1.0 and free["graph_steps"] == 50
    same = tune.best(4096, 1.0, 1.0)
    assert same["lanes_per_atom"] == 32 and "skin" not in same and same["graph_steps"] == 50
    other = tune.best(4096, 1.0, 0.5)          # the lanes measured at that skin, the winner's launch form
    assert other["lanes_per_atom"] == 16 and other["graph_steps"] == 50 and "skin" not in other
    unknown = tune.best(4096, 1.0, 0.7)        # no per-skin record: the winner's lanes
    assert unknown["lanes_per_atom"] == 32
    missing = tune.best(1 << 20, 1.0, None)    # no entry: defaults
    assert missing == tune.DEFAULT


def test_bucket_names():
    assert tune.bucket(4096, 1.0) == "n12_rho1.00"
    assert tune.bucket(262144, 0.95) == "n18_rho0.95"
    assert tune.bucket(5000, 1.0) == "n12_rho1.00"
