"""Host logic of the launch-shape autotuner: candidate set and the JSON cache."""
import json

from paper_1311_5551_amd import autotune


def test_candidates_are_the_supported_shapes():
    assert set(autotune.CANDIDATES) == {(b, p) for b in (64, 128, 256) for p in (1, 2, 4, 8, 16)}


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    key = autotune.cache_key("gfx950", 0, 1, 1, 97_000_000)
    assert key.endswith("2^26")
    assert autotune.cache_load(path, key) is None
    res = {"lepton": {"block": 256, "ppt": 4, "ns_per_million_particle_steps": 30.0},
           "photon": {"block": 256, "ppt": 8, "ns_per_million_particle_steps": 6.4}, "trials": [1, 2]}
    autotune.cache_store(path, key, res)
    got = autotune.cache_load(path, key)
    assert got == {k: v for k, v in res.items() if k != "trials"}
    autotune.cache_store(path, "other", res)
    assert set(json.load(open(path))) == {key, "other"}


def test_combine_sums_per_particle_times():
    r1 = {"trials": [], "times": {"lepton": {"256/1": 1.0, "256/4": 3.0}, "photon": {"256/1": 10.0, "256/8": 11.0}}}
    r2 = {"trials": [], "times": {"lepton": {"256/1": 5.0, "256/4": 1.5}, "photon": {"256/1": 9.0, "256/8": 6.0}}}
    c = autotune.combine([r1, r2], weighted=False)
    assert (c["lepton"]["block"], c["lepton"]["ppt"]) == (256, 4)
    assert (c["photon"]["block"], c["photon"]["ppt"]) == (256, 8)
    assert c["photon"]["score"] == 17.0
    empty = {"trials": [], "times": {"lepton": {}, "photon": {}}}
    assert autotune.combine([empty])["photon"] is None


def test_combine_weights_points_by_population():
    # per-particle times favour 256/1 at a small point, 256/4 at a large one: the large point decides
    r1 = {"trials": [], "times": {"lepton": {"256/1": 1.0, "256/4": 2.0}, "photon": {}},
          "particles_per_step": {"lepton": 1e4, "photon": 0}}
    r2 = {"trials": [], "times": {"lepton": {"256/1": 3.0, "256/4": 2.5}, "photon": {}},
          "particles_per_step": {"lepton": 1e6, "photon": 0}}
    c = autotune.combine([r1, r2])
    assert (c["lepton"]["block"], c["lepton"]["ppt"]) == (256, 4)
    assert autotune.combine([r1, r2], weighted=False)["lepton"]["ppt"] == 1
    assert c["photon"] is None
