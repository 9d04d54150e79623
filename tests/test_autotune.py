"""Host logic of the autotuner: graph classes, size buckets, lookup of the
nearest stored entry and overlaying tuned knobs on the paper defaults."""
import json
import types

import paper_1701_01170_amd.autotune as at


def fake(V, E, maxdeg):
    return types.SimpleNamespace(n_vertices=V, n_edges=E, max_degree=maxdeg)


def test_graph_class_and_bucket():
    assert at.graph_class(fake(1 << 22, 128_000_000, 163_000)) == "scalefree"
    assert at.graph_class(fake(1 << 22, 16_769_024, 4)) == "mesh"
    assert at.size_bucket(fake(10, 1 << 20, 5)) == 20
    assert at.size_bucket(fake(10, 3 << 20, 5)) == 22  # log2(3 Mi) = 21.58 rounds to 22


def test_lookup_nearest_bucket(tmp_path, monkeypatch):
    monkeypatch.setattr(at, "TUNING_DIR", str(tmp_path))
    db = {"arch": "gfx950", "entries": [
        {"class": "scalefree", "kind": "bfs", "log2_edges": 19, "opts": {"lb_chunk": 2048}},
        {"class": "scalefree", "kind": "bfs", "log2_edges": 27, "opts": {"lb_chunk": 8192}},
        {"class": "mesh", "kind": "bfs", "log2_edges": 24, "opts": {"lb_chunk": 4096}},
    ]}
    (tmp_path / "gfx950.json").write_text(json.dumps(db))
    g = fake(1 << 22, 100_000_000, 100_000)  # scalefree, bucket 27
    assert at.lookup(g, "bfs") == {"lb_chunk": 8192}
    assert at.lookup(fake(1 << 14, 400_000, 3000), "bfs") == {"lb_chunk": 2048}
    assert at.lookup(g, "sssp") is None
    assert at.lookup(fake(1 << 22, 16_000_000, 4), "bfs") == {"lb_chunk": 4096}


def test_tuner_sweeps_every_launch_knob(monkeypatch):
    """The coordinate search visits the workgroup size, both TWC tier cut-offs
    (on a graph that expands with TWC) and the BFS filter, and never asks for
    a tier split the library rejects (block tier below the wave tier)."""
    seen = []

    def fake_time(g, kind, sources, knobs, reps=1):
        seen.append(dict(knobs))
        w, b = knobs.get("twc_wave_min", 0), knobs.get("twc_block_min", 0)
        assert not (w > 0 and b > 0 and b < w)
        return 1.0 + 0.01 * (knobs.get("adv_block") == 512) - 0.5 * (knobs.get("twc_wave_min") == 32)

    monkeypatch.setattr(at, "_time", fake_time)
    g = fake(1 << 20, 4 << 20, 4)  # average degree 4: below the LB cut of 5, so TWC
    best, best_ms, base = at.tune(g, "bfs", [0], log=lambda m: None)
    keys = {k for kn in seen for k, v in kn.items() if v}
    assert {"adv_block", "twc_wave_min", "twc_block_min", "bfs_filter"} <= keys
    assert {kn.get("adv_block") for kn in seen} >= {128, 256, 512}
    assert best["twc_wave_min"] == 32 and best_ms == 0.5
    assert set(best) == set(at.KNOBS)


def test_tuner_starts_from_the_stored_setting(monkeypatch):
    """A combination that no single knob change from the defaults reaches (here
    two knobs that only pay together) is kept when it is the stored setting."""
    def fake_time(g, kind, sources, knobs, reps=1):
        both = knobs.get("lb_chunk") == 4096 and knobs.get("adv_block") == 256
        return 0.4 if both else 1.0

    stored = {"lb_chunk": 4096, "adv_block": 256}
    monkeypatch.setattr(at, "_time", fake_time)
    monkeypatch.setattr(at, "lookup", lambda g, kind, arch=at.ARCH: dict(stored))
    g = fake(1 << 20, 16 << 20, 4)
    best, best_ms, base = at.tune(g, "bfs_multi", [0], log=lambda m: None)
    assert best_ms == 0.4 and base == 1.0
    assert best["lb_chunk"] == 4096 and best["adv_block"] == 256
