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
