"""Host logic of the measurement tooling: the rocprofv3 summaries written to
profiles/ and the kernel-source hash that ties a traffic summary to the
kernels it was measured on (CPU only, synthetic rocpd databases)."""
import json
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1701_01170_amd import rocprof_summary as rs  # noqa: E402

MANGLED_LB = "void gr::(anonymous namespace)::k_push_lb<gr::SsspMark<true>, 4, 1>(int const*)"
MANGLED_LB_F = "void gr::(anonymous namespace)::k_push_lb<gr::SsspMark<false>, 4, 1>(int const*)"
MANGLED_LB_32 = "void gr::(anonymous namespace)::k_push_lb<gr::SsspMark<true>, 32, 1>(int const*)"
COPY = "void gr::(anonymous namespace)::k_copy16(uint4 const*, uint4*, long)"


def _kernels_db(path, rows):
    os.makedirs(path, exist_ok=True)
    c = sqlite3.connect(os.path.join(path, "run_results.db"))
    c.execute("create table kernels (name text, duration integer)")
    c.executemany("insert into kernels values (?, ?)", rows)
    c.commit()
    c.close()


def _counters_db(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    c = sqlite3.connect(os.path.join(path, "run_results.db"))
    c.execute("create table counters_collection "
              "(dispatch_id integer, kernel_name text, counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)",
                  [(i, n, counter, v) for i, (n, v) in enumerate(rows)])
    c.commit()
    c.close()


def test_short_name():
    assert rs.short_name(MANGLED_LB) == "k_push_lb<SsspMark<true>, 4, 1>"
    assert rs.short_name(COPY) == "k_copy16"


def test_stats_counts_durations_and_groups(tmp_path):
    d = str(tmp_path / "stats")
    # durations in ns
    _kernels_db(d, [(MANGLED_LB, 1000), (MANGLED_LB, 3000), (MANGLED_LB_F, 2000),
                    (MANGLED_LB_32, 10000), (COPY, 4000)])
    out = str(tmp_path / "k.md")
    rs.stats(d, out, "cmd", ["tuned=k_push_lb<SsspMark<\\w+>, 4, 1>"])
    text = open(out).read()
    assert "Command: `cmd`" in text
    assert f"Kernel source hash: `{rs.kernel_source_hash()}`" in text
    # 2 calls, 4.0 us total, 2.00 us average, min 1.00, max 3.00, 4 / 20 of all time
    assert "| `k_push_lb<SsspMark<true>, 4, 1>` | 2 | 4.0 | 2.00 | 1.00 | 3.00 | 20.0 |" in text
    # the most expensive kernel is listed first
    body = [l for l in text.splitlines() if l.startswith("| `")]
    assert body[0].startswith("| `k_push_lb<SsspMark<true>, 32, 1>`")
    # the group takes both 4-edge launches of either filter flavour, not the 32-edge one
    assert "| tuned (`k_push_lb<SsspMark<\\w+>, 4, 1>`) | 3 | 6.0 | 2.00 |" in text


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    copy_bytes = 1 << 20  # 1024 KiB read and written per copy launch
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    # FETCH_SIZE reads half the copied bytes (scale 2), WRITE_SIZE all of them (scale 1)
    _counters_db(fd, "FETCH_SIZE", [(COPY, 512.0), (COPY, 512.0), (MANGLED_LB, 100.0),
                                    (MANGLED_LB_F, 300.0), (MANGLED_LB_32, 9999.0)])
    _counters_db(wd, "WRITE_SIZE", [(COPY, 1024.0), (MANGLED_LB, 10.0), (MANGLED_LB_F, 30.0)])
    out = str(tmp_path / "t.json")
    rs.traffic(fd, wd, "k_push_lb<SsspMark<\\w+>, 4, 1>", copy_bytes, out, "cmd")
    j = json.load(open(out))
    assert j["fetch"]["scale"] == pytest.approx(2.0)
    assert j["write"]["scale"] == pytest.approx(1.0)
    assert j["fetch"]["launches"] == 2 and j["write"]["launches"] == 2
    # per launch: fetch 200 KiB x 2 + write 20 KiB x 1 = 420 KiB
    assert j["l2_fabric_bytes_per_launch"] == 420 * 1024
    # unscaled: fetch 200 KiB + write 20 KiB
    assert j["unscaled_bytes_per_launch"] == 220 * 1024
    assert "upper bound" in j["meaning"]
    assert j["kernel_source_hash"] == rs.kernel_source_hash()


def test_traffic_needs_the_copy_kernel(tmp_path):
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    _counters_db(fd, "FETCH_SIZE", [(MANGLED_LB, 100.0)])
    _counters_db(wd, "WRITE_SIZE", [(MANGLED_LB, 10.0)])
    with pytest.raises(RuntimeError):
        rs.traffic(fd, wd, "k_push_lb", 1 << 20, str(tmp_path / "t.json"), "cmd")


def test_kernel_source_hash_tracks_the_sources():
    h = rs.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert rs.kernel_source_hash() == h


def test_committed_traffic_summary_names_its_kernel():
    # the committed summary carries the fields the benchmark reads
    p = os.path.join(ROOT, "profiles", "traffic_k_push_lb_sssp_rmat22.json")
    j = json.load(open(p))
    assert j["l2_fabric_bytes_per_launch"] > 0
    assert len(j["kernel_source_hash"]) == 16
    assert "FETCH_SIZE" in j["command"] and "WRITE_SIZE" in j["command"]


def test_algorithmic_bytes_per_launch():
    import bench
    # SSSP relaxation (any form but the refill): 16 B per edge, 12 B per
    # frontier vertex, 4 B per output vertex
    for k in (0, 1, 2, 6, 8, 9, 10):
        assert bench.algorithmic_bytes("sssp", k, 10, 1000, 7) == 16000 + 120 + 28
    # priority-queue refill: 16 B per far-pile entry read
    assert bench.algorithmic_bytes("sssp", 7, 0, 0, 7, n_in=50) == 800
    # BFS push: 4 B per edge, 12 B per frontier vertex, 12 B per new vertex
    for k in (0, 1, 2, 3, 6):
        assert bench.algorithmic_bytes("bfs", k, 10, 1000, 7) == 4000 + 120 + 84
    # pull over the bitmap: V / 4 bitmap bytes, 8 B per unvisited vertex,
    # 4 B per neighbour scanned, 12 B per vertex found
    for k in (4, 5):
        assert bench.algorithmic_bytes("bfs", k, 10, 1000, 7, n_in=300, inspected=900,
                                       V=4096) == 1024 + 2400 + 3600 + 84
    # pull over the list: 12 B per entry, 4 B per neighbour scanned, 12 B per hit
    assert bench.algorithmic_bytes("bfs", 11, 10, 1000, 7, n_in=300, inspected=900,
                                   V=4096) == 3600 + 3600 + 84
    # every trace kernel code the library documents has a kernel name
    assert {k for (_, k) in bench.KERNEL_NAMES} == set(range(12))


def test_accumulate_and_roofline():
    import bench

    class T:
        def __init__(self, kernel, n_f, m_f, n_next, n_in, inspected, us):
            self.kernel, self.n_f, self.m_f, self.n_next = kernel, n_f, m_f, n_next
            self.n_in, self.inspected, self.kernel_us = n_in, inspected, us

    pk = {}
    buf = [T(2, 10, 1000, 7, 10, 1000, 2.0), T(4, 0, 0, 5, 100, 40, 1.0), T(2, 1, 10, 0, 1, 10, 2.0)]
    tot = bench.accumulate(pk, "bfs", buf, 3, 64)
    assert pk[("bfs", 2)] == [2, 4.0, (4000 + 120 + 84) + (40 + 12)]
    assert pk[("bfs", 4)] == [1, 1.0, 16 + 800 + 160 + 60]
    assert tot == 4204 + 52 + 1036
    r = bench.roofline_of(pk, ("bfs", 2))
    assert r["kernel"] == "k_push_lb<BfsVisit>" and r["launches"] == 2
    assert r["achieved"] == round(4256 / 4e-6 / 1e9, 1) and r["peak"] == 8000.0
    assert r["frac"] == round(4256 / 4e-6 / 1e9 / 8000.0, 4)


def test_counters_averages_and_ratios(tmp_path):
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    os.makedirs(a)
    c = sqlite3.connect(os.path.join(a, "run_results.db"))
    c.execute("create table counters_collection "
              "(dispatch_id integer, kernel_name text, counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", [
        (0, MANGLED_LB, "SQ_WAVE_CYCLES", 100.0), (0, MANGLED_LB, "SQ_WAIT_ANY", 80.0),
        (0, MANGLED_LB, "SQ_WAVES", 4.0),
        (1, MANGLED_LB_F, "SQ_WAVE_CYCLES", 300.0), (1, MANGLED_LB_F, "SQ_WAIT_ANY", 280.0),
        (1, MANGLED_LB_F, "SQ_WAVES", 4.0),
        (2, COPY, "SQ_WAVE_CYCLES", 5.0), (2, COPY, "SQ_WAIT_ANY", 0.0), (2, COPY, "SQ_WAVES", 1.0)])
    c.commit()
    c.close()
    _counters_db(b, "TCC_HIT_sum", [(MANGLED_LB, 30.0), (COPY, 1.0)])
    c = sqlite3.connect(os.path.join(b, "run_results.db"))
    c.execute("insert into counters_collection values (5, ?, 'TCC_MISS_sum', 90.0)", (MANGLED_LB,))
    c.commit()
    c.close()
    out = str(tmp_path / "c.md")
    rs.counters(out, "cmd", "relax=k_push_lb<SsspMark<\\w+>, 4, 1>", [a, b])
    text = open(out).read()
    assert "| `SQ_WAVE_CYCLES` | 2 | 200 |" in text
    assert "| `SQ_WAIT_ANY` | 2 | 180 |" in text
    assert "| waves waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES) | 0.9 |" in text
    assert "| average wave lifetime in cycles (SQ_WAVE_CYCLES / SQ_WAVES) | 50 |" in text
    assert "| L2 hit rate (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)) | 0.25 |" in text
