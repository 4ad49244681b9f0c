"""Host logic of bench.py's HBM record (no GPU): the calibration of the two
counter runs and the digest that ties the record to the kernel sources."""
import importlib.util
import json
import os
import sqlite3

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)

KERNEL = "void ss::(anonymous namespace)::k_trsv_level<HIP_vector_type<double, 2u>, false, 8, 3>(int, int, ...)"
KERNEL_UP = "void ss::(anonymous namespace)::k_trsv_level<HIP_vector_type<double, 2u>, true, 8, 3>(int, int, ...)"
KERNEL_C64 = "void ss::(anonymous namespace)::k_trsv_level<HIP_vector_type<float, 2u>, false, 8, 3>(int, int, ...)"
COPY = "__amd_rocclr_copyBuffer"


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id int, kernel_name text, grid_size int, "
                "counter_name text, value real)")
    for d, (k, g, v) in enumerate(rows):
        # two counter instances per dispatch, summed by the reader
        con.execute("insert into counters_collection values (?, ?, ?, ?, ?)", (d, k, g, counter, v / 2))
        con.execute("insert into counters_collection values (?, ?, ?, ?, ?)", (d, k, g, counter, v / 2))
    con.commit()
    con.close()


def test_traffic_record_scales_each_counter_by_the_copy(tmp_path):
    copy_kib = bench.COPY_BYTES / 1024
    grid = bench.COPY_BYTES // 2048
    # the copy reads its bytes twice over in FETCH_SIZE (factor 1/2) and once in WRITE_SIZE.
    # Two applications, each one launch per level: lower levels 300 and 200, upper 250;
    # a complex64 launch is not counted.  The calibration copy is the first copy with its
    # grid; a later copy with the same grid (another size) is not used.
    app_f = [(KERNEL, 4096, 300.0), (KERNEL, 2048, 200.0), (KERNEL_UP, 4096, 250.0)]
    app_w = [(KERNEL, 4096, 40.0), (KERNEL, 2048, 20.0), (KERNEL_UP, 4096, 30.0)]
    _db(tmp_path / "f.db", "FETCH_SIZE", [(COPY, 512, 3.0), (COPY, grid, copy_kib / 2)] + app_f
        + [(KERNEL_C64, grid, 7.0)] + app_f + [(COPY, grid, 77.0)])
    _db(tmp_path / "w.db", "WRITE_SIZE", [(COPY, grid, copy_kib)] + app_w + app_w + [(COPY, grid, 99.0)])
    out = tmp_path / "traffic.json"
    rec = bench.write_traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), 2, str(out))
    assert json.load(open(out)) == rec
    assert rec["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert rec["calibration"]["write_factor"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(750.0 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(90.0 * 1024)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(750.0 * 1024 * 2.0 + 90.0 * 1024)
    assert rec["sources_sha256"] == bench.source_digest(bench.KERNEL_SOURCE)
    assert rec["kernel_match"] == bench.KERNEL_MATCH
    assert rec["dispatches"] == {"fetch": 6, "write": 6}
    assert rec["applications"] == 2


def test_traffic_record_needs_the_solver_and_the_copy(tmp_path):
    grid = bench.COPY_BYTES // 2048
    _db(tmp_path / "f.db", "FETCH_SIZE", [(KERNEL, grid, 1000.0)])
    _db(tmp_path / "w.db", "WRITE_SIZE", [(COPY, grid, 1.0), (KERNEL, grid, 1.0)])
    with pytest.raises(SystemExit):
        bench.write_traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), 1, str(tmp_path / "t.json"))


def test_source_digest_follows_included_headers(tmp_path):
    (tmp_path / "src").mkdir()
    (tmp_path / "inc").mkdir()
    (tmp_path / "src" / "k.hip").write_text('#include "a.hpp"\n#include "../inc/b.h"\nint k;\n')
    (tmp_path / "src" / "a.hpp").write_text('#include "c.hpp"\nint a;\n')
    (tmp_path / "src" / "c.hpp").write_text("int c;\n")
    (tmp_path / "inc" / "b.h").write_text("int b;\n")
    d0 = bench.source_digest("src/k.hip", str(tmp_path))
    assert d0 == bench.source_digest("src/k.hip", str(tmp_path))
    for f in ("src/c.hpp", "inc/b.h", "src/k.hip"):
        p = tmp_path / f
        old = p.read_text()
        p.write_text(old + "// changed\n")
        assert bench.source_digest("src/k.hip", str(tmp_path)) != d0, f
        p.write_text(old)
    assert bench.source_digest("src/k.hip", str(tmp_path)) == d0
    # a header nobody includes does not count
    (tmp_path / "src" / "unused.hpp").write_text("int u;\n")
    assert bench.source_digest("src/k.hip", str(tmp_path)) == d0


def test_committed_record_matches_the_current_sources():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        pytest.skip("no counter record committed for the current dominant kernel")
    rec = json.load(open(path))
    assert rec["kernel_match"] == bench.KERNEL_MATCH
    assert rec["sources_sha256"] == bench.source_digest(rec["source"])
