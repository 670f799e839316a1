"""Host logic of bench.py, on the CPU: the serving sweep's request counts and
the rocprofv3 summary (parsing of the trace and counter databases, counter
calibration against device copies, HBM bytes per launch, the traffic table
that bench.py reads back)."""
import json
import os
import sqlite3

import pytest

import bench

V32 = "void wp::pass_kernel<float, float, 512, true, 1, 0>(wp::PassArgs)"
E32 = "void wp::edge_pass_kernel<float, float, 512, true, 1, 0>(wp::PassArgs)"
K32 = "void wp::pass_kernel<float, float, 512, false, 2, 1>(wp::PassArgs)"
V64 = "void wp::pass_kernel<double, double, 512, true, 1, 0>(wp::PassArgs)"
COPY = "__amd_rocclr_copyBuffer"
G32, G64, GCOPY = 8388608, 16777216, 4194304


def test_sweep_counts_within_limit():
    rates = [0.25, 0.5, 0.75, 0.9, 1.1]
    # 1100 requests per rate at C = 25 req/s: about 411 s asked
    count, warm, projected = bench.sweep_counts(1000, 100, rates, 25.0, 180.0)
    assert projected == pytest.approx(sum(1100 / (f * 25.0) for f in rates))
    assert sum((count + warm) / (f * 25.0) for f in rates) <= 180.0 + 1e-9
    assert count == int(1000 * 180.0 / projected) and warm == int(100 * 180.0 / projected)
    # no limit, or a limit that the asked counts meet: unchanged
    assert bench.sweep_counts(1000, 100, rates, 25.0, 0.0)[:2] == (1000, 100)
    assert bench.sweep_counts(300, 30, rates, 25.0, 1e6)[:2] == (300, 30)
    # floors of 100 measured and 10 warm-up requests
    assert bench.sweep_counts(1000, 100, rates, 0.01, 1.0)[:2] == (100, 10)


def _trace_db(path, launches):
    """launches: (name, grid, stream, duration_ns) in launch order."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    db = sqlite3.connect(path)
    db.execute("create table kernels (name text, start integer, duration integer, stream_id integer, "
               "grid_size integer)")
    t = 0
    for name, grid, stream, dur in launches:
        db.execute("insert into kernels values (?, ?, ?, ?, ?)", (name, t, dur, stream, grid))
        t += dur + 1000
    db.commit()


def _counter_db(path, rows):
    """rows: (kernel, grid, counter, value) per dispatch."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
               "value real, grid_size integer)")
    for i, (k, g, c, v) in enumerate(rows):
        db.execute("insert into counters_collection values (?, ?, ?, ?, ?)", (i, k, c, v, g))
    db.commit()


@pytest.fixture
def profile_dir(tmp_path):
    base = str(tmp_path)
    # in-step launches (short runs on stream 0, between other kernels), then
    # a back-to-back run of five
    launches = []
    for _ in range(4):
        launches += [(V32, G32, 0, 560000), (K32, G32 // 8, 0, 100000), (K32, G32 // 8, 1, 100000)]
    launches += [(V32, G32, 0, 580000)] * 5
    launches += [(E32, G32, 0, 440000), (V64, G64, 0, 970000), (K32, G32, 0, 440000)]
    launches += [(COPY, GCOPY, 0, 420000)] * 3
    _trace_db(os.path.join(base, "trace", "trace_results.db"), launches)
    fetch, write, sq = [], [], []
    # a 1 GiB copy reads FETCH_SIZE = 512 MiB and WRITE_SIZE = 1 GiB, except
    # one dispatch that reports twice as much: the median calibrates
    for v in (512, 512, 1024):
        fetch.append((COPY, GCOPY, "FETCH_SIZE", v * 1024))
    for v in (1024, 2048, 1024):
        write.append((COPY, GCOPY, "WRITE_SIZE", v * 1024))
    for name, grid, gib in ((V32, G32, 1), (E32, G32, 1), (K32, G32, 1), (V64, G64, 2)):
        for _ in range(3):
            fetch.append((name, grid, "FETCH_SIZE", gib * 512 * 1024))
            write.append((name, grid, "WRITE_SIZE", gib * 1024 * 1024))
            sq += [(name, grid, "SQ_WAVES", 131072.0), (name, grid, "SQ_INSTS_VALU", 131072.0 * 1961),
                   (name, grid, "SQ_INSTS_LDS", 1e6), (name, grid, "SQ_LDS_BANK_CONFLICT", 5e4)]
    _counter_db(os.path.join(base, "fetch", "fetch_results.db"), fetch)
    _counter_db(os.path.join(base, "write", "write_results.db"), write)
    _counter_db(os.path.join(base, "sq", "sq_results.db"), sq)
    return base


def test_rocprof_summary_bytes_and_traffic_table(profile_dir, capsys):
    assert bench.rocprof_summary(profile_dir, 512) == 0
    out = capsys.readouterr().out
    assert "scale 2.0000" in out and "scale 1.0000" in out  # median, not the outlier
    row = next(l for l in out.splitlines() if l.startswith("| `pass<float,float,512,strided,V,t0>`"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    # kernel, part, launches, avg, in-step launches, in-step avg, b2b avg, read GB, write GB, GB/s, conflicts, VALU
    assert cells[2] == "9" and cells[4] == "4" and float(cells[5]) == pytest.approx(560.0)
    assert float(cells[6]) == pytest.approx(580.0)
    assert float(cells[7]) == pytest.approx(1.074, abs=1e-3) and float(cells[8]) == pytest.approx(1.074, abs=1e-3)
    assert float(cells[11]) == pytest.approx(1961)
    t = json.load(open(os.path.join(profile_dir, "traffic.json")))
    assert t["kernel_hash"] == bench.kernel_hash()
    assert t["entries"]["softcore_3d_512:c64:axis0:t0"]["bytes_per_launch"] == 2 * (1 << 30)
    assert t["entries"]["softcore_3d_512:c64:edge:t0"]["bytes_per_launch"] == 2 * (1 << 30)
    assert t["entries"]["softcore_3d_512:c64:last:t1"]["bytes_per_launch"] == 2 * (1 << 30)
    assert t["entries"]["softcore_3d_512:c128:axis0:t0"]["bytes_per_launch"] == 4 * (1 << 30)


def test_rocprof_summary_precision_filter(profile_dir, capsys):
    assert bench.rocprof_summary(profile_dir, 512, "c128") == 0
    out = capsys.readouterr().out
    assert "`pass<double,double,512,strided,V,t0>`" in out
    assert "`pass<float," not in out and "`edge<float," not in out


def test_rocprof_summary_trace_only(profile_dir, capsys):
    for d in ("sq", "fetch", "write"):
        os.remove(os.path.join(profile_dir, d, f"{d}_results.db"))
        os.rmdir(os.path.join(profile_dir, d))
    assert bench.rocprof_summary(profile_dir, 512) == 0
    out = capsys.readouterr().out
    row = next(l for l in out.splitlines() if l.startswith("| `pass<float,float,512,strided,V,t0>`"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == str(G32) and cells[2] == "9" and cells[5] == "4"


def test_traffic_for_reads_the_committed_table():
    # the committed table answers only for the kernel sources it was taken on
    t = json.load(open(bench.TRAFFIC_FILE))
    got = bench.traffic_for("axis0", "softcore_3d_512", "c64", 0)
    if t["kernel_hash"] == bench.kernel_hash():
        assert got == t["entries"]["softcore_3d_512:c64:axis0:t0"]["bytes_per_launch"]
    else:
        assert got is None


def test_kernel_hash_ignores_comments_only():
    code = "int f(int a) {\n  // twice\n  return 2 * a; /* doubled */\n}\n"
    recommented = "int f(int a) {   // doubled\n  /* a block\n     comment */ return 2 * a;\n}\n"
    changed = "int f(int a) {\n  // twice\n  return 3 * a;\n}\n"
    assert bench.code_only(code) == bench.code_only(recommented)
    assert bench.code_only(code) != bench.code_only(changed)
    assert bench.code_only(code) == "int f(int a) { return 2 * a; }"
