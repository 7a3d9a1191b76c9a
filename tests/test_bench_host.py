"""Host-side logic of bench.py on synthetic inputs (no GPU): the counter and
traffic summaries from rocprofv3 --pmc databases (the calibration by the
1 GiB copy kernel and the derived issue share), the kernel-trace table, and
the refusal of more than one GPU."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

HOP = "void tmk::k_dslash_walk<2, false, 0, false, false, true, 0, 2>(tmk::DslashArgs)"
COPY = "tmk::k_stream_copy(unsigned int __vector(4) const*, unsigned int __vector(4)*, unsigned long)"
CT = "void tmk::k_contract<1, false, 9>(tmk::Geom, void const*, char const*)"


def _db(path, rows):
    """A database with the one table the summaries read."""
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()
    return str(path)


def test_counter_summary_calibration_and_issue_share(tmp_path):
    # the copy reads 1 GiB, FETCH_SIZE counts half of it (64 B per 128 B request)
    copy_fetch_kib = (1 << 30) / 1024 / 2
    fetch = _db(tmp_path / "f_results.db", [(COPY, "FETCH_SIZE", copy_fetch_kib)] * 2 +
                [(CT, "FETCH_SIZE", 1000.0), (CT, "FETCH_SIZE", 3000.0)])
    write = _db(tmp_path / "w_results.db", [(COPY, "WRITE_SIZE", (1 << 30) / 1024)] +
                [(CT, "WRITE_SIZE", 10.0)])
    # 2.4e6 cycles per XCD; 1024 SIMDs x 2.4e6 / 4 = 6.144e8 wave instructions fill them
    sq = _db(tmp_path / "s_results.db", [(CT, "SQ_INSTS_VALU", 3.072e8), (CT, "GRBM_GUI_ACTIVE", 8 * 2.4e6),
                                          (CT, "TCC_HIT_sum", 3.0), (CT, "TCC_MISS_sum", 1.0),
                                          (HOP, "SQ_INSTS_VALU", 1.0)])
    out = tmp_path / "c.json"
    bench.counter_summary(str(out), "k_contract<1, false, 9>", "--contract-only", [fetch, write, sq],
                          sites=1000, sources=12)
    d = json.load(open(out))
    assert d["dispatches"]["FETCH_SIZE"] == 2
    assert d["per_dispatch_means"]["FETCH_SIZE"] == pytest.approx(2000.0)
    assert d["derived"]["fetch_scale"] == pytest.approx(2.0, rel=1e-4)
    assert d["derived"]["fetch_bytes_per_dispatch"] == pytest.approx(2000 * 1024 * 2.0, rel=1e-4)
    assert d["derived"]["write_scale"] == pytest.approx(1.0, rel=1e-4)
    assert d["derived"]["valu_issue_busy"] == pytest.approx(0.5, abs=1e-3)
    assert d["derived"]["valu_lane_instructions_per_site_source"] == pytest.approx(3.072e8 * 64 / 12000, rel=1e-6)
    assert d["derived"]["l2_hit_rate"] == pytest.approx(0.75)
    # 3.072e8 wave instructions over 1024 SIMDs at four cycles each and 2.4 GHz
    assert d["derived"]["valu_issue_floor_us_at_2400MHz"] == pytest.approx(3.072e8 * 4 / 1024 / 2400, abs=0.1)
    # the hop's row is not mixed in, and every command names committed files only
    assert d["per_dispatch_means"]["SQ_INSTS_VALU"] == pytest.approx(3.072e8)
    assert all("_work" not in c for c in d["commands"])
    assert d["commands"][-1].startswith("python3 bench.py --counter-summary")


def test_counter_summary_without_the_kernel_fails(tmp_path):
    db = _db(tmp_path / "x_results.db", [(COPY, "FETCH_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        bench.counter_summary(str(tmp_path / "o.json"), "k_contract", "--contract-only", [db], sites=1, sources=1)


def test_traffic_from_scales_by_the_copy(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    fetch = _db(tmp_path / "fetch_results.db", [(COPY, "FETCH_SIZE", (1 << 30) / 1024 / 2)] +
                [(HOP, "FETCH_SIZE", 800000.0)] * 3)
    write = _db(tmp_path / "write_results.db", [(COPY, "WRITE_SIZE", (1 << 30) / 1024)] + [(HOP, "WRITE_SIZE", 600000.0)])
    bench.write_traffic(fetch, write, "tsm-batched-32c64")
    d = json.load(open(out))
    assert d["fetch_bytes_per_launch"] == pytest.approx(800000 * 1024 * 2, rel=1e-4)
    assert d["write_bytes_per_launch"] == pytest.approx(600000 * 1024, rel=1e-4)
    assert d["hbm_bytes_per_launch"] == d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert d["kernel_hash"] == bench.kernel_hash() and d["dispatches"] == [3, 1]


def test_kernel_hash_ignores_comments_only():
    src = 'int f(int x) { // twice\n  return 2 * x;  /* doubled */ }\nconst char *s = "// kept";\n'
    same = 'int f(int x)\n{\n    return 2 * x;\n}\n// a note\nconst char *s = "// kept";'
    assert bench.code_text(src) == bench.code_text(same)
    assert bench.code_text(src) != bench.code_text(src.replace("2 * x", "3 * x"))
    assert bench.code_text(src) != bench.code_text(src.replace('"// kept"', '"// gone"'))
    assert len(bench.kernel_hash()) == 16


def test_trace_summary_table(tmp_path):
    (tmp_path / "b_kernel_stats.csv").write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs,StdDev\n"
        f'"{HOP}",4,4000000,1000000,80,900000,1100000,0\n'
        f'"{COPY}",2,1000000,500000,20,500000,500000,0\n')
    (tmp_path / "b_kernel_trace.csv").write_text(
        "Kernel_Name,VGPR_Count,Accum_VGPR_Count,Scratch_Size,Grid_Size_X,Grid_Size_Y,Workgroup_Size_X\n"
        f'"{HOP}",60,0,0,1572864,1,512\n'
        f'"{COPY}",28,0,0,16777216,1,256\n')
    txt = bench.trace_summary(str(tmp_path), "rocprofv3 ... -- python3 bench.py --roofline-only")
    lines = [l for l in txt.splitlines() if not l.startswith("#") and not l.startswith("kernel")]
    assert lines[0].startswith(HOP[:40]) and " 4 " in lines[0] and "80.0%" in lines[0] and "1572864 512" in lines[0]
    assert "1000.00" in lines[0]  # average in microseconds
    assert txt.splitlines()[-1] == "# 2 kernels, 6 dispatches, 5.0 ms of kernel time"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_committed_bench_line_keeps_the_contract():
    """The committed bench line (profiles/) carries every field of the output
    contract, and its figures agree with one another: value from the step
    time, the roofline fraction from the algorithmic bytes and the launch
    time, the traffic record keyed to the current Dslash code."""
    d = json.load(open(os.path.join(ROOT, "profiles", "bench_tsm_32c64_line.json")))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    c = d["config"]
    assert d["n_gpus"] == 1 and c["workload"] == "tsm-batched-32c64" and c["lattice"] == [32, 32, 32, 64]
    assert d["value"] == pytest.approx((c["n_hp"] + c["n_lp"]) / (d["ms_per_step"] / 1e3), rel=2e-3)
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["alg_bytes_per_launch"] == 1440 * 32 ** 3 * 64 // 2
    assert r["achieved"] == pytest.approx(r["alg_bytes_per_launch"] / (r["launch_us"] * 1e-6) / 1e9, rel=2e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=2e-3) and r["peak"] == 8000.0
    stale = "the profiles predate the current Dslash code: refresh the bench line and the traffic record"
    assert r["kernel_hash"] == bench.kernel_hash(), stale
    traffic = json.load(open(os.path.join(ROOT, "profiles", "dslash_f16_traffic.json")))
    assert traffic["kernel_hash"] == bench.kernel_hash(), stale
    assert r["traffic"] == traffic["hbm_bytes_per_launch"]
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
