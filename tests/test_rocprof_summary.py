"""The rocprofv3 summaries on synthetic counter files: calibration against the
copy kernel, the dominant launch's bytes, and the block bookkeeping of the
evaluation-suite traffic run (markers, every kernel of a call, call counts)
and of the per-variant run of the bandwidth workload (rows grouped by shape)."""
import csv
import json
import os

import pytest

from paper_2609_01864_amd import rocprof_summary as R

HDR = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for i, (name, grid, kib) in enumerate(rows):
            w.writerow([i + 1, grid, name, counter, kib])


def test_suite_traffic_blocks(tmp_path):
    calib = 1 << 30
    meta = {"mode": "traffic_suite", "source_hash": "abc", "copy_kernel_bytes": calib, "copy_threads": calib // 16,
            "blocks": [{"workload": "w", "M": 4, "N": 8, "variant": "two_pass", "k": 1, "marker_threads": 256,
                        "launches": 2, "algorithmic_bytes": 3000.0},
                       {"workload": "w", "M": 4, "N": 8, "variant": "split", "k": 4, "marker_threads": 512,
                        "launches": 2, "algorithmic_bytes": 2000.0}]}
    mp = tmp_path / "meta.json"
    mp.write_text(json.dumps(meta) + "\n")
    copy = "credit::k_copy(u32x4 const*, u32x4*, long)"
    tp = "void credit::k_twopass<9, 0, 256>(credit::RowArgs)"
    rs = "void credit::k_resident<9, 0, 4>(credit::RowArgs)"
    cr = "credit::k_colreduce(float const*, float*, int, long)"
    fl = "credit::k_flush_read(u32x4 const*, long, unsigned int*)"

    def seq(f):  # FETCH counts 0.5 KiB per KiB moved, WRITE 1.0
        kib = lambda b: f * b / 1024.0
        return [(copy, calib // 16, kib(calib)),                     # calibration
                (rs, 1024, 999.0),                                  # before any marker: ignored
                (copy, 256, 1.0), (copy, 256, 1.0),                 # marker of block 0
                (fl, 99, 5000.0), (tp, 4096, kib(2900)), (fl, 99, 5000.0), (tp, 4096, kib(3100)),
                (copy, 512, 1.0),                                   # marker of block 1
                (fl, 99, 5000.0), (rs, 1024, kib(1800)), (cr, 64, kib(200)),
                (fl, 99, 5000.0), (rs, 1024, kib(1800)), (cr, 64, kib(200))]

    _write(tmp_path / "f", "FETCH_SIZE", seq(0.5))
    _write(tmp_path / "w", "WRITE_SIZE", seq(1.0))
    out = tmp_path / "s.json"
    R.main(["suite", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--bench", str(mp),
            "--json", str(out), "--out", str(tmp_path / "s.md")])
    rows = json.load(open(out))["rows"]
    # each counter recovers the bytes of one call: 3000 (two-pass), 2000 (split
    # row kernel 1800 + column reduction 200), once per counter
    assert rows[0]["fetch_bytes"] == 3000 and rows[0]["write_bytes"] == 3000
    assert rows[1]["fetch_bytes"] == 2000 and rows[1]["write_bytes"] == 2000
    assert rows[1]["ratio_to_algorithmic"] == pytest.approx(2.0)
    assert "33.3%" in (tmp_path / "s.md").read_text()


def test_plans_traffic_groups_by_shape(tmp_path):
    # --traffic-plans: per width a two-pass row, optionally a row-resident row,
    # then a split row; every reduction is against the two-pass row of its width
    calib = 1 << 30
    blk = lambda N, v, k, m, alg: {"workload": "ln", "M": 2, "N": N, "variant": v, "k": k, "marker_threads": m,
                                   "launches": 1, "algorithmic_bytes": alg}
    meta = {"mode": "traffic_plans", "source_hash": "abc", "copy_kernel_bytes": calib, "copy_threads": calib // 16,
            "blocks": [blk(8, "two_pass", 1, 256, 1200.0), blk(8, "resident", 1, 512, 800.0),
                       blk(8, "split", 2, 768, 800.0), blk(16, "two_pass", 1, 1024, 2400.0),
                       blk(16, "split", 4, 1280, 1600.0)]}
    mp = tmp_path / "meta.json"
    mp.write_text(json.dumps(meta) + "\n")
    copy = "credit::k_copy(u32x4 const*, u32x4*, long)"
    tp = "void credit::k_twopass<1, 0, 256>(credit::RowArgs)"
    rs = "void credit::k_resident<1, 0, 4>(credit::RowArgs)"

    def seq(f):
        kib = lambda b: f * b / 1024.0
        return [(copy, calib // 16, kib(calib)),
                (copy, 256, 1.0), (tp, 64, kib(1000)),   # width 8: the reread partly cached
                (copy, 512, 1.0), (rs, 64, kib(800)),
                (copy, 768, 1.0), (rs, 128, kib(800)),
                (copy, 1024, 1.0), (tp, 64, kib(2400)),  # width 16: the reread reaches HBM
                (copy, 1280, 1.0), (rs, 256, kib(1600))]

    _write(tmp_path / "f", "FETCH_SIZE", seq(0.5))
    _write(tmp_path / "w", "WRITE_SIZE", seq(1.0))
    R.main(["suite", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--bench", str(mp),
            "--json", str(tmp_path / "s.json"), "--out", str(tmp_path / "s.md")])
    rows = json.load(open(tmp_path / "s.json"))["rows"]
    assert [r["fetch_bytes"] for r in rows] == [1000, 800, 800, 2400, 1600]
    md = (tmp_path / "s.md").read_text()
    assert "variants of the bandwidth workload" in md
    lines = [ln for ln in md.splitlines() if ln.startswith("| ln |")]
    assert "row-resident" in lines[1] and lines[1].endswith("| 20.0% |")
    assert "split k=2" in lines[2] and lines[2].endswith("| 20.0% |")
    assert lines[3].endswith("|  |") and lines[4].endswith("| 33.3% |")


def test_suite_traffic_rejects_a_missing_call(tmp_path):
    calib = 1 << 30
    meta = {"mode": "traffic_suite", "copy_kernel_bytes": calib, "copy_threads": calib // 16,
            "blocks": [{"workload": "w", "M": 1, "N": 1, "variant": "two_pass", "k": 1, "marker_threads": 256,
                        "launches": 3, "algorithmic_bytes": 1.0}]}
    mp = tmp_path / "meta.json"
    mp.write_text(json.dumps(meta) + "\n")
    rows = [("credit::k_copy(x)", calib // 16, 512.0), ("credit::k_copy(x)", 256, 1.0),
            ("void credit::k_twopass<0, 0, 256>(credit::RowArgs)", 8, 1.0)]
    _write(tmp_path / "f", "FETCH_SIZE", rows)
    _write(tmp_path / "w", "WRITE_SIZE", rows)
    with pytest.raises(SystemExit):
        R.main(["suite", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--bench", str(mp),
                "--json", str(tmp_path / "s.json"), "--out", str(tmp_path / "s.md")])


def test_suite_traffic_rejects_runs_with_different_blocks(tmp_path):
    calib = 1 << 30
    blk = {"workload": "w", "M": 1, "N": 1, "variant": "split", "k": 8, "marker_threads": 256, "launches": 1,
           "algorithmic_bytes": 1.0}
    meta = {"mode": "traffic_suite", "copy_kernel_bytes": calib, "copy_threads": calib // 16, "blocks": [blk]}
    (tmp_path / "f.json").write_text(json.dumps(meta) + "\n")
    (tmp_path / "w.json").write_text(json.dumps(dict(meta, blocks=[dict(blk, k=4)])) + "\n")
    rows = [("credit::k_copy(x)", calib // 16, 512.0), ("credit::k_copy(x)", 256, 1.0),
            ("void credit::k_resident<0, 0, 1>(credit::RowArgs)", 8, 1.0)]
    _write(tmp_path / "f", "FETCH_SIZE", rows)
    _write(tmp_path / "w", "WRITE_SIZE", rows)
    with pytest.raises(SystemExit, match="different blocks"):
        R.main(["suite", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"),
                "--bench", str(tmp_path / "f.json"), "--bench-write", str(tmp_path / "w.json"),
                "--json", str(tmp_path / "s.json"), "--out", str(tmp_path / "s.md")])


def _dominant_bench(kernel="ln:N=8:plan=2,4", grid=4096, alg=4000.0):
    return {"copy_kernel_bytes": 1 << 30, "source_hash": "abc",
            "roofline": {"kernel": kernel, "kernel_symbol": "void credit::k_resident<1, 0, 32>",
                         "grid_threads": grid, "algorithmic_bytes_per_launch": alg}}


def test_dominant_traffic_calibrated_per_counter(tmp_path):
    calib = 1 << 30
    b = _dominant_bench()
    (tmp_path / "b.json").write_text(json.dumps(b) + "\n")
    dom = "void credit::k_resident<1, 0, 32>(credit::RowArgs)"
    copy = "credit::k_copy(u32x4 const*, u32x4*, long)"

    def seq(f, moved):  # the dominant launch moves `moved` bytes in this direction
        kib = lambda x: f * x / 1024.0
        return [(copy, calib // 16, kib(calib)), (dom, 4096, kib(moved)), (dom, 4096, kib(moved)),
                (dom, 4096, kib(100 * moved))]  # same kernel and grid, another shape: excluded

    _write(tmp_path / "f", "FETCH_SIZE", seq(0.5, 2100))
    _write(tmp_path / "w", "WRITE_SIZE", seq(1.0, 2000))
    out = tmp_path / "t.json"
    R.main(["traffic", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--bench",
            str(tmp_path / "b.json"), "--bench-write", str(tmp_path / "b.json"), "--json", str(out),
            "--out", str(tmp_path / "t.md")])
    e = json.load(open(out))["kernels"]["ln:N=8:plan=2,4"]
    assert e["fetch_bytes"] == 2100 and e["write_bytes"] == 2000 and e["bytes_per_launch"] == 4100
    assert "ratio 1.025" in (tmp_path / "t.md").read_text()


def test_dominant_traffic_rejects_runs_with_different_launches(tmp_path):
    (tmp_path / "f.json").write_text(json.dumps(_dominant_bench()) + "\n")
    (tmp_path / "w.json").write_text(json.dumps(_dominant_bench(kernel="ln:N=8:plan=2,8", grid=8192)) + "\n")
    with pytest.raises(SystemExit, match="different dominant launches"):
        R.main(["traffic", "--fetch", str(tmp_path), "--write", str(tmp_path), "--bench", str(tmp_path / "f.json"),
                "--bench-write", str(tmp_path / "w.json"), "--json", str(tmp_path / "t.json"),
                "--out", str(tmp_path / "t.md")])


def test_counters_median_and_ratios(tmp_path):
    bench = {"roofline": {"kernel": "layernorm_fwd:N=8:plan=2,2", "kernel_symbol": "void credit::k_resident<1, 0, 1>",
                          "grid_threads": 128, "algorithmic_bytes_per_launch": 8.0 * 1000, "avg_launch_us": 10.0},
             "source_hash": "h"}
    bp = tmp_path / "b.json"
    bp.write_text(json.dumps(bench) + "\n")
    d = tmp_path / "sq"
    d.mkdir()
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR + ["Start_Timestamp", "End_Timestamp"])
        k = "void credit::k_resident<1, 0, 1>(credit::RowArgs)"
        # (dispatch, grid, duration us, {counter: value})
        disp = [(1, 128, 10.0, {"SQ_WAVES": 2, "SQ_INSTS_VALU": 100, "SQ_ACTIVE_INST_LDS": 50,
                                "SQ_LDS_BANK_CONFLICT": 5}),
                (2, 128, 11.0, {"SQ_WAVES": 2, "SQ_INSTS_VALU": 300}),
                (3, 128, 9.0, {"SQ_WAVES": 2, "SQ_INSTS_VALU": 200}),
                (4, 64, 10.0, {"SQ_INSTS_VALU": 9999}),  # another grid: ignored
                (5, 128, 1.0, {"SQ_WAVES": 2, "SQ_INSTS_VALU": 7})]  # same kernel and grid, another shape
        t = 1000
        for did, g, us, cs in disp:
            for c, v in cs.items():
                w.writerow([did, g, k, c, v, t, t + int(us * 1000)])
            t += 100000
    out = tmp_path / "c.json"
    R.main(["counters", "--pmc", str(d), "--bench", str(bp), "--json", str(out), "--out", str(tmp_path / "c.md")])
    res = json.load(open(out))
    assert res["median_per_dispatch"]["SQ_INSTS_VALU"] == 200.0
    assert res["median_per_dispatch"]["SQ_WAVES"] == 2.0
    md = (tmp_path / "c.md").read_text()
    assert "| SQ_INSTS_VALU | 200 | 100 | 0.2 |" in md
    assert "1 dispatches of the same kernel and grid" in md
    assert "0.1000" in md  # 5 conflict cycles per 50 active LDS cycles
