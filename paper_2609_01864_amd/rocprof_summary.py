"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_2609_01864_amd.rocprof_summary trace  --trace DIR --bench BENCH.json --out profiles/X.md
    python -m paper_2609_01864_amd.rocprof_summary traffic --fetch DIR --write DIR --bench BENCH.json \
        --bench-write BENCH_W.json --json profiles/traffic.json --out profiles/Y.md

trace    per-kernel dispatch counts and average durations from a
         `rocprofv3 --kernel-trace --stats --output-format csv` run of the
         benchmark, with the benchmark's own HIP-event average for its dominant
         kernel beside the trace's average for the same kernel and grid.
traffic  HBM bytes per launch of the dominant kernel from two `--pmc` runs
         (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each divided by the
         counter-per-byte factor the same counter reads on the plain copy
         kernel (k_copy moves a known number of bytes each way).
counters the SQ counters of one `--pmc` run (occupancy, instruction mix, LDS
         bank conflicts) for the dominant kernel and grid: the median per
         dispatch, with per-wave and per-element ratios.
suite    the same two counters over the launch sequence of
         `bench.py --traffic-suite` (two-pass and every legal split-row plan
         of every evaluation-suite workload at N = 65536) or of
         `bench.py --traffic-plans` (two-pass, row-resident where legal and
         every legal split-row plan of the bandwidth workload at each width),
         each block behind a marker copy launch: bytes per operator call,
         summed over every kernel the call launches, and the reduction of
         each plan against the two-pass kernel of the same shape.

    python -m paper_2609_01864_amd.rocprof_summary suite --fetch DIR --write DIR --bench META.json \
        --bench-write META_W.json --json profiles/suite_traffic.json --out profiles/Z.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import statistics
import sys


CLOCK_HZ = 2.4e9  # MI355X peak engine clock (the launch's cycles for the coverage figure)


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def _rows(path: str):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _grid(r) -> int:
    for k in ("Grid_Size", "Grid_Size_X", "grid_size", "Grid_X"):
        if k in r and r[k] not in ("", None):
            return int(float(r[k]))
    return -1


def _dur_us(r) -> float:
    s = r.get("Start_Timestamp") or r.get("start")
    e = r.get("End_Timestamp") or r.get("end")
    return (int(e) - int(s)) / 1e3


def kernel_name(bench: dict) -> tuple:
    """(demangled name prefix, grid in work-items) of the dominant launch."""
    d = bench["roofline"]
    return d["kernel_symbol"], int(d["grid_threads"])


def trace(args):
    bench = json.loads(open(args.bench).read().strip().splitlines()[-1])
    rows = _rows(_find(args.trace, "kernel_trace.csv"))
    by = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("kernel_name")
        by.setdefault(name, []).append(r)
    sym, grid = kernel_name(bench)
    avg = bench["roofline"]["avg_launch_us"]
    same = [_dur_us(r) for r in rows if (r.get("Kernel_Name") or "").startswith(sym) and _grid(r) == grid]
    # other shapes of the workload can launch the same kernel instance with the
    # same grid; the dominant launch's dispatches are those within a factor
    # 1.5 of the benchmark's own average for it
    dom = [d for d in same if avg / 1.5 <= d <= avg * 1.5]
    lines = [f"# rocprofv3 kernel trace: {args.title}", "",
             f"Command: `{args.command}`", "",
             f"Dominant kernel (benchmark roofline): `{sym}` grid {grid} work-items", "",
             f"* benchmark HIP-event average over the timed steps: {bench['roofline']['avg_launch_us']:.2f} us",
             f"* rocprofv3 average of the same kernel and grid: {statistics.mean(dom):.2f} us over {len(dom)} "
             f"dispatches (median {statistics.median(dom):.2f} us); {len(same) - len(dom)} other dispatches of "
             f"this kernel and grid (other shapes, outside 1/1.5..1.5x of the benchmark average) excluded"
             if dom else "* (not found in trace)",
             "", "| kernel | dispatches | total ms | avg us |", "|---|---:|---:|---:|"]
    tot = []
    for name, rs in by.items():
        ds = [_dur_us(r) for r in rs]
        tot.append((sum(ds), name, len(ds), statistics.mean(ds)))
    for s, name, n, avg in sorted(tot, reverse=True)[:25]:
        short = name if len(name) < 90 else name[:87] + "..."
        lines.append(f"| `{short}` | {n} | {s / 1e3:.2f} | {avg:.2f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines[:10]))


def _counter_rows(d: str, counter: str):
    rows = _rows(_find(d, "counter_collection.csv"))
    out = []
    for r in rows:
        if (r.get("Counter_Name") or r.get("counter_name")) != counter:
            continue
        out.append((r.get("Kernel_Name") or "", _grid(r), float(r.get("Counter_Value") or r.get("value"))))
    return out


def traffic(args):
    bench = json.loads(open(args.bench).read().strip().splitlines()[-1])
    sym, grid = kernel_name(bench)
    if args.bench_write:  # the WRITE_SIZE run must have timed the same dominant launch
        other = json.loads(open(args.bench_write).read().strip().splitlines()[-1])
        if (other["roofline"]["kernel"], kernel_name(other)) != (bench["roofline"]["kernel"], (sym, grid)):
            raise SystemExit("the FETCH_SIZE and WRITE_SIZE runs timed different dominant launches")
    copy_bytes = float(bench["copy_kernel_bytes"])  # bytes read (= bytes written) per copy launch
    res = {}
    for counter, d in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        rows = _counter_rows(d, counter)
        # counters are summed over the dispatch's instances by rocprofv3
        cp = [v for n, g, v in rows if n.startswith("credit::k_copy")]
        same = [v for n, g, v in rows if n.startswith(sym) and g == grid]
        if not cp or not same:
            raise SystemExit(f"{counter}: copy dispatches {len(cp)}, dominant dispatches {len(same)}")
        factor = statistics.median(cp) * 1024.0 / copy_bytes  # counter bytes per real byte
        # other shapes may launch the same kernel and grid: keep the dispatches
        # within a factor 2 of the dominant launch's algorithmic bytes for this
        # direction (read: inputs, write: outputs; half each for these ops)
        expect = 0.5 * bench["roofline"]["algorithmic_bytes_per_launch"] * factor / 1024.0
        dom = [v for v in same if expect / 2 <= v <= expect * 2]
        if not dom:
            raise SystemExit(f"{counter}: no dispatch near {expect:.0f} KiB among {sorted(same)[:8]}")
        res[counter] = {"kib_per_dispatch": statistics.median(dom), "copy_kib_per_dispatch": statistics.median(cp),
                        "dispatches": len(dom), "excluded": len(same) - len(dom),
                        "factor": factor, "bytes_per_launch": statistics.median(dom) * 1024.0 / factor}
    total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    key = bench["roofline"]["kernel"]
    entry = {"bytes_per_launch": round(total), "fetch_bytes": round(res["FETCH_SIZE"]["bytes_per_launch"]),
             "write_bytes": round(res["WRITE_SIZE"]["bytes_per_launch"]),
             "algorithmic_bytes": bench["roofline"]["algorithmic_bytes_per_launch"],
             "source_hash": bench["source_hash"], "kernel_symbol": sym, "grid_threads": grid,
             "copy_factor_fetch": res["FETCH_SIZE"]["factor"], "copy_factor_write": res["WRITE_SIZE"]["factor"]}
    data = {"kernels": {}}
    if os.path.exists(args.json):
        data = json.load(open(args.json))
    data.setdefault("kernels", {})[key] = entry
    json.dump(data, open(args.json, "w"), indent=1)
    lines = [f"# HBM traffic of the dominant kernel: {args.title}", "",
             f"Commands: `{args.command}` with `--pmc FETCH_SIZE` and, separately, `--pmc WRITE_SIZE`", "",
             f"Kernel `{sym}`, grid {grid} work-items ({key})", "",
             "| counter | kernel KiB/dispatch | copy-kernel KiB/dispatch | counter bytes per byte moved | HBM bytes/launch |",
             "|---|---:|---:|---:|---:|"]
    for c, r in res.items():
        lines.append(f"| {c} | {r['kib_per_dispatch']:.0f} | {r['copy_kib_per_dispatch']:.0f} | {r['factor']:.4f} | "
                     f"{r['bytes_per_launch']:.4e} |")
    alg = entry["algorithmic_bytes"]
    lines += ["", "Dispatches used (kept / other shapes sharing kernel and grid, outside 0.5..2x of the expected "
                  "bytes): " + ", ".join(f"{c} {r['dispatches']}/{r['excluded']}" for c, r in res.items()),
              "", f"Total {total:.4e} bytes per launch against {alg:.4e} algorithmic bytes "
                  f"(ratio {total / alg:.3f}).", "",
              f"The copy kernel moves {copy_bytes:.0f} bytes each way per launch."]
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


_OP_KERNEL = re.compile(r"credit::k_(twopass|resident|multirow|colreduce1|colreduce|colstats)\b")
_MAIN_KERNEL = re.compile(r"credit::k_(twopass|resident|multirow)\b")


def _counter_seq(d: str, counter: str):
    """(kernel name, grid, value) of every dispatch, in dispatch order."""
    rows = _rows(_find(d, "counter_collection.csv"))
    out = []
    for r in rows:
        if (r.get("Counter_Name") or r.get("counter_name")) != counter:
            continue
        out.append((int(r.get("Dispatch_Id") or 0), r.get("Kernel_Name") or "", _grid(r),
                    float(r.get("Counter_Value") or r.get("value"))))
    out.sort()
    return [(n, g, v) for _, n, g, v in out]


def suite(args):
    meta = json.loads(open(args.bench).read().strip().splitlines()[-1])
    assert meta.get("mode") in ("traffic_suite", "traffic_plans"), "not a --traffic-suite / --traffic-plans run"
    blocks = meta["blocks"]
    if args.bench_write:  # the WRITE_SIZE run must have launched the same blocks
        other = json.loads(open(args.bench_write).read().strip().splitlines()[-1])["blocks"]
        if other != blocks:
            raise SystemExit("the FETCH_SIZE and WRITE_SIZE runs launched different blocks")
    by_marker = {b["marker_threads"]: i for i, b in enumerate(blocks)}
    per = {}
    for counter, d in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        seq = _counter_seq(d, counter)
        cp = [v for n, g, v in seq if "credit::k_copy" in n and g == meta["copy_threads"]]
        if not cp:
            raise SystemExit(f"{counter}: no calibration copy dispatch")
        factor = statistics.median(cp) * 1024.0 / meta["copy_kernel_bytes"]
        sums = [0.0] * len(blocks)
        mains = [0] * len(blocks)
        cur = None
        for n, g, v in seq:
            if "credit::k_copy" in n:
                cur = by_marker.get(g, cur if g != meta["copy_threads"] else None)
                continue
            if cur is None or not _OP_KERNEL.search(n):
                continue
            sums[cur] += v
            mains[cur] += 1 if _MAIN_KERNEL.search(n) else 0
        for i, b in enumerate(blocks):
            if mains[i] != b["launches"]:
                raise SystemExit(f"{counter}: block {i} ({b['workload']} {b['variant']}) has {mains[i]} main "
                                 f"dispatches, expected {b['launches']}")
            per.setdefault(i, {})[counter] = sums[i] / mains[i] * 1024.0 / factor
        per.setdefault("factor", {})[counter] = factor
    rows = []
    for i, b in enumerate(blocks):
        tot = per[i]["FETCH_SIZE"] + per[i]["WRITE_SIZE"]
        rows.append(dict(b, fetch_bytes=round(per[i]["FETCH_SIZE"]), write_bytes=round(per[i]["WRITE_SIZE"]),
                         bytes_per_call=round(tot), ratio_to_algorithmic=round(tot / b["algorithmic_bytes"], 4)))
    out = {"source_hash": meta.get("source_hash"), "factors": per["factor"], "rows": rows}
    json.dump(out, open(args.json, "w"), indent=1)
    what = "evaluation-suite workloads" if meta["mode"] == "traffic_suite" else "variants of the bandwidth workload"
    lines = [f"# HBM traffic of the {what}: {args.title}", "",
             f"Commands: `{args.command}` with `--pmc FETCH_SIZE` and, separately, `--pmc WRITE_SIZE`", "",
             "Bytes per operator call, summed over every kernel the call launches (row kernel and, for",
             "LayerNorm backward, the column reductions), averaged over the calls of its block; counters",
             f"divided by what they read per byte on a 1 GiB copy (FETCH {per['factor']['FETCH_SIZE']:.4f}, "
             f"WRITE {per['factor']['WRITE_SIZE']:.4f}).", "",
             "| workload | M x N | plan | HBM bytes/call | algorithmic | ratio | reduction vs two-pass |",
             "|---|---|---|---:|---:|---:|---:|"]
    base = None  # each (workload, M, N) group opens with its two-pass row
    for r in rows:
        if r["variant"] == "two_pass":
            base, rr = r, ""
        else:
            same = base is not None and (base["workload"], base["M"], base["N"]) == (r["workload"], r["M"], r["N"])
            rr = f"{100 * (1.0 - r['bytes_per_call'] / base['bytes_per_call']):.1f}%" if same else ""
        plan = {"two_pass": "two-pass", "resident": "row-resident"}.get(r["variant"], f"split k={r['k']}")
        lines.append(f"| {r['workload']} | {r['M']} x {r['N']} | {plan} | {r['bytes_per_call']:.4e} | "
                     f"{r['algorithmic_bytes']:.4e} | {r['ratio_to_algorithmic']:.3f} | {rr} |")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(args):
    bench = json.loads(open(args.bench).read().strip().splitlines()[-1])
    sym, grid = kernel_name(bench)
    rows = _rows(_find(args.pmc, "counter_collection.csv"))
    # one row per (dispatch, counter); other shapes can launch the same kernel
    # instance with the same grid (the row-resident plan of a narrower row),
    # so a dispatch counts only when its duration lies within 1/1.5..1.5x of
    # the benchmark's own average for the dominant launch (both timed under
    # the same counter collection)
    avg = float(bench["roofline"]["avg_launch_us"])
    disp, excluded = {}, set()
    for r in rows:
        if not (r.get("Kernel_Name") or "").startswith(sym) or _grid(r) != grid:
            continue
        did = r.get("Dispatch_Id") or r.get("dispatch_id")
        if not avg / 1.5 <= _dur_us(r) <= avg * 1.5:
            excluded.add(did)
            continue
        disp.setdefault(did, {})[r.get("Counter_Name")] = float(r.get("Counter_Value") or 0.0)
    vals = {}
    for d in disp.values():
        for c, v in d.items():
            vals.setdefault(c, []).append(v)
    if not vals:
        raise SystemExit(f"no dispatch of {sym} with grid {grid} near {avg:.1f} us")
    med = {c: statistics.median(v) for c, v in vals.items()}
    n_disp = min(len(v) for v in vals.values())
    key = bench["roofline"]["kernel"]
    # elements per launch: stated by single-workload runs, else FP32 in + out
    elems = bench["roofline"].get("elements_per_launch") or bench["roofline"]["algorithmic_bytes_per_launch"] / 8.0
    waves = med.get("SQ_WAVES", 0.0)
    lines = [f"# SQ counters of the dominant kernel: {args.title}", "",
             f"Command: `{args.command}`", "",
             f"Kernel `{sym}`, grid {grid} work-items ({key}); median over {n_disp} dispatches "
             f"({len(excluded)} dispatches of the same kernel and grid outside 1/1.5..1.5x of the benchmark's "
             f"{avg:.1f} us excluded: other shapes)", "",
             "| counter | per dispatch | per wave | per element |", "|---|---:|---:|---:|"]
    for c in sorted(med):
        pw = med[c] / waves if waves else float("nan")
        lines.append(f"| {c} | {med[c]:.4g} | {pw:.4g} | {med[c] / elems:.4g} |")
    if med.get("SQ_ACTIVE_INST_LDS"):
        lines += ["", f"LDS bank-conflict cycles per active LDS instruction cycle: "
                      f"{med.get('SQ_LDS_BANK_CONFLICT', 0.0) / med['SQ_ACTIVE_INST_LDS']:.4f}"]
    if waves:
        lines += ["", f"Waves per dispatch {waves:.0f} (grid / 64 = {grid / 64:.0f})."]
    gui = med.get("GRBM_GUI_ACTIVE")
    avg_us = bench["roofline"].get("avg_launch_us")
    if gui and avg_us:
        # GRBM_GUI_ACTIVE counts the busy cycles of every XCD the collection
        # covers: over the launch's duration it tells how many XCDs the SQ sums
        # (which are summed over the same units) include
        xcds = gui / (avg_us * 1e-6 * CLOCK_HZ)
        lines += ["", f"Coverage: GRBM_GUI_ACTIVE is {xcds:.2f}x the launch's cycles ({avg_us:.1f} us at "
                      f"{CLOCK_HZ / 1e9:.1f} GHz), i.e. the counters sum over about {round(xcds)} of the 8 XCDs; "
                      f"SQ_BUSY_CYCLES / GRBM_GUI_ACTIVE = {med.get('SQ_BUSY_CYCLES', 0.0) / gui:.2f} "
                      f"(the SQ units per XCD counted).  Full-chip figures per element, scaled by "
                      f"8 / {xcds:.2f}:", ""]
        lines += ["| counter | per element, full chip |", "|---|---:|"]
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS"):
            if c in med:
                lines.append(f"| {c} | {med[c] / elems * 8.0 / xcds:.4g} |")
        if med.get("SQ_WAVE_CYCLES") and med.get("SQ_BUSY_CYCLES"):
            lines += ["", f"SQ_WAVE_CYCLES / SQ_BUSY_CYCLES = {med['SQ_WAVE_CYCLES'] / med['SQ_BUSY_CYCLES']:.2f} "
                          f"(resident waves per counted SQ unit, in the counter's units)."]
    out = {"kernel": key, "kernel_symbol": sym, "grid_threads": grid, "dispatches": n_disp,
           "median_per_dispatch": med, "source_hash": bench.get("source_hash")}
    json.dump(out, open(args.json, "w"), indent=1)
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "traffic", "suite", "counters"])
    ap.add_argument("--pmc")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--bench", required=True)
    ap.add_argument("--bench-write", help="traffic / suite: the JSON of the WRITE_SIZE run, checked against --bench")
    ap.add_argument("--json", default="profiles/traffic.json")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="python3 bench.py")
    args = ap.parse_args(argv)
    {"trace": trace, "traffic": traffic, "suite": suite, "counters": counters}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
